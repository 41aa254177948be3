"""GPU parity: every kernel through the C ABI against the FP64 oracle.

Tolerances: FP64 paths 1e-12 (links: max |entry difference|; fields:
normwise and max-abs relative; norms relative; plaquettes absolute), FP32
paths 1e-5 after one step, both compared with the FP64 oracle evaluated on the
same FP64 inputs.
"""

import numpy as np
import pytest
import torch

import latgen
import oracle
import paper_1105_2279_amd as q
from gpuhelp import (FORMAT_IDS, FORMATS, ape, assert_bench_geometry, bench_ctx, chain, ctx, dev, link_err, need_gpu,
                     plaquette, rel_err, shift, su3_defects, tol)
from lathelp import gauge_links, pure_gauge

pytestmark = pytest.mark.gpu

RAGGED = (3, 5, 4, 7)  # V = 420: not a multiple of 64, every extent different


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


# ------------------------------------------------------------ pack / unpack
@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
def test_pack_unpack_roundtrip(prec, fmt):
    U = latgen.haar_links(RAGGED, 3)
    V = q.links_to_host(ctx(), RAGGED, q.links_to_device(ctx(), RAGGED, U, prec, fmt), prec, fmt)
    if prec == q.F64:
        assert np.array_equal(V, U)
    else:
        r = U.real.astype(np.float32).astype(np.float64) + 1j * U.imag.astype(np.float32).astype(np.float64)
        if fmt == q.LINK18:
            assert np.array_equal(V, r)
        else:
            assert np.array_equal(V[..., :2, :], r[..., :2, :])
            assert np.max(np.abs(V[..., 2, :] - U[..., 2, :])) < 1e-6
    psi = latgen.dirac_field(RAGGED, 4)
    P = q.fermion_to_host(ctx(), RAGGED, q.fermion_to_device(ctx(), RAGGED, psi, prec), prec)
    if prec == q.F64:
        assert np.array_equal(P, psi)
    else:
        assert np.max(np.abs(P - psi)) < 1e-6 * np.max(np.abs(psi))


# ------------------------------------------------------- shift expression
@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
@pytest.mark.parametrize("L", [(16, 16, 16, 32), RAGGED, (2, 2, 2, 2)], ids=["16x16x16x32", "ragged", "2^4"])
def test_shift_mul_axpy(prec, fmt, L):
    seeds = latgen.SEEDS["shift_16x16x16x32"]
    U = latgen.haar_links(L, seeds["links"])
    psi, phi = latgen.dirac_field(L, seeds["psi"]), latgen.dirac_field(L, seeds["phi"])
    chi, n2 = shift(L, U, psi, phi, 0.3, prec, fmt)
    ref, n2ref = oracle.shift_mul_axpy(U, psi, phi, 0.3)
    e_norm, e_max = rel_err(chi, ref)
    assert e_norm < tol(prec) and e_max < tol(prec), (e_norm, e_max)
    assert abs(n2 - n2ref) < tol(prec) * n2ref


@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
def test_shift_benched_shape_and_geometry(prec, fmt):
    """The shift expression at 32^3x64 in the stored launch geometry the
    benchmark times, element by element against the oracle."""
    L = (32, 32, 32, 64)
    assert_bench_geometry("SHIFT", q.OP_SHIFT, L, prec, fmt)
    seeds = latgen.SEEDS["shift_16x16x16x32"]
    U = latgen.haar_links(L, seeds["links"])
    psi, phi = latgen.dirac_field(L, seeds["psi"]), latgen.dirac_field(L, seeds["phi"])
    chi, n2 = shift(L, U, psi, phi, 0.3, prec, fmt, context=bench_ctx())
    ref, n2ref = oracle.shift_mul_axpy(U, psi, phi, 0.3)
    e_norm, e_max = rel_err(chi, ref)
    print(f"shift 32^3x64 {prec}/{fmt}: rel {e_norm:.2e} max {e_max:.2e}", flush=True)
    assert e_norm < tol(prec) and e_max < tol(prec), (e_norm, e_max)
    assert abs(n2 - n2ref) < tol(prec) * n2ref


@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
@pytest.mark.parametrize("L", [RAGGED, (16, 8, 4, 8), (2, 6, 2, 6)], ids=["ragged", "16x8x4x8", "2x6x2x6"])
@pytest.mark.parametrize("mask,sign", [(0xF, -1), (0x5, 1), (0x8, -1), (0x6, 1), (0x0, 1)])
def test_shift_direction_mask_and_backward_hop(prec, fmt, L, mask, sign):
    U = latgen.haar_links(L, 31 + mask)
    psi, phi = latgen.dirac_field(L, 32), latgen.dirac_field(L, 33)
    chi, n2 = shift(L, U, psi, phi, 0.3, prec, fmt, mask=mask, sign=sign)
    ref, n2ref = oracle.shift_expr(U, psi, phi, 0.3, mask, sign)
    e_norm, e_max = rel_err(chi, ref)
    assert e_norm < tol(prec) and e_max < tol(prec), (e_norm, e_max)
    assert abs(n2 - n2ref) < tol(prec) * n2ref


def test_forward_plus_backward_shift_is_the_hop():
    """sign +1 plus sign -1 over one mask is the hopping term of qdpx_eval_hop."""
    L = (8, 8, 4, 6)
    U = latgen.haar_links(L, 41)
    psi = latgen.dirac_field(L, 42)
    c = ctx()
    Ud = q.links_to_device(c, L, U, q.F64, q.LINK18, dev())
    pd = q.fermion_to_device(c, L, psi, q.F64, dev())
    f, b, h = (q.alloc_fermion(L, q.F64, dev()) for _ in range(3))
    q.qdpx_eval_shift_mul_axpy(c, L, q.F64, q.LINK18, Ud, pd, None, 0.0, f, dir_mask=0xB, sign=1)
    q.qdpx_eval_shift_mul_axpy(c, L, q.F64, q.LINK18, Ud, pd, None, 0.0, b, dir_mask=0xB, sign=-1)
    q.qdpx_eval_hop(c, L, q.F64, q.LINK18, Ud, pd, h, 0xB)
    fh, bh, hh = (q.fermion_to_host(c, L, t, q.F64) for t in (f, b, h))
    assert max(rel_err(fh + bh, hh)) < 1e-14


def test_shift_rejects_bad_mask_and_sign():
    L = (4, 4, 4, 4)
    c = ctx()
    U = q.alloc_links(L, q.F64, q.LINK18, dev())
    psi, chi = q.alloc_fermion(L, q.F64, dev()), q.alloc_fermion(L, q.F64, dev())
    with pytest.raises(q.QdpxError, match="dir_mask"):
        q.qdpx_eval_shift_mul_axpy(c, L, q.F64, q.LINK18, U, psi, None, 0.3, chi, dir_mask=0x10)
    with pytest.raises(q.QdpxError, match="sign"):
        q.qdpx_eval_shift_mul_axpy(c, L, q.F64, q.LINK18, U, psi, None, 0.3, chi, sign=0)


def test_shift_without_phi():
    L = RAGGED
    U = latgen.haar_links(L, 5)
    psi = latgen.dirac_field(L, 6)
    chi, n2 = shift(L, U, psi, None, 0.3, q.F64, q.LINK18)
    ref, n2ref = oracle.shift_mul_axpy(U, psi, None, 0.3)
    assert max(rel_err(chi, ref)) < 1e-12
    assert abs(n2 - n2ref) < 1e-12 * n2ref


@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
@pytest.mark.parametrize("n", [1, 8])
def test_shift_chain(prec, fmt, n):
    L = (8, 8, 8, 16)
    U = latgen.haar_links(L, 11)
    psi, phi = latgen.dirac_field(L, 12), latgen.dirac_field(L, 13)
    got, norms = chain(L, U, psi, phi, 0.3, 0.1, n, prec, fmt)
    ref, rnorms = oracle.shift_chain(U, psi, phi, 0.3, 0.1, n)
    # FP32 rounding compounds over the iterations; the bound grows with n.
    t = tol(prec) * (1 if prec == q.F64 else max(1, n))
    assert max(rel_err(got, ref)) < t
    assert np.max(np.abs(norms - rnorms) / rnorms) < t


# -------------------------------------------------------------- plaquette
@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
@pytest.mark.parametrize("L", [(4, 4, 4, 4), RAGGED, (8, 8, 8, 16)], ids=["4^4", "ragged", "8^3x16"])
def test_plaquette(prec, fmt, L):
    U = latgen.haar_links(L, 21)
    U = oracle.ape_step(U, 0.5)  # a plaquette away from zero
    got = plaquette(L, U, prec, fmt)
    ref = oracle.plaquette(U)
    assert np.max(np.abs(got - ref)) < tol(prec), (got, ref)


@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
def test_degenerate_w_gives_nan(prec, fmt):
    """Links that vanish on four t slices make W vanish on the links whose
    staples all touch them; the projection then writes NaN at exactly the
    links where the oracle's projection reports a degenerate W, and the
    oracle's value everywhere else."""
    L = (8, 8, 4, 10)
    U = latgen.haar_links(L, 51)
    U[2:6] = 0.0
    W = oracle.ape_w(U, 0.5)
    Vref, nbad = oracle.reunitarise(W)
    assert nbad > 0
    bad = np.isnan(Vref).any(axis=(-1, -2))
    assert np.isnan(Vref[bad]).all()
    V, _ = ape(L, U, prec, fmt, 1, with_plaq=False)
    assert np.array_equal(np.isnan(V).any(axis=(-1, -2)), bad)
    assert np.isnan(V[bad]).all()
    assert link_err(V[~bad], Vref[~bad]) < tol(prec)


@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
def test_step_plaquettes_are_the_fp64_plaquette_of_the_links(prec, fmt):
    """The plaquettes qdpx_ape_smear reports for its input and for every
    step's output are the FP64 plaquette (qdpx_plaquette) of those links:
    the same values bit for bit for FP32 links, to FP64 rounding for FP64
    links (whose per-step traces are fused into the step kernel)."""
    L = (16, 8, 8, 8)
    U = latgen.haar_links(L, 71)
    c = ctx()
    cur = q.links_to_device(c, L, U, prec, fmt, dev())
    work_p = q.alloc_workspace(q.OP_PLAQ, L, prec, fmt, 1, dev())
    n = 3
    full = torch.zeros(3 * (n + 1), dtype=torch.float64, device=dev())
    out = q.alloc_links(L, prec, fmt, dev())
    q.qdpx_ape_smear(c, L, prec, fmt, cur, out, 0.5, n, full, q.alloc_workspace(q.OP_APE, L, prec, fmt, n, dev()))
    ref = []
    for k in range(n + 1):  # plaquette of the input, then of each step's output
        p = torch.zeros(3, dtype=torch.float64, device=dev())
        q.qdpx_plaquette(c, L, prec, fmt, cur, p, work_p)
        ref.append(p)
        if k < n:
            nxt = q.alloc_links(L, prec, fmt, dev())
            q.qdpx_ape_smear(c, L, prec, fmt, cur, nxt, 0.5, 1, None, q.alloc_workspace(q.OP_APE, L, prec, fmt, 1,
                                                                                           dev()))
            cur = nxt
    ref = torch.cat(ref)
    torch.cuda.synchronize()
    if prec == q.F32:
        assert torch.equal(full, ref), (full - ref).abs().max()
    else:
        assert float((full - ref).abs().max()) < 1e-14


def test_plaquette_unit_links_exact():
    L = (4, 4, 4, 8)
    for prec, fmt in FORMATS:
        got = plaquette(L, latgen.unit_links(L), prec, fmt)
        assert np.max(np.abs(got - 1.0)) < 1e-15


# ----------------------------------------------------------------- APE
@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
@pytest.mark.parametrize("L", [(4, 4, 4, 4), RAGGED, (8, 8, 8, 16)], ids=["4^4", "ragged", "8^3x16"])
def test_ape_one_step(prec, fmt, L):
    U = latgen.haar_links(L, latgen.SEEDS["ape_4x4x4x4"]["links"])
    V, plaq = ape(L, U, prec, fmt, 1)
    Vref = oracle.ape_step(U, 0.5)
    assert link_err(V, Vref) < tol(prec)
    assert np.max(np.abs(plaq[0] - oracle.plaquette(U))) < tol(prec)
    assert np.max(np.abs(plaq[1] - oracle.plaquette(Vref))) < tol(prec)
    u, d = su3_defects(V)
    assert u < (1e-14 if prec == q.F64 else 1e-6) and d < (1e-14 if prec == q.F64 else 1e-6)


@pytest.mark.parametrize("n", [2, 3])
def test_ape_multi_step_fp64(n):
    L = (4, 6, 4, 8)
    U = latgen.haar_links(L, 31)
    V, plaq = ape(L, U, q.F64, q.LINK18, n)
    Vk = U
    refs = [oracle.plaquette(U)]
    for _ in range(n):
        Vk = oracle.ape_step(Vk, 0.5)
        refs.append(oracle.plaquette(Vk))
    assert link_err(V, Vk) < 1e-12
    assert np.max(np.abs(plaq - np.array(refs))) < 1e-12
    assert np.all(np.diff(plaq[:, 0]) > 0)


@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
def test_ape_fixed_points(prec, fmt):
    L = (4, 4, 6, 4)
    I = latgen.unit_links(L)
    V, plaq = ape(L, I, prec, fmt, 2)
    assert np.max(np.abs(V - I)) < (1e-15 if prec == q.F64 else 1e-7)
    assert np.max(np.abs(plaq - 1.0)) < (1e-14 if prec == q.F64 else 1e-6)
    U = pure_gauge(latgen.haar_gauge(L, 41))
    V, plaq = ape(L, U, prec, fmt, 1)
    assert np.max(np.abs(V - U)) < (1e-13 if prec == q.F64 else 1e-5)


def test_ape_torus_gauge_covariance():
    L = (4, 4, 4, 6)
    U = latgen.haar_links(L, 51)
    g = latgen.torus_gauge(L, 52)
    V, _ = ape(L, U, q.F64, q.LINK18, 1)
    Vg, _ = ape(L, gauge_links(U, g), q.F64, q.LINK18, 1)
    assert np.max(np.abs(Vg - gauge_links(V, g))) < 1e-13


# --------------------------------------------- bench-size sampled parity
@pytest.fixture(scope="module")
def big_links():
    L = (32, 32, 32, 64)
    return L, latgen.haar_links(L, latgen.SEEDS["ape_32x32x32x64"]["links"])


@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
def test_ape_32x32x32x64_sampled(big_links, prec, fmt):
    """The benchmark's lattice in the launch geometry the benchmark times."""
    L, U = big_links
    assert_bench_geometry("APE", q.OP_APE, L, prec, fmt)
    V, plaq = ape(L, U, prec, fmt, 1, context=bench_ctx())
    rng = np.random.default_rng(99)
    V4 = V.reshape(-1, 4, 3, 3)
    n = 4096
    sites = rng.integers(0, V4.shape[0], n)
    # include the lattice corners and faces (wrap-around)
    sites[:4] = [0, V4.shape[0] - 1, 31, 32 * 32 * 32 * 63]
    mus = rng.integers(0, 4, n)
    ref = oracle.ape_links(U, 0.5, sites, mus)
    assert np.max(np.abs(V4[sites, mus] - ref)) < tol(prec)
    assert abs(plaq[0, 0] - oracle.plaquette(U)[0]) < tol(prec)
    u, d = su3_defects(V4[sites, mus])
    assert u < (1e-14 if prec == q.F64 else 1e-6)


# ------------------------------------------------ tuning and graph replay
@pytest.mark.parametrize("L", [(8, 6, 4, 10), (16, 8, 4, 8)], ids=["linear_groups", "brick_groups"])
def test_geometries_are_bit_identical(L):
    # (8, 6, 4, 10): V = 1920, 64-site groups of consecutive sites and partial
    # last tiles; (16, 8, 4, 8): 16x4 bricks, where the t window and the XCD
    # slab walk reorder groups
    U = latgen.haar_links(L, 61)
    psi, phi = latgen.dirac_field(L, 62), latgen.dirac_field(L, 63)
    c = ctx()
    results_ape, results_shift = [], []
    # the LDS tile of the FP32 step (0 none, 1 own links, 2 own and backward
    # links, 3 also each plane's upper product passed between its two waves,
    # 4 own links and the products)
    # is one more launch choice that must not change a bit
    for block, ns, xcd, tw, lds in [(256, 1, 1, 1, 2), (256, 1, 0, 2, 1), (512, 2, 1, 4, 0), (256, 4, 0, 8, 2),
                                    (256, 2, 2, 1, 0), (512, 1, 2, 1, 1), (512, 2, 2, 1, 2), (256, 1, 1, 1, 3),
                                    (512, 1, 2, 1, 3), (512, 2, 0, 2, 3), (256, 4, 1, 1, 3), (256, 1, 2, 1, 4),
                                    (512, 2, 1, 1, 4)]:
        if L[3] % tw:
            tw = 2
        q.qdpx_tune_set(c, q.OP_APE, L, q.F32, q.LINK12, block, ns, xcd, tw, lds)
        results_ape.append(ape(L, U, q.F32, q.LINK12, 2))
    for block, ns, xcd, tw in [(256, 1, 1, 1), (256, 8, 0, 2), (256, 2, 1, 8), (256, 4, 0, 2), (256, 2, 2, 1)]:
        if L[3] % tw:
            tw = 1
        q.qdpx_tune_set(c, q.OP_SHIFT, L, q.F64, q.LINK18, block, ns, xcd, tw)
        results_shift.append(shift(L, U, psi, phi, 0.3, q.F64, q.LINK18))
    for V, p in results_ape[1:]:
        assert np.array_equal(V, results_ape[0][0]) and np.array_equal(p, results_ape[0][1])
    for chi, n2 in results_shift[1:]:
        assert np.array_equal(chi, results_shift[0][0]) and n2 == results_shift[0][1]
    q.qdpx_tune_set(c, q.OP_APE, L, q.F32, q.LINK12, 256, 1, 1, 1)
    q.qdpx_tune_set(c, q.OP_SHIFT, L, q.F64, q.LINK18, 256, 1, 1, 1)


@pytest.mark.parametrize("fmt", [q.LINK12, q.LINK18], ids=["f32_12", "f32_18"])
@pytest.mark.parametrize("L", [(3, 5, 4, 7), (5, 3, 4, 6), (8, 6, 4, 10)], ids=["V420", "V360", "V1920"])
def test_shared_plane_products_on_ragged_lattices(L, fmt):
    """LDS tiles 3 and 4 (each plane's upper product formed by one wave and
    read by the other through LDS, between block barriers) on lattices whose last
    group is partial or whose group count is odd, so that a 512-thread block
    also holds a group past the end (also with two or four groups per wave):
    the same bits as level 0, and the oracle to 1e-5 after one step."""
    U = latgen.haar_links(L, 77)
    c = q.Context(0)
    res = []
    for block, ns, lds in ((256, 1, 0), (256, 1, 3), (512, 1, 3), (256, 1, 4), (512, 1, 4), (512, 2, 4),
                           (256, 4, 3)):
        q.qdpx_tune_set(c, q.OP_APE, L, q.F32, fmt, block, ns, 0, 1, lds)
        res.append(ape(L, U, q.F32, fmt, 2, context=c))
    for V, p in res[1:]:
        assert np.array_equal(V, res[0][0]) and np.array_equal(p, res[0][1])
    V1, _ = ape(L, U, q.F32, fmt, 1, context=c)
    assert link_err(V1, oracle.ape_step(U, 0.5)) < 1e-5
    c.close()


def test_tuner_picks_a_valid_geometry():
    c = q.Context(0)
    L = (8, 8, 8, 8)
    q.qdpx_tune(c, q.OP_APE, L, q.F32, q.LINK12)
    b, n, x, tw, lds = q.qdpx_tune_get(c, q.OP_APE, L, q.F32, q.LINK12)
    assert b in (256, 512) and n in (1, 2, 4) and x in (0, 1, 2) and tw in (1, 2, 4, 8) and lds in (0, 1, 2, 3, 4)
    q.qdpx_tune(c, q.OP_SHIFT, L, q.F64, q.LINK18)
    b, n, x, tw, lds = q.qdpx_tune_get(c, q.OP_SHIFT, L, q.F64, q.LINK18)
    assert b == 256 and n in (1, 2, 4, 8) and x in (0, 1, 2) and tw in (1, 2, 4, 8) and lds == 0
    c.close()


def test_graph_replay_matches_eager():
    L = (8, 8, 4, 8)
    prec, fmt = q.F32, q.LINK12
    c = ctx()
    U = latgen.haar_links(L, 71)
    Ud = q.links_to_device(c, L, U, prec, fmt, dev())
    out = q.alloc_links(L, prec, fmt, dev())
    plaq = torch.zeros(9, dtype=torch.float64, device=dev())
    work = q.alloc_workspace(q.OP_APE, L, prec, fmt, 2, dev())
    q.qdpx_ape_smear(c, L, prec, fmt, Ud, out, 0.5, 2, plaq, work)
    torch.cuda.synchronize()
    eager_out, eager_plaq = out.clone(), plaq.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        q.qdpx_ape_smear(c, L, prec, fmt, Ud, out, 0.5, 2, plaq, work)
    for _ in range(3):
        out.zero_()
        plaq.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager_out)
        assert torch.equal(plaq, eager_plaq)


def test_capture_rejects_tuning():
    L = (4, 4, 4, 4)
    c = ctx()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    err = None
    with torch.cuda.graph(g, stream=s):
        try:
            q.qdpx_tune(c, q.OP_APE, L, q.F64, q.LINK18, stream=s)
        except q.QdpxError as e:
            err = e
    assert err is not None and err.code == -6


# ------------------------------------------------------------- validation
def test_validation_errors():
    c = ctx()
    L = (4, 4, 4, 4)
    U = q.links_to_device(c, L, latgen.haar_links(L, 1), q.F64, q.LINK18)
    out = q.alloc_links(L, q.F64, q.LINK18)
    small = q.empty_bytes(16)
    work = q.alloc_workspace(q.OP_APE, L, q.F64, q.LINK18, 2)
    with pytest.raises(q.QdpxError) as e:
        q.qdpx_ape_smear(c, L, q.F64, q.LINK18, U, U, 0.5, 1, None, work)
    assert e.value.code == -2  # aliasing
    with pytest.raises(q.QdpxError) as e:
        q.qdpx_ape_smear(c, L, q.F64, q.LINK18, U, out, 0.5, 2, None, small)
    assert e.value.code == -3  # workspace too small
    with pytest.raises(q.QdpxError) as e:
        q.qdpx_ape_smear(c, L, q.F64, q.LINK18, U, out, 0.5, 0, None, work)
    assert e.value.code == -1  # n_steps < 1
    with pytest.raises(q.QdpxError) as e:
        q.qdpx_ape_smear(c, L, q.F64, q.LINK12, U, out, 0.5, 1, None, work)
    assert e.value.code == -5  # LINK12 with FP64
    with pytest.raises(q.QdpxError) as e:
        q.qdpx_ape_smear(c, (1, 4, 4, 4), q.F64, q.LINK18, U, out, 0.5, 1, None, work)
    assert e.value.code == -1
    psi = q.alloc_fermion(L, q.F64)
    with pytest.raises(q.QdpxError) as e:
        q.qdpx_eval_shift_mul_axpy(c, L, q.F64, q.LINK18, U, psi, None, 0.3, psi, None, None)
    assert e.value.code == -2
    with pytest.raises(q.QdpxError) as e:
        q.qdpx_shift_chain(c, L, q.F64, q.LINK18, U, psi, None, 0.3, 0.1, 0, None, work)
    assert e.value.code == -1
    with pytest.raises(q.QdpxError) as e:
        q.qdpx_tune_set(c, q.OP_APE, L, q.F64, q.LINK18, 1024, 1, 1, 1)
    assert e.value.code == -1
    for op, prec, fmt, lds in ((q.OP_APE, q.F32, q.LINK12, 5), (q.OP_APE, q.F64, q.LINK18, 1),
                               (q.OP_SHIFT, q.F32, q.LINK12, 1)):  # LDS tiles only for the FP32 APE step
        with pytest.raises(q.QdpxError) as e:
            q.qdpx_tune_set(c, op, L, prec, fmt, 256, 1, 1, 1, lds)
        assert e.value.code == -1


def test_misaligned_links_rejected():
    """Link fields are accessed 16 bytes at a time: a pointer that is only
    8-byte aligned is refused before anything is launched."""
    c = ctx()
    L = (4, 4, 4, 4)
    for prec, fmt in FORMATS:
        lb = q.qdpx_links_bytes(L, prec, fmt)
        big = q.empty_bytes(2 * lb + 64)
        good, mis = big[:lb], big[lb + 40:2 * lb + 40]  # offset 40 = 8 mod 16
        aos = torch.from_numpy(latgen.haar_links(L, 2).view(np.float64).ravel()).to(dev())
        q.qdpx_pack_links(c, L, aos, prec, fmt, good)
        work = q.alloc_workspace(q.OP_APE, L, prec, fmt, 2)
        wbig = q.empty_bytes(q.qdpx_workspace_bytes(q.OP_APE, L, prec, fmt, 2) + 64)
        for call in (lambda: q.qdpx_pack_links(c, L, aos, prec, fmt, mis),
                     lambda: q.qdpx_ape_smear(c, L, prec, fmt, good, mis, 0.5, 1, None, work),
                     lambda: q.qdpx_ape_smear(c, L, prec, fmt, mis, good, 0.5, 1, None, work),
                     lambda: q.qdpx_ape_smear(c, L, prec, fmt, good, q.alloc_links(L, prec, fmt), 0.5, 2, None,
                                              wbig[8:]),
                     lambda: q.qdpx_plaquette(c, L, prec, fmt, mis, torch.zeros(3, dtype=torch.float64, device=dev()),
                                              work)):
            with pytest.raises(q.QdpxError) as e:
                call()
            assert e.value.code == -1 and "aligned" in str(e.value)
        # Dirac fields: 16-byte aligned (FP32 components are read in pairs)
        fb = q.qdpx_fermion_bytes(L, prec)
        fbig = q.empty_bytes(3 * fb + 64)
        psi, chi = fbig[:fb], fbig[fb + 64:2 * fb + 64]
        off = 8  # aligned to a complex element in either precision, not to 16 bytes
        bad = fbig[2 * fb + 64 + off:3 * fb + 64 + off - 16]
        shift_ws = q.alloc_workspace(q.OP_SHIFT, L, prec, fmt, 1)
        for call in (lambda: q.qdpx_eval_hop(c, L, prec, fmt, good, bad, chi, 0xF),
                     lambda: q.qdpx_eval_hop(c, L, prec, fmt, good, psi, bad, 0xF),
                     lambda: q.qdpx_eval_shift_mul_axpy(c, L, prec, fmt, good, psi, None, 0.3, bad, None, None),
                     lambda: q.qdpx_eval_shift_mul_axpy(c, L, prec, fmt, good, psi, None, 0.3, chi,
                                                        torch.zeros(1, dtype=torch.float64, device=dev()),
                                                        shift_ws[8:])):
            with pytest.raises(q.QdpxError) as e:
                call()
            assert e.value.code == -1 and "aligned" in str(e.value)
    torch.cuda.synchronize()
