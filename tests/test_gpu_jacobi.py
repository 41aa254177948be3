"""Jacobi smearing on the GPU (section 7) against the oracle.

The hopping term H and the smearing iteration are compared element by
element with ``oracle.hop`` / ``oracle.jacobi_smear`` on seeded inputs over
the three link formats, direction masks, a ragged lattice (odd extents, no
brick), a brick lattice and a lattice with a 2-site direction.  At
32^3x64 the whole field is compared after a few iterations, and two
properties that hold at any size are checked on the GPU's own operators:
H is Hermitian, and the truncated series satisfies
K chi_N = s_0 - (kappa H)^{N+1} s_0 with K = 1 - kappa H (section 7)."""

import numpy as np
import pytest
import torch

import latgen
import oracle
import paper_1105_2279_amd as q
from gpuhelp import FORMAT_IDS, FORMATS, assert_bench_geometry, bench_ctx, ctx, dev, need_gpu, rel_err, tol

pytestmark = pytest.mark.gpu

LATTICES = [(4, 4, 4, 4), (3, 5, 4, 7), (16, 8, 4, 8), (2, 6, 2, 6)]
KAPPA = 0.21


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _inputs(L, seed):
    return latgen.haar_links(L, seed), latgen.dirac_field(L, seed + 1)


def gpu_hop(L, U, psi, prec, fmt, mask):
    c = ctx()
    Ud = q.links_to_device(c, L, U, prec, fmt, dev())
    pd = q.fermion_to_device(c, L, psi, prec, dev())
    out = q.alloc_fermion(L, prec, dev())
    q.qdpx_eval_hop(c, L, prec, fmt, Ud, pd, out, mask)
    return q.fermion_to_host(c, L, out, prec)


def gpu_jacobi(L, U, chi, prec, fmt, kappa, n, norm, mask, context=None):
    c = context or ctx()
    Ud = q.links_to_device(c, L, U, prec, fmt, dev())
    cd = q.fermion_to_device(c, L, chi, prec, dev())
    work = q.alloc_workspace(q.OP_JACOBI, L, prec, fmt, n, dev())
    q.qdpx_jacobi_smear(c, L, prec, fmt, Ud, cd, kappa, n, norm, mask, work)
    return q.fermion_to_host(c, L, cd, prec)


@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
@pytest.mark.parametrize("L", LATTICES, ids=lambda L: "x".join(map(str, L)))
@pytest.mark.parametrize("mask", [0xF, 0x7, 0x8, 0x5])
def test_hop_matches_oracle(L, prec, fmt, mask):
    U, psi = _inputs(L, 2100 + sum(L))
    got = gpu_hop(L, U, psi, prec, fmt, mask)
    ref = oracle.hop(U, psi, mask)
    nrm, mx = rel_err(got, ref)
    assert nrm < tol(prec) and mx < tol(prec), (nrm, mx)


def test_hop_empty_mask_is_zero():
    L = (4, 4, 4, 4)
    U, psi = _inputs(L, 2200)
    got = gpu_hop(L, U, psi, q.F64, q.LINK18, 0)
    assert np.all(got == 0)


@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
@pytest.mark.parametrize("L", LATTICES, ids=lambda L: "x".join(map(str, L)))
@pytest.mark.parametrize("n,norm,mask", [(1, 1.0, 0xF), (2, 3.5, 0x7), (5, 0.75, 0xF)])
def test_jacobi_matches_oracle(L, prec, fmt, n, norm, mask):
    U, chi = _inputs(L, 2300 + sum(L))
    got = gpu_jacobi(L, U, chi, prec, fmt, KAPPA, n, norm, mask)
    ref = oracle.jacobi_smear(U, chi, KAPPA, n, norm, mask)
    nrm, mx = rel_err(got, ref)
    # Each iteration adds at most one rounding of a 48-term sum per component:
    # the stated one-application tolerance per iteration.
    assert nrm < n * tol(prec) and mx < n * tol(prec), (nrm, mx)


@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
def test_jacobi_full_lattice_32x32x32x64(prec, fmt):
    L = (32, 32, 32, 64)
    assert_bench_geometry("JACOBI", q.OP_JACOBI, L, prec, fmt)  # the geometry the benchmark times
    U, chi = _inputs(L, 2400)
    n = 3
    got = gpu_jacobi(L, U, chi, prec, fmt, KAPPA, n, 2.0, 0x7, context=bench_ctx())
    ref = oracle.jacobi_smear(U, chi, KAPPA, n, 2.0, 0x7)
    nrm, mx = rel_err(got, ref)
    print(f"32^3x64 {prec}/{fmt}: rel {nrm:.2e} max {mx:.2e}", flush=True)
    assert nrm < n * tol(prec) and mx < n * tol(prec), (nrm, mx)  # per iteration


def test_hop_is_hermitian_on_gpu():
    """<phi, H psi> = <H phi, psi> for the GPU's own H at 32^3x64 in FP64."""
    L = (32, 32, 32, 64)
    U = latgen.haar_links(L, 2500)
    psi, phi = latgen.dirac_field(L, 2501), latgen.dirac_field(L, 2502)
    c = ctx()
    Ud = q.links_to_device(c, L, U, q.F64, q.LINK18, dev())
    pd = q.fermion_to_device(c, L, psi, q.F64, dev())
    fd = q.fermion_to_device(c, L, phi, q.F64, dev())
    hp, hf = q.alloc_fermion(L, q.F64, dev()), q.alloc_fermion(L, q.F64, dev())
    q.qdpx_eval_hop(c, L, q.F64, q.LINK18, Ud, pd, hp, 0xF)
    q.qdpx_eval_hop(c, L, q.F64, q.LINK18, Ud, fd, hf, 0xF)
    Hpsi, Hphi = q.fermion_to_host(c, L, hp, q.F64), q.fermion_to_host(c, L, hf, q.F64)
    a = np.vdot(phi.ravel(), Hpsi.ravel())
    b = np.vdot(Hphi.ravel(), psi.ravel())
    scale = np.linalg.norm(phi) * np.linalg.norm(Hpsi)
    assert abs(a - b) < 1e-12 * scale, (a, b)


def test_truncated_series_identity_on_gpu():
    """K chi_N = s_0 - (kappa H)^{N+1} s_0, all operators on the GPU (FP64)."""
    L = (24, 24, 24, 48)
    U, s0 = _inputs(L, 2600)
    n = 6
    c = ctx()
    prec, fmt = q.F64, q.LINK18
    Ud = q.links_to_device(c, L, U, prec, fmt, dev())
    chi = q.fermion_to_device(c, L, s0, prec, dev())
    work = q.alloc_workspace(q.OP_JACOBI, L, prec, fmt, n, dev())
    q.qdpx_jacobi_smear(c, L, prec, fmt, Ud, chi, KAPPA, n, 1.0, 0xF, work)
    h = q.alloc_fermion(L, prec, dev())
    q.qdpx_eval_hop(c, L, prec, fmt, Ud, chi, h, 0xF)
    chiN = q.fermion_to_host(c, L, chi, prec)
    lhs = chiN - KAPPA * q.fermion_to_host(c, L, h, prec)
    p = q.fermion_to_device(c, L, s0, prec, dev())
    t = q.alloc_fermion(L, prec, dev())
    for _ in range(n + 1):
        q.qdpx_eval_hop(c, L, prec, fmt, Ud, p, t, 0xF)
        p, t = t, p
    tail = KAPPA ** (n + 1) * q.fermion_to_host(c, L, p, prec)
    rhs = s0 - tail
    nrm, _ = rel_err(lhs, rhs)
    assert nrm < 1e-13, nrm
    assert np.linalg.norm(tail) > 1e-3 * np.linalg.norm(s0)  # the tail is not negligible


def test_jacobi_launch_geometry_bit_identical():
    """Every launch geometry computes each site identically."""
    L = (16, 8, 4, 8)
    U, chi = _inputs(L, 2700)
    c = q.Context(0)
    prec, fmt = q.F32, q.LINK12
    outs = []
    for cfg in [(256, 1, 0, 1), (256, 2, 1, 1), (256, 4, 1, 2), (256, 1, 1, 4), (256, 1, 2, 1), (256, 8, 0, 8)]:
        q.qdpx_tune_set(c, q.OP_JACOBI, L, prec, fmt, *cfg)
        Ud = q.links_to_device(c, L, U, prec, fmt, dev())
        cd = q.fermion_to_device(c, L, chi, prec, dev())
        work = q.alloc_workspace(q.OP_JACOBI, L, prec, fmt, 3, dev())
        q.qdpx_jacobi_smear(c, L, prec, fmt, Ud, cd, KAPPA, 3, 1.5, 0xF, work)
        outs.append(q.fermion_to_host(c, L, cd, prec))
    for o in outs[1:]:
        assert np.array_equal(o.view(np.float64), outs[0].view(np.float64))


def test_jacobi_tune_and_graph_replay():
    L = (16, 16, 16, 32)
    U, chi = _inputs(L, 2800)
    c = q.Context(0)
    prec, fmt = q.F32, q.LINK12
    q.qdpx_tune(c, q.OP_JACOBI, L, prec, fmt)
    cfg = q.qdpx_tune_get(c, q.OP_JACOBI, L, prec, fmt)
    assert cfg[0] == 256
    Ud = q.links_to_device(c, L, U, prec, fmt, dev())
    base = q.fermion_to_device(c, L, chi, prec, dev())
    cd = base.clone()
    work = q.alloc_workspace(q.OP_JACOBI, L, prec, fmt, 4, dev())
    eager = cd.clone()
    q.qdpx_jacobi_smear(c, L, prec, fmt, Ud, eager, KAPPA, 4, 2.0, 0xF, work)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            q.qdpx_jacobi_smear(c, L, prec, fmt, Ud, cd, KAPPA, 4, 2.0, 0xF, work, stream=s)
    for _ in range(3):
        cd.copy_(base)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(cd, eager)


def test_jacobi_validation_errors():
    L = (4, 4, 4, 4)
    c = ctx()
    prec, fmt = q.F64, q.LINK18
    U, chi = _inputs(L, 2900)
    Ud = q.links_to_device(c, L, U, prec, fmt, dev())
    cd = q.fermion_to_device(c, L, chi, prec, dev())
    work = q.alloc_workspace(q.OP_JACOBI, L, prec, fmt, 1, dev())
    with pytest.raises(q.QdpxError):
        q.qdpx_jacobi_smear(c, L, prec, fmt, Ud, cd, KAPPA, 0, 1.0, 0xF, work)
    with pytest.raises(q.QdpxError):
        q.qdpx_jacobi_smear(c, L, prec, fmt, Ud, cd, KAPPA, 1, 0.0, 0xF, work)
    with pytest.raises(q.QdpxError):
        q.qdpx_jacobi_smear(c, L, prec, fmt, Ud, cd, KAPPA, 1, 1.0, 0x1F, work)
    with pytest.raises(q.QdpxError):
        q.qdpx_jacobi_smear(c, L, prec, fmt, Ud, cd, KAPPA, 1, 1.0, 0xF, work[: work.numel() // 2])
    with pytest.raises(q.QdpxError):
        q.qdpx_eval_hop(c, L, prec, fmt, Ud, cd, cd, 0xF)  # out aliases psi
    # Nothing above launched: chi is untouched.
    assert np.array_equal(q.fermion_to_host(c, L, cd, prec), chi)
