"""APE smearing restricted to a subset of directions (smear_mask) on the GPU
against the FP64 oracle: smeared links within the stated tolerances (FP64
1e-12, FP32 1e-5 per step), the other directions copied bit for bit, and the
plaquettes of the separate plaquette pass bit-identical to the fused ones."""

import numpy as np
import pytest
import torch

import latgen
import oracle
import paper_1105_2279_amd as q
from gpuhelp import FORMAT_IDS, FORMATS, ctx, dev, link_err, need_gpu, tol

pytestmark = pytest.mark.gpu

LATTICES = [(4, 4, 4, 4), (3, 5, 4, 7), (16, 8, 4, 8)]


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def run(L, U, prec, fmt, n, mask, with_plaq=True, context=None):
    c = context or ctx()
    Ud = q.links_to_device(c, L, U, prec, fmt, dev())
    out = q.alloc_links(L, prec, fmt, dev())
    plaq = torch.zeros(3 * (n + 1), dtype=torch.float64, device=dev()) if with_plaq else None
    work = q.alloc_workspace(q.OP_APE, L, prec, fmt, n, dev())
    q.qdpx_ape_smear(c, L, prec, fmt, Ud, out, 0.5, n, plaq, work, smear_mask=mask)
    V = q.links_to_host(c, L, out, prec, fmt)
    Uin = q.links_to_host(c, L, Ud, prec, fmt)
    torch.cuda.synchronize()
    return V, Uin, (plaq.cpu().numpy().reshape(-1, 3) if with_plaq else None)


@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
@pytest.mark.parametrize("L", LATTICES, ids=lambda L: "x".join(map(str, L)))
@pytest.mark.parametrize("mask", [0x7, 0x5, 0x1, 0x0])
@pytest.mark.parametrize("n", [1, 2])
def test_masked_ape_matches_oracle(L, prec, fmt, mask, n):
    U = latgen.haar_links(L, 4100 + sum(L))
    V, Uin, plaq = run(L, U, prec, fmt, n, mask)
    ref = oracle.ape_smear(U, 0.5, n, mask)
    assert link_err(V, ref) < n * tol(prec)
    for mu in range(4):
        if not (mask >> mu) & 1:
            # copied through every step: identical to the stored input
            assert np.array_equal(V[..., mu, :, :].view(np.float64), Uin[..., mu, :, :].view(np.float64))
    # plaquettes of the input and of the output
    assert np.max(np.abs(plaq[0] - oracle.plaquette(U))) < tol(prec)
    assert np.max(np.abs(plaq[n] - oracle.plaquette(ref))) < n * tol(prec)  # per step


@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
def test_masked_links_do_not_depend_on_plaquette_request(prec, fmt):
    L = (16, 8, 4, 8)
    U = latgen.haar_links(L, 4200)
    a, _, _ = run(L, U, prec, fmt, 3, 0x7, with_plaq=True)
    b, _, _ = run(L, U, prec, fmt, 3, 0x7, with_plaq=False)
    assert np.array_equal(a.view(np.float64), b.view(np.float64))


@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
def test_plaquette_pass_equals_fused(prec, fmt):
    """The input plaquette with a partial mask (always the plaquette pass)
    equals the full-mask one: bit for bit for FP32 links (the same pass), to
    FP64 rounding for FP64 links (whose full-mask steps fuse it into the step
    kernel through the row identity)."""
    L = (8, 8, 8, 8)
    U = latgen.haar_links(L, 4300)
    _, _, p_masked = run(L, U, prec, fmt, 1, 0x7)
    _, _, p_full = run(L, U, prec, fmt, 1, 0xF)
    if prec == q.F32:
        assert np.array_equal(p_masked[0], p_full[0])
    else:
        assert np.max(np.abs(p_masked[0] - p_full[0])) < 1e-14


def test_full_mask_is_the_default():
    L = (4, 4, 4, 4)
    U = latgen.haar_links(L, 4400)
    a, _, pa = run(L, U, q.F32, q.LINK12, 2, 0xF)
    c = ctx()
    Ud = q.links_to_device(c, L, U, q.F32, q.LINK12, dev())
    out = q.alloc_links(L, q.F32, q.LINK12, dev())
    plaq = torch.zeros(9, dtype=torch.float64, device=dev())
    work = q.alloc_workspace(q.OP_APE, L, q.F32, q.LINK12, 2, dev())
    q.qdpx_ape_smear(c, L, q.F32, q.LINK12, Ud, out, 0.5, 2, plaq, work)
    b = q.links_to_host(c, L, out, q.F32, q.LINK12)
    assert np.array_equal(a.view(np.float64), b.view(np.float64))
    assert np.array_equal(pa.ravel(), plaq.cpu().numpy())


def test_spatial_smearing_32x32x32x64_sampled():
    L = (32, 32, 32, 64)
    U = latgen.haar_links(L, latgen.SEEDS["ape_32x32x32x64"]["links"])
    V, Uin, _ = run(L, U, q.F32, q.LINK12, 1, 0x7, with_plaq=False)
    rng = np.random.default_rng(7)
    sites = rng.integers(0, latgen.volume(L), 4000)
    mus = rng.integers(0, 3, 4000)
    ref = oracle.ape_links(U, 0.5, sites, mus, 0x7)
    got = V.reshape(-1, 4, 3, 3)[sites, mus]
    assert np.max(np.abs(got - ref)) < tol(q.F32)
    assert np.array_equal(V[..., 3, :, :].view(np.float64), Uin[..., 3, :, :].view(np.float64))


def test_mask_validation():
    L = (4, 4, 4, 4)
    c = ctx()
    U = q.links_to_device(c, L, latgen.haar_links(L, 4500), q.F64, q.LINK18, dev())
    out = q.alloc_links(L, q.F64, q.LINK18, dev())
    work = q.alloc_workspace(q.OP_APE, L, q.F64, q.LINK18, 1, dev())
    with pytest.raises(q.QdpxError):
        q.qdpx_ape_smear(c, L, q.F64, q.LINK18, U, out, 0.5, 1, None, work, smear_mask=0x10)


@pytest.mark.parametrize("fmt", [q.LINK12, q.LINK18], ids=["f32_12", "f32_18"])
@pytest.mark.parametrize("mask", [0x7, 0x5])
def test_masked_links_do_not_depend_on_the_lds_tile(fmt, mask):
    """The FP32 step's LDS tile (none, own links, own and backward links,
    and each plane's upper product formed once and passed through LDS)
    changes where links and products come from, never a bit of the result,
    also when only some directions are smeared."""
    L = (16, 8, 4, 8)
    U = latgen.haar_links(L, 4500 + mask)
    c = q.Context(0)
    res = []
    for block, lds in ((256, 0), (256, 1), (256, 2), (256, 3), (512, 3), (256, 4)):
        q.qdpx_tune_set(c, q.OP_APE, L, q.F32, fmt, block, 1, 1, 1, lds)
        res.append(run(L, U, q.F32, fmt, 2, mask, context=c))
    for V, _, p in res[1:]:
        assert np.array_equal(V.view(np.float64), res[0][0].view(np.float64))
        assert np.array_equal(p, res[0][2])
    c.close()
