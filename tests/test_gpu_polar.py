"""APE smearing with the bi-covariant (polar) projection on the GPU against
the FP64 oracle, and the property that motivates it: the whole smearing step
commutes with a random SU(3) gauge transformation, checked on the GPU's own
output (FP64 to 1e-12)."""

import numpy as np
import pytest
import torch

import latgen
import oracle
import paper_1105_2279_amd as q
from gpuhelp import FORMAT_IDS, FORMATS, ctx, dev, link_err, need_gpu, su3_defects, tol
from lathelp import gauge_links

pytestmark = pytest.mark.gpu

LATTICES = [(4, 4, 4, 4), (3, 5, 4, 7), (16, 8, 4, 8)]


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def run(L, U, prec, fmt, n, mask=0xF, with_plaq=True):
    c = ctx()
    Ud = q.links_to_device(c, L, U, prec, fmt, dev())
    out = q.alloc_links(L, prec, fmt, dev())
    plaq = torch.zeros(3 * (n + 1), dtype=torch.float64, device=dev()) if with_plaq else None
    work = q.alloc_workspace(q.OP_APE, L, prec, fmt, n, dev())
    q.qdpx_ape_smear(c, L, prec, fmt, Ud, out, 0.5, n, plaq, work, smear_mask=mask, projection=q.PROJ_POLAR)
    V = q.links_to_host(c, L, out, prec, fmt)
    torch.cuda.synchronize()
    return V, (plaq.cpu().numpy().reshape(-1, 3) if with_plaq else None)


@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
@pytest.mark.parametrize("L", LATTICES, ids=lambda L: "x".join(map(str, L)))
@pytest.mark.parametrize("mask,n", [(0xF, 1), (0xF, 2), (0x7, 1)])
def test_polar_matches_oracle(L, prec, fmt, mask, n):
    U = latgen.haar_links(L, 5100 + sum(L))
    V, plaq = run(L, U, prec, fmt, n, mask)
    ref = oracle.ape_smear(U, 0.5, n, mask, proj=1)
    assert link_err(V, ref) < n * tol(prec)
    u, d = su3_defects(V.reshape(-1, 3, 3))
    assert u < (1e-13 if prec == q.F64 else 1e-6) and d < (1e-13 if prec == q.F64 else 1e-6)
    assert np.max(np.abs(plaq[0] - oracle.plaquette(U))) < tol(prec)
    assert np.max(np.abs(plaq[n] - oracle.plaquette(ref))) < n * tol(prec)  # per step


def test_polar_step_commutes_with_haar_gauge_transformation():
    L = (16, 16, 16, 32)
    U = latgen.haar_links(L, 5200)
    g = latgen.haar_gauge(L, 5201)
    V, _ = run(L, U, q.F64, q.LINK18, 1, with_plaq=False)
    Vg, _ = run(L, gauge_links(U, g), q.F64, q.LINK18, 1, with_plaq=False)
    err = link_err(Vg, gauge_links(V, g))
    print(f"max |V[gU] - g V[U] g^dag| = {err:.2e}", flush=True)
    assert err < 1e-12


def test_polar_fixed_point_unit_links():
    L = (8, 8, 4, 8)
    U = latgen.unit_links(L)
    for prec, fmt in FORMATS:
        V, plaq = run(L, U, prec, fmt, 3)
        assert link_err(V, U) < (1e-14 if prec == q.F64 else 1e-7)
        assert np.max(np.abs(plaq - 1.0)) < 1e-7


def test_polar_32x32x32x64_sampled():
    L = (32, 32, 32, 64)
    U = latgen.haar_links(L, latgen.SEEDS["ape_32x32x32x64"]["links"])
    V, _ = run(L, U, q.F32, q.LINK12, 1, with_plaq=False)
    rng = np.random.default_rng(8)
    sites = rng.integers(0, latgen.volume(L), 3000)
    mus = rng.integers(0, 4, 3000)
    ref = oracle.ape_links(U, 0.5, sites, mus, proj=1)
    got = V.reshape(-1, 4, 3, 3)[sites, mus]
    assert np.max(np.abs(got - ref)) < tol(q.F32)


def test_projection_validation():
    L = (4, 4, 4, 4)
    c = ctx()
    U = q.links_to_device(c, L, latgen.haar_links(L, 5300), q.F64, q.LINK18, dev())
    out = q.alloc_links(L, q.F64, q.LINK18, dev())
    work = q.alloc_workspace(q.OP_APE, L, q.F64, q.LINK18, 1, dev())
    with pytest.raises(q.QdpxError):
        q.qdpx_ape_smear(c, L, q.F64, q.LINK18, U, out, 0.5, 1, None, work, projection=2)
