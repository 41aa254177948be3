"""The shift expression's no-allocation entry point
(qdpx_eval_shift_mul_axpy_noalloc) against the workspace entry point: two
calls in a row on different lattices, the second smaller, each compared
field and norm bit for bit with qdpx_eval_shift_mul_axpy (the same kernels
and reduction order) and with the oracle to the stated tolerance; sizes
beyond its fixed scratch memory are refused."""

import numpy as np
import pytest
import torch

import latgen
import oracle
import paper_1105_2279_amd as q
from gpuhelp import FORMAT_IDS, FORMATS, ctx, dev, need_gpu, rel_err, tol

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def both(c, L, U, psi, phi, prec, fmt, mask, sign):
    Ud = q.links_to_device(c, L, U, prec, fmt, dev())
    pd = q.fermion_to_device(c, L, psi, prec, dev())
    fd = q.fermion_to_device(c, L, phi, prec, dev())
    chi_w, chi_n = q.alloc_fermion(L, prec, dev()), q.alloc_fermion(L, prec, dev())
    n_w = torch.zeros(1, dtype=torch.float64, device=dev())
    n_n = torch.full((1,), float("nan"), dtype=torch.float64, device=dev())
    work = q.alloc_workspace(q.OP_SHIFT, L, prec, fmt, 1, dev())
    q.qdpx_eval_shift_mul_axpy(c, L, prec, fmt, Ud, pd, fd, 0.3, chi_w, n_w, work, dir_mask=mask, sign=sign)
    q.qdpx_eval_shift_mul_axpy_noalloc(c, L, prec, fmt, Ud, pd, fd, 0.3, chi_n, n_n, dir_mask=mask, sign=sign)
    torch.cuda.synchronize()
    # the fields on the lattice's sites (the SoA padding is never written)
    return (q.fermion_to_host(c, L, chi_w, prec), q.fermion_to_host(c, L, chi_n, prec), float(n_w.item()),
            float(n_n.item()))


@pytest.mark.parametrize("prec,fmt", FORMATS, ids=FORMAT_IDS)
@pytest.mark.parametrize("mask,sign", [(0xF, 1), (0xB, -1)])
def test_noalloc_matches_workspace_entry_point(prec, fmt, mask, sign):
    c = ctx()
    # the larger lattice first, then a smaller (ragged) one: the second call
    # must not see anything the first left in the scratch memory
    for L, seed in (((16, 16, 16, 32), 61), ((3, 5, 4, 7), 62)):
        U = latgen.haar_links(L, seed)
        psi, phi = latgen.dirac_field(L, seed + 100), latgen.dirac_field(L, seed + 200)
        chi_w, chi_n, n_w, n_n = both(c, L, U, psi, phi, prec, fmt, mask, sign)
        assert np.array_equal(chi_w.view(np.float64), chi_n.view(np.float64))
        assert n_n == n_w, (n_n, n_w)
        ref, n_ref = oracle.shift_expr(U, psi, phi, 0.3, mask, sign)
        assert max(rel_err(chi_n, ref)) < tol(prec)
        assert abs(n_n - n_ref) < tol(prec) * n_ref


def test_noalloc_without_norm_and_size_limit():
    c = ctx()
    L = (8, 8, 8, 8)
    U = latgen.haar_links(L, 63)
    psi = latgen.dirac_field(L, 64)
    Ud = q.links_to_device(c, L, U, q.F64, q.LINK18, dev())
    pd = q.fermion_to_device(c, L, psi, q.F64, dev())
    chi = q.alloc_fermion(L, q.F64, dev())
    q.qdpx_eval_shift_mul_axpy_noalloc(c, L, q.F64, q.LINK18, Ud, pd, None, 0.0, chi)
    ref, _ = oracle.shift_expr(U, psi, None, 0.0)
    assert max(rel_err(q.fermion_to_host(c, L, chi, q.F64), ref)) < 1e-12
    # 2^25 + 1 sites and beyond are refused before anything is launched
    big = (256, 256, 256, 4)
    with pytest.raises(q.QdpxError, match="exceed"):
        q.qdpx_eval_shift_mul_axpy_noalloc(c, big, q.F32, q.LINK12, Ud, pd, None, 0.0, chi)
