"""Helpers for the GPU parity tests: run the library through its C ABI on
seeded inputs and bring results back in the canonical complex128 layout."""

import numpy as np
import pytest
import torch

import paper_1105_2279_amd as q

FORMATS = [(q.F64, q.LINK18), (q.F32, q.LINK18), (q.F32, q.LINK12)]
FORMAT_IDS = ["f64_18", "f32_18", "f32_12"]

TOL_F64 = 1e-12  # links: max |entry difference|; fields: relative
TOL_F32 = 1e-5


def tol(prec):
    return TOL_F64 if prec == q.F64 else TOL_F32


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_ctx = None


def ctx():
    global _ctx
    if _ctx is None:
        _ctx = q.Context(0)
    return _ctx


_bench_ctx = None


def bench_ctx():
    """A context holding the stored launch table: the geometries bench.py times."""
    global _bench_ctx
    if _bench_ctx is None:
        from paper_1105_2279_amd import tuning

        _bench_ctx = tuning.context(0)
    return _bench_ctx


FMT_NAMES = {(q.F64, q.LINK18): ("F64", "LINK18"), (q.F32, q.LINK18): ("F32", "LINK18"),
             (q.F32, q.LINK12): ("F32", "LINK12")}


def assert_bench_geometry(op_name, op, L, prec, fmt):
    """The geometry bench_ctx() launches for this shape is the stored one."""
    from paper_1105_2279_amd import tuning

    stored = tuning.read()[(op_name, *FMT_NAMES[(prec, fmt)], tuple(L))]
    assert q.qdpx_tune_get(bench_ctx(), op, L, prec, fmt) == stored
    assert q.qdpx_tune_source(bench_ctx(), op, L, prec, fmt) == "table"


def dev():
    return torch.device("cuda:0")


def ape(L, U, prec, fmt, n_steps, alpha=0.5, with_plaq=True, context=None):
    c = context or ctx()
    Ud = q.links_to_device(c, L, U, prec, fmt, dev())
    out = q.alloc_links(L, prec, fmt, dev())
    plaq = torch.zeros(3 * (n_steps + 1), dtype=torch.float64, device=dev()) if with_plaq else None
    work = q.alloc_workspace(q.OP_APE, L, prec, fmt, n_steps, dev())
    q.qdpx_ape_smear(c, L, prec, fmt, Ud, out, alpha, n_steps, plaq, work)
    V = q.links_to_host(c, L, out, prec, fmt)
    torch.cuda.synchronize()
    return V, (plaq.cpu().numpy().reshape(-1, 3) if with_plaq else None)


def plaquette(L, U, prec, fmt):
    c = ctx()
    Ud = q.links_to_device(c, L, U, prec, fmt, dev())
    plaq = torch.zeros(3, dtype=torch.float64, device=dev())
    work = q.alloc_workspace(q.OP_PLAQ, L, prec, fmt, 1, dev())
    q.qdpx_plaquette(c, L, prec, fmt, Ud, plaq, work)
    return plaq.cpu().numpy()


def shift(L, U, psi, phi, a, prec, fmt, mask=0xF, sign=1, context=None):
    c = context or ctx()
    Ud = q.links_to_device(c, L, U, prec, fmt, dev())
    pd = q.fermion_to_device(c, L, psi, prec, dev())
    fd = q.fermion_to_device(c, L, phi, prec, dev()) if phi is not None else None
    chi = q.alloc_fermion(L, prec, dev())
    n2 = torch.zeros(1, dtype=torch.float64, device=dev())
    work = q.alloc_workspace(q.OP_SHIFT, L, prec, fmt, 1, dev())
    q.qdpx_eval_shift_mul_axpy(c, L, prec, fmt, Ud, pd, fd, a, chi, n2, work, dir_mask=mask, sign=sign)
    return q.fermion_to_host(c, L, chi, prec), float(n2.item())


def chain(L, U, psi, phi, a, cc, n, prec, fmt):
    c = ctx()
    Ud = q.links_to_device(c, L, U, prec, fmt, dev())
    pd = q.fermion_to_device(c, L, psi, prec, dev())
    fd = q.fermion_to_device(c, L, phi, prec, dev()) if phi is not None else None
    norms = torch.zeros(n, dtype=torch.float64, device=dev())
    work = q.alloc_workspace(q.OP_CHAIN, L, prec, fmt, n, dev())
    q.qdpx_shift_chain(c, L, prec, fmt, Ud, pd, fd, a, cc, n, norms, work)
    return q.fermion_to_host(c, L, pd, prec), norms.cpu().numpy()


def rel_err(x, ref):
    """(normwise relative error, max-abs error / max |ref|)."""
    d = x - ref
    return (float(np.linalg.norm(d.ravel()) / np.linalg.norm(ref.ravel())),
            float(np.max(np.abs(d)) / np.max(np.abs(ref))))


def link_err(V, Vref):
    return float(np.max(np.abs(V - Vref)))


def su3_defects(V):
    eye = np.eye(3)
    d = np.conj(np.swapaxes(V, -1, -2)) @ V - eye
    u = float(np.max(np.sqrt(np.sum(np.abs(d) ** 2, axis=(-1, -2)))))
    det = float(np.max(np.abs(np.linalg.det(V) - 1.0)))
    return u, det
