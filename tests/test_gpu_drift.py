"""Ten APE steps on the 32^3x64 lattice: FP32-12 (and FP64) GPU path against
the FP64 oracle step by step.  Reports per iteration the largest entry
difference and the largest unitarity defect; bounds them at the stated
tolerances (FP64 1e-12 at every step; FP32 1e-5 after one step and a drift
bound of 1e-5 per step)."""

import numpy as np
import pytest
import torch

import latgen
import oracle
import paper_1105_2279_amd as q
from gpuhelp import assert_bench_geometry, bench_ctx, dev, need_gpu, su3_defects

pytestmark = pytest.mark.gpu

L = (32, 32, 32, 64)
N = 10


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def test_ten_steps_step_by_step_against_oracle():
    c = bench_ctx()  # the launch geometry the benchmark times
    for prec, fmt in ((q.F64, q.LINK18), (q.F32, q.LINK12)):
        assert_bench_geometry("APE", q.OP_APE, L, prec, fmt)
    U = latgen.haar_links(L, latgen.SEEDS["ape_32x32x32x64"]["links"])
    cur = {fmt: q.links_to_device(c, L, U, prec, fmt, dev()) for prec, fmt in ((q.F64, q.LINK18), (q.F32, q.LINK12))}
    prec_of = {q.LINK18: q.F64, q.LINK12: q.F32}
    work = {fmt: q.alloc_workspace(q.OP_APE, L, prec_of[fmt], fmt, 1, dev()) for fmt in cur}
    ref = U
    rows = []
    for k in range(1, N + 1):
        ref = oracle.ape_step(ref, 0.5)
        errs = {}
        for fmt in cur:
            prec = prec_of[fmt]
            out = q.alloc_links(L, prec, fmt, dev())
            q.qdpx_ape_smear(c, L, prec, fmt, cur[fmt], out, 0.5, 1, None, work[fmt])
            cur[fmt] = out
            V = q.links_to_host(c, L, out, prec, fmt)
            d = float(np.max(np.abs(V - ref)))
            u, _ = su3_defects(V.reshape(-1, 3, 3)[:: 97])  # every 97th link
            errs[fmt] = (d, u)
        rows.append((k, errs[q.LINK18], errs[q.LINK12]))
        print(f"step {k}: fp64 max|dV| {errs[q.LINK18][0]:.2e} defect {errs[q.LINK18][1]:.2e}; "
              f"fp32-12 max|dV| {errs[q.LINK12][0]:.2e} defect {errs[q.LINK12][1]:.2e}", flush=True)
        assert errs[q.LINK18][0] < 1e-12
        assert errs[q.LINK12][0] < 1e-5 * k
        assert errs[q.LINK12][1] < 1e-6
    torch.cuda.synchronize()


def test_n_steps_call_equals_chained_single_steps():
    c = bench_ctx()
    Ls = (16, 16, 16, 32)
    U = latgen.haar_links(Ls, 77)
    prec, fmt = q.F32, q.LINK12
    Ud = q.links_to_device(c, Ls, U, prec, fmt, dev())
    out = q.alloc_links(Ls, prec, fmt, dev())
    work = q.alloc_workspace(q.OP_APE, Ls, prec, fmt, 4, dev())
    q.qdpx_ape_smear(c, Ls, prec, fmt, Ud, out, 0.5, 4, None, work)
    cur = Ud
    for _ in range(4):
        nxt = q.alloc_links(Ls, prec, fmt, dev())
        q.qdpx_ape_smear(c, Ls, prec, fmt, cur, nxt, 0.5, 1, None, work)
        cur = nxt
    a = q.links_to_host(c, Ls, out, prec, fmt)
    b = q.links_to_host(c, Ls, cur, prec, fmt)
    assert np.array_equal(a.view(np.float64), b.view(np.float64))
