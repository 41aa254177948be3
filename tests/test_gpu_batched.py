"""GPU tests of the persistent batched APE kernel: bit-identity with the
single-lattice path, parity with the oracle, graph replay, the 64-lattice
batch of uneven extents, and the bounded-wait failure path (forced from the
host with a tiny spin limit, so every wave still exits normally)."""

import os

import numpy as np
import pytest
import torch

import latgen
import oracle
import paper_1105_2279_amd as q
from gpuhelp import ctx, dev, need_gpu

pytestmark = pytest.mark.gpu

MIXED = [(4, 4, 4, 4), (3, 5, 4, 7), (8, 8, 8, 16), (6, 4, 4, 8), (12, 12, 12, 24), (2, 2, 2, 2)]


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def run_single(c, L, Ud, prec, fmt, n):
    out = q.alloc_links(L, prec, fmt, dev())
    plaq = torch.zeros(3 * (n + 1), dtype=torch.float64, device=dev())
    work = q.alloc_workspace(q.OP_APE, L, prec, fmt, n, dev())
    q.qdpx_ape_smear(c, L, prec, fmt, Ud, out, 0.5, n, plaq, work)
    return out, plaq


def run_batched(c, Ls, Uds, prec, fmt, n, work=None, outs=None, plaq=None):
    outs = outs if outs is not None else [q.alloc_links(L, prec, fmt, dev()) for L in Ls]
    plaq = plaq if plaq is not None else torch.zeros(3 * len(Ls), dtype=torch.float64, device=dev())
    work = work if work is not None else q.alloc_workspace(q.OP_BATCHED, Ls, prec, fmt, len(Ls), dev())
    q.qdpx_ape_smear_batched(c, Ls, prec, fmt, Uds, outs, 0.5, n, plaq, work)
    return outs, plaq, work


def same_links(c, L, a, b, prec, fmt):
    """Bitwise equality of the valid entries (the SoA padding is never written)."""
    A = q.links_to_host(c, L, a, prec, fmt)
    B = q.links_to_host(c, L, b, prec, fmt)
    return np.array_equal(A.view(np.float64), B.view(np.float64))


def status_of(work):
    return int(work[4:8].cpu().numpy().view(np.uint32)[0])


@pytest.mark.parametrize("prec,fmt", [(q.F64, q.LINK18), (q.F32, q.LINK12), (q.F32, q.LINK18)],
                         ids=["f64_18", "f32_12", "f32_18"])
@pytest.mark.parametrize("n", [1, 2, 3])
def test_batched_bit_identical_to_single(prec, fmt, n):
    c = ctx()
    Us = [latgen.haar_links(L, 100 + i) for i, L in enumerate(MIXED)]
    Uds = [q.links_to_device(c, L, U, prec, fmt, dev()) for L, U in zip(MIXED, Us)]
    outs, plaq, work = run_batched(c, MIXED, Uds, prec, fmt, n)
    torch.cuda.synchronize()
    assert status_of(work) == 0
    for i, L in enumerate(MIXED):
        o1, p1 = run_single(c, L, Uds[i], prec, fmt, n)
        torch.cuda.synchronize()
        assert same_links(c, L, outs[i], o1, prec, fmt), f"lattice {i} {L}"
        assert torch.equal(plaq[3 * i:3 * i + 3], p1[3 * n:3 * n + 3]), f"lattice {i} {L}"
    # parity of one lattice with the oracle
    V = q.links_to_host(c, MIXED[2], outs[2], prec, fmt)
    Vref = oracle.ape_smear(Us[2], 0.5, n)
    tol = 1e-12 if prec == q.F64 else 1e-5 * n
    assert np.max(np.abs(V - Vref)) < tol
    assert np.max(np.abs(plaq[6:9].cpu().numpy() - oracle.plaquette(Vref))) < tol


@pytest.mark.parametrize("block", [256, 512])
@pytest.mark.parametrize("chunk", [1, 3, 64])
def test_batched_geometry_does_not_change_results(block, chunk):
    c = q.Context(0)
    prec, fmt = q.F32, q.LINK12
    Uds = [q.links_to_device(c, L, latgen.haar_links(L, 200 + i), prec, fmt, dev()) for i, L in enumerate(MIXED)]
    ref_outs, ref_plaq, _ = run_batched(c, MIXED, Uds, prec, fmt, 2)
    q.qdpx_tune_set(c, q.OP_BATCHED, MIXED[0], prec, fmt, block, chunk, 1)
    outs, plaq, work = run_batched(c, MIXED, Uds, prec, fmt, 2)
    torch.cuda.synchronize()
    assert status_of(work) == 0
    for L, a, b in zip(MIXED, outs, ref_outs):
        assert same_links(c, L, a, b, prec, fmt)
    assert torch.equal(plaq, ref_plaq)
    c.close()


@pytest.mark.parametrize("prec,fmt", [(q.F64, q.LINK18), (q.F32, q.LINK12)], ids=["f64_18", "f32_12"])
def test_batched_autotuner(prec, fmt, tmp_path):
    """qdpx_tune_batched picks a geometry on the batch itself, writes it to
    the context's launch table, and the tuned batch gives the same bits."""
    table = str(tmp_path / "table.json")
    c = q.Context(0, tune_cache=table)
    Uds = [q.links_to_device(c, L, latgen.haar_links(L, 250 + i), prec, fmt, dev()) for i, L in enumerate(MIXED)]
    ref_outs, ref_plaq, _ = run_batched(c, MIXED, Uds, prec, fmt, 2)
    q.qdpx_tune_batched(c, MIXED, prec, fmt, 2)
    assert q.qdpx_tune_source(c, q.OP_BATCHED, MIXED[0], prec, fmt) == "tuned"
    block, chunk, _, _, _ = q.qdpx_tune_get(c, q.OP_BATCHED, MIXED[0], prec, fmt)
    assert block in (256, 512) and chunk in (1, 2, 4, 8)
    outs, plaq, work = run_batched(c, MIXED, Uds, prec, fmt, 2)
    torch.cuda.synchronize()
    assert status_of(work) == 0
    for L, a, b in zip(MIXED, outs, ref_outs):
        assert same_links(c, L, a, b, prec, fmt)
    assert torch.equal(plaq, ref_plaq)
    c.close()
    c2 = q.Context(0, tune_cache=table)
    assert q.qdpx_tune_get(c2, q.OP_BATCHED, MIXED[0], prec, fmt) == (block, chunk, 1, 1, 0)
    assert q.qdpx_tune_source(c2, q.OP_BATCHED, MIXED[0], prec, fmt) == "table"
    c2.close()


def test_batched_graph_replay():
    c = ctx()
    prec, fmt = q.F32, q.LINK12
    Ls = MIXED[:4]
    Uds = [q.links_to_device(c, L, latgen.haar_links(L, 300 + i), prec, fmt, dev()) for i, L in enumerate(Ls)]
    outs, plaq, work = run_batched(c, Ls, Uds, prec, fmt, 3)  # eager call builds the device table
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    eager_plaq = plaq.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        q.qdpx_ape_smear_batched(c, Ls, prec, fmt, Uds, outs, 0.5, 3, plaq, work, stream=s)
    for _ in range(3):
        for o in outs:
            o.zero_()
        plaq.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert status_of(work) == 0
        for L, a, b in zip(Ls, outs, eager):
            assert same_links(c, L, a, b, prec, fmt)
        assert torch.equal(plaq, eager_plaq)


def test_batched_first_call_cannot_be_captured():
    c = q.Context(0)
    prec, fmt = q.F32, q.LINK12
    Ls = MIXED[:2]
    Uds = [q.links_to_device(c, L, latgen.haar_links(L, 1), prec, fmt, dev()) for L in Ls]
    outs = [q.alloc_links(L, prec, fmt, dev()) for L in Ls]
    work = q.alloc_workspace(q.OP_BATCHED, Ls, prec, fmt, len(Ls), dev())
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    err = None
    with torch.cuda.graph(g, stream=s):
        try:
            q.qdpx_ape_smear_batched(c, Ls, prec, fmt, Uds, outs, 0.5, 1, None, work, stream=s)
        except q.QdpxError as e:
            err = e
    assert err is not None and err.code == -6
    c.close()


def test_batched_validation():
    c = ctx()
    prec, fmt = q.F32, q.LINK12
    Ls = MIXED[:2]
    Uds = [q.links_to_device(c, L, latgen.haar_links(L, 1), prec, fmt, dev()) for L in Ls]
    work = q.alloc_workspace(q.OP_BATCHED, Ls, prec, fmt, len(Ls), dev())
    with pytest.raises(q.QdpxError) as e:  # output aliases an input of another lattice
        q.qdpx_ape_smear_batched(c, Ls, prec, fmt, Uds, [q.alloc_links(Ls[0], prec, fmt), Uds[0]], 0.5, 1,
                                 None, work)
    assert e.value.code == -2
    with pytest.raises(q.QdpxError) as e:
        q.qdpx_ape_smear_batched(c, Ls, prec, fmt, Uds, [q.alloc_links(L, prec, fmt) for L in Ls], 0.5, 1, None,
                                 work[:100])
    assert e.value.code == -3
    with pytest.raises(q.QdpxError) as e:  # an empty batch
        q.qdpx_ape_smear_batched(c, [], prec, fmt, [], [], 0.5, 1, None, work)
    assert e.value.code == -1 and "n_lat" in str(e.value)
    with pytest.raises(q.QdpxError) as e:  # workspace only 8-byte aligned (it holds intermediate links)
        need = q.qdpx_workspace_bytes(q.OP_BATCHED, Ls, prec, fmt)
        q.qdpx_ape_smear_batched(c, Ls, prec, fmt, Uds, [q.alloc_links(L, prec, fmt) for L in Ls], 0.5, 1, None,
                                 q.empty_bytes(need + 64)[8:])
    assert e.value.code == -1 and "aligned" in str(e.value)
    with pytest.raises(q.QdpxError) as e:
        big = (64, 64, 64, 32)  # beyond the per-lattice limit of the batched kernel
        q.qdpx_workspace_bytes(q.OP_BATCHED, [big], prec, fmt)
        q.qdpx_ape_smear_batched(c, [big], prec, fmt, [Uds[0]], [Uds[1]], 0.5, 1, None, work)
    assert e.value.code in (-5, -3)


def test_batched_timeout_path_reports_and_drains():
    # A zero spin limit makes every wait that is not satisfied at once give up:
    # the kernel must still finish, flag the status word, and leave the library
    # usable for the next call.
    c = q.Context(0)
    prec, fmt = q.F32, q.LINK12
    Ls = [(32, 32, 32, 32)]
    Uds = [q.links_to_device(c, Ls[0], latgen.haar_links(Ls[0], 7), prec, fmt, dev())]
    outs = [q.alloc_links(Ls[0], prec, fmt, dev())]
    work = q.alloc_workspace(q.OP_BATCHED, Ls, prec, fmt, 1, dev())
    old = os.environ.get("QDPX_SPIN_LIMIT")
    os.environ["QDPX_SPIN_LIMIT"] = "0"
    try:
        q.qdpx_ape_smear_batched(c, Ls, prec, fmt, Uds, outs, 0.5, 2, None, work)
        torch.cuda.synchronize()
    finally:
        if old is None:
            del os.environ["QDPX_SPIN_LIMIT"]
        else:
            os.environ["QDPX_SPIN_LIMIT"] = old
    assert status_of(work) == 1
    q.qdpx_ape_smear_batched(c, Ls, prec, fmt, Uds, outs, 0.5, 2, None, work)
    torch.cuda.synchronize()
    assert status_of(work) == 0
    ref, _ = run_single(c, Ls[0], Uds[0], prec, fmt, 2)
    torch.cuda.synchronize()
    assert same_links(c, Ls[0], outs[0], ref, prec, fmt)
    c.close()


def test_batch_of_64_uneven_lattices():
    """The 64-lattice batch (extents drawn from 8^4, 12^3x24, 16^3x32, 24^3x48),
    5 APE steps + final plaquettes, FP32-12: bit-identical to the per-lattice
    launch loop; lattice 0 sampled against the oracle."""
    c = ctx()
    prec, fmt = q.F32, q.LINK12
    Ls = latgen.batch_extents()
    seed0 = latgen.SEEDS["batch_64"]["first_lattice"]
    Uds, host0 = [], None
    for i, L in enumerate(Ls):
        U = latgen.haar_links(L, seed0 + i)
        if i == 0:
            host0 = U
        Uds.append(q.links_to_device(c, L, U, prec, fmt, dev()))
    outs, plaq, work = run_batched(c, Ls, Uds, prec, fmt, 5)
    torch.cuda.synchronize()
    assert status_of(work) == 0
    for i, L in enumerate(Ls):
        o1, p1 = run_single(c, L, Uds[i], prec, fmt, 5)
        torch.cuda.synchronize()
        assert same_links(c, L, outs[i], o1, prec, fmt), i
        assert torch.equal(plaq[3 * i:3 * i + 3], p1[15:18]), i
        del o1, p1
    V = q.links_to_host(c, Ls[0], outs[0], prec, fmt)
    Vref = oracle.ape_smear(host0, 0.5, 5)
    assert np.max(np.abs(V - Vref)) < 5e-5
    p = plaq.cpu().numpy().reshape(-1, 3)
    assert np.all(p[:, 0] > 0.5)  # five steps raise the Haar plaquette far above 0
