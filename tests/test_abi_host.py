"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, sizes follow the documented layout and invalid arguments return a
status code with a message.  No kernel runs here."""

import ctypes
import os
import re

import pytest

import paper_1105_2279_amd as q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "qdpx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qdpx_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 20
    h = q.lib()
    for n in names:
        assert hasattr(h, n), n
    assert sorted(q.EXPORTS) == names


def test_version():
    assert "gfx950" in q.qdpx_version()


def test_sizes_follow_layout():
    L = (4, 4, 4, 4)
    assert q.qdpx_site_stride(L) == 256
    assert q.qdpx_site_stride((3, 5, 4, 7)) == 512  # 420 rounded up to 256
    assert q.qdpx_links_bytes(L, q.F64, q.LINK18) == 256 * 4 * 9 * 16
    assert q.qdpx_links_bytes(L, q.F32, q.LINK18) == 256 * 4 * 9 * 8
    assert q.qdpx_links_bytes(L, q.F32, q.LINK12) == 256 * 4 * 6 * 8
    assert q.qdpx_fermion_bytes(L, q.F64) == 256 * 12 * 16
    assert q.qdpx_fermion_bytes(L, q.F32) == 256 * 12 * 8
    big = (48, 48, 48, 96)
    assert q.qdpx_links_bytes(big, q.F64, q.LINK18) == 10616832 * 4 * 9 * 16  # > 2^32 bytes


def test_workspace_sizes():
    L = (16, 16, 16, 32)
    for op in (q.OP_SHIFT, q.OP_PLAQ):
        assert q.qdpx_workspace_bytes(op, L, q.F64, q.LINK18) > 0
    one = q.qdpx_workspace_bytes(q.OP_APE, L, q.F32, q.LINK12, 1)
    two = q.qdpx_workspace_bytes(q.OP_APE, L, q.F32, q.LINK12, 2)
    assert two - one >= q.qdpx_links_bytes(L, q.F32, q.LINK12)
    assert q.qdpx_workspace_bytes(q.OP_CHAIN, L, q.F64, q.LINK18, 8) >= q.qdpx_fermion_bytes(L, q.F64)


@pytest.mark.parametrize("L", [(1, 4, 4, 4), (4, 4, 4, 4097), (4096, 4096, 4096, 2), (512, 512, 512, 2)])
def test_invalid_extents(L):
    assert q.qdpx_links_bytes(L, q.F64, q.LINK18) == 0
    assert q.lib().qdpx_last_error().decode()
    assert q.qdpx_site_stride(L) == -1


def test_link12_needs_fp32():
    assert q.qdpx_links_bytes((4, 4, 4, 4), q.F64, q.LINK12) == 0
    assert "LINK12" in q.lib().qdpx_last_error().decode()


def test_null_context_rejected_everywhere():
    h = q.lib()
    g = ctypes.byref(q.geom((4, 4, 4, 4)))
    EINVAL = -1
    assert h.qdpx_pack_links(None, g, 1, 0, 0, 2, None) == EINVAL
    assert h.qdpx_unpack_links(None, g, 1, 0, 0, 2, None) == EINVAL
    assert h.qdpx_pack_fermion(None, g, 1, 0, 2, None) == EINVAL
    assert h.qdpx_unpack_fermion(None, g, 1, 0, 2, None) == EINVAL
    assert h.qdpx_eval_shift_mul_axpy(None, g, 0, 0, 1, 2, 3, 0.3, 0xF, 1, 4, None, None, 0, None) == EINVAL
    assert h.qdpx_shift_chain(None, g, 0, 0, 1, 2, 3, 0.3, 0.1, 8, None, None, 0, None) == EINVAL
    assert h.qdpx_ape_smear(None, g, 0, 0, 1, 2, 0.5, 1, 0xF, 0, None, None, 0, None) == EINVAL
    assert h.qdpx_plaquette(None, g, 0, 0, 1, 2, 3, 0, None) == EINVAL
    assert h.qdpx_free_all(None) == EINVAL
    assert h.qdpx_tune_save(None, None) == EINVAL
    assert h.qdpx_create(None, 0, None) == EINVAL
    assert "NULL" in h.qdpx_last_error().decode()
    assert h.qdpx_destroy(None) == 0


def test_python_binding_raises_on_status():
    with pytest.raises(q.QdpxError) as ei:
        q._check(-1, "qdpx_demo")
    assert "QDPX_EINVAL" in str(ei.value)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without libqdpx.so the binding raises instead of falling back to
    anything else."""
    monkeypatch.setattr(q, "_lib", None)
    monkeypatch.setattr(q, "LIB_PATH", str(tmp_path / "libqdpx.so"))
    with pytest.raises(ImportError, match="no fallback"):
        q.lib()
