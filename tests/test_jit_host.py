"""Run-time compiled expression kernels, host side: the generator accepts the
expression language and rejects malformed input with a reason, and its source
compiles with hipRTC for gfx950 into a code object free of packed FP32
instructions (no GPU needed)."""

import ctypes
import os
import re
import shutil
import subprocess

import pytest

import paper_1105_2279_amd as q

HOP = "(sum 0xF (add (umul m (shift f0 + m)) (shift (uadj m f0) - m)))"
JACOBI = f"(add f1 (scale s0 {HOP}))"


def test_generate_valid_expressions():
    for e, nf, ns in [(HOP, 1, 0), (JACOBI, 2, 1), ("(sub (shift (umul 2 (shift f1 - 0)) + 3) f0)", 2, 0),
                      ("(scale s1 (sum 0x5 (uadj m (shift f0 + m))))", 1, 2)]:
        for prec, fmt in ((q.F64, q.LINK18), (q.F32, q.LINK18), (q.F32, q.LINK12)):
            src = q.jit_generate(e, prec, fmt, nf, ns)
            assert "qdpx_jit_kernel" in src and ("double" in src) == (prec == q.F64 or "(double)" in src)


@pytest.mark.parametrize("e,nf,ns", [(JACOBI, 2, 1), ("(add (shift f0 + 1) (scale s0 f0))", 1, 1),
                                     ("(sub (scale s1 (shift f1 - 2)) (scale s0 (shift f0 + 3)))", 2, 2),
                                     ("(scale s2 (sum 0xF (umul m (shift (scale s1 f0) + m))))", 1, 3)])
def test_generated_locals_never_shadow_parameters(e, nf, ns):
    """Every name the kernel declares in its body differs from its parameter
    names, so a scalar or field argument is never hidden by a local (the
    site index of a shift once took the name of scalar 0)."""
    src = q.jit_generate(e, q.F64, q.LINK18, nf, ns)
    sig = src[src.index("qdpx_jit_kernel("):]
    params = re.findall(r"(\w+)\s*[,)]", sig[:sig.index("{")])
    body = sig[sig.index("{"):]
    assert {"U", "out", "partials"} <= set(params) and len(params) == 8 + nf + ns
    for p in params:
        # a declaration "type p = ...", "type p;" or a continued one ", p = ..."
        decl = rf"(?:\b(?:int|spinor|link|double|cx|real)\s+|,\s*){p}\s*[=;]"
        assert not re.search(decl, body), p
    for k in range(ns):
        assert f"real scal{k}" in sig


@pytest.mark.parametrize("bad", ["(umul m f0)", "(sum 0x10 f0)", "(add f0)", "(shift f0 * 1)", "(scale s3 f0)",
                                 "(sum 0x3 (sum 0x1 f0))", "(add f0 f1) f0", "(frob f0)", "f2", "(umul 4 f0)"])
def test_generate_rejects_malformed(bad):
    with pytest.raises(q.QdpxError) as ei:
        q.jit_generate(bad, q.F64, q.LINK18, 2, 1)
    assert ei.value.code == q.EINVAL


def test_generate_rejects_unsupported_format():
    with pytest.raises(q.QdpxError):
        q.jit_generate(HOP, q.F64, q.LINK12, 1, 0)


def test_source_compiles_with_hiprtc_without_packed_fp32(tmp_path):
    lib = "/opt/rocm/lib/libhiprtc.so"
    objdump = "/opt/rocm/llvm/bin/llvm-objdump"
    if not os.path.exists(lib) or not os.path.exists(objdump):
        pytest.skip("hipRTC or llvm-objdump not installed")
    h = ctypes.CDLL(lib)
    for prec, fmt in ((q.F32, q.LINK12), (q.F64, q.LINK18)):
        src = q.jit_generate(JACOBI, prec, fmt, 2, 1)
        prog = ctypes.c_void_p()
        assert h.hiprtcCreateProgram(ctypes.byref(prog), src.encode(), b"qdpx_jit.hip", 0, None, None) == 0
        opts = [b"-O3", b"-std=c++17", b"-Xclang", b"-target-feature", b"-Xclang", b"-packed-fp32-ops",
                b"--offload-arch=gfx950"]
        assert h.hiprtcCompileProgram(prog, len(opts), (ctypes.c_char_p * len(opts))(*opts)) == 0
        n = ctypes.c_size_t()
        h.hiprtcGetCodeSize(prog, ctypes.byref(n))
        code = ctypes.create_string_buffer(n.value)
        h.hiprtcGetCode(prog, code)
        h.hiprtcDestroyProgram(ctypes.byref(prog))
        co = tmp_path / f"k{prec}.co"
        co.write_bytes(code.raw)
        dis = subprocess.run([objdump, "-d", str(co)], capture_output=True, text=True, check=True).stdout
        assert "v_fma" in dis or "v_fmac" in dis
        assert "v_pk_" not in dis
