"""Python binding of the qdpx HIP library (``libqdpx.so``, C ABI in ``include/qdpx.h``).

Argument marshalling only: every function below passes device pointers of
torch tensors, sizes and the current HIP stream to the C entry point of the
same name, and raises :class:`QdpxError` on a non-zero status.  Every step of
the computation runs in the library's HIP kernels; there is no other code
path, and importing this package fails loudly when the library is missing.
"""

from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqdpx.so")

F64, F32 = 0, 1
LINK18, LINK12 = 0, 1
OP_SHIFT, OP_CHAIN, OP_APE, OP_PLAQ, OP_BATCHED, OP_JACOBI = 0, 1, 2, 3, 4, 5
PROJ_GRAM_SCHMIDT, PROJ_POLAR = 0, 1
OK, EINVAL, EALIAS, ENOMEM, EHIP, EUNSUPPORTED, ECAPTURE = 0, -1, -2, -3, -4, -5, -6

STATUS = {
    0: "QDPX_OK",
    -1: "QDPX_EINVAL",
    -2: "QDPX_EALIAS",
    -3: "QDPX_ENOMEM",
    -4: "QDPX_EHIP",
    -5: "QDPX_EUNSUPPORTED",
    -6: "QDPX_ECAPTURE",
}

# Every symbol declared in include/qdpx.h.
EXPORTS = (
    "qdpx_create", "qdpx_destroy", "qdpx_free_all", "qdpx_last_error", "qdpx_version",
    "qdpx_site_stride", "qdpx_links_bytes", "qdpx_fermion_bytes", "qdpx_workspace_bytes",
    "qdpx_pack_links", "qdpx_unpack_links", "qdpx_pack_fermion", "qdpx_unpack_fermion",
    "qdpx_eval_shift_mul_axpy", "qdpx_shift_chain", "qdpx_ape_smear", "qdpx_plaquette",
    "qdpx_ape_smear_batched", "qdpx_tune", "qdpx_tune_get", "qdpx_tune_set",
    "qdpx_eval_hop", "qdpx_jacobi_smear", "qdpx_tune_save", "qdpx_tune_batched",
    "qdpx_eval_shift_mul_axpy_noalloc",
    "qdpx_jit_generate", "qdpx_jit_compile", "qdpx_jit_info", "qdpx_jit_eval",
)


class QdpxError(RuntimeError):
    def __init__(self, code: int, fn: str, msg: str):
        super().__init__(f"{fn} -> {STATUS.get(code, code)}: {msg}")
        self.code = code


class Geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4)]


def geom(L) -> Geom:
    g = Geom()
    for d in range(4):
        g.L[d] = int(L[d])
    return g


_P = ctypes.c_void_p
_G = ctypes.POINTER(Geom)
_lib = None


def lib():
    """The loaded ``libqdpx.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1105_2279_amd.build` "
            "(or __graft_entry__.build()); there is no fallback path"
        )
    h = ctypes.CDLL(LIB_PATH)
    i32, sz, dbl = ctypes.c_int, ctypes.c_size_t, ctypes.c_double
    sig = {
        "qdpx_create": (i32, [ctypes.POINTER(_P), i32, ctypes.c_char_p]),
        "qdpx_tune_save": (i32, [_P, ctypes.c_char_p]),
        "qdpx_destroy": (i32, [_P]),
        "qdpx_free_all": (i32, [_P]),
        "qdpx_last_error": (ctypes.c_char_p, []),
        "qdpx_version": (ctypes.c_char_p, []),
        "qdpx_site_stride": (ctypes.c_int64, [_G]),
        "qdpx_links_bytes": (sz, [_G, i32, i32]),
        "qdpx_fermion_bytes": (sz, [_G, i32]),
        "qdpx_workspace_bytes": (sz, [i32, _G, i32, i32, i32]),
        "qdpx_pack_links": (i32, [_P, _G, _P, i32, i32, _P, _P]),
        "qdpx_unpack_links": (i32, [_P, _G, _P, i32, i32, _P, _P]),
        "qdpx_pack_fermion": (i32, [_P, _G, _P, i32, _P, _P]),
        "qdpx_unpack_fermion": (i32, [_P, _G, _P, i32, _P, _P]),
        "qdpx_eval_shift_mul_axpy": (i32, [_P, _G, i32, i32, _P, _P, _P, dbl, ctypes.c_uint32, i32, _P, _P, _P, sz,
                                           _P]),
        "qdpx_eval_shift_mul_axpy_noalloc": (i32, [_P, _G, i32, i32, _P, _P, _P, dbl, ctypes.c_uint32, i32, _P, _P,
                                                   _P]),
        "qdpx_shift_chain": (i32, [_P, _G, i32, i32, _P, _P, _P, dbl, dbl, i32, _P, _P, sz, _P]),
        "qdpx_ape_smear": (i32, [_P, _G, i32, i32, _P, _P, dbl, i32, ctypes.c_uint32, i32, _P, _P, sz, _P]),
        "qdpx_plaquette": (i32, [_P, _G, i32, i32, _P, _P, _P, sz, _P]),
        "qdpx_ape_smear_batched": (i32, [_P, i32, _G, i32, i32, ctypes.POINTER(_P), ctypes.POINTER(_P), dbl, i32,
                                         _P, _P, sz, _P]),
        "qdpx_tune": (i32, [_P, i32, _G, i32, i32, _P]),
        "qdpx_tune_batched": (i32, [_P, i32, _G, i32, i32, i32, _P]),
        "qdpx_eval_hop": (i32, [_P, _G, i32, i32, _P, _P, _P, ctypes.c_uint32, _P]),
        "qdpx_jit_generate": (i32, [ctypes.c_char_p, i32, i32, i32, i32, _P, sz, ctypes.POINTER(sz)]),
        "qdpx_jit_compile": (i32, [_P, ctypes.c_char_p, i32, i32, i32, i32, ctypes.POINTER(i32)]),
        "qdpx_jit_info": (i32, [_P, i32, ctypes.POINTER(i32), _P, sz]),
        "qdpx_jit_eval": (i32, [_P, i32, _G, _P, _P, _P, _P, _P, _P, sz, _P]),
        "qdpx_jacobi_smear": (i32, [_P, _G, i32, i32, _P, _P, dbl, i32, dbl, ctypes.c_uint32, _P, sz, _P]),
        "qdpx_tune_get": (i32, [_P, i32, _G, i32, i32] + [ctypes.POINTER(ctypes.c_int32)] * 6),
        "qdpx_tune_set": (i32, [_P, i32, _G, i32, i32] + [ctypes.c_int32] * 5),
    }
    for name, (res, args) in sig.items():
        f = getattr(h, name)
        f.restype = res
        f.argtypes = args
    _lib = h
    return h


def _check(code: int, fn: str) -> None:
    if code != 0:
        raise QdpxError(code, fn, lib().qdpx_last_error().decode())


def _ptr(t):
    """Device pointer of a tensor (or None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("qdpx takes device tensors only")
    if not t.is_contiguous():
        raise ValueError("qdpx takes contiguous tensors only")
    return t.data_ptr()


def _stream(stream=None):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _nbytes(t) -> int:
    return 0 if t is None else t.numel() * t.element_size()


# --------------------------------------------------------------------- context
class Context:
    """Owns one ``qdpx_ctx`` (tuned geometries, cached tables).  ``tune_cache``:
    path of a launch-table file the library reads now and rewrites when it
    tunes (None: the library takes ``$QDPX_TUNE_CACHE`` if set)."""

    def __init__(self, device: int = 0, tune_cache=None):
        p = _P()
        path = None if tune_cache is None else os.fsencode(tune_cache)
        _check(lib().qdpx_create(ctypes.byref(p), int(device), path), "qdpx_create")
        self._p = p
        self.device = int(device)

    @property
    def handle(self):
        return self._p

    def close(self):
        if getattr(self, "_p", None):
            lib().qdpx_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------- sizes
def qdpx_version() -> str:
    return lib().qdpx_version().decode()


def qdpx_site_stride(L) -> int:
    return int(lib().qdpx_site_stride(ctypes.byref(geom(L))))


def qdpx_links_bytes(L, prec, fmt) -> int:
    return int(lib().qdpx_links_bytes(ctypes.byref(geom(L)), prec, fmt))


def qdpx_fermion_bytes(L, prec) -> int:
    return int(lib().qdpx_fermion_bytes(ctypes.byref(geom(L)), prec))


def qdpx_workspace_bytes(op, L, prec, fmt, n=1) -> int:
    if op == OP_BATCHED:
        arr = (Geom * len(L))(*[geom(x) for x in L])
        return int(lib().qdpx_workspace_bytes(op, arr, prec, fmt, len(L)))
    return int(lib().qdpx_workspace_bytes(op, ctypes.byref(geom(L)), prec, fmt, int(n)))


def empty_bytes(nbytes: int, device="cuda") -> torch.Tensor:
    """Uninitialised device buffer of ``nbytes`` bytes (uint8 tensor)."""
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def alloc_links(L, prec, fmt, device="cuda") -> torch.Tensor:
    return empty_bytes(qdpx_links_bytes(L, prec, fmt), device)


def alloc_fermion(L, prec, device="cuda") -> torch.Tensor:
    return empty_bytes(qdpx_fermion_bytes(L, prec), device)


def alloc_workspace(op, L, prec, fmt, n=1, device="cuda") -> torch.Tensor:
    return empty_bytes(qdpx_workspace_bytes(op, L, prec, fmt, n), device)


# ----------------------------------------------------------------- entry points
def qdpx_pack_links(ctx, L, aos, prec, fmt, soa, stream=None):
    _check(lib().qdpx_pack_links(ctx.handle, ctypes.byref(geom(L)), _ptr(aos), prec, fmt, _ptr(soa),
                                 _stream(stream)), "qdpx_pack_links")


def qdpx_unpack_links(ctx, L, soa, prec, fmt, aos, stream=None):
    _check(lib().qdpx_unpack_links(ctx.handle, ctypes.byref(geom(L)), _ptr(soa), prec, fmt, _ptr(aos),
                                   _stream(stream)), "qdpx_unpack_links")


def qdpx_pack_fermion(ctx, L, aos, prec, soa, stream=None):
    _check(lib().qdpx_pack_fermion(ctx.handle, ctypes.byref(geom(L)), _ptr(aos), prec, _ptr(soa),
                                   _stream(stream)), "qdpx_pack_fermion")


def qdpx_unpack_fermion(ctx, L, soa, prec, aos, stream=None):
    _check(lib().qdpx_unpack_fermion(ctx.handle, ctypes.byref(geom(L)), _ptr(soa), prec, _ptr(aos),
                                     _stream(stream)), "qdpx_unpack_fermion")


def qdpx_eval_shift_mul_axpy(ctx, L, prec, fmt, U, psi, phi, a, chi, norm2=None, work=None, stream=None,
                             dir_mask=0xF, sign=1):
    _check(lib().qdpx_eval_shift_mul_axpy(ctx.handle, ctypes.byref(geom(L)), prec, fmt, _ptr(U), _ptr(psi),
                                          _ptr(phi), float(a), int(dir_mask), int(sign), _ptr(chi), _ptr(norm2),
                                          _ptr(work), _nbytes(work), _stream(stream)), "qdpx_eval_shift_mul_axpy")


def qdpx_eval_shift_mul_axpy_noalloc(ctx, L, prec, fmt, U, psi, phi, a, chi, norm2=None, stream=None, dir_mask=0xF,
                                     sign=1):
    _check(lib().qdpx_eval_shift_mul_axpy_noalloc(ctx.handle, ctypes.byref(geom(L)), prec, fmt, _ptr(U), _ptr(psi),
                                                  _ptr(phi), float(a), int(dir_mask), int(sign), _ptr(chi),
                                                  _ptr(norm2), _stream(stream)), "qdpx_eval_shift_mul_axpy_noalloc")


def qdpx_shift_chain(ctx, L, prec, fmt, U, psi, phi, a, c, n_iter, norms=None, work=None, stream=None):
    _check(lib().qdpx_shift_chain(ctx.handle, ctypes.byref(geom(L)), prec, fmt, _ptr(U), _ptr(psi), _ptr(phi),
                                  float(a), float(c), int(n_iter), _ptr(norms), _ptr(work), _nbytes(work),
                                  _stream(stream)), "qdpx_shift_chain")


def qdpx_ape_smear(ctx, L, prec, fmt, U_in, U_out, alpha, n_steps, plaq=None, work=None, stream=None,
                   smear_mask=0xF, projection=0):
    _check(lib().qdpx_ape_smear(ctx.handle, ctypes.byref(geom(L)), prec, fmt, _ptr(U_in), _ptr(U_out),
                                float(alpha), int(n_steps), int(smear_mask), int(projection), _ptr(plaq),
                                _ptr(work), _nbytes(work), _stream(stream)), "qdpx_ape_smear")


def qdpx_plaquette(ctx, L, prec, fmt, U, plaq, work, stream=None):
    _check(lib().qdpx_plaquette(ctx.handle, ctypes.byref(geom(L)), prec, fmt, _ptr(U), _ptr(plaq), _ptr(work),
                                _nbytes(work), _stream(stream)), "qdpx_plaquette")


def qdpx_ape_smear_batched(ctx, Ls, prec, fmt, U_in, U_out, alpha, n_steps, plaq=None, work=None, stream=None):
    n = len(Ls)
    garr = (Geom * n)(*[geom(x) for x in Ls])
    pin = (_P * n)(*[_ptr(t) for t in U_in])
    pout = (_P * n)(*[_ptr(t) for t in U_out])
    _check(lib().qdpx_ape_smear_batched(ctx.handle, n, garr, prec, fmt, pin, pout, float(alpha), int(n_steps),
                                        _ptr(plaq), _ptr(work), _nbytes(work), _stream(stream)),
           "qdpx_ape_smear_batched")


def qdpx_eval_hop(ctx, L, prec, fmt, U, psi, out, dir_mask=0xF, stream=None):
    _check(lib().qdpx_eval_hop(ctx.handle, ctypes.byref(geom(L)), prec, fmt, _ptr(U), _ptr(psi), _ptr(out),
                               int(dir_mask), _stream(stream)), "qdpx_eval_hop")


def qdpx_jacobi_smear(ctx, L, prec, fmt, U, chi, kappa, n_iter, norm=1.0, dir_mask=0xF, work=None, stream=None):
    _check(lib().qdpx_jacobi_smear(ctx.handle, ctypes.byref(geom(L)), prec, fmt, _ptr(U), _ptr(chi), float(kappa),
                                   int(n_iter), float(norm), int(dir_mask), _ptr(work), _nbytes(work),
                                   _stream(stream)), "qdpx_jacobi_smear")


def jit_generate(expr, prec, fmt, n_fields, n_scalars=0) -> str:
    """HIP source of the run-time compiled kernel for an expression (no device needed)."""
    need = ctypes.c_size_t(0)
    _check(lib().qdpx_jit_generate(expr.encode(), prec, fmt, n_fields, n_scalars, None, 0, ctypes.byref(need)),
           "qdpx_jit_generate")
    buf = ctypes.create_string_buffer(need.value)
    _check(lib().qdpx_jit_generate(expr.encode(), prec, fmt, n_fields, n_scalars, buf, need.value, None),
           "qdpx_jit_generate")
    return buf.value.decode()


def qdpx_jit_compile(ctx, expr, prec, fmt, n_fields, n_scalars=0) -> int:
    k = ctypes.c_int32(-1)
    _check(lib().qdpx_jit_compile(ctx.handle, expr.encode(), prec, fmt, n_fields, n_scalars, ctypes.byref(k)),
           "qdpx_jit_compile")
    return k.value


def qdpx_jit_info(ctx, kernel):
    """(came from the on-disk cache, generated source)."""
    fc = ctypes.c_int32(0)
    buf = ctypes.create_string_buffer(1 << 20)
    _check(lib().qdpx_jit_info(ctx.handle, kernel, ctypes.byref(fc), buf, len(buf)), "qdpx_jit_info")
    return bool(fc.value), buf.value.decode()


def qdpx_jit_eval(ctx, kernel, L, U, fields, scalars, out, norm2=None, work=None, stream=None):
    ptrs = (ctypes.c_void_p * max(1, len(fields)))(*[_ptr(f) for f in fields])
    sc = (ctypes.c_double * max(1, len(scalars)))(*[float(x) for x in scalars])
    _check(lib().qdpx_jit_eval(ctx.handle, kernel, ctypes.byref(geom(L)), _ptr(U), ptrs, sc, _ptr(out), _ptr(norm2),
                               _ptr(work), _nbytes(work), _stream(stream)), "qdpx_jit_eval")


def qdpx_tune(ctx, op, L, prec, fmt, stream=None):
    _check(lib().qdpx_tune(ctx.handle, op, ctypes.byref(geom(L)), prec, fmt, _stream(stream)), "qdpx_tune")


def qdpx_tune_batched(ctx, Ls, prec, fmt, n_steps, stream=None):
    n = len(Ls)
    garr = (Geom * n)(*[geom(x) for x in Ls])
    _check(lib().qdpx_tune_batched(ctx.handle, n, garr, prec, fmt, int(n_steps), _stream(stream)),
           "qdpx_tune_batched")


TUNE_SOURCES = ("default", "table", "tuned", "set")


def _tune_get(ctx, op, L, prec, fmt):
    b, n, x, t, d, src = (ctypes.c_int32() for _ in range(6))
    _check(lib().qdpx_tune_get(ctx.handle, op, ctypes.byref(geom(L)), prec, fmt, ctypes.byref(b), ctypes.byref(n),
                               ctypes.byref(x), ctypes.byref(t), ctypes.byref(d), ctypes.byref(src)),
           "qdpx_tune_get")
    return (int(b.value), int(n.value), int(x.value), int(t.value), int(d.value)), TUNE_SOURCES[src.value]


def qdpx_tune_get(ctx, op, L, prec, fmt):
    """(block, sites_per_thread, xcd_map, t_window, lds_tile) remembered for this case."""
    return _tune_get(ctx, op, L, prec, fmt)[0]


def qdpx_tune_source(ctx, op, L, prec, fmt) -> str:
    """Where the remembered geometry came from: "default", "table", "tuned" or "set"."""
    return _tune_get(ctx, op, L, prec, fmt)[1]


def qdpx_tune_save(ctx, path=None):
    _check(lib().qdpx_tune_save(ctx.handle, None if path is None else os.fsencode(path)), "qdpx_tune_save")


def qdpx_tune_set(ctx, op, L, prec, fmt, block, sites_per_thread, xcd_map, t_window=1, lds_tile=None):
    """lds_tile None: the default (4 for the FP32 APE step, else 0)."""
    if lds_tile is None:
        lds_tile = 4 if (op == OP_APE and prec == F32) else 0
    _check(lib().qdpx_tune_set(ctx.handle, op, ctypes.byref(geom(L)), prec, fmt, int(block),
                               int(sites_per_thread), int(xcd_map), int(t_window), int(lds_tile)), "qdpx_tune_set")


# ------------------------------------------------- host <-> device conveniences
def links_to_device(ctx, L, links_c128, prec, fmt, device="cuda", stream=None) -> torch.Tensor:
    """Copy canonical complex128 links (Lt, Lz, Ly, Lx, 4, 3, 3) to the device and pack them."""
    aos = torch.from_numpy(_as_f64(links_c128)).to(device)
    soa = alloc_links(L, prec, fmt, device)
    qdpx_pack_links(ctx, L, aos, prec, fmt, soa, stream)
    return soa


def fermion_to_device(ctx, L, field_c128, prec, device="cuda", stream=None) -> torch.Tensor:
    aos = torch.from_numpy(_as_f64(field_c128)).to(device)
    soa = alloc_fermion(L, prec, device)
    qdpx_pack_fermion(ctx, L, aos, prec, soa, stream)
    return soa


def links_to_host(ctx, L, soa, prec, fmt, stream=None):
    """Unpack SoA links into a complex128 numpy array (Lt, Lz, Ly, Lx, 4, 3, 3)."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    aos = torch.empty((Lt, Lz, Ly, Lx, 4, 3, 3, 2), dtype=torch.float64, device=soa.device)
    qdpx_unpack_links(ctx, L, soa, prec, fmt, aos, stream)
    return aos.cpu().numpy().view("complex128").reshape(Lt, Lz, Ly, Lx, 4, 3, 3)


def fermion_to_host(ctx, L, soa, prec, stream=None):
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    aos = torch.empty((Lt, Lz, Ly, Lx, 4, 3, 2), dtype=torch.float64, device=soa.device)
    qdpx_unpack_fermion(ctx, L, soa, prec, aos, stream)
    return aos.cpu().numpy().view("complex128").reshape(Lt, Lz, Ly, Lx, 4, 3)


def _as_f64(a):
    import numpy as np

    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a.view(np.float64).reshape(a.shape + (2,))
