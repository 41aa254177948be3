"""FP64 CPU oracle for the lattice hot path (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product library never does.

The arithmetic lives in ``oracle.c`` (plain C, FP64, explicit real/imag
operations, compiled with ``-O2 -fopenmp -ffp-contract=off``); this module
builds it with gcc when asked and wraps it with ctypes over numpy arrays in the
host canonical layout of ``latgen``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc; returns the path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_L = ctypes.POINTER(ctypes.c_long)


def lib():
    """The loaded oracle library.

    ``ORACLE_LIB`` may name another build of ``oracle.c`` (the mutation tests
    use it to run the pins against deliberately broken copies)."""
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        h = ctypes.CDLL(path)
        h.oracle_neumaier_sum.argtypes = [ctypes.c_long, _D]
        h.oracle_neumaier_sum.restype = ctypes.c_double
        h.oracle_num_threads.restype = ctypes.c_int
        h.oracle_set_num_threads.argtypes = [ctypes.c_int]
        h.oracle_shift_mul_axpy.argtypes = [_I, _D, _D, _D, ctypes.c_double, _D, _D]
        h.oracle_shift_expr.argtypes = [_I, _D, _D, _D, ctypes.c_double, ctypes.c_uint, ctypes.c_int, _D, _D]
        h.oracle_shift_chain.argtypes = [_I, _D, _D, _D, ctypes.c_double, ctypes.c_double, ctypes.c_int, _D]
        h.oracle_staple_sums.argtypes = [_I, _D, _D, _D]
        h.oracle_ape_w.argtypes = [_I, _D, ctypes.c_double, ctypes.c_uint, _D]
        h.oracle_reunitarise.argtypes = [ctypes.c_long, _D, _D]
        h.oracle_reunitarise.restype = ctypes.c_long
        h.oracle_polar_project.argtypes = [ctypes.c_long, _D, _D]
        h.oracle_polar_project.restype = ctypes.c_long
        h.oracle_ape_step.argtypes = [_I, _D, ctypes.c_double, ctypes.c_uint, ctypes.c_int, _D]
        h.oracle_ape_step.restype = ctypes.c_long
        h.oracle_ape_smear.argtypes = [_I, _D, ctypes.c_double, ctypes.c_uint, ctypes.c_int, ctypes.c_int, _D]
        h.oracle_ape_smear.restype = ctypes.c_long
        h.oracle_ape_links.argtypes = [_I, _D, ctypes.c_double, ctypes.c_uint, ctypes.c_int, ctypes.c_long, _L, _I, _D]
        h.oracle_ape_links.restype = ctypes.c_long
        h.oracle_plaquette.argtypes = [_I, _D, _D]
        h.oracle_shift_sites.argtypes = [_I, _D, _D, _D, ctypes.c_double, ctypes.c_long, _L, _D]
        h.oracle_hop.argtypes = [_I, _D, _D, ctypes.c_uint, _D]
        h.oracle_jacobi_smear.argtypes = [_I, _D, _D, ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_uint]
        _lib = h
    return _lib


# ---------------------------------------------------------------------------
# numpy wrappers.  Arrays are complex128 in the latgen canonical shapes:
# links (Lt, Lz, Ly, Lx, 4, 3, 3), fermions (Lt, Lz, Ly, Lx, 4, 3).
# ---------------------------------------------------------------------------

def _extents(links_or_field):
    Lt, Lz, Ly, Lx = links_or_field.shape[:4]
    return (ctypes.c_int * 4)(Lx, Ly, Lz, Lt)


def _dp(a):
    assert a.dtype == np.complex128 or a.dtype == np.float64, a.dtype
    assert a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads(int(n))


def neumaier_sum(x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().oracle_neumaier_sum(x.size, _dp(x)))


def shift_mul_axpy(U, psi, phi=None, a=0.0):
    """chi = sum_mu U_mu(x) psi(x+mu) + a*phi(x); returns (chi, |chi|^2)."""
    U, psi = _c(U), _c(psi)
    chi = np.empty_like(psi)
    n2 = ctypes.c_double(0.0)
    phi_p = None
    if phi is not None:
        phi = _c(phi)
        phi_p = _dp(phi)
    lib().oracle_shift_mul_axpy(_extents(U), _dp(U), _dp(psi), phi_p, float(a), _dp(chi), ctypes.byref(n2))
    return chi, float(n2.value)


def shift_expr(U, psi, phi=None, a=0.0, mask=0xF, sign=+1):
    """chi = sum_{mu in mask} h_mu(x) + a*phi(x) with the forward hop
    h_mu = U_mu(x) psi(x+mu) (sign > 0) or the backward hop
    h_mu = U_mu(x-mu)^dag psi(x-mu) (sign < 0); returns (chi, |chi|^2)."""
    U, psi = _c(U), _c(psi)
    chi = np.empty_like(psi)
    n2 = ctypes.c_double(0.0)
    phi_p = None
    if phi is not None:
        phi = _c(phi)
        phi_p = _dp(phi)
    lib().oracle_shift_expr(_extents(U), _dp(U), _dp(psi), phi_p, float(a), ctypes.c_uint(mask), int(sign),
                            _dp(chi), ctypes.byref(n2))
    return chi, float(n2.value)


def shift_chain(U, psi, phi, a, c, n_iter):
    """n_iter times: chi = shift_mul_axpy(U, psi, phi, a); psi -= c*chi.
    Returns (final psi, array of |chi_k|^2)."""
    U = _c(U)
    psi = _c(psi).copy()
    norms = np.zeros(max(int(n_iter), 1), dtype=np.float64)
    phi_p = None
    if phi is not None:
        phi = _c(phi)
        phi_p = _dp(phi)
    lib().oracle_shift_chain(_extents(U), _dp(U), _dp(psi), phi_p, float(a), float(c), int(n_iter), _dp(norms))
    return psi, norms[: int(n_iter)]


def staple_sums(U):
    """(upper, lower) staple sums per link, each shaped like U."""
    U = _c(U)
    up, lo = np.empty_like(U), np.empty_like(U)
    lib().oracle_staple_sums(_extents(U), _dp(U), _dp(up), _dp(lo))
    return up, lo


def ape_w(U, alpha, mask=0xF):
    U = _c(U)
    W = np.empty_like(U)
    lib().oracle_ape_w(_extents(U), _dp(U), float(alpha), ctypes.c_uint(mask), _dp(W))
    return W


def reunitarise(W):
    """Row Gram-Schmidt projection of any (..., 3, 3) array; returns (V, n_degenerate)."""
    W = _c(W)
    V = np.empty_like(W)
    n = W.size // 9
    bad = lib().oracle_reunitarise(n, _dp(W), _dp(V))
    return V, int(bad)


def polar_project(W):
    """Polar (bi-covariant) projection of any (..., 3, 3) array; returns (V, n_degenerate)."""
    W = _c(W)
    V = np.empty_like(W)
    n = W.size // 9
    bad = lib().oracle_polar_project(n, _dp(W), _dp(V))
    return V, int(bad)


def ape_step(U, alpha, mask=0xF, proj=0):
    """One APE step; links of directions outside mask are copied.  proj 0:
    row Gram-Schmidt; 1: polar (bi-covariant) projection."""
    U = _c(U)
    V = np.empty_like(U)
    bad = lib().oracle_ape_step(_extents(U), _dp(U), float(alpha), ctypes.c_uint(mask), int(proj), _dp(V))
    if bad:
        raise FloatingPointError(f"{bad} degenerate links in the APE projection")
    return V


def ape_smear(U, alpha, n_steps, mask=0xF, proj=0):
    U = _c(U)
    V = np.empty_like(U)
    bad = lib().oracle_ape_smear(_extents(U), _dp(U), float(alpha), ctypes.c_uint(mask), int(proj), int(n_steps),
                                 _dp(V))
    if bad:
        raise FloatingPointError(f"{bad} degenerate links in the APE projection")
    return V


def ape_links(U, alpha, sites, mus, mask=0xF, proj=0):
    """One APE step evaluated only at the given (flat site, mu) pairs; (n, 3, 3)."""
    U = _c(U)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    mus = np.ascontiguousarray(mus, dtype=np.int32)
    out = np.empty((sites.size, 3, 3), dtype=np.complex128)
    bad = lib().oracle_ape_links(
        _extents(U), _dp(U), float(alpha), ctypes.c_uint(mask), int(proj), sites.size, sites.ctypes.data_as(_L),
        mus.ctypes.data_as(_I), _dp(out)
    )
    if bad:
        raise FloatingPointError(f"{bad} degenerate links in the APE projection")
    return out


def plaquette(U):
    """(total, spatial, temporal) average plaquette, each 1 on unit links."""
    U = _c(U)
    out = np.zeros(3, dtype=np.float64)
    lib().oracle_plaquette(_extents(U), _dp(U), _dp(out))
    return out


def shift_sites(U, psi, phi, a, sites):
    """chi at the given flat sites only; (n, 4, 3)."""
    U, psi = _c(U), _c(psi)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((sites.size, 4, 3), dtype=np.complex128)
    phi_p = None
    if phi is not None:
        phi = _c(phi)
        phi_p = _dp(phi)
    lib().oracle_shift_sites(_extents(U), _dp(U), _dp(psi), phi_p, float(a), sites.size, sites.ctypes.data_as(_L),
                             _dp(out))
    return out


def hop(U, psi, mask=0xF):
    """(H psi)(x) = sum_{mu in mask} [U_mu(x) psi(x+mu) + U_mu(x-mu)^dag psi(x-mu)]."""
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    lib().oracle_hop(_extents(U), _dp(U), _dp(psi), int(mask), _dp(out))
    return out


def jacobi_smear(U, chi, kappa, n_iter, norm=1.0, mask=0xF):
    """(1/norm) sum_{n=0}^{n_iter} (kappa H)^n chi: the truncated series of
    K^{-1} = (1 - kappa H)^{-1} applied to the source chi."""
    U = _c(U)
    chi = _c(chi).copy()
    lib().oracle_jacobi_smear(_extents(U), _dp(U), _dp(chi), float(kappa), int(n_iter), float(norm), int(mask))
    return chi
