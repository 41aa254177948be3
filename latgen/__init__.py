"""Seeded synthetic lattice inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and shapes them into gauge links and
Dirac fields.  It holds none of the smearing / shift-expression arithmetic:
that lives separately in the oracle (CPU, FP64) and in the HIP library.

Conventions (host canonical layout, used by everything that exchanges data):

* Extents are ``L = (Lx, Ly, Lz, Lt)``; direction mu = 0, 1, 2, 3 is x, y, z, t.
* Arrays are C-ordered ``[t][z][y][x]`` so the flat site index is
  ``x + Lx*(y + Ly*(z + Lz*t))``.
* Links: complex128 ``[Lt, Lz, Ly, Lx, 4, 3, 3]``, element ``[..., mu, a, b]`` is
  ``U_mu(x)_{ab}`` (row a, column b); as float64 the trailing axis is (re, im).
* Dirac fields: complex128 ``[Lt, Lz, Ly, Lx, 4, 3]`` (spin, colour).

Every generator draws per t-slice from ``numpy.random.default_rng([seed, t])`` so
that a lattice can be produced slice by slice and the same seed always gives
the same bits.
"""

from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

__all__ = [
    "volume",
    "haar_su3",
    "haar_links",
    "near_unit_links",
    "unit_links",
    "dirac_field",
    "haar_gauge",
    "torus_gauge",
    "batch_extents",
    "BATCH_CHOICES",
    "SEEDS",
]

# Seeds of the named workloads (one per input array).
SEEDS = {
    "ape_4x4x4x4": {"links": 1105},
    "shift_16x16x16x32": {"links": 1205, "psi": 1206, "phi": 1207},
    "ape_32x32x32x64": {"links": 1305},
    "batch_64": {"extents": 1400, "first_lattice": 1405},
    "large_48x48x48x96": {"links_haar": 1505, "links_near_unit": 1506, "psi": 1507, "phi": 1508, "gauge": 1509},
    # Jacobi smearing on the Table 1 lattices: seed + Lx
    "jacobi_table1": {"links": 3000, "chi": 3001},
}

# Extents drawn for the 64-lattice batch (Lx, Ly, Lz, Lt).
BATCH_CHOICES = ((8, 8, 8, 8), (12, 12, 12, 24), (16, 16, 16, 32), (24, 24, 24, 48))


def volume(L) -> int:
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    return Lx * Ly * Lz * Lt


def _slices(Lt, fill):
    """Call fill(t) for every t-slice.  Each slice draws from its own
    generator, so the result does not depend on the order or on the number of
    threads; large lattices are filled by a thread pool (numpy releases the
    interpreter lock inside its array operations)."""
    workers = min(16, os.cpu_count() or 1, Lt)
    if workers <= 1 or Lt < 8:
        for t in range(Lt):
            fill(t)
        return
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(fill, range(Lt)))


def _check_extents(L):
    if len(L) != 4 or any(int(v) < 1 for v in L):
        raise ValueError(f"extents must be 4 positive integers, got {L!r}")
    return tuple(int(v) for v in L)


def _complex_gaussian(rng, shape):
    # Real and imaginary parts independent standard normals.
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def haar_su3(rng, n: int) -> np.ndarray:
    """``n`` Haar-distributed SU(3) matrices, shape (n, 3, 3) complex128.

    A complex Gaussian 3x3 matrix is orthonormalised column by column (this is
    its QR factor with a positive real diagonal in R, which makes the unitary
    factor Haar on U(3)); the result is then multiplied by the cube root of
    conj(det) taken on the principal branch so that det = 1.
    """
    z = _complex_gaussian(rng, (n, 3, 3))
    q = np.empty_like(z)
    for j in range(3):
        v = z[:, :, j].copy()
        # two projection passes keep the columns orthonormal to rounding
        for _ in range(2):
            for k in range(j):
                proj = np.sum(q[:, :, k].conj() * v, axis=1)
                v -= proj[:, None] * q[:, :, k]
        v /= np.sqrt(np.sum(v.real ** 2 + v.imag ** 2, axis=1))[:, None]
        q[:, :, j] = v
    det = np.linalg.det(q)
    phase = np.exp(-1j * np.angle(det) / 3.0)
    return q * phase[:, None, None]


def haar_links(L, seed: int) -> np.ndarray:
    """Haar-random SU(3) links, shape (Lt, Lz, Ly, Lx, 4, 3, 3)."""
    Lx, Ly, Lz, Lt = _check_extents(L)
    out = np.empty((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
    per_slice = Lz * Ly * Lx * 4

    def fill(t):
        out[t] = haar_su3(np.random.default_rng([seed, t]), per_slice).reshape(Lz, Ly, Lx, 4, 3, 3)

    _slices(Lt, fill)
    return out


def _gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    return lam


def near_unit_links(L, seed: int, eps: float = 0.1) -> np.ndarray:
    """Links ``exp(i*eps*H)`` with ``H = sum_a w_a lambda_a / 2``, ``w_a ~ N(0,1)``.

    The matrix exponential is the library routine (torch.linalg.matrix_exp,
    on the CPU, one call per t-slice).
    """
    import torch

    Lx, Ly, Lz, Lt = _check_extents(L)
    lam_half = _gell_mann() / 2.0
    out = np.empty((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
    per_slice = Lz * Ly * Lx * 4

    def fill(t):
        w = np.random.default_rng([seed, t]).standard_normal((per_slice, 8))
        h = np.einsum("na,aij->nij", w, lam_half)
        u = torch.linalg.matrix_exp(torch.from_numpy(1j * eps * h)).numpy()
        out[t] = u.reshape(Lz, Ly, Lx, 4, 3, 3)

    _slices(Lt, fill)
    return out


def unit_links(L) -> np.ndarray:
    Lx, Ly, Lz, Lt = _check_extents(L)
    out = np.zeros((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
    out[..., 0, 0] = out[..., 1, 1] = out[..., 2, 2] = 1.0
    return out


def dirac_field(L, seed: int) -> np.ndarray:
    """Dirac field with 4 spins x 3 colours, re/im parts i.i.d. N(0,1)."""
    Lx, Ly, Lz, Lt = _check_extents(L)
    out = np.empty((Lt, Lz, Ly, Lx, 4, 3), dtype=np.complex128)

    def fill(t):
        out[t] = _complex_gaussian(np.random.default_rng([seed, t]), (Lz, Ly, Lx, 4, 3))

    _slices(Lt, fill)
    return out


def haar_gauge(L, seed: int) -> np.ndarray:
    """One Haar SU(3) matrix per site, shape (Lt, Lz, Ly, Lx, 3, 3)."""
    Lx, Ly, Lz, Lt = _check_extents(L)
    out = np.empty((Lt, Lz, Ly, Lx, 3, 3), dtype=np.complex128)

    def fill(t):
        out[t] = haar_su3(np.random.default_rng([seed, t]), Lz * Ly * Lx).reshape(Lz, Ly, Lx, 3, 3)

    _slices(Lt, fill)
    return out


def torus_gauge(L, seed: int) -> np.ndarray:
    """Diagonal SU(3) matrices diag(e^{i a}, e^{i b}, e^{-i(a+b)}), a, b uniform."""
    Lx, Ly, Lz, Lt = _check_extents(L)
    out = np.zeros((Lt, Lz, Ly, Lx, 3, 3), dtype=np.complex128)
    for t in range(Lt):
        rng = np.random.default_rng([seed, t])
        th = rng.uniform(-np.pi, np.pi, (Lz, Ly, Lx, 2))
        out[t, ..., 0, 0] = np.exp(1j * th[..., 0])
        out[t, ..., 1, 1] = np.exp(1j * th[..., 1])
        out[t, ..., 2, 2] = np.exp(-1j * (th[..., 0] + th[..., 1]))
    return out


def batch_extents(n: int = 64, seed: int = 1400):
    """Extents of the uneven batch: each drawn uniformly from ``BATCH_CHOICES``."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(BATCH_CHOICES), size=n)
    return [BATCH_CHOICES[i] for i in idx]


def as_real(a: np.ndarray) -> np.ndarray:
    """Contiguous float64 view with a trailing (re, im) axis."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a.view(np.float64).reshape(a.shape + (2,))


def as_complex(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.view(np.complex128).reshape(a.shape[:-1])
