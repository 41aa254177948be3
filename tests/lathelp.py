"""numpy helpers for the tests: periodic shifts, gauge transformations, SU(3) checks.

Arrays use the latgen canonical shapes: links (Lt, Lz, Ly, Lx, 4, 3, 3),
fermions (Lt, Lz, Ly, Lx, 4, 3), gauge matrices (Lt, Lz, Ly, Lx, 3, 3).
Direction mu = 0..3 (x, y, z, t) is array axis 3 - mu.
"""

import numpy as np


def axis(mu: int) -> int:
    return 3 - mu


def fwd(a, mu):
    """a(x + mu) at x (periodic)."""
    return np.roll(a, -1, axis=axis(mu))


def bwd(a, mu):
    """a(x - mu) at x (periodic)."""
    return np.roll(a, +1, axis=axis(mu))


def dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def gauge_links(U, g):
    """U_mu(x) -> g(x) U_mu(x) g(x+mu)^dagger."""
    out = np.empty_like(U)
    for mu in range(4):
        out[..., mu, :, :] = g @ U[..., mu, :, :] @ dag(fwd(g, mu))
    return out


def gauge_fermion(psi, g):
    """psi(x) -> g(x) psi(x) on colour, for each spin."""
    return np.einsum("...ab,...sb->...sa", g, psi)


def pure_gauge(g):
    """U_mu(x) = g(x) g(x+mu)^dagger: a gauge transform of unit links."""
    shape = g.shape[:4] + (4, 3, 3)
    U = np.empty(shape, dtype=np.complex128)
    for mu in range(4):
        U[..., mu, :, :] = g @ dag(fwd(g, mu))
    return U


def unitarity_defect(V):
    """max over matrices of the Frobenius norm of V^dagger V - 1."""
    eye = np.eye(3)
    d = dag(V) @ V - eye
    return float(np.max(np.sqrt(np.sum(np.abs(d) ** 2, axis=(-1, -2)))))


def det_defect(V):
    return float(np.max(np.abs(np.linalg.det(V) - 1.0)))


def max_abs(a):
    return float(np.max(np.abs(a))) if a.size else 0.0
