"""Pins of the FP64 oracle's Jacobi smearing (the paper's application,
section 7): the hopping term H of the smearing operator K = 1 - kappa H and
the smeared source, the truncated power series of K^{-1} applied to the
source, (1/norm) sum_{n=0}^{N} (kappa H)^n s0."""

import numpy as np
import pytest

import latgen
import oracle
from lathelp import gauge_fermion, gauge_links, max_abs


def fields(L, seed):
    return latgen.haar_links(L, seed), latgen.dirac_field(L, seed + 1), latgen.dirac_field(L, seed + 2)


@pytest.mark.parametrize("mask", [0xF, 0x7, 0x9])
def test_hop_is_hermitian(mask):
    U, psi, phi = fields((3, 4, 2, 5), 10)
    lhs = np.vdot(phi, oracle.hop(U, psi, mask))
    rhs = np.vdot(oracle.hop(U, phi, mask), psi)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


@pytest.mark.parametrize("mask", [0xF, 0x7])
def test_hop_unit_links_is_array_shifts(mask):
    L = (4, 3, 5, 2)
    psi = latgen.dirac_field(L, 3)
    ref = np.zeros_like(psi)
    for mu in range(4):
        if (mask >> mu) & 1:
            ref += np.roll(psi, -1, axis=3 - mu) + np.roll(psi, +1, axis=3 - mu)
    assert max_abs(oracle.hop(latgen.unit_links(L), psi, mask) - ref) < 1e-15 * 8


def test_hop_forward_part_is_the_shift_expression():
    # H = F + F^dagger where F psi = sum_mu U_mu(x) psi(x+mu) (pinned separately)
    U, psi, phi = fields((3, 4, 2, 5), 20)
    f_psi, _ = oracle.shift_mul_axpy(U, psi)
    h_psi = oracle.hop(U, psi)
    # <phi, (H - F) psi> = <F phi, psi>
    lhs = np.vdot(phi, h_psi - f_psi)
    f_phi, _ = oracle.shift_mul_axpy(U, phi)
    rhs = np.vdot(f_phi, psi)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_hop_gauge_covariant():
    L = (3, 4, 2, 5)
    U, psi, _ = fields(L, 30)
    g = latgen.haar_gauge(L, 33)
    a = oracle.hop(gauge_links(U, g), gauge_fermion(psi, g))
    b = gauge_fermion(oracle.hop(U, psi), g)
    assert max_abs(a - b) < 1e-13


@pytest.mark.parametrize("mask", [0xF, 0x7])
def test_jacobi_unit_links_fourier_closed_form(mask):
    # unit links: H is diagonal in momentum space with eigenvalue
    # h(p) = sum_{mu in mask} 2 cos(2 pi p_mu / L_mu), so the truncated
    # series is (1/norm) sum_{k=0}^{N} (kappa h)^k s0 mode by mode.
    L = (4, 3, 5, 6)
    s0 = latgen.dirac_field(L, 40)
    kappa, n, norm = 0.21, 5, 1.7
    got = oracle.jacobi_smear(latgen.unit_links(L), s0, kappa, n, norm, mask)
    Lx, Ly, Lz, Lt = L
    kt, kz, ky, kx = np.meshgrid(*(np.arange(m) for m in (Lt, Lz, Ly, Lx)), indexing="ij")
    parts = [2 * np.cos(2 * np.pi * kx / Lx), 2 * np.cos(2 * np.pi * ky / Ly),
             2 * np.cos(2 * np.pi * kz / Lz), 2 * np.cos(2 * np.pi * kt / Lt)]
    h = sum(p for mu, p in enumerate(parts) if (mask >> mu) & 1)[..., None, None]
    S = np.fft.fftn(s0, axes=(0, 1, 2, 3))
    acc = sum((kappa * h) ** k for k in range(n + 1)) * S
    ref = np.fft.ifftn(acc, axes=(0, 1, 2, 3)) / norm
    assert max_abs(got - ref) < 1e-12


@pytest.mark.parametrize("n", [0, 1, 4])
def test_jacobi_solves_k_up_to_truncation(n):
    # K chi_N = (1 - kappa H) chi_N = s0 - (kappa H)^{N+1} s0   (norm = 1)
    U, s0, _ = fields((3, 4, 2, 5), 50)
    kappa = 0.15
    chi = oracle.jacobi_smear(U, s0, kappa, n, 1.0)
    lhs = chi - kappa * oracle.hop(U, chi)
    t = s0
    for _ in range(n + 1):
        t = kappa * oracle.hop(U, t)
    assert max_abs(lhs - (s0 - t)) < 1e-13


def test_hop_is_forward_plus_backward_shift():
    # H = F + B, the forward and the backward hop of the shift expression
    L = (3, 4, 2, 5)
    U, psi, _ = fields(L, 70)
    for mask in (0xF, 0x6):
        f, _ = oracle.shift_expr(U, psi, None, 0.0, mask, +1)
        b, _ = oracle.shift_expr(U, psi, None, 0.0, mask, -1)
        assert max_abs(oracle.hop(U, psi, mask) - (f + b)) < 1e-14


def test_jacobi_matches_recursion_of_the_listing():
    # the listing's recursion chi <- s0 + kappa H chi, started from s0 and
    # run N times, reaches the same series (up to rounding)
    U, s0, _ = fields((3, 4, 2, 5), 80)
    kappa, n, norm = 0.2, 6, 2.5
    chi = s0.copy()
    for _ in range(n):
        chi = s0 + kappa * oracle.hop(U, chi)
    assert max_abs(oracle.jacobi_smear(U, s0, kappa, n, norm) - chi / norm) < 1e-13


def test_shift_sites_equals_full_evaluation():
    L = (3, 4, 2, 5)
    U, psi, phi = fields(L, 60)
    chi, _ = oracle.shift_mul_axpy(U, psi, phi, 0.3)
    sites = np.array([0, 7, 29, 119, 64])
    got = oracle.shift_sites(U, psi, phi, 0.3, sites)
    assert np.array_equal(got, chi.reshape(-1, 4, 3)[sites])
