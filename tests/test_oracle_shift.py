"""Pins of the FP64 oracle's shift expression and expression chain.

chi(x) = sum_mu U_mu(x) psi(x+mu) + a phi(x)   (forward hop of the smearing
operator of section 7 plus the axpy of expression E_3).
"""

import math

import numpy as np
import pytest

import latgen
import oracle
from lathelp import bwd, dag, fwd, gauge_fermion, gauge_links, max_abs

A = 0.3


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (2, 3, 4, 5), (5, 1, 2, 3)])
def test_unit_links_is_array_shift(L):
    U = latgen.unit_links(L)
    psi = latgen.dirac_field(L, 1)
    phi = latgen.dirac_field(L, 2)
    chi, n2 = oracle.shift_mul_axpy(U, psi, phi, A)
    ref = sum(np.roll(psi, -1, axis=3 - mu) for mu in range(4)) + A * phi
    assert max_abs(chi - ref) < 1e-15 * 8
    assert n2 == pytest.approx(float(np.sum(np.abs(ref) ** 2)), rel=1e-14)


def test_single_site_single_direction_brute_force():
    # psi nonzero at one site only: chi is nonzero exactly at the four sites
    # x with x + mu = that site, where it equals U_mu(x) psi.
    L = (3, 4, 5, 6)
    U = latgen.haar_links(L, 3)
    psi = np.zeros((6, 5, 4, 3, 4, 3), dtype=np.complex128)
    v = latgen.dirac_field((1, 1, 1, 1), 4)[0, 0, 0, 0]
    tgt = (2, 3, 1, 2)  # (t, z, y, x)
    psi[tgt] = v
    chi, _ = oracle.shift_mul_axpy(U, psi)
    expect = np.zeros_like(psi)
    for mu in range(4):
        src = list(tgt)
        ax = 3 - mu
        src[ax] = (src[ax] - 1) % psi.shape[ax]
        src = tuple(src)
        expect[src] += np.einsum("ab,sb->sa", U[src][mu], v)
    assert max_abs(chi - expect) < 1e-15 * 4


def test_gauge_covariance():
    L = (4, 3, 2, 5)
    U = latgen.haar_links(L, 5)
    psi, phi = latgen.dirac_field(L, 6), latgen.dirac_field(L, 7)
    g = latgen.haar_gauge(L, 8)
    chi, n2 = oracle.shift_mul_axpy(U, psi, phi, A)
    chig, n2g = oracle.shift_mul_axpy(gauge_links(U, g), gauge_fermion(psi, g), gauge_fermion(phi, g), A)
    assert max_abs(chig - gauge_fermion(chi, g)) < 1e-13
    assert n2g == pytest.approx(n2, rel=1e-13)


def test_forward_hop_adjoint_is_backward_hop():
    # <phi, H psi> = <H^dagger phi, psi> with (H^dagger phi)(x) = sum_mu U_mu(x-mu)^dagger phi(x-mu)
    L = (3, 4, 2, 5)
    U = latgen.haar_links(L, 9)
    psi, phi = latgen.dirac_field(L, 10), latgen.dirac_field(L, 11)
    hpsi, _ = oracle.shift_mul_axpy(U, psi)
    hdag_phi = np.zeros_like(phi)
    for mu in range(4):
        um = bwd(U[..., mu, :, :], mu)
        hdag_phi += np.einsum("...ab,...sb->...sa", dag(um), bwd(phi, mu))
    lhs = np.vdot(phi, hpsi)
    rhs = np.vdot(hdag_phi, psi)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_norm_expectation():
    # unitary rows and independent Gaussians: E|chi|^2 = 12 (4*2 + a^2*2) V
    L = (8, 8, 8, 8)
    V = np.prod(L)
    U = latgen.haar_links(L, 1205)
    psi, phi = latgen.dirac_field(L, 1206), latgen.dirac_field(L, 1207)
    _, n2 = oracle.shift_mul_axpy(U, psi, phi, A)
    expect = 12 * (8 + 2 * A * A) * V
    assert abs(n2 / expect - 1) < 5 / math.sqrt(12 * V)


def test_phi_none_equals_zero_phi():
    L = (2, 2, 3, 2)
    U = latgen.haar_links(L, 1)
    psi = latgen.dirac_field(L, 2)
    a, n_a = oracle.shift_mul_axpy(U, psi, None, A)
    b, n_b = oracle.shift_mul_axpy(U, psi, np.zeros_like(psi), A)
    assert np.array_equal(a, b) and n_a == n_b


def test_chain_unit_links_fourier_closed_form():
    # With unit links the hop is sum_mu T_mu, diagonal in momentum space with
    # eigenvalue h(k) = sum_mu exp(2 pi i k_mu / L_mu).  Each chain step is
    # psi <- (1 - c h) psi - c a phi.
    L = (4, 3, 5, 2)
    U = latgen.unit_links(L)
    psi, phi = latgen.dirac_field(L, 12), latgen.dirac_field(L, 13)
    c, n = 0.1, 8
    got, norms = oracle.shift_chain(U, psi, phi, A, c, n)
    ax = (0, 1, 2, 3)
    P, F = np.fft.fftn(psi, axes=ax), np.fft.fftn(phi, axes=ax)
    Lt, Lz, Ly, Lx = psi.shape[:4]
    kt, kz, ky, kx = np.meshgrid(*(np.arange(m) for m in (Lt, Lz, Ly, Lx)), indexing="ij")
    h = (np.exp(2j * np.pi * kx / Lx) + np.exp(2j * np.pi * ky / Ly)
         + np.exp(2j * np.pi * kz / Lz) + np.exp(2j * np.pi * kt / Lt))[..., None, None]
    ref_norms = []
    for _ in range(n):
        X = h * P + A * F
        ref_norms.append(float(np.sum(np.abs(X) ** 2)) / np.prod(L))  # Parseval
        P = P - c * X
    ref = np.fft.ifftn(P, axes=ax)
    assert max_abs(got - ref) < 1e-13
    assert np.allclose(norms, ref_norms, rtol=1e-13, atol=0)


def test_chain_is_iterated_expression():
    L = (2, 3, 2, 4)
    U = latgen.haar_links(L, 14)
    psi, phi = latgen.dirac_field(L, 15), latgen.dirac_field(L, 16)
    got, norms = oracle.shift_chain(U, psi, phi, A, 0.1, 3)
    p = psi.copy()
    for k in range(3):
        chi, n2 = oracle.shift_mul_axpy(U, p, phi, A)
        assert norms[k] == n2
        p = p - 0.1 * chi
    assert np.array_equal(got, p)


# ------------------------------------------------- direction mask and sign
# chi = sum_{mu in mask} h_mu + a phi with the forward hop U_mu(x) psi(x+mu)
# (sign +1) or the backward hop U_mu(x-mu)^dag psi(x-mu) (sign -1), the two
# terms of the smearing operator K of section 7.

@pytest.mark.parametrize("mask", [0xF, 0x7, 0x9, 0x2, 0x0])
@pytest.mark.parametrize("sign", [+1, -1])
def test_masked_unit_links_is_array_shift(mask, sign):
    # unit links: the hops are plain periodic array shifts (textbook roll)
    L = (4, 3, 5, 2)
    psi, phi = latgen.dirac_field(L, 21), latgen.dirac_field(L, 22)
    chi, n2 = oracle.shift_expr(latgen.unit_links(L), psi, phi, A, mask, sign)
    ref = A * phi
    for mu in range(4):
        if (mask >> mu) & 1:
            ref = ref + np.roll(psi, -sign, axis=3 - mu)
    assert max_abs(chi - ref) < 1e-15 * 8
    assert n2 == pytest.approx(float(np.sum(np.abs(ref) ** 2)), rel=1e-14)


@pytest.mark.parametrize("mask", [0xF, 0x5, 0x8])
def test_backward_is_adjoint_of_forward(mask):
    # <phi, F psi> = <B phi, psi>: the backward hop is the adjoint of the
    # forward one, direction by direction (pins the dagger and the link site)
    L = (3, 4, 2, 5)
    U = latgen.haar_links(L, 23)
    psi, phi = latgen.dirac_field(L, 24), latgen.dirac_field(L, 25)
    f_psi, _ = oracle.shift_expr(U, psi, None, 0.0, mask, +1)
    b_phi, _ = oracle.shift_expr(U, phi, None, 0.0, mask, -1)
    lhs, rhs = np.vdot(phi, f_psi), np.vdot(b_phi, psi)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_backward_single_site_brute_force():
    # psi nonzero at one site y: the backward hop is nonzero exactly at the
    # four sites y + mu, where it equals U_mu(y)^dag psi(y)
    L = (3, 4, 5, 6)
    U = latgen.haar_links(L, 26)
    psi = np.zeros((6, 5, 4, 3, 4, 3), dtype=np.complex128)
    v = latgen.dirac_field((1, 1, 1, 1), 27)[0, 0, 0, 0]
    y = (2, 3, 1, 2)  # (t, z, y, x)
    psi[y] = v
    chi, _ = oracle.shift_expr(U, psi, None, 0.0, 0xF, -1)
    expect = np.zeros_like(psi)
    for mu in range(4):
        dst = list(y)
        ax = 3 - mu
        dst[ax] = (dst[ax] + 1) % psi.shape[ax]
        expect[tuple(dst)] += np.einsum("ab,sb->sa", dag(U[y][mu]), v)
    assert max_abs(chi - expect) < 1e-15 * 4


@pytest.mark.parametrize("sign", [+1, -1])
def test_masked_gauge_covariance(sign):
    L = (4, 3, 2, 5)
    U = latgen.haar_links(L, 28)
    psi, phi = latgen.dirac_field(L, 29), latgen.dirac_field(L, 30)
    g = latgen.haar_gauge(L, 31)
    chi, n2 = oracle.shift_expr(U, psi, phi, A, 0xB, sign)
    chig, n2g = oracle.shift_expr(gauge_links(U, g), gauge_fermion(psi, g), gauge_fermion(phi, g), A, 0xB, sign)
    assert max_abs(chig - gauge_fermion(chi, g)) < 1e-13
    assert n2g == pytest.approx(n2, rel=1e-13)


def test_masks_add_up():
    # the hop over a mask is the sum of the hops over a split of the mask
    L = (3, 4, 2, 5)
    U = latgen.haar_links(L, 32)
    psi = latgen.dirac_field(L, 33)
    for sign in (+1, -1):
        full, _ = oracle.shift_expr(U, psi, None, 0.0, 0xF, sign)
        parts = sum(oracle.shift_expr(U, psi, None, 0.0, 1 << mu, sign)[0] for mu in range(4))
        assert max_abs(full - parts) < 1e-14
