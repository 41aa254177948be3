"""Pins of the FP64 oracle's APE step, reunitarisation and plaquette.

Each pin is fixed by mathematics independent of the oracle's own code:
fixed points, gauge covariance, closed forms for abelian links, a library QR,
trace identities and Haar statistics.  Together they fail on a dropped staple,
a wrong staple orientation or shift, a transposed or non-daggered operand, a
wrong combination weight and a wrong projection.
"""

import math

import numpy as np
import pytest

import latgen
import oracle
from lathelp import (bwd, dag, det_defect, fwd, gauge_links, max_abs, pure_gauge,
                     unitarity_defect)

ALPHA = 0.5


def small_haar(L=(4, 4, 4, 4), seed=1105):
    return latgen.haar_links(L, seed)


# ---------------------------------------------------------------- fixed points
def test_unit_links_fixed_point():
    U = latgen.unit_links((4, 4, 4, 4))
    V = oracle.ape_step(U, ALPHA)
    assert max_abs(V - U) <= 1e-15
    assert np.allclose(oracle.plaquette(U), 1.0, atol=0, rtol=1e-15)
    assert np.allclose(oracle.plaquette(V), 1.0, atol=1e-15)


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (2, 3, 4, 5)])
def test_pure_gauge_fixed_point(L):
    # U_mu(x) = g(x) g(x+mu)^dagger is a gauge copy of the unit field: every
    # staple equals U_mu(x), so W = U and the projection returns U.
    g = latgen.haar_gauge(L, 21)
    U = pure_gauge(g)
    W = oracle.ape_w(U, ALPHA)
    assert max_abs(W - U) < 1e-14
    V = oracle.ape_step(U, ALPHA)
    assert max_abs(V - U) < 1e-14
    assert abs(oracle.plaquette(U)[0] - 1.0) < 1e-14


# ---------------------------------------------------------- gauge covariance
def test_w_gauge_covariant_haar():
    U = small_haar()
    g = latgen.haar_gauge((4, 4, 4, 4), 33)
    W = oracle.ape_w(U, ALPHA)
    Wg = oracle.ape_w(gauge_links(U, g), ALPHA)
    assert max_abs(Wg - gauge_links(W, g)) < 1e-13


def test_step_gauge_covariant_torus():
    # Row Gram-Schmidt commutes with right multiplication by SU(3) and with left
    # multiplication by diagonal unitaries, so the full step is covariant under
    # torus-valued gauge transformations.
    U = small_haar()
    g = latgen.torus_gauge((4, 4, 4, 4), 34)
    V = oracle.ape_step(U, ALPHA)
    Vg = oracle.ape_step(gauge_links(U, g), ALPHA)
    assert max_abs(Vg - gauge_links(V, g)) < 1e-13


def test_plaquette_gauge_invariant_haar():
    U = small_haar((2, 3, 4, 5), 40)
    g = latgen.haar_gauge((2, 3, 4, 5), 41)
    assert np.max(np.abs(oracle.plaquette(gauge_links(U, g)) - oracle.plaquette(U))) < 1e-15


# ------------------------------------------------------------ SU(3) output
def test_output_special_unitary():
    V = oracle.ape_step(small_haar(), ALPHA)
    assert unitarity_defect(V) < 1e-14
    assert det_defect(V) < 1e-14


# ---------------------------------------------------- abelian closed form
def _abelian(L, seed):
    rng = np.random.default_rng(seed)
    Lx, Ly, Lz, Lt = L
    th = rng.uniform(-np.pi, np.pi, (Lt, Lz, Ly, Lx, 4, 2))
    ang = np.concatenate([th, -(th[..., :1] + th[..., 1:])], axis=-1)  # (.., 4, 3)
    U = np.zeros((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
    for k in range(3):
        U[..., k, k] = np.exp(1j * ang[..., k])
    return ang, U


@pytest.mark.parametrize("L,mask", [((4, 4, 4, 4), 0xF), ((2, 3, 4, 5), 0xF), ((4, 4, 4, 4), 0x7),
                                    ((2, 3, 4, 5), 0xB)])
def test_abelian_closed_form(L, mask):
    # For diagonal links each colour component is a U(1) field with angle
    # th_mu(x); the staples become phases of sums of angles.  A smeared link
    # mixes (1 - alpha) of itself with alpha times the average of its staples
    # in the smeared directions; the other links are left alone.
    ang, U = _abelian(L, 55)
    W = oracle.ape_w(U, ALPHA, mask)
    V = oracle.ape_step(U, ALPHA, mask)
    dirs = [nu for nu in range(4) if (mask >> nu) & 1]
    Wexp = np.zeros(U.shape[:5] + (3,), dtype=np.complex128)
    for mu in range(4):
        th_mu = ang[..., mu, :]
        staples = []
        for nu in dirs:
            if nu == mu:
                continue
            th_nu = ang[..., nu, :]
            up = th_nu + fwd(th_mu, nu) - fwd(th_nu, mu)
            lo = -bwd(th_nu, nu) + bwd(th_mu, nu) + fwd(bwd(th_nu, nu), mu)
            staples += [np.exp(1j * up), np.exp(1j * lo)]
        Wexp[..., mu, :] = (1 - ALPHA) * np.exp(1j * th_mu) + ALPHA * np.mean(staples, axis=0)
    diag = np.diagonal(W, axis1=-2, axis2=-1)
    assert max_abs(diag - Wexp) < 1e-14
    off = W.copy()
    for k in range(3):
        off[..., k, k] = 0
    assert max_abs(off) == 0.0
    v0 = Wexp[..., 0] / np.abs(Wexp[..., 0])
    v1 = Wexp[..., 1] / np.abs(Wexp[..., 1])
    v2 = np.exp(-1j * (np.angle(Wexp[..., 0]) + np.angle(Wexp[..., 1])))
    vd = np.diagonal(V, axis1=-2, axis2=-1)
    for mu in range(4):
        if mu in dirs:
            assert max_abs(vd[..., mu, 0] - v0[..., mu]) < 1e-14
            assert max_abs(vd[..., mu, 1] - v1[..., mu]) < 1e-14
            assert max_abs(vd[..., mu, 2] - v2[..., mu]) < 1e-14
        else:
            assert np.array_equal(V[..., mu, :, :], U[..., mu, :, :])


# ------------------------------------------------- polar (bi-covariant) projection
def _phase_fixed(Vu):
    d = np.linalg.det(Vu)
    return Vu * np.exp(-1j * np.angle(d) / 3)[..., None, None]


def test_polar_matches_library_polar_decomposition():
    # The unitary factor of scipy's polar decomposition, with the phase of its
    # determinant removed on the principal branch.
    import scipy.linalg
    W = oracle.ape_w(small_haar((2, 3, 2, 2), 90), ALPHA).reshape(-1, 3, 3)
    W = np.concatenate([W, latgen._complex_gaussian(np.random.default_rng(91), (50, 3, 3))])
    V, bad = oracle.polar_project(W)
    assert bad == 0
    ref = _phase_fixed(np.array([scipy.linalg.polar(w)[0] for w in W]))
    assert max_abs(V - ref) < 1e-13


def test_polar_projection_is_bicovariant_and_su3():
    # well-conditioned inputs, as APE combinations are (the inverse square root
    # of W^dag W loses accuracy as the square of W's condition number)
    rng = np.random.default_rng(92)
    W = latgen.haar_su3(rng, 200) + 0.1 * latgen._complex_gaussian(rng, (200, 3, 3))
    g = latgen.haar_su3(rng, 200)
    h = latgen.haar_su3(rng, 200)
    V, _ = oracle.polar_project(W)
    Vg, _ = oracle.polar_project(g @ W @ dag(h))
    assert max_abs(Vg - g @ V @ dag(h)) < 1e-13
    assert unitarity_defect(V) < 1e-14 and det_defect(V) < 1e-14
    # a scaled SU(3) matrix projects to itself
    U = latgen.haar_su3(rng, 50)
    Vs, _ = oracle.polar_project(2.5 * U)
    assert max_abs(Vs - U) < 1e-14


def test_polar_step_gauge_covariant_haar():
    # With a bi-covariant projection the whole smearing step commutes with a
    # random (Haar) gauge transformation.
    U = small_haar()
    g = latgen.haar_gauge((4, 4, 4, 4), 93)
    for mask in (0xF, 0x7):
        V = oracle.ape_step(U, ALPHA, mask, proj=1)
        Vg = oracle.ape_step(gauge_links(U, g), ALPHA, mask, proj=1)
        assert max_abs(Vg - gauge_links(V, g)) < 1e-13


def test_polar_fixed_points():
    U = latgen.unit_links((2, 3, 2, 3))
    assert max_abs(oracle.ape_step(U, ALPHA, proj=1) - U) < 1e-15
    g = latgen.haar_gauge((2, 3, 4, 5), 94)
    P = pure_gauge(g)
    assert max_abs(oracle.ape_step(P, ALPHA, proj=1) - P) < 1e-13


def test_polar_abelian_closed_form():
    # Diagonal W: the polar factor is the diagonal of phases; the determinant
    # phase (principal branch) is then split evenly over the three entries.
    L = (3, 2, 4, 2)
    ang, U = _abelian(L, 95)
    W = oracle.ape_w(U, ALPHA)
    V = oracle.ape_step(U, ALPHA, proj=1)
    wd = np.diagonal(W, axis1=-2, axis2=-1)
    ph = wd / np.abs(wd)
    ph = ph * np.exp(-1j * np.angle(np.prod(ph, axis=-1)) / 3)[..., None]
    assert max_abs(np.diagonal(V, axis1=-2, axis2=-1) - ph) < 1e-14
    off = V.copy()
    for k in range(3):
        off[..., k, k] = 0
    assert max_abs(off) < 1e-15


# ------------------------------------------------- spatial-only smearing
def test_spatial_smearing_leaves_temporal_links_and_ignores_them():
    # With the three spatial directions smeared, temporal links are copied,
    # and spatial links depend on spatial links only.
    L = (4, 3, 2, 5)
    U = latgen.haar_links(L, 80)
    V = oracle.ape_step(U, ALPHA, 0x7)
    assert np.array_equal(V[..., 3, :, :], U[..., 3, :, :])
    U2 = U.copy()
    U2[..., 3, :, :] = latgen.haar_links(L, 81)[..., 3, :, :]
    V2 = oracle.ape_step(U2, ALPHA, 0x7)
    assert np.array_equal(V2[..., :3, :, :], V[..., :3, :, :])


def test_spatial_smearing_is_per_time_slice():
    # Each t-slice smears on its own: the slice taken as an Lt = 1 lattice
    # gives the same spatial links.
    L = (3, 4, 2, 3)
    U = latgen.haar_links(L, 82)
    V = oracle.ape_step(U, ALPHA, 0x7)
    for t in range(L[3]):
        Vt = oracle.ape_step(U[t:t + 1].copy(), ALPHA, 0x7)
        assert np.array_equal(Vt[0, ..., :3, :, :], V[t, ..., :3, :, :])


def test_masked_step_gauge_covariant_torus():
    U = small_haar()
    g = latgen.torus_gauge((4, 4, 4, 4), 83)
    for mask in (0x7, 0x5):
        V = oracle.ape_step(U, ALPHA, mask)
        Vg = oracle.ape_step(gauge_links(U, g), ALPHA, mask)
        assert max_abs(Vg - gauge_links(V, g)) < 1e-13


def test_single_direction_mask_only_projects():
    # One smeared direction has no staples: W = (1 - alpha) U, which projects
    # back to U.
    U = small_haar((2, 3, 2, 2), 84)
    V = oracle.ape_step(U, ALPHA, 0x2)
    assert max_abs(V - U) < 1e-14
    assert np.array_equal(oracle.ape_step(U, ALPHA, 0x0), U)


def test_abelian_plaquette_closed_form():
    L = (3, 4, 2, 5)
    ang, U = _abelian(L, 56)
    tot = sp = tp = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            ph = ang[..., mu, :] + fwd(ang[..., nu, :], mu) - fwd(ang[..., mu, :], nu) - ang[..., nu, :]
            s = float(np.sum(np.cos(ph)))
            tot += s
            if nu == 3:
                tp += s
            else:
                sp += s
    V = np.prod(L)
    ref = np.array([tot / (18 * V), sp / (9 * V), tp / (9 * V)])
    assert np.max(np.abs(oracle.plaquette(U) - ref)) < 1e-15


# -------------------------------------------- reunitarisation vs library QR
def test_reunitarise_matches_qr_of_transpose():
    # Row Gram-Schmidt of W is the unitary factor of the LQ decomposition
    # W = L Q; numpy's QR of W^T with the phases of R's diagonal removed
    # gives Q^T, whose first two columns are rows 0 and 1 of the result.
    rng = np.random.default_rng(77)
    W = rng.standard_normal((500, 3, 3)) + 1j * rng.standard_normal((500, 3, 3))
    V, bad = oracle.reunitarise(W)
    assert bad == 0
    q, r = np.linalg.qr(np.swapaxes(W, -1, -2))
    ph = np.diagonal(r, axis1=-2, axis2=-1)
    ph = ph / np.abs(ph)
    q = q * ph[:, None, :]
    assert max_abs(V[:, 0, :] - q[:, :, 0]) < 1e-14
    assert max_abs(V[:, 1, :] - q[:, :, 1]) < 1e-14
    assert unitarity_defect(V) < 1e-14
    assert det_defect(V) < 1e-14


def test_reunitarise_degenerate_counts():
    W = np.zeros((3, 3, 3), dtype=np.complex128)
    W[0] = np.eye(3)
    W[1][1, 1] = 1.0  # zero first row
    W[2][0, 0] = 1.0
    W[2][1, 0] = 2.0  # second row parallel to the first
    V, bad = oracle.reunitarise(W)
    assert bad == 2
    assert np.all(np.isfinite(V[0])) and np.all(np.isnan(V[1])) and np.all(np.isnan(V[2]))


def test_reunitarise_of_scaled_su3_is_identity_map():
    U = latgen.haar_su3(np.random.default_rng(5), 200)
    V, bad = oracle.reunitarise(3.7 * U)
    assert bad == 0
    assert max_abs(V - U) < 1e-14


# ---------------------------------------------- staple / plaquette identity
def test_staple_plaquette_identity():
    # sum_x sum_mu sum_{nu != mu} Re Tr[U_mu(x) S_mu(x)^dagger] equals twice the
    # sum of Re Tr over all plaquettes, for the upper and for the lower staples.
    L = (2, 3, 4, 5)
    U = latgen.haar_links(L, 60)
    up, lo = oracle.staple_sums(U)
    V = np.prod(L)
    plaq_sum = oracle.plaquette(U)[0] * 18 * V
    s_up = float(np.sum(U * np.conj(up)).real)
    s_lo = float(np.sum(U * np.conj(lo)).real)
    assert abs(s_up - 2 * plaq_sum) < 1e-12 * max(1.0, abs(plaq_sum))
    assert abs(s_lo - 2 * plaq_sum) < 1e-12 * max(1.0, abs(plaq_sum))


def test_w_is_weighted_staple_sum():
    # W = (1-alpha) U + (alpha/6)(S_up + S_lo), for any alpha
    U = latgen.haar_links((2, 2, 3, 3), 61)
    up, lo = oracle.staple_sums(U)
    for alpha in (0.0, 0.3, 0.5, 1.0):
        W = oracle.ape_w(U, alpha)
        assert max_abs(W - ((1 - alpha) * U + alpha / 6 * (up + lo))) < 1e-14


def test_upper_staple_single_plane_brute_force():
    # On a lattice that is trivial (unit links) except one random link, only
    # the staples that contain that link differ from 1.
    L = (3, 3, 3, 3)
    U = latgen.unit_links(L)
    X = latgen.haar_su3(np.random.default_rng(9), 1)[0]
    # link U_1 (y-direction) at site (x,y,z,t) = (1,1,1,1)
    U[1, 1, 1, 1, 1] = X
    up, lo = oracle.staple_sums(U)
    # upper staple of U_0 at (1,1,1,1) in nu=1: U_1(x) U_0(x+y) U_1(x+x)^dag = X
    # lower staple of U_0 at (1,2,1,1) in nu=1: U_1(x-y)^dag U_0(x-y) U_1(x-y+x) = X^dag
    # upper staple of U_0 at (0,1,1,1) in nu=1: U_1(x) U_0(x+y) U_1(x+x)^dag = X^dag
    # lower staple of U_0 at (0,2,1,1) in nu=1: U_1(x-y)^dag U_0(x-y) U_1(x-y+x) = X
    I = np.eye(3)
    assert max_abs(up[1, 1, 1, 1, 0] - (X + 2 * I)) < 1e-15
    assert max_abs(lo[1, 1, 2, 1, 0] - (X.conj().T + 2 * I)) < 1e-15
    assert max_abs(up[1, 1, 1, 0, 0] - (X.conj().T + 2 * I)) < 1e-15
    assert max_abs(lo[1, 1, 2, 0, 0] - (X + 2 * I)) < 1e-15
    # a link far away sees only unit staples
    assert max_abs(up[0, 0, 0, 0, 3] - 3 * I) < 1e-15


# --------------------------------------------------------- Haar statistics
def test_haar_plaquette_zero_mean_and_rises():
    L = (4, 4, 4, 4)
    V = np.prod(L)
    sigma = 1.0 / math.sqrt(108 * V)
    U = latgen.haar_links(L, 1105)
    p0 = oracle.plaquette(U)[0]
    assert abs(p0) < 5 * sigma
    U1 = oracle.ape_step(U, ALPHA)
    p1 = oracle.plaquette(U1)[0]
    assert p1 > p0 + 5 * sigma
    U2 = oracle.ape_step(U1, ALPHA)
    assert oracle.plaquette(U2)[0] > p1 + 5 * sigma


def test_smear_is_iterated_step():
    U = latgen.haar_links((2, 3, 2, 3), 70)
    V = oracle.ape_smear(U, ALPHA, 3)
    W = oracle.ape_step(oracle.ape_step(oracle.ape_step(U, ALPHA), ALPHA), ALPHA)
    assert np.array_equal(V, W)
    assert np.array_equal(oracle.ape_smear(U, ALPHA, 0), U)


def test_sampled_links_equal_full_step():
    U = latgen.haar_links((2, 3, 4, 5), 71)
    V = oracle.ape_step(U, ALPHA)
    rng = np.random.default_rng(0)
    sites = rng.integers(0, 120, 50)
    mus = rng.integers(0, 4, 50)
    got = oracle.ape_links(U, ALPHA, sites, mus)
    flat = V.reshape(-1, 4, 3, 3)
    assert np.array_equal(got, flat[sites, mus])


# ------------------------------------------------------------- reductions
def test_neumaier_matches_fsum():
    rng = np.random.default_rng(4)
    x = rng.standard_normal(4096) * np.exp(rng.uniform(-20, 20, 4096))
    x = np.concatenate([x, [1e16, 1.0, -1e16]])
    assert oracle.neumaier_sum(x) == pytest.approx(math.fsum(x), rel=0, abs=abs(math.fsum(x)) * 1e-15 + 1e-300)
    assert oracle.neumaier_sum(np.array([1e16, 1.0, -1e16])) == 1.0
