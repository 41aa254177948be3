"""Input generators: Haar moments, SU(3) properties, determinism, 12-real rebuild."""

import numpy as np
import pytest

import latgen
from lathelp import det_defect, unitarity_defect


def test_haar_su3_is_special_unitary():
    U = latgen.haar_su3(np.random.default_rng(7), 20000)
    assert unitarity_defect(U) < 1e-14
    assert det_defect(U) < 1e-14


def test_haar_moments():
    # Haar SU(3): E[Tr U] = 0, E|Tr U|^2 = 1, E|U_ij|^2 = 1/3, E[(Re Tr U)^2] = 1/2.
    n = 200000
    U = latgen.haar_su3(np.random.default_rng(11), n)
    tr = np.trace(U, axis1=-2, axis2=-1)
    se = 1.0 / np.sqrt(n)
    assert abs(np.mean(tr)) < 6 * se
    assert abs(np.mean(np.abs(tr) ** 2) - 1.0) < 6 * 1.5 * se
    assert abs(np.mean(np.abs(U) ** 2) - 1.0 / 3.0) < 6 * se
    assert abs(np.mean(tr.real ** 2) - 0.5) < 6 * se
    # the third-moment that separates SU(3) from U(3): E[Tr U^3]... E[(Tr U)^3] = 1 for SU(3)
    assert abs(np.mean(tr ** 3) - 1.0) < 6 * 3 * se


def test_haar_links_deterministic_and_slice_seeded():
    L = (3, 2, 2, 4)
    a = latgen.haar_links(L, 5)
    b = latgen.haar_links(L, 5)
    assert a.shape == (4, 2, 2, 3, 4, 3, 3)
    assert np.array_equal(a.view(np.float64), b.view(np.float64))
    # slice t of a larger-t lattice equals slice t of a smaller one with the same seed
    c = latgen.haar_links((3, 2, 2, 2), 5)
    assert np.array_equal(c.view(np.float64), a[:2].view(np.float64))
    assert not np.array_equal(latgen.haar_links(L, 6), a)


def test_row3_is_conj_cross_of_rows_1_2():
    # 12-real compression rebuilds row 3 as conj(r1 x r2); exact for SU(3).
    U = latgen.haar_su3(np.random.default_rng(3), 5000)
    r3 = np.conj(np.cross(U[:, 0, :], U[:, 1, :]))
    assert np.max(np.abs(r3 - U[:, 2, :])) < 1e-15 * 4


def test_near_unit_links():
    U = latgen.near_unit_links((2, 2, 2, 2), 9, eps=0.1)
    assert unitarity_defect(U) < 1e-14
    assert det_defect(U) < 1e-14
    dist = np.abs(U - np.eye(3)).max()
    assert 0.0 < dist < 0.6


def test_dirac_field_moments():
    psi = latgen.dirac_field((4, 4, 4, 8), 1)
    assert psi.shape == (8, 4, 4, 4, 4, 3)
    v = np.abs(psi) ** 2
    assert abs(v.mean() - 2.0) < 0.1


def test_gauge_generators():
    g = latgen.haar_gauge((2, 2, 2, 2), 3)
    assert unitarity_defect(g) < 1e-14 and det_defect(g) < 1e-14
    t = latgen.torus_gauge((2, 2, 2, 2), 3)
    assert unitarity_defect(t) < 1e-14 and det_defect(t) < 1e-14
    off = t.copy()
    for i in range(3):
        off[..., i, i] = 0
    assert np.abs(off).max() == 0


def test_batch_extents():
    ext = latgen.batch_extents()
    assert len(ext) == 64
    assert set(ext) <= set(latgen.BATCH_CHOICES)
    assert ext == latgen.batch_extents()
    assert len(set(ext)) == 4


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (2, 3, 4, 5)])
def test_as_real_roundtrip(L):
    U = latgen.haar_links(L, 1)
    r = latgen.as_real(U)
    assert r.shape == U.shape + (2,)
    assert np.array_equal(latgen.as_complex(r), U)
