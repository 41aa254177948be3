"""Pins of the reference expression evaluator: the hopping term of the
smearing operator, the shift expression and the Jacobi update written as
expressions equal the C oracle's dedicated routines (themselves pinned);
shifts compose and invert; unit links reduce hops to array rolls."""

import numpy as np
import pytest

import latgen
import oracle
from oracle import expr
from lathelp import bwd, fwd

HOP = "(sum 0xF (add (umul m (shift f0 + m)) (shift (uadj m f0) - m)))"
L = (4, 3, 2, 5)


@pytest.fixture(scope="module")
def data():
    return latgen.haar_links(L, 600), latgen.dirac_field(L, 601), latgen.dirac_field(L, 602)


def test_hop_expression_is_the_hopping_term(data):
    U, psi, _ = data
    assert np.max(np.abs(expr.evaluate(HOP, U, [psi]) - oracle.hop(U, psi))) < 1e-13
    spatial = HOP.replace("0xF", "0x7")
    assert np.max(np.abs(expr.evaluate(spatial, U, [psi]) - oracle.hop(U, psi, 0x7))) < 1e-13


def test_shift_expression(data):
    U, psi, phi = data
    e = "(add (sum 0xF (umul m (shift f0 + m))) (scale s0 f1))"
    ref, _ = oracle.shift_mul_axpy(U, psi, phi, 0.3)
    assert np.max(np.abs(expr.evaluate(e, U, [psi, phi], [0.3]) - ref)) < 1e-13


def test_jacobi_update_expression(data):
    U, chi, _ = data
    # one iteration of the listing: chi = s0 + kappa H psi with psi = s0 = chi
    e = f"(add f0 (scale s0 {HOP}))"
    got = expr.evaluate(e, U, [chi], [0.21])
    ref = oracle.jacobi_smear(U, chi, 0.21, 1)
    assert np.max(np.abs(got - ref)) < 1e-13


def test_shifts_compose_and_invert(data):
    U, psi, _ = data
    assert np.array_equal(expr.evaluate("(shift (shift f0 + 2) - 2)", U, [psi]), psi)
    assert np.array_equal(expr.evaluate("(shift f0 + 3)", U, [psi]), fwd(psi, 3))
    assert np.array_equal(expr.evaluate("(shift f0 - 1)", U, [psi]), bwd(psi, 1))


def test_unit_links_and_sub_scale(data):
    _, psi, phi = data
    U = latgen.unit_links(L)
    got = expr.evaluate("(sub (umul 1 (shift f0 + 1)) (scale s0 (uadj 2 f1)))", U, [psi, phi], [2.0])
    assert np.allclose(got, fwd(psi, 1) - 2.0 * phi, atol=1e-15)


def test_parse_errors():
    with pytest.raises(ValueError):
        expr.evaluate("(umul m f0)", latgen.unit_links(L), [np.zeros(L[::-1] + (4, 3))])
    with pytest.raises(ValueError):
        expr.parse("(add f0 f1) f2")


def test_uadj_undoes_umul_and_empty_sum_is_zero(data):
    """For SU(3) links U^dag U = 1, so uadj inverts umul site by site in either
    order; a sum over no direction is the zero field."""
    U, psi, _ = data
    for mu in range(4):
        for e in (f"(uadj {mu} (umul {mu} f0))", f"(umul {mu} (uadj {mu} f0))"):
            assert np.max(np.abs(expr.evaluate(e, U, [psi]) - psi)) < 1e-14, e
    zero = expr.evaluate("(sum 0x0 (umul m f0))", U, [psi])
    assert zero.shape == psi.shape and not np.any(zero)
