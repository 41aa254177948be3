"""The oracle's pins catch plausible mistakes.

Each case copies ``oracle/oracle.c``, plants one mistake (a wrong shift, a
missing dagger, a transposed product, a dropped staple, a wrong weight, a
missing conjugate, a wrong sign or normalisation, a mask ignored, an extra or
unscaled series term), compiles the copy with the
oracle's own flags, and runs the pin tests against it in a fresh process.
The pins must fail for every mutant.  Nothing here touches the GPU.
"""

import os
import re
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_ape.py", "tests/test_oracle_shift.py", "tests/test_oracle_jacobi.py"]

MUTANTS = {
    "upper_staple_wrong_shift": ("mat3 b = load_link(U, hop(g, s, nu, +1), mu);",
                                 "mat3 b = load_link(U, hop(g, s, mu, +1), mu);"),
    "upper_staple_missing_dagger": ("mat3 cd = m_dag(&c);\n    mat3 ab = m_mul(&a, &b);",
                                    "mat3 cd = c;\n    mat3 ab = m_mul(&a, &b);"),
    "lower_staple_wrong_diagonal": ("mat3 c = load_link(U, hop(g, sm, mu, +1), nu);",
                                    "mat3 c = load_link(U, hop(g, s, mu, +1), nu);"),
    "lower_staple_transposed_product": ("mat3 ab = m_mul(&ad, &b);", "mat3 ab = m_mul(&b, &ad);"),
    "lower_staple_dropped": ("S = m_add(&S, &sl);", "S = m_add(&S, &su);"),
    "combine_wrong_weight": ("alpha / n : 0.0", "alpha / (n + 2) : 0.0"),
    "mask_ignored_in_staples": ("if (nu == mu || !((mask >> nu) & 1u)) continue;", "if (nu == mu) continue;"),
    "masked_direction_smeared": ("if (!((mask >> mu) & 1u)) {\n        *V = load_link(U, s, mu);",
                                 "if (0) {\n        *V = load_link(U, s, mu);"),
    "row3_missing_conj": ("V->e[2][1] = c_conj(c_sub(c_mul(u[2], v[0]), c_mul(u[0], v[2])));",
                          "V->e[2][1] = c_sub(c_mul(u[2], v[0]), c_mul(u[0], v[2]));"),
    "gram_schmidt_no_conj": ("d = c_add(d, c_mul(c_conj(u[j]), W->e[1][j]));",
                             "d = c_add(d, c_mul(u[j], W->e[1][j]));"),
    "plaquette_wrong_order": ("mat3 abc = m_mul(&ab, &cd);\n    mat3 p = m_mul(&abc, &dd);",
                              "mat3 abc = m_mul(&ab, &dd);\n    mat3 p = m_mul(&abc, &cd);"),
    "plaquette_wrong_norm": ("out[0] = (ssum + tsum) / (18.0 * (double)g.V);",
                             "out[0] = (ssum + tsum) / (9.0 * (double)g.V);"),
    "shift_backward": ("long fwd = hop(g, s, mu, +1);", "long fwd = hop(g, s, mu, -1);"),
    "shift_dagger_link": ("c_mul(u.e[ca][cb], load_fermion(psi, fwd, sp, cb))",
                          "c_mul(c_conj(u.e[cb][ca]), load_fermion(psi, fwd, sp, cb))"),
    "axpy_per_direction": ("acc[sp][c] = c_add(acc[sp][c], c_scale(a, load_fermion(phi, s, sp, c)));",
                           "acc[sp][c] = c_add(acc[sp][c], c_scale(4.0 * a, load_fermion(phi, s, sp, c)));"),
    "chain_wrong_sign": ("psi[i] = psi[i] - c * chi[i];", "psi[i] = psi[i] + c * chi[i];"),
    "hop_wrong_axis": ("c[mu] = ((c[mu] + step) % g->L[mu] + g->L[mu]) % g->L[mu];",
                       "c[(mu + 1) % 4] = ((c[(mu + 1) % 4] + step) % g->L[(mu + 1) % 4]"
                       " + g->L[(mu + 1) % 4]) % g->L[(mu + 1) % 4];"),
    "hop_backward_no_dagger": ("c_mul(c_conj(ub.e[cb][ca]), load_fermion(psi, bwd, sp, cb))",
                               "c_mul(ub.e[ca][cb], load_fermion(psi, bwd, sp, cb))"),
    "hop_backward_wrong_link_site": ("mat3 ub = load_link(U, bwd, mu);", "mat3 ub = load_link(U, s, mu);"),
    "jacobi_extra_term": ("for (int n = 1; n <= n_iter; ++n) {", "for (int n = 0; n <= n_iter; ++n) {"),
    "jacobi_term_not_scaled": ("term[i] = kappa * h[i];", "term[i] = h[i];"),
    "jacobi_norm_multiplied": ("chi[i] = sum[i] / norm;", "chi[i] = sum[i] * norm;"),
    "shift_backward_no_dagger": ("c_mul(c_conj(lb.e[cb][ca]), load_fermion(psi, back, sp, cb))",
                                 "c_mul(lb.e[ca][cb], load_fermion(psi, back, sp, cb))"),
    "shift_backward_link_at_x": ("mat3 lb = load_link(U, back, mu);", "mat3 lb = load_link(U, s, mu);"),
    "shift_mask_ignored": ("if (!((mask >> mu) & 1u)) continue;\n        if (sign > 0) {",
                           "if (0) continue;\n        if (sign > 0) {"),
    "polar_inverse_not_sqrt": ("f[k] = 1.0 / sqrt(lam[k]);", "f[k] = 1.0 / lam[k];"),
    "polar_no_phase_fix": ("double ph = -atan2(d.im, d.re) / 3.0;", "double ph = 0.0 * atan2(d.im, d.re);"),
    "polar_wrong_side": ("mat3 H = m_mul(&Wd, W);", "mat3 H = m_mul(W, &Wd);"),
    "jacobi_rotation_sign": ("A[k][p] = A[p][k] = c * akp - sn * akq;", "A[k][p] = A[p][k] = c * akp + sn * akq;"),
    "norm_drops_imag": ("static double c_abs2(cplx a) { return a.re * a.re + a.im * a.im; }",
                        "static double c_abs2(cplx a) { return a.re * a.re + a.im * a.im * 0.0 + 0.0 * a.re; }"),
}


def _build_mutant(name, tmp_path):
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not unique/present"
    path_c = tmp_path / f"{name}.c"
    path_so = tmp_path / f"lib{name}.so"
    path_c.write_text(src.replace(old, new))
    subprocess.run(["gcc", *oracle.CFLAGS, str(path_c), "-o", str(path_so), "-lm"], check=True)
    return str(path_so)


def test_unmutated_source_passes(tmp_path):
    so = tmp_path / "liborig.so"
    subprocess.run(["gcc", *oracle.CFLAGS, os.path.join(ROOT, "oracle", "oracle.c"), "-o", str(so), "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", *PIN_FILES], cwd=ROOT, env=env,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    so = _build_mutant(name, tmp_path)
    env = dict(os.environ, ORACLE_LIB=so)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", *PIN_FILES], cwd=ROOT, env=env,
                       capture_output=True, text=True)
    assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout[-1500:]}"
    assert re.search(r"\d+ failed", r.stdout), r.stdout[-1500:]
