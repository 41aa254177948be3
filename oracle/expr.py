"""Reference evaluator of lattice field expressions (test infrastructure).

Evaluates the expression language of the library's run-time compiled kernels
in complex128 with numpy, one whole-lattice array operation per node, from
the definition of each node:

    fK                field argument K (Dirac field, 4 spins x 3 colours)
    (shift E + mu)    E evaluated at x + mu;  (shift E - mu): at x - mu
    (umul mu E)       U_mu(x) E(x)            (colour matrix on each spin)
    (uadj mu E)       U_mu(x)^dagger E(x)
    (add E F)  (sub E F)  (scale sK E)        sK = scalar argument K
    (sum MASK E)      sum over the directions mu in MASK (hex bit mask) of
                      E with the direction variable m set to mu

A direction is a digit 0..3 (x, y, z, t) or the variable m of the enclosing
sum.  This is the QDP++ style of section 4 of the paper: the listing's
hopping term is (sum 0xF (add (umul m (shift f0 + m)) (shift (uadj m f0) - m))).
Only ``tests/`` use this module.
"""

from __future__ import annotations

import numpy as np


def tokenize(text: str):
    return text.replace("(", " ( ").replace(")", " ) ").split()


def parse(text: str):
    toks = tokenize(text)
    pos = 0

    def node():
        nonlocal pos
        t = toks[pos]
        pos += 1
        if t != "(":
            return t
        items = []
        while toks[pos] != ")":
            items.append(node())
        pos += 1
        return items

    tree = node()
    if pos != len(toks):
        raise ValueError("trailing tokens in expression")
    return tree


def _axis(mu: int) -> int:
    return 3 - mu  # canonical layout (Lt, Lz, Ly, Lx, ...)


def evaluate(text: str, U, fields, scalars=()):
    """Value of the expression for links U (Lt, Lz, Ly, Lx, 4, 3, 3) and
    fields [(Lt, Lz, Ly, Lx, 4, 3)], as a complex128 field."""
    U = np.asarray(U, dtype=np.complex128)
    fields = [np.asarray(f, dtype=np.complex128) for f in fields]

    def direction(tok, m):
        if tok == "m":
            if m is None:
                raise ValueError("direction variable m outside a sum")
            return m
        d = int(tok)
        if not 0 <= d <= 3:
            raise ValueError(f"direction {tok}")
        return d

    def ev(n, m):
        if isinstance(n, str):
            if n[0] != "f":
                raise ValueError(f"unknown leaf {n}")
            return fields[int(n[1:])]
        op = n[0]
        if op == "shift":
            _, e, sign, d = n
            mu = direction(d, m)
            step = {"+": -1, "-": +1}[sign]  # E(x + mu) is the array rolled by -1 along mu
            return np.roll(ev(e, m), step, axis=_axis(mu))
        if op in ("umul", "uadj"):
            _, d, e = n
            mu = direction(d, m)
            u = U[..., mu, :, :]
            if op == "uadj":
                u = np.conj(np.swapaxes(u, -1, -2))
            return np.einsum("...ab,...sb->...sa", u, ev(e, m))
        if op == "add":
            return ev(n[1], m) + ev(n[2], m)
        if op == "sub":
            return ev(n[1], m) - ev(n[2], m)
        if op == "scale":
            return scalars[int(n[1][1:])] * ev(n[2], m)
        if op == "sum":
            mask = int(n[1], 16)
            acc = 0
            for mu in range(4):
                if (mask >> mu) & 1:
                    acc = acc + ev(n[2], mu)
            return acc if not isinstance(acc, int) else np.zeros_like(fields[0])
        raise ValueError(f"unknown operation {op}")

    return ev(parse(text), None)
