"""Stored launch geometries.

``qdpx_tune`` times the candidate launch geometries of an operation on one
lattice shape and keeps the fastest in a context; this module stores such
choices in a JSON table so that later processes launch the same geometry
without re-tuning (and so that timing and counter runs measure the same
kernels).  Entries are keyed by (operation, precision, link format,
extents).

    python -m paper_1105_2279_amd.tuning [--out PATH]

tunes the shapes listed in ``SHAPES`` on the current GPU and writes the table.
"""

from __future__ import annotations

import argparse
import json
import os

from . import (F32, F64, LINK12, LINK18, OP_APE, OP_CHAIN, OP_JACOBI, OP_SHIFT, Context, qdpx_tune, qdpx_tune_get,
               qdpx_tune_set)

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "launch_table_mi355x.json")

_OPS = {"APE": OP_APE, "SHIFT": OP_SHIFT, "CHAIN": OP_CHAIN, "JACOBI": OP_JACOBI}
_PRECS = {"F64": F64, "F32": F32}
_FMTS = {"LINK18": LINK18, "LINK12": LINK12}
_FORMATS = (("F32", "LINK12"), ("F64", "LINK18"), ("F32", "LINK18"))
_TABLE1 = ((8, 8, 8, 16), (12, 12, 12, 24), (16, 16, 16, 32), (20, 20, 20, 40), (24, 24, 24, 48), (32, 32, 32, 64))

# The shapes the benchmark launches.
SHAPES = ([("APE", p, f, (32, 32, 32, 64)) for p, f in _FORMATS]
          + [("SHIFT", p, f, (32, 32, 32, 64)) for p, f in _FORMATS]
          + [("JACOBI", p, f, L) for L in _TABLE1 for p, f in _FORMATS])


def _key(op, prec, fmt, L):
    return (op, prec, fmt, tuple(int(x) for x in L))


def read(path=TABLE):
    """{(op, prec, fmt, L): (block, groups_per_wave, xcd_map, t_window)}; empty if there is no table."""
    try:
        with open(path) as fh:
            rows = json.load(fh)["entries"]
    except FileNotFoundError:
        return {}
    return {_key(r["op"], r["prec"], r["fmt"], r["L"]): tuple(r["launch"]) for r in rows}


def load(ctx, path=TABLE):
    """Set every stored geometry in ctx; returns the keys set."""
    table = read(path)
    for (op, prec, fmt, L), cfg in table.items():
        qdpx_tune_set(ctx, _OPS[op], L, _PRECS[prec], _FMTS[fmt], *cfg)
    return set(table)


def ensure(ctx, op, prec, fmt, L, table_keys):
    """Launch geometry for one shape: the stored one if ctx was loaded with
    it, else tuned now.  Returns (geometry, "table" | "tuned")."""
    names = ({v: k for k, v in _OPS.items()}[op], {v: k for k, v in _PRECS.items()}[prec],
             {v: k for k, v in _FMTS.items()}[fmt])
    if _key(*names, L) in table_keys:
        return qdpx_tune_get(ctx, op, L, prec, fmt), "table"
    qdpx_tune(ctx, op, L, prec, fmt)
    return qdpx_tune_get(ctx, op, L, prec, fmt), "tuned"


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()
    import torch

    torch.cuda.init()
    ctx = Context(0)
    rows = []
    for op, prec, fmt, L in SHAPES:
        qdpx_tune(ctx, _OPS[op], L, _PRECS[prec], _FMTS[fmt])
        cfg = qdpx_tune_get(ctx, _OPS[op], L, _PRECS[prec], _FMTS[fmt])
        rows.append({"op": op, "prec": prec, "fmt": fmt, "L": list(L), "launch": list(cfg)})
        print(f"{op} {prec} {fmt} {L}: {cfg}", flush=True)
    ctx.close()
    with open(args.out, "w") as fh:
        json.dump({"device": torch.cuda.get_device_properties(0).gcnArchName, "entries": rows}, fh, indent=1)
        fh.write("\n")
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
