"""Stored launch geometries.

``qdpx_tune`` times the candidate launch geometries of an operation on one
lattice shape and keeps the fastest in a context.  A context created with a
launch-table file (``Context(device, tune_cache=path)``, or
``$QDPX_TUNE_CACHE``) reads the file in the library and writes every tuned
geometry back to it, so later processes launch the same geometry without
re-tuning (and timing and counter runs measure the same kernels).  Entries
are keyed by (operation, precision, link format, extents).  ``TABLE`` is the
table stored with the package for the benchmark's shapes.

    python -m paper_1105_2279_amd.tuning [--out PATH] [--missing]

tunes the shapes listed in ``SHAPES``, and the batched call on the
benchmark's batch of 64 lattices (``BATCH_FORMATS``), on the current GPU into
that table.  Batched entries are keyed by the first lattice's extents.
"""

from __future__ import annotations

import argparse
import json
import os

from . import (F32, F64, LINK12, LINK18, OP_APE, OP_BATCHED, OP_CHAIN, OP_JACOBI, OP_SHIFT, Context, _tune_get,
               qdpx_tune, qdpx_tune_batched)

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "launch_table_mi355x.json")

_OPS = {"APE": OP_APE, "SHIFT": OP_SHIFT, "CHAIN": OP_CHAIN, "JACOBI": OP_JACOBI, "BATCHED": OP_BATCHED}
_PRECS = {"F64": F64, "F32": F32}
_FMTS = {"LINK18": LINK18, "LINK12": LINK12}
_FORMATS = (("F32", "LINK12"), ("F64", "LINK18"), ("F32", "LINK18"))
_TABLE1 = ((8, 8, 8, 16), (12, 12, 12, 24), (16, 16, 16, 32), (20, 20, 20, 40), (24, 24, 24, 48), (32, 32, 32, 64))

# The shapes the benchmark launches.
SHAPES = ([("APE", p, f, (32, 32, 32, 64)) for p, f in _FORMATS]
          + [("SHIFT", p, f, (32, 32, 32, 64)) for p, f in _FORMATS]
          + [("JACOBI", p, f, L) for L in _TABLE1 for p, f in _FORMATS]
          + [(op, p, f, (48, 48, 48, 96)) for op in ("APE", "CHAIN") for p, f in _FORMATS[:2]])
# The batched call: 5 APE steps over the benchmark's 64 lattices.
BATCH_FORMATS = (("F32", "LINK12"), ("F64", "LINK18"))
BATCH_STEPS = 5


def _key(op, prec, fmt, L):
    return (op, prec, fmt, tuple(int(x) for x in L))


def default_lds_tile(op, prec):
    """The library's LDS tile for an entry stored without one."""
    return 4 if (op == "APE" and prec == "F32") else 0


def read(path=TABLE):
    """{(op, prec, fmt, L): (block, groups_per_wave, xcd_map, t_window, lds_tile)}
    as stored in the file (lds_tile the default where an entry has none);
    empty if there is no table (for inspection: contexts read the file in the
    library)."""
    try:
        with open(path) as fh:
            rows = json.load(fh)["entries"]
    except FileNotFoundError:
        return {}
    out = {}
    for r in rows:
        launch = list(r["launch"])
        if len(launch) == 4:
            launch.append(default_lds_tile(r["op"], r["prec"]))
        out[_key(r["op"], r["prec"], r["fmt"], r["L"])] = tuple(launch)
    return out


def context(device=0, path=TABLE):
    """A context that launches the stored geometries (and stores what it tunes)."""
    return Context(device, tune_cache=path)


def ensure(ctx, op, prec, fmt, L):
    """Launch geometry for one shape: the one the context read from its
    table, else tuned now.  Returns (geometry, "table" | "tuned" | "set")."""
    cfg, src = _tune_get(ctx, op, L, prec, fmt)
    if src == "default":
        qdpx_tune(ctx, op, L, prec, fmt)
        cfg, src = _tune_get(ctx, op, L, prec, fmt)
    return cfg, src


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--missing", action="store_true", help="tune only the shapes the table does not hold yet")
    args = ap.parse_args()
    import torch

    torch.cuda.init()
    ctx = Context(0, tune_cache=args.out)
    have = read(args.out) if args.missing else {}
    for op, prec, fmt, L in SHAPES:
        if _key(op, prec, fmt, L) in have:
            continue
        qdpx_tune(ctx, _OPS[op], L, _PRECS[prec], _FMTS[fmt])  # written to the table by the library
        cfg, _ = _tune_get(ctx, _OPS[op], L, _PRECS[prec], _FMTS[fmt])
        print(f"{op} {prec} {fmt} {L}: {cfg}", flush=True)
    import sys

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from latgen import batch_extents  # the benchmark's batch of extents

    Ls = batch_extents()
    for prec, fmt in BATCH_FORMATS:
        if _key("BATCHED", prec, fmt, Ls[0]) in have:
            continue
        qdpx_tune_batched(ctx, Ls, _PRECS[prec], _FMTS[fmt], BATCH_STEPS)
        cfg, _ = _tune_get(ctx, OP_BATCHED, Ls[0], _PRECS[prec], _FMTS[fmt])
        print(f"BATCHED {prec} {fmt} {len(Ls)} lattices from {tuple(Ls[0])}: {cfg}", flush=True)
    ctx.close()
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
