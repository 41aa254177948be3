"""Benchmark: APE link smearing on a 32^3 x 64 lattice on one MI355X.

One timed step = 10 APE smearing steps (alpha = 0.5, one qdpx_ape_smear
call) of Haar-random SU(3) links, staple products in FP32 with links stored
as 12 reals, FP64 reunitarisation, then the FP64 plaquette of the smeared
links (qdpx_plaquette).  ``value`` is link updates per second,
4 * V * 10 * K / elapsed, with the links already resident in HBM.  The same
steps with the plaquette of every step's output are reported beside it.

The same JSON line carries the plain all-FP64 path for comparison, the
roofline of the dominant kernel (the APE step kernel, timed with HIP events
on its own stream), the FP64 CPU oracle timed on the host (cpu_baseline), and
secondary figures for the shift expression.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

L = (32, 32, 32, 64)
N_APE = 10
ALPHA = 0.5

# Peaks of the MI355X (published): HBM3E 8 TB/s; FP64 vector 78.6 TFLOP/s.
# FP32 vector is 157.3 TFLOP/s only with packed (two-wide) FP32 FMA; this
# library is built with packed FP32 disabled, so its FP32 arithmetic issues at
# the same rate as FP64: 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz.
PEAK_HBM_GBS = 8000.0
PEAK_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12  # 78.64

# Algorithmic work per link update of one APE step, the method's own count
# (the staple algorithm without reuse: 12 full 3x3 complex products of 198
# flop, the staple sum, the combination and the FP64 projection, plus for
# 12-real links the row-2 rebuild of the link read): the per-unit figure the
# roofline object is quoted on.
ALGO_FLOPS_PER_LINK = {"f32_12": 2562 + 126, "f64_18": 2646, "f32_18": 2646}

# Work per link update as this implementation executes it: rows 0
# and 1 of the six staples (two 2x3 by 3x3 complex products each), the
# combination, the FP64 projection, and the row-2 rebuilds of the links read
# as rows 0 and 1.  The FP32 step forms each plane's upper product
# P = U_mu(x+nu) U_nu(x+mu)^dag (rows 0 and 1, row 2 rebuilt) and the upper
# staple from it; at LDS tile levels 3 and 4 P is formed once per plane for
# the two link updates that share it (54 complex FMA per plane instead of
# 2 x 36), else by each.  Rebuilds per FP32-12 update: 3 per lower staple
# (2 with the backward links staged, plus 1 for staging), 2 per upper staple
# formed alone, 6 per plane at levels 3 and 4 from the shared product (4 per
# plane, 2 per link update: its link, P by the producer, P re-read by
# producer and consumer).  FP32-18 links are read whole: only P's row 2 is
# rebuilt (once per upper staple alone, 3 times per shared plane).  FP64
# update: 10 rebuilds (one backward link, three per plane).
CMAC_FLOPS = 8
LOWER_CMAC = 3 * 2 * 18  # three lower staples, two 2x3 by 3x3 products each
UPPER_CMAC = {False: 3 * 2 * 18, True: 3 * 54 // 2}  # upper staples: each alone / from a shared product
COMBINE_FLOPS = 12 * 2 * 3
PROJECT_FLOPS = 126
REBUILD_FLOPS = 42


def flops_per_link(name, lds=0):
    """Flop per link update of the APE step for a link format and LDS tile level."""
    shared = name != "f64_18" and lds in (3, 4)
    cmac = LOWER_CMAC + UPPER_CMAC[shared]
    if name == "f64_18":
        rebuilds2 = 2 * 10  # twice the rebuilds per link update
    elif name == "f32_12":
        staged = lds in (2, 3)
        rebuilds2 = 2 * (3 * (2 if staged else 3) + (1 if staged else 0)) + 2 * 6
    else:  # f32_18: only the products' row 2
        rebuilds2 = 3 * 3 if shared else 2 * 3
    return cmac * CMAC_FLOPS + COMBINE_FLOPS + PROJECT_FLOPS + rebuilds2 * REBUILD_FLOPS // 2


# Compulsory HBM bytes per link update: read the link once (the FP64 step
# reads rows 0 and 1 only), write it once.
BYTES_PER_LINK = {"f32_12": 2 * 48, "f64_18": 96 + 144, "f32_18": 2 * 72}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources of each counted kernel; a counter summary in profiles/ records
# their hash, and its HBM traffic is reported only while they are unchanged.
APE_SOURCES = ["su3_device.hpp", "ape_device.hpp", "ape.hip", "qdpx_impl.hpp"]
HOP_SOURCES = ["su3_device.hpp", "fields.hip", "qdpx_impl.hpp"]
APE_COUNTERS_MD = os.path.join(ROOT, "profiles", "ape_step_32x32x32x64_counters.md")
HOP_COUNTERS_MD = os.path.join(ROOT, "profiles", "jacobi_hop_32x32x32x64_counters.md")


def kernel_source_hash(sources):
    import hashlib

    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_1105_2279_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(md, sources, name):
    """HBM bytes per launch of one kernel from a committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel calibration), or None
    if the summary is missing or was taken on different kernel sources."""
    try:
        text = open(md).read()
    except OSError:
        return None
    import re

    m = re.search(r"source hash: `([0-9a-f]+)`", text)
    if not m or m.group(1) != kernel_source_hash(sources):
        return None
    m = re.search(r"traffic %s: ([0-9.eE+]+) bytes per launch" % re.escape(name), text)
    return float(m.group(1)) if m else None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=30)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extras", action="store_true")
    p.add_argument("--profile", action="store_true",
                   help="short run for hardware-counter profiling: one 1 GiB device copy (the calibration "
                        "kernel of known size), then two plaquette-free calls and two timed steps (10 APE steps and "
                        "the plaquette) of each APE link format, then four Jacobi hop launches per format, four "
                        "shift-expression launches (FP64-18, FP32-12), two batched calls on the 64-lattice batch "
                        "(FP32-12, FP64-18); no JSON line")
    return p.parse_args()


def time_calls(torch, fn, k, stream):
    """HIP-event elapsed milliseconds of k back-to-back calls on `stream`."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(k):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU t-slab design is not built",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import latgen
    import paper_1105_2279_amd as q
    from paper_1105_2279_amd import tuning

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    ctx = tuning.context(0)  # launches the stored geometries (the launch table the library reads)
    V = latgen.volume(L)
    t = time.time()
    U = latgen.haar_links(L, latgen.SEEDS["ape_32x32x32x64"]["links"])
    log(f"generated {L} Haar links in {time.time() - t:.1f} s")

    paths = {"f32_12": (q.F32, q.LINK12), "f64_18": (q.F64, q.LINK18), "f32_18": (q.F32, q.LINK18)}
    dev_links = {}
    for name, (prec, fmt) in paths.items():
        dev_links[name] = q.links_to_device(ctx, L, U, prec, fmt, dev)
    torch.cuda.synchronize()
    # launch geometry: the stored table of autotuner results, or the
    # autotuner now for shapes it lacks (not timed)
    tuned = {}
    for name, (prec, fmt) in paths.items():
        cfg, src = tuning.ensure(ctx, q.OP_APE, prec, fmt, L)
        tuned[name] = dict(zip(("block", "groups_per_wave", "xcd_map", "t_window", "lds_tile"), cfg), source=src)
        log(f"APE {name} launch: {tuned[name]}")

    works = {}

    def make_call(name, with_plaq=True, n=N_APE):
        prec, fmt = paths[name]
        out = q.alloc_links(L, prec, fmt, dev)
        work = q.alloc_workspace(q.OP_APE, L, prec, fmt, n, dev)
        works[name] = work
        plaq = torch.zeros(3 * (n + 1), dtype=torch.float64, device=dev) if with_plaq else None
        src = dev_links[name]

        def call():
            q.qdpx_ape_smear(ctx, L, prec, fmt, src, out, ALPHA, n, plaq, work, stream)

        return call, out, plaq

    results = {}

    def timed_step(name, per_step=False):
        """The timed workload on one link format: 10 APE steps (one
        qdpx_ape_smear call) and the FP64 plaquette of the smeared links
        (qdpx_plaquette), or with per_step the plaquette of the input and of
        every step's output from the smearing call itself.  Returns
        (enqueue(stream), output links, plaquettes)."""
        prec, fmt = paths[name]
        out = q.alloc_links(L, prec, fmt, dev)
        work = q.alloc_workspace(q.OP_APE, L, prec, fmt, N_APE, dev)
        work_p = q.alloc_workspace(q.OP_PLAQ, L, prec, fmt, 1, dev)
        plaq = torch.zeros(3 * (N_APE + 1) if per_step else 3, dtype=torch.float64, device=dev)
        src = dev_links[name]

        def enqueue(st):
            if per_step:
                q.qdpx_ape_smear(ctx, L, prec, fmt, src, out, ALPHA, N_APE, plaq, work, st)
            else:
                q.qdpx_ape_smear(ctx, L, prec, fmt, src, out, ALPHA, N_APE, None, work, st)
                q.qdpx_plaquette(ctx, L, prec, fmt, out, plaq, work_p, st)

        return enqueue, out, plaq

    def graph_of(enqueue):
        """The calls recorded once into a HIP graph (replayed on `stream`)."""
        enqueue(stream)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream()
        cs.wait_stream(stream)
        with torch.cuda.graph(g, stream=cs):
            enqueue(cs)
        g.replay()
        torch.cuda.synchronize()
        return g

    if args.profile:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
        # after tuning: two plaquette-free calls (the roofline kernel, mode 0)
        # then two timed steps (10 APE steps + the plaquette), per link format
        for name in paths:
            call, _, _ = make_call(name, with_plaq=False)
            call()
            call()
            step, _, _ = timed_step(name)
            step(stream)
            step(stream)
        # then, per format, the tuned Jacobi hop kernel, four launches
        psi = latgen.dirac_field(L, latgen.SEEDS["ape_32x32x32x64"]["links"] + 1)
        for name, (prec, fmt) in paths.items():
            tuning.ensure(ctx, q.OP_JACOBI, prec, fmt, L)
            pd = q.fermion_to_device(ctx, L, psi, prec, dev)
            h = q.alloc_fermion(L, prec, dev)
            for _ in range(4):
                q.qdpx_eval_hop(ctx, L, prec, fmt, dev_links[name], pd, h, 0xF, stream)
            torch.cuda.synchronize()
            del pd, h
        # the shift expression of the bench line, four launches per format
        profile_shift(torch, q, ctx, dev, stream, latgen)
        # the batched call on the 64-lattice batch, two calls per format
        profile_batched(torch, q, ctx, dev, stream, latgen)
        torch.cuda.synchronize()
        log("profile run done")
        ctx.close()
        return

    # ---------------------------------------------------------------- headline
    # One step = 10 APE steps + the FP64 plaquette of the result: the two
    # calls' kernel launches recorded once into a HIP graph and replayed.
    head, head_out, head_plaq = timed_step("f32_12")
    graph = graph_of(head)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps of {N_APE} FP32-12 APE steps + FP64 plaquette (graph replay)")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = 4.0 * V * N_APE * args.steps / elapsed
    log(f"headline: {value / 1e9:.2f} G link-updates/s, {1e3 * elapsed / args.steps:.3f} ms/step")
    # the same calls launched eagerly, for comparison
    for _ in range(2):
        head(stream)
    ms_eager = time_calls(torch, lambda: head(stream), args.steps, stream) / args.steps
    log(f"eager launches: {ms_eager:.3f} ms/step")
    # spread of single steps: graph replays each bracketed by its own events
    singles = sorted(time_calls(torch, graph.replay, 1, stream) for _ in range(max(20, args.steps)))
    spread = {"replays": len(singles), "median_ms": singles[len(singles) // 2], "min_ms": singles[0],
              "max_ms": singles[-1]}
    log(f"single steps: median {spread['median_ms']:.3f} ms, min {spread['min_ms']:.3f} ms")

    # ---------------------------------------- per-kernel timing of each path
    kernel = {}
    per_step_plaq = {}
    reps = max(3, args.steps // 3)
    for name in paths:
        call, _, _ = make_call(name, with_plaq=False)
        call()
        ms = time_calls(torch, call, reps, stream)
        per_kernel_s = ms / 1e3 / (reps * N_APE)
        kernel[name] = per_kernel_s
        log(f"{name}: APE kernel {per_kernel_s * 1e6:.1f} us")
        if name != "f32_12":
            # the same timed step as the headline (graph replay), other link format
            gr = graph_of(timed_step(name)[0])
            ms = time_calls(torch, gr.replay, reps, stream)
            results[name] = 4.0 * V * N_APE * reps / (ms / 1e3)
            log(f"{name}: {results[name] / 1e9:.2f} G link-updates/s (graph replay)")
            del gr
        if name != "f32_18":
            # the same 10 steps with the plaquette of every step's output
            gr = graph_of(timed_step(name, per_step=True)[0])
            ms = time_calls(torch, gr.replay, reps, stream) / reps
            per_step_plaq[name] = {"ms_per_step": ms, "link_updates_per_s": 4.0 * V * N_APE / (ms / 1e3)}
            log(f"{name}: {ms:.3f} ms with the plaquette of every step (graph replay)")
            del gr
    results["f32_12"] = value

    # ------------------------------ per-step errors (outside every timed region)
    samp_sites, samp_mus = error_sample(np, V)
    steps = step_by_step(torch, q, ctx, dev, stream, paths, dev_links, samp_sites, samp_mus)
    same_as_call = bool(torch.equal(steps["f32_12_final"], head_out))
    log(f"step-by-step FP32-12 output identical to the timed call: {same_as_call}")

    def roof(name):
        t_k = kernel[name]
        fpl = ALGO_FLOPS_PER_LINK[name]
        achieved = fpl * 4 * V / t_k / 1e12
        # what the kernel executes at its LDS tile level (fewer flops where
        # each plane's upper product is shared)
        fpl_x = flops_per_link(name, tuned[name]["lds_tile"])
        achieved_x = fpl_x * 4 * V / t_k / 1e12
        hbm = BYTES_PER_LINK[name] * 4 * V / t_k / 1e9
        return {
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": round(PEAK_VALU_TFLOPS, 2),
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_VALU_TFLOPS, 4),
            "traffic": measured_traffic(APE_COUNTERS_MD, APE_SOURCES, name),
            "kernel": {"f32_12": "k_ape_step<float,2>", "f64_18": "k_ape_step<double,3>",
                       "f32_18": "k_ape_step<float,3>"}[name],
            "kernel_us": round(t_k * 1e6, 2),
            "flops_per_link_update": fpl,
            "flops_per_link_update_executed": fpl_x,
            "achieved_executed": round(achieved_x, 3),
            "frac_executed": round(achieved_x / PEAK_VALU_TFLOPS, 4),
            "hbm_gbs_algorithmic": round(hbm, 1),
            "hbm_frac_algorithmic": round(hbm / PEAK_HBM_GBS, 4),
        }

    roofline = roof("f32_12")

    # --------------------------------------------------------- extras
    batch_check = None
    extras = {
        "fp64_18_link_updates_per_s": results["f64_18"],
        "fp32_18_link_updates_per_s": results["f32_18"],
        "speedup_fp32_12_vs_fp64": results["f32_12"] / results["f64_18"],
        "f32_12_eager_ms_per_step": ms_eager,
        "f32_12_eager_link_updates_per_s": 4.0 * V * N_APE / (ms_eager / 1e3),
        "f32_12_single_step_ms": spread,
        "ape_kernel_roofline": {k: roof(k) for k in paths},
        "tuned_launch": tuned,
        "plaquette_after_10_steps_f32_12": [float(x) for x in head_plaq.cpu().numpy()[-3:]],
        "with_plaquette_of_every_step": per_step_plaq,
        "errors_per_step_32x32x32x64": {
            "note": "step k = 1..10 of the timed workload; FP32-12 and FP64-18 GPU paths against each other on "
                    "every link, SU(3) defects on every link, and against the FP64 oracle on "
                    f"{len(samp_sites)} sampled links (the oracle's steps of the cpu_baseline leg)",
            "max_abs_f32_12_minus_f64_gpu": steps["d32_64"],
            "f32_12_max_unitarity_defect": steps["u32"],
            "f32_12_max_det_defect": steps["det32"],
            "f64_18_max_unitarity_defect": steps["u64"],
            "f64_18_max_det_defect": steps["det64"],
            "plaquette_f32_12": steps["plaq32"],
            "plaquette_f64_18": steps["plaq64"],
            "step_by_step_identical_to_timed_call": same_as_call,
        },
    }
    if not args.no_extras:
        extras.update(shift_extras(torch, q, ctx, dev, stream, latgen, np))
        bx, batch_check = batched_extras(torch, q, ctx, dev, stream, latgen)
        extras.update(bx)
        extras.update(jacobi_extras(torch, q, ctx, dev, stream, latgen))
        extras.update(jit_extras(torch, q, ctx, dev, stream, latgen))
        extras.update(pack_extras(torch, q, ctx, dev, stream, latgen, U))
        extras.update(large_extras(torch, q, ctx, dev, stream, latgen, np))

    # ------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu_baseline:
        cpu, oracle_err = cpu_baseline(U, steps, samp_sites, samp_mus)
        extras["errors_per_step_32x32x32x64"].update(oracle_err)
        if batch_check is not None:
            extras["batched_64_lattices"].update(batch_oracle_check(batch_check))
        extras["cpu_oracle_host"] = cpu_host_context(latgen)

    line = {
        "metric": "APE link-updates/s + HBM GB/s fraction, FP32/batched vs FP64, 32^3x64",
        "value": value,
        "unit": "link-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 staples / f64 projection and plaquette",
        "data": "synthetic: Haar-random SU(3) links, seed 1305",
        "config": {
            "workload": "APE smearing, 10 steps alpha=0.5 then the FP64 plaquette of the smeared links, "
                        "32^3x64 periodic, links FP32 12-real, FP64 projection",
            "lattice": list(L),
            "sites": V,
            "ape_steps_per_step": N_APE,
            "parallelism": "1 GPU",
            "tuned_launch": tuned["f32_12"],
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


# Algorithmic bytes per site of the shift expression: 4 links (FP64 links are
# read as rows 0 and 1, 96 B each), psi, phi and chi once each.
SHIFT_FORMATS = (("f64_18", "F64", "LINK18", 960), ("f32_12", "F32", "LINK12", 480))


_SHIFT_HOST = {}


def shift_inputs(torch, q, ctx, dev, latgen, Ls, prec, fmt):
    """Links, psi and phi of the shift expression on the device (host arrays generated once per shape)."""
    if Ls not in _SHIFT_HOST:
        seeds = latgen.SEEDS["shift_16x16x16x32"]
        _SHIFT_HOST[Ls] = (latgen.haar_links(Ls, seeds["links"]), latgen.dirac_field(Ls, seeds["psi"]),
                           latgen.dirac_field(Ls, seeds["phi"]))
    U, psi, phi = _SHIFT_HOST[Ls]
    return (q.links_to_device(ctx, Ls, U, prec, fmt, dev), q.fermion_to_device(ctx, Ls, psi, prec, dev),
            q.fermion_to_device(ctx, Ls, phi, prec, dev))


def profile_shift(torch, q, ctx, dev, stream, latgen):
    Ls = (32, 32, 32, 64)
    for name, p, f, _ in SHIFT_FORMATS:
        prec, fmt = getattr(q, p), getattr(q, f)
        Ud, pd, fd = shift_inputs(torch, q, ctx, dev, latgen, Ls, prec, fmt)
        chi = q.alloc_fermion(Ls, prec, dev)
        n2 = torch.zeros(1, dtype=torch.float64, device=dev)
        work = q.alloc_workspace(q.OP_SHIFT, Ls, prec, fmt, 1, dev)
        cfg, src = tuning_ensure(q, ctx, q.OP_SHIFT, prec, fmt, Ls)
        log(f"profile shift {name}: launch {cfg} ({src})")
        for _ in range(4):
            q.qdpx_eval_shift_mul_axpy(ctx, Ls, prec, fmt, Ud, pd, fd, 0.3, chi, n2, work, stream)
        torch.cuda.synchronize()
        del Ud, pd, fd, chi, work


def profile_batched(torch, q, ctx, dev, stream, latgen):
    """The batched call on the benchmark's 64 lattices, two calls per format.
    The counters measure cost, which does not depend on the link values, so
    the links are drawn from one pool of 2^20 Haar matrices instead of
    generated lattice by lattice (seconds instead of a minute per pass)."""
    import numpy as np

    Ls = latgen.batch_extents()
    pool = latgen.haar_su3(np.random.default_rng(latgen.SEEDS["batch_64"]["first_lattice"]), 1 << 20)

    def links(i, L):
        n = 4 * latgen.volume(L)
        idx = (np.arange(n, dtype=np.int64) * 7919 + 104729 * i) % len(pool)
        return pool[idx].reshape(L[3], L[2], L[1], L[0], 4, 3, 3)

    for name, prec, fmt in (("f32_12", q.F32, q.LINK12), ("f64_18", q.F64, q.LINK18)):
        src = q.qdpx_tune_source(ctx, q.OP_BATCHED, Ls[0], prec, fmt)
        if src == "default":  # tuning launches the same kernels: keep them out of the counted run
            raise SystemExit("profile: the launch table holds no batched entry for this batch; run the tuner first")
        Uds = [q.links_to_device(ctx, L, links(i, L), prec, fmt, dev) for i, L in enumerate(Ls)]
        outs = [q.alloc_links(L, prec, fmt, dev) for L in Ls]
        plaq = torch.zeros(3 * len(Ls), dtype=torch.float64, device=dev)
        work = q.alloc_workspace(q.OP_BATCHED, Ls, prec, fmt, len(Ls), dev)
        log(f"profile batched {name}: launch {q.qdpx_tune_get(ctx, q.OP_BATCHED, Ls[0], prec, fmt)} ({src})")
        for _ in range(2):
            q.qdpx_ape_smear_batched(ctx, Ls, prec, fmt, Uds, outs, ALPHA, 5, plaq, work, stream)
        torch.cuda.synchronize()
        del Uds, outs, work


def tuning_ensure(q, ctx, op, prec, fmt, Ls):
    from paper_1105_2279_amd import tuning

    return tuning.ensure(ctx, op, prec, fmt, Ls)


def pack_extras(torch, q, ctx, dev, stream, latgen, U):
    """Boundary staging at 32^3x64: the canonical FP64 links (already in device
    memory) into each library layout and back, outside every timed step."""
    Ls = (32, 32, 32, 64)
    V = latgen.volume(Ls)
    aos = torch.from_numpy(U.view("float64").reshape(-1)).to(dev)
    back = torch.empty_like(aos)
    aos_bytes = aos.numel() * 8
    out = {}
    for name, prec, fmt in (("f64_18", q.F64, q.LINK18), ("f32_18", q.F32, q.LINK18), ("f32_12", q.F32, q.LINK12)):
        soa = q.alloc_links(Ls, prec, fmt, dev)
        pack = lambda: q.qdpx_pack_links(ctx, Ls, aos, prec, fmt, soa, stream)
        unpack = lambda: q.qdpx_unpack_links(ctx, Ls, soa, prec, fmt, back, stream)
        pack(), unpack()
        torch.cuda.synchronize()
        ms_p = time_calls(torch, pack, 5, stream) / 5
        ms_u = time_calls(torch, unpack, 5, stream) / 5
        moved = aos_bytes + soa.numel()
        out[name] = {"pack_ms": ms_p, "unpack_ms": ms_u, "pack_gbs": moved / (ms_p / 1e3) / 1e9,
                     "unpack_gbs": moved / (ms_u / 1e3) / 1e9}
        log(f"pack {name}: {ms_p:.2f} ms, unpack {ms_u:.2f} ms for {V} sites")
        del soa
    return {"pack_unpack_links_32x32x32x64": out}


def shift_extras(torch, q, ctx, dev, stream, latgen, np):
    """Shift expression chi = sum_mu U psi(x+mu) + a phi at 32^3x64 (FP64 and FP32-12)."""
    from paper_1105_2279_amd import tuning

    Ls = (32, 32, 32, 64)
    V = latgen.volume(Ls)
    out = {}
    for name, p, f, bytes_site in SHIFT_FORMATS:
        prec, fmt = getattr(q, p), getattr(q, f)
        Ud, pd, fd = shift_inputs(torch, q, ctx, dev, latgen, Ls, prec, fmt)
        chi = q.alloc_fermion(Ls, prec, dev)
        n2 = torch.zeros(1, dtype=torch.float64, device=dev)
        work = q.alloc_workspace(q.OP_SHIFT, Ls, prec, fmt, 1, dev)
        tuning.ensure(ctx, q.OP_SHIFT, prec, fmt, Ls)

        def call():
            q.qdpx_eval_shift_mul_axpy(ctx, Ls, prec, fmt, Ud, pd, fd, 0.3, chi, n2, work, stream)

        call()
        reps = 20
        ms = time_calls(torch, call, reps, stream)
        t = ms / 1e3 / reps
        gbs = bytes_site * V / t / 1e9
        out[f"shift_{name}_32x32x32x64"] = {
            "tuned_launch": q.qdpx_tune_get(ctx, q.OP_SHIFT, Ls, prec, fmt),
            "sites_per_s": V / t,
            "us_per_call": t * 1e6,
            "hbm_gbs_algorithmic": gbs,
            "hbm_frac": gbs / PEAK_HBM_GBS,
        }
        log(f"shift {name}: {t * 1e6:.1f} us, {gbs:.0f} GB/s")
        del Ud, pd, fd, chi, work
    return out


# Jacobi smearing (section 7): flops per site and iteration as counted here:
# 8 SU(3) x colour-vector products per spin component (4 x 8 x 66), the sum
# of the 8 hop terms (7 x 12 complex adds) and chi = s0 + kappa h (12 x 4).
JACOBI_FLOPS_SITE_ITER = 4 * 8 * 66 + 7 * 12 * 2 + 12 * 4  # 2328
# Sustained GFLOPS of the whole smearing routine in the paper's Table 1
# (GTX 480 GPU, Xeon E5507 CPU): context only, the flop convention and the
# number of iterations are not stated there.
JACOBI_PAPER_GFLOPS = {
    (8, 8, 8, 16): {"sp_gpu": 1.64, "dp_gpu": 1.49},
    (12, 12, 12, 24): {"sp_gpu": 6.53, "dp_gpu": 4.41},
    (16, 16, 16, 32): {"sp_gpu": 11.86, "dp_gpu": 6.26},
    (20, 20, 20, 40): {"sp_gpu": 16.56, "dp_gpu": 7.51},
    (24, 24, 24, 48): {"sp_gpu": 19.09, "dp_gpu": 7.91},
    (32, 32, 32, 64): {"sp_gpu": 21.31, "dp_gpu": None},
}
N_JACOBI = 20
KAPPA_JACOBI = 0.21


def jacobi_extras(torch, q, ctx, dev, stream, latgen):
    """The whole Jacobi routine (copy, N_JACOBI fused hop+axpy iterations,
    division by the norm) on the lattices of the paper's Table 1, FP32 with
    12-real and 18-real links and FP64, each call replayed from a HIP graph;
    plus the hop kernel alone at 32^3x64 against the HBM roofline."""
    from paper_1105_2279_amd import tuning

    out = {}
    paths = (("sp_f32_12", q.F32, q.LINK12, 48, 96), ("sp_f32_18", q.F32, q.LINK18, 72, 96),
             ("dp_f64_18", q.F64, q.LINK18, 96, 192))  # link bytes read: FP64 rows 0 and 1
    for L, paper in JACOBI_PAPER_GFLOPS.items():
        V = latgen.volume(L)
        seeds = latgen.SEEDS["jacobi_table1"]
        U = latgen.haar_links(L, seeds["links"] + L[0])
        chi = latgen.dirac_field(L, seeds["chi"] + L[0])
        row = {"paper_gtx480_gflops": paper}
        for name, prec, fmt, link_b, ferm_b in paths:
            Ud = q.links_to_device(ctx, L, U, prec, fmt, dev)
            cd = q.fermion_to_device(ctx, L, chi, prec, dev)
            work = q.alloc_workspace(q.OP_JACOBI, L, prec, fmt, N_JACOBI, dev)
            tuning.ensure(ctx, q.OP_JACOBI, prec, fmt, L)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            s = torch.cuda.Stream()
            s.wait_stream(stream)
            with torch.cuda.graph(g, stream=s):
                q.qdpx_jacobi_smear(ctx, L, prec, fmt, Ud, cd, KAPPA_JACOBI, N_JACOBI, 1.0, 0xF, work, s)
            g.replay()
            reps = 10
            ms = time_calls(torch, g.replay, reps, stream) / reps
            gflops = JACOBI_FLOPS_SITE_ITER * V * N_JACOBI / (ms / 1e3) / 1e9
            row[name] = {"ms_per_call": round(ms, 4), "gflops": round(gflops, 1),
                         "tuned_launch": q.qdpx_tune_get(ctx, q.OP_JACOBI, L, prec, fmt)}
            if L == (32, 32, 32, 64):
                h = q.alloc_fermion(L, prec, dev)

                def hop():
                    q.qdpx_eval_hop(ctx, L, prec, fmt, Ud, cd, h, 0xF, stream)

                hop()
                t = time_calls(torch, hop, 20, stream) / 20 / 1e3
                # compulsory bytes: 4 links, psi, out (the iteration adds s0)
                gbs = (4 * link_b + 2 * ferm_b) * V / t / 1e9
                row[name]["hop_kernel"] = {"us": round(t * 1e6, 2), "hbm_gbs_algorithmic": round(gbs, 1),
                                           "hbm_frac": round(gbs / PEAK_HBM_GBS, 4),
                                           "traffic": measured_traffic(HOP_COUNTERS_MD, HOP_SOURCES,
                                                                       name.split("_", 1)[1])}
                del h
            log(f"jacobi {L} {name}: {ms:.3f} ms / {N_JACOBI} iterations, {gflops:.0f} GFLOPS")
            del Ud, cd, work, g
        out["x".join(map(str, L))] = row
    return {"jacobi_smearing": {"iterations": N_JACOBI, "kappa": KAPPA_JACOBI, "directions": 4,
                                "flops_per_site_iteration": JACOBI_FLOPS_SITE_ITER, "lattices": out}}


def jit_extras(torch, q, ctx, dev, stream, latgen):
    """The listing's hopping term as a run-time compiled expression kernel
    (generated, compiled with hipRTC or loaded from the on-disk cache) against
    the hand-written hop kernel, 32^3x64."""
    Lj = (32, 32, 32, 64)
    V = latgen.volume(Lj)
    hop = "(sum 0xF (add (umul m (shift f0 + m)) (shift (uadj m f0) - m)))"
    U = latgen.haar_links(Lj, 1305)
    psi = latgen.dirac_field(Lj, 1306)
    out = {}
    # link bytes read: FP64 links as rows 0 and 1 (both kernels)
    for name, prec, fmt, link_b, ferm_b in (("f32_12", q.F32, q.LINK12, 48, 96), ("f64_18", q.F64, q.LINK18, 96, 192)):
        t0 = time.perf_counter()
        k = q.qdpx_jit_compile(ctx, hop, prec, fmt, 1, 0)
        t_compile = time.perf_counter() - t0
        cached, _ = q.qdpx_jit_info(ctx, k)
        Ud = q.links_to_device(ctx, Lj, U, prec, fmt, dev)
        pd = q.fermion_to_device(ctx, Lj, psi, prec, dev)
        o1, o2 = q.alloc_fermion(Lj, prec, dev), q.alloc_fermion(Lj, prec, dev)

        def jit():
            q.qdpx_jit_eval(ctx, k, Lj, Ud, [pd], [], o1, stream=stream)

        def hand():
            q.qdpx_eval_hop(ctx, Lj, prec, fmt, Ud, pd, o2, 0xF, stream)

        jit()
        hand()
        tj = time_calls(torch, jit, 20, stream) / 20 / 1e3
        th = time_calls(torch, hand, 20, stream) / 20 / 1e3
        gbs = (4 * link_b + 2 * ferm_b) * V / tj / 1e9
        out[name] = {"compile_or_load_s": round(t_compile, 3), "from_disk_cache": bool(cached),
                     "jit_us": round(tj * 1e6, 1), "hand_written_us": round(th * 1e6, 1),
                     "jit_hbm_gbs_algorithmic": round(gbs, 1), "jit_over_hand": round(tj / th, 3)}
        log(f"jit hop {name}: {tj * 1e6:.1f} us (hand-written {th * 1e6:.1f} us), compile/load {t_compile:.2f} s")
        del Ud, pd, o1, o2
    return {"jit_hop_32x32x32x64": out}


LARGE = (48, 48, 48, 96)
N_LARGE_APE = 20
N_CHAIN = 8


def large_extras(torch, q, ctx, dev, stream, latgen, np):
    """The large single lattice, 48^3x96: 20 APE steps and the plaquette of
    the result (the per-step plaquettes from one more, untimed call), then
    the fused shift-expression chain psi <- psi - 0.1 chi,
    chi = sum_mu U_mu(x) psi(x+mu) + 0.3 phi, 8 times on the smeared links;
    FP32-12 (FP64 projection and reductions) against the plain FP64-18 GPU
    path.  Haar links are timed (each call replayed from a HIP graph) and
    compared; near-unit links are compared; unit links are checked as a fixed
    point."""
    from paper_1105_2279_amd import tuning

    Ls = LARGE
    V = latgen.volume(Ls)
    seeds = latgen.SEEDS["large_48x48x48x96"]
    t = time.time()
    U = latgen.haar_links(Ls, seeds["links_haar"])
    psi = latgen.dirac_field(Ls, seeds["psi"])
    phi = latgen.dirac_field(Ls, seeds["phi"])
    log(f"large: generated 48^3x96 Haar links and fields in {time.time() - t:.1f} s")
    paths = (("f32_12", q.F32, q.LINK12, 48, 480), ("f64_18", q.F64, q.LINK18, 96, 960))  # bytes read per link, per site
    res, full, psi_out, norms_out = {}, {}, {}, {}
    for name, prec, fmt, link_b, site_b in paths:
        launch = {"ape": tuning.ensure(ctx, q.OP_APE, prec, fmt, Ls),
                  "chain": tuning.ensure(ctx, q.OP_CHAIN, prec, fmt, Ls)}
        Ud = q.links_to_device(ctx, Ls, U, prec, fmt, dev)
        Vd = q.alloc_links(Ls, prec, fmt, dev)
        work = q.alloc_workspace(q.OP_APE, Ls, prec, fmt, N_LARGE_APE, dev)
        work_p = q.alloc_workspace(q.OP_PLAQ, Ls, prec, fmt, 1, dev)
        plaq = torch.zeros(3 * (N_LARGE_APE + 1), dtype=torch.float64, device=dev)
        plaq_end = torch.zeros(3, dtype=torch.float64, device=dev)
        pd = q.fermion_to_device(ctx, Ls, psi, prec, dev)
        pd0 = pd.clone()
        fd = q.fermion_to_device(ctx, Ls, phi, prec, dev)
        norms = torch.zeros(N_CHAIN, dtype=torch.float64, device=dev)
        cwork = q.alloc_workspace(q.OP_CHAIN, Ls, prec, fmt, N_CHAIN, dev)
        torch.cuda.synchronize()
        graphs = []
        def smear_and_plaquette(st):
            q.qdpx_ape_smear(ctx, Ls, prec, fmt, Ud, Vd, ALPHA, N_LARGE_APE, None, work, st)
            q.qdpx_plaquette(ctx, Ls, prec, fmt, Vd, plaq_end, work_p, st)

        for fn in (smear_and_plaquette,
                   lambda st: q.qdpx_shift_chain(ctx, Ls, prec, fmt, Vd, pd, fd, 0.3, 0.1, N_CHAIN, norms, cwork,
                                                 st)):
            g = torch.cuda.CUDAGraph()
            cs = torch.cuda.Stream()
            cs.wait_stream(stream)
            with torch.cuda.graph(g, stream=cs):
                fn(cs)
            graphs.append(g)
        g_ape, g_chain = graphs
        g_ape.replay()
        g_chain.replay()
        torch.cuda.synchronize()
        ms_ape = time_calls(torch, g_ape.replay, 3, stream) / 3
        ms_chain = time_calls(torch, g_chain.replay, 3, stream) / 3
        # the results: the smeared links are those of every replay (and of
        # the untimed call that reports every step's plaquette); the chain
        # runs once more from the initial psi
        q.qdpx_ape_smear(ctx, Ls, prec, fmt, Ud, Vd, ALPHA, N_LARGE_APE, plaq, work, stream)
        pd.copy_(pd0)
        g_chain.replay()
        torch.cuda.synchronize()
        full[name] = unpack_device(torch, q, ctx, Ls, Vd, prec, fmt, dev).reshape(-1, 3, 3)
        psi_out[name] = torch.empty((V, 4, 3, 2), dtype=torch.float64, device=dev)  # canonical FP64 layout
        q.qdpx_unpack_fermion(ctx, Ls, pd, prec, psi_out[name])
        norms_out[name] = norms.cpu().numpy()
        u, d = su3_defects_device(torch, full[name])
        ups = 4.0 * V * N_LARGE_APE / (ms_ape / 1e3)
        res[name] = {
            "launch": {k: {"geometry": v[0], "source": v[1]} for k, v in launch.items()},
            "ape_20_steps_and_plaquette_ms": round(ms_ape, 3),
            "final_plaquette_of_timed_call": [float(x) for x in plaq_end.cpu().numpy()],
            "final_plaquette_equals_per_step_call": bool(torch.equal(plaq_end, plaq[-3:])),
            "ape_link_updates_per_s": ups,
            "ape_hbm_gbs_algorithmic": round(BYTES_PER_LINK[name] * ups / 1e9, 1),
            "chain_8_iterations_ms": round(ms_chain, 3),
            "chain_hbm_gbs_algorithmic": round(site_b * V * N_CHAIN / (ms_chain / 1e3) / 1e9, 1),
            "chain_hbm_frac": round(site_b * V * N_CHAIN / (ms_chain / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
            "plaquettes": plaq.cpu().numpy().reshape(-1, 3)[[0, 1, 5, 10, 20]].tolist(),
            "max_unitarity_defect": u,
            "max_det_defect": d,
            "chain_norms": norms_out[name].tolist(),
        }
        log(f"large {name}: 20 APE steps + plaquette {ms_ape:.2f} ms ({ups / 1e9:.2f} G link-updates/s), chain "
            f"{ms_chain:.2f} ms ({res[name]['chain_hbm_gbs_algorithmic']} GB/s)")
        del Ud, Vd, work, work_p, pd, pd0, fd, cwork, g_ape, g_chain, graphs
    d_links = float((full["f32_12"] - full["f64_18"]).abs().max())
    dpsi = psi_out["f32_12"] - psi_out["f64_18"]
    ref = psi_out["f64_18"]
    chain_rel = float(dpsi.square().sum().sqrt() / ref.square().sum().sqrt())
    chain_maxrel = float(dpsi.abs().max() / ref.abs().max())
    norm_rel = float(np.max(np.abs(norms_out["f32_12"] - norms_out["f64_18"]) / norms_out["f64_18"]))
    del full, psi_out, dpsi, ref
    log(f"large: after 20 steps max |V32 - V64| {d_links:.2e}; chain psi rel. difference {chain_rel:.2e}")
    # near-unit links: FP32-12 against FP64 after 20 steps; unit links: fixed point
    t = time.time()
    Un = latgen.near_unit_links(Ls, seeds["links_near_unit"])
    log(f"large: generated near-unit links in {time.time() - t:.1f} s")
    near, pl = {}, {}
    for name, prec, fmt, _, _ in paths:
        Ud = q.links_to_device(ctx, Ls, Un, prec, fmt, dev)
        Vd = q.alloc_links(Ls, prec, fmt, dev)
        work = q.alloc_workspace(q.OP_APE, Ls, prec, fmt, N_LARGE_APE, dev)
        plaq = torch.zeros(3 * (N_LARGE_APE + 1), dtype=torch.float64, device=dev)
        q.qdpx_ape_smear(ctx, Ls, prec, fmt, Ud, Vd, ALPHA, N_LARGE_APE, plaq, work, stream)
        near[name] = unpack_device(torch, q, ctx, Ls, Vd, prec, fmt, dev).reshape(-1, 3, 3)
        pl[name] = plaq.cpu().numpy().reshape(-1, 3)
        del Ud, Vd, work
    del Un
    un32, _ = su3_defects_device(torch, near["f32_12"])
    d_near = float((near["f32_12"] - near["f64_18"]).abs().max())
    del near
    Uu = latgen.unit_links(Ls)
    Ud = q.links_to_device(ctx, Ls, Uu, q.F32, q.LINK12, dev)
    del Uu
    Vd = q.alloc_links(Ls, q.F32, q.LINK12, dev)
    work = q.alloc_workspace(q.OP_APE, Ls, q.F32, q.LINK12, N_LARGE_APE, dev)
    plaq = torch.zeros(3 * (N_LARGE_APE + 1), dtype=torch.float64, device=dev)
    q.qdpx_ape_smear(ctx, Ls, q.F32, q.LINK12, Ud, Vd, ALPHA, N_LARGE_APE, plaq, work, stream)
    unit = unpack_device(torch, q, ctx, Ls, Vd, q.F32, q.LINK12, dev).reshape(-1, 3, 3)
    eye = torch.eye(3, dtype=torch.complex128, device=dev)
    unit_dev = float((unit - eye).abs().max())
    unit_plaq = float(plaq.abs().sub(1.0).abs().max())
    del unit, Ud, Vd, work
    log(f"large: near-unit max |V32 - V64| {d_near:.2e}; unit links max |V - 1| {unit_dev:.2e}")
    speed = res["f32_12"]["ape_link_updates_per_s"] / res["f64_18"]["ape_link_updates_per_s"]
    return {"large_48x48x48x96": {
        "sites": V, "ape_steps": N_LARGE_APE, "chain_iterations": N_CHAIN, "a": 0.3, "c": 0.1,
        "haar": res,
        "ape_speedup_f32_12_vs_f64": speed,
        "chain_speedup_f32_12_vs_f64": res["f64_18"]["chain_8_iterations_ms"] / res["f32_12"]["chain_8_iterations_ms"],
        "errors": {
            "haar_max_abs_f32_12_minus_f64_after_20_steps": d_links,
            "chain_psi_rel_norm_f32_12_vs_f64": chain_rel,
            "chain_psi_max_abs_over_max_ref_f32_12_vs_f64": chain_maxrel,
            "chain_norms_max_rel_f32_12_vs_f64": norm_rel,
            "near_unit_max_abs_f32_12_minus_f64_after_20_steps": d_near,
            "near_unit_f32_12_max_unitarity_defect": un32,
            "near_unit_plaquette_f32_12_input_and_20": [pl["f32_12"][0].tolist(), pl["f32_12"][-1].tolist()],
            "near_unit_plaquette_f64_18_input_and_20": [pl["f64_18"][0].tolist(), pl["f64_18"][-1].tolist()],
            "unit_links_f32_12_max_abs_v_minus_1_after_20_steps": unit_dev,
            "unit_links_f32_12_max_abs_plaquette_minus_1": unit_plaq,
        },
    }}


def batched_extras(torch, q, ctx, dev, stream, latgen):
    """64 lattices with extents drawn from 8^4, 12^3x24, 16^3x32, 24^3x48; 5 APE
    steps + final FP64 plaquettes, FP32-12 and FP64-18: the batched call (its
    launch geometry from the autotuner on this batch) replayed from a
    captured HIP graph, against the loop of 64 single-lattice calls (5 steps
    and the plaquette of the result each) in both formats.  Returns the
    extras and lattice 0's links (input, FP32-12 and FP64-18 results) for the
    oracle check of the cpu_baseline leg."""
    import numpy as np

    n = 5
    Ls = latgen.batch_extents()
    seed0 = latgen.SEEDS["batch_64"]["first_lattice"]
    t = time.time()
    hosts = [latgen.haar_links(L, seed0 + i) for i, L in enumerate(Ls)]
    log(f"batched: generated 64 lattices in {time.time() - t:.1f} s")
    sites = sum(latgen.volume(L) for L in Ls)
    updates = 4.0 * sites * n
    reps = 10
    res, check = {}, {"U": hosts[0], "L": Ls[0]}
    for name, prec, fmt in (("f32_12", q.F32, q.LINK12), ("f64_18", q.F64, q.LINK18)):
        Uds = [q.links_to_device(ctx, L, U, prec, fmt, dev) for L, U in zip(Ls, hosts)]
        # launch geometry: the stored one for this batch, else the autotuner now
        src = q.qdpx_tune_source(ctx, q.OP_BATCHED, Ls[0], prec, fmt)
        if src == "default":
            q.qdpx_tune_batched(ctx, Ls, prec, fmt, n)
            src = q.qdpx_tune_source(ctx, q.OP_BATCHED, Ls[0], prec, fmt)
        geometry = q.qdpx_tune_get(ctx, q.OP_BATCHED, Ls[0], prec, fmt)
        outs = [q.alloc_links(L, prec, fmt, dev) for L in Ls]
        plaq = torch.zeros(3 * len(Ls), dtype=torch.float64, device=dev)
        work = q.alloc_workspace(q.OP_BATCHED, Ls, prec, fmt, len(Ls), dev)
        q.qdpx_ape_smear_batched(ctx, Ls, prec, fmt, Uds, outs, ALPHA, n, plaq, work, stream)  # builds the table
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream()
        cs.wait_stream(stream)
        with torch.cuda.graph(g, stream=cs):
            q.qdpx_ape_smear_batched(ctx, Ls, prec, fmt, Uds, outs, ALPHA, n, plaq, work, cs)
        g.replay()
        torch.cuda.synchronize()
        ms_graph = time_calls(torch, g.replay, reps, stream) / reps
        status = int(work[4:8].cpu().numpy().view("uint32")[0])

        loop_out = [q.alloc_links(L, prec, fmt, dev) for L in Ls]
        loop_plaq = [torch.zeros(3, dtype=torch.float64, device=dev) for _ in Ls]
        loop_work = [q.alloc_workspace(q.OP_APE, L, prec, fmt, n, dev) for L in Ls]
        loop_wp = [q.alloc_workspace(q.OP_PLAQ, L, prec, fmt, 1, dev) for L in Ls]

        def loop():
            for i, L in enumerate(Ls):
                q.qdpx_ape_smear(ctx, L, prec, fmt, Uds[i], loop_out[i], ALPHA, n, None, loop_work[i], stream)
                q.qdpx_plaquette(ctx, L, prec, fmt, loop_out[i], loop_plaq[i], loop_wp[i], stream)

        loop()
        torch.cuda.synchronize()
        ms_loop = time_calls(torch, loop, reps, stream) / reps
        same_links = all(np.array_equal(q.links_to_host(ctx, L, a, prec, fmt).view(np.float64),
                                        q.links_to_host(ctx, L, b, prec, fmt).view(np.float64))
                         for L, a, b in zip(Ls[:8], outs[:8], loop_out[:8]))
        same_plaq = all(torch.equal(plaq[3 * i:3 * i + 3], loop_plaq[i]) for i in range(len(Ls)))
        check[name] = q.links_to_host(ctx, Ls[0], outs[0], prec, fmt)
        res[name] = {
            "launch": {"block": geometry[0], "groups_per_ticket": geometry[1], "source": src},
            "link_updates_per_s_persistent_graph": updates / (ms_graph / 1e3),
            "link_updates_per_s_per_lattice_loop": updates / (ms_loop / 1e3),
            "ms_persistent_graph": ms_graph,
            "ms_per_lattice_loop": ms_loop,
            "speedup_vs_loop": ms_loop / ms_graph,
            "status": status,
            "links_identical_to_loop_first_8_lattices": bool(same_links),
            "final_plaquettes_identical_to_loop": bool(same_plaq),
        }
        log(f"batched {name}: graph {ms_graph:.2f} ms, loop {ms_loop:.2f} ms, geometry {geometry} ({src}), "
            f"status {status}, identical links {same_links}, plaquettes {same_plaq}")
        del Uds, outs, work, loop_out, loop_work, loop_wp, g
    d32 = float(abs(check["f32_12"] - check["f64_18"]).max())
    return {
        "batched_64_lattices": {
            "sites": sites,
            "ape_steps": n,
            **res,
            "speedup_batched_f32_12_vs_f64_18_loop": res["f64_18"]["ms_per_lattice_loop"] / res["f32_12"]["ms_persistent_graph"],
            "speedup_batched_f32_12_vs_batched_f64_18": res["f64_18"]["ms_persistent_graph"] / res["f32_12"]["ms_persistent_graph"],
            "lattice0_max_abs_f32_12_minus_f64_18": d32,
        }
    }, check


def cpu_baseline(U, steps, samp_sites, samp_mus):
    """The FP64 oracle on the host: whole APE steps over the full 32^3x64
    lattice, repeated until at least 10 s of work (at least N_APE, at most 40
    steps).  Only the steps are timed.  The oracle's links after steps
    1..N_APE are the reference of the per-step errors of both GPU paths (on
    the sampled links), and its plaquettes (untimed) of their plaquettes."""
    import numpy as np

    import oracle

    V = U.shape[0] * U.shape[1] * U.shape[2] * U.shape[3]
    flat = U.reshape(V, 4, 3, 3)
    threads = oracle.num_threads()
    log(f"cpu baseline: oracle APE steps on {L} with {threads} threads")
    err = {"oracle_max_abs_f32_12": [], "oracle_max_abs_f64_18": [], "oracle_plaquette_abs_err_f32_12": [],
           "oracle_plaquette_abs_err_f64_18": [], "oracle_plaquette": []}
    p0 = oracle.plaquette(U)
    err["oracle_plaquette_input"] = [float(x) for x in p0]
    n, t, cur = 0, 0.0, U
    while (t < 10.0 or n < N_APE) and n < 40:
        t0 = time.perf_counter()
        cur = oracle.ape_step(cur, ALPHA)
        t += time.perf_counter() - t0
        n += 1
        if n <= N_APE:
            ref = cur.reshape(V, 4, 3, 3)[samp_sites, samp_mus]
            err["oracle_max_abs_f32_12"].append(float(np.max(np.abs(steps["s32"][n - 1] - ref))))
            err["oracle_max_abs_f64_18"].append(float(np.max(np.abs(steps["s64"][n - 1] - ref))))
            p = oracle.plaquette(cur)
            err["oracle_plaquette"].append([float(x) for x in p])
            err["oracle_plaquette_abs_err_f32_12"].append(float(np.max(np.abs(np.array(steps["plaq32"][n]) - p))))
            err["oracle_plaquette_abs_err_f64_18"].append(float(np.max(np.abs(np.array(steps["plaq64"][n]) - p))))
    del flat
    log(f"cpu baseline: {n} steps in {t:.1f} s; step-10 oracle error FP32-12 "
        f"{err['oracle_max_abs_f32_12'][-1]:.2e}, FP64 {err['oracle_max_abs_f64_18'][-1]:.2e}")
    return {
        "value": 4.0 * V * n / t,
        "unit": "link-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{n} FP64 APE steps over the full {L[0]}^3x{L[3]} lattice ({4 * V * n} link updates) "
                  f"in {t:.2f} s",
    }, err


def batch_oracle_check(check):
    """Part of the cpu_baseline leg: the FP64 oracle's 5 steps on lattice 0 of
    the batch against both formats' batched results."""
    import numpy as np

    import oracle

    ref = oracle.ape_smear(check["U"], ALPHA, 5)
    e32 = float(np.max(np.abs(check["f32_12"] - ref)))
    e64 = float(np.max(np.abs(check["f64_18"] - ref)))
    log(f"batch lattice 0 {check['L']}: oracle error FP32-12 {e32:.2e}, FP64 {e64:.2e}")
    return {"lattice0": list(check["L"]), "lattice0_oracle_max_abs_f32_12": e32, "lattice0_oracle_max_abs_f64_18": e64}


def error_sample(np, V, n=4096, seed=1305 + 77):
    """Links (site, direction) at which the GPU results are compared with the oracle."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(V, size=n, replace=False)), rng.integers(0, 4, n)


def su3_defects_device(torch, m, chunk=1 << 22):
    """(max ||V^dag V - 1||_F, max |det V - 1|) over (n, 3, 3) complex128 on the
    device, by explicit elementwise sums (no batched library products)."""
    eye = torch.eye(3, dtype=torch.complex128, device=m.device)
    u = d = 0.0
    for i in range(0, m.shape[0], chunk):
        x = m[i:i + chunk]
        gram = (x.conj().unsqueeze(-1) * x.unsqueeze(-2)).sum(-3) - eye  # sum_k conj(x_ki) x_kj
        u = max(u, float(gram.abs().square().sum((-1, -2)).sqrt().max()))
        det = (x[:, 0, 0] * (x[:, 1, 1] * x[:, 2, 2] - x[:, 1, 2] * x[:, 2, 1])
               - x[:, 0, 1] * (x[:, 1, 0] * x[:, 2, 2] - x[:, 1, 2] * x[:, 2, 0])
               + x[:, 0, 2] * (x[:, 1, 0] * x[:, 2, 1] - x[:, 1, 1] * x[:, 2, 0]))
        d = max(d, float((det - 1.0).abs().max()))
    return u, d


def unpack_device(torch, q, ctx, Ls, soa, prec, fmt, dev):
    """SoA links -> device complex128 tensor (V, 4, 3, 3) in the canonical order."""
    n = Ls[0] * Ls[1] * Ls[2] * Ls[3]
    aos = torch.empty((n, 4, 3, 3, 2), dtype=torch.float64, device=dev)
    q.qdpx_unpack_links(ctx, Ls, soa, prec, fmt, aos)
    return torch.view_as_complex(aos)


def step_by_step(torch, q, ctx, dev, stream, paths, dev_links, samp_sites, samp_mus):
    """The timed workload one APE step per call (bit-identical to one call of
    N_APE steps), FP32-12 and FP64-18 side by side: after every step the two
    outputs are compared on every link, their SU(3) defects are taken on
    every link, and the sampled links are kept for the oracle comparison."""
    sel_s = torch.from_numpy(samp_sites).to(dev)
    sel_m = torch.from_numpy(samp_mus).to(dev)
    res = {"d32_64": [], "u32": [], "det32": [], "u64": [], "det64": [], "s32": [], "s64": []}
    cur, bufs, plaq = {}, {}, {}
    for name in ("f32_12", "f64_18"):
        prec, fmt = paths[name]
        cur[name] = dev_links[name]
        bufs[name] = [q.alloc_links(L, prec, fmt, dev), q.alloc_links(L, prec, fmt, dev)]
        plaq[name] = torch.zeros(3 * (N_APE + 1), dtype=torch.float64, device=dev)
    for k in range(N_APE):
        full = {}
        for name in ("f32_12", "f64_18"):
            prec, fmt = paths[name]
            out = bufs[name][k & 1]
            p2 = torch.zeros(6, dtype=torch.float64, device=dev)
            work = q.alloc_workspace(q.OP_APE, L, prec, fmt, 1, dev)
            q.qdpx_ape_smear(ctx, L, prec, fmt, cur[name], out, ALPHA, 1, p2, work, stream)
            if k == 0:
                plaq[name][0:3] = p2[0:3]
            plaq[name][3 * (k + 1):3 * (k + 2)] = p2[3:6]
            cur[name] = out
            full[name] = unpack_device(torch, q, ctx, L, out, prec, fmt, dev).reshape(-1, 4, 3, 3)
            tag = "32" if name == "f32_12" else "64"
            u, d = su3_defects_device(torch, full[name].reshape(-1, 3, 3))
            res["u" + tag].append(u)
            res["det" + tag].append(d)
            res["s" + tag].append(full[name][sel_s, sel_m].cpu().numpy())
        res["d32_64"].append(float((full["f32_12"] - full["f64_18"]).abs().max()))
        del full
        log(f"step {k + 1}: max |V32 - V64| {res['d32_64'][-1]:.2e}, FP32 unitarity defect {res['u32'][-1]:.2e}")
    res["plaq32"] = plaq["f32_12"].cpu().numpy().reshape(-1, 3).tolist()
    res["plaq64"] = plaq["f64_18"].cpu().numpy().reshape(-1, 3).tolist()
    res["f32_12_final"] = cur["f32_12"]
    return res


def cpu_host_context(latgen):
    """The host the oracle ran on (CPU model, logical CPUs, memory) and the
    oracle's single-thread rate: one FP64 APE step on 16^3x32."""
    import oracle

    model, mem_gb = "unknown", None
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), model)
        with open("/proc/meminfo") as fh:
            kb = next((int(l.split()[1]) for l in fh if l.startswith("MemTotal")), None)
            mem_gb = None if kb is None else round(kb / 2**20, 1)
    except OSError:
        pass
    Ls = (16, 16, 16, 32)
    U = latgen.haar_links(Ls, latgen.SEEDS["shift_16x16x16x32"]["links"])
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.ape_step(U, ALPHA)
        t = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    rate = 4.0 * latgen.volume(Ls) / t
    log(f"cpu baseline: one thread {rate / 1e6:.2f} M link-updates/s on {model}")
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "mem_gb": mem_gb, "threads_used": threads,
            "single_thread_link_updates_per_s": rate, "single_thread_sample": "1 FP64 APE step on 16^3x32"}


if __name__ == "__main__":
    main()
