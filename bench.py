#!/usr/bin/env python3
"""Throughput of the RBL force path on one MI355X.

Workload: N = 1,000,000 LJ particles, density 0.8442, T = 1.0 (FCC lattice +
0.05 sigma jitter, Maxwell-Boltzmann velocities; synthetic, seeded), core
radius r_s = 1.5, cut-off r_c = 3.5, skin 0.3, lists rebuilt every 10 steps,
velocity Verlet at dt = 0.005.  One step = one pass of the whole path:
kick/drift, (every 10th step) binning + list build + batch draw, the force
and the mean-force reduction.

Variants timed back to back on the same GPU, each for --steps steps after
--warmup steps: RBL in the mixed form (FP32 pair arithmetic, FP64
classification and accumulation; the headline ``value``), RBL in FP64, and
the full Verlet list (direct truncation at r_c) in both precisions; batch
sizes P = 5, 10, 20 for the mixed RBL.

Prints one JSON line (rank 0, N = 1 GPU).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

RS, RC, SKIN, DT, K_REBUILD = 1.5, 3.5, 0.3, 0.005, 10
N, RHO, TEMP = 1_000_000, 0.8442, 1.0
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=100_000,
                    help="rows of the N = 1M state the CPU oracle leg processes")
    ap.add_argument("--variants", default="all", help="comma list or 'all'")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (a reference for "
                         "the HBM byte counters of a profiler run)")
    return ap.parse_args()


def force_algorithmic_bytes(ctx, n, P, mean_core):
    """Algorithmic HBM bytes of one pre-drawn RBL force launch: per particle
    the own position (double4, 32 B), core row length (4 B) and entries
    (4 B each), shell length (4 B), P batch entries (4 B each) and the force
    written (3 x 8 B).  Neighbour positions are gathered from cache."""
    return n * (32 + 4 + 4 * mean_core + 4 + 4 * P + 24)


def run_variant(name, x0, v0, box, precision, P, use_full, steps, warmup, torch):
    from paper_2105_04884_amd import Context, KIND_FORCE_RBL, KIND_FORCE_FULL, KIND_BUILD, \
        KIND_BIN, KIND_INTEGRATE, KIND_REDUCE, KIND_PREDRAW
    lists = ("full",) if use_full else ("core", "shell")
    x = x0.clone()
    v = v0.clone()
    ctx = Context(N, precision=precision, lists=lists, skin=SKIN)
    ctx.build(x, box, RS, RC)
    if warmup > 0:
        ctx.step(x, v, nsteps=warmup, dt=DT, P=P, seed=1, step0=0, rebuild_every=K_REBUILD,
                 use_full=use_full)
    step0 = warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status, _ = ctx.step(x, v, nsteps=steps, dt=DT, P=P, seed=1, step0=step0,
                         rebuild_every=K_REBUILD, use_full=use_full)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # second pass of the same length with per-kernel HIP events on the
    # context's stream (the events add small gaps, so it is not the clock of
    # `value`)
    ctx.set_profiling(True)
    ctx.step(x, v, nsteps=steps, dt=DT, P=P, seed=1, step0=step0 + steps,
             rebuild_every=K_REBUILD, use_full=use_full)
    kinds = {"force_rbl": KIND_FORCE_RBL, "force_full": KIND_FORCE_FULL, "build": KIND_BUILD,
             "binning": KIND_BIN, "integrate": KIND_INTEGRATE, "reduce": KIND_REDUCE,
             "predraw": KIND_PREDRAW}
    stats = {k: ctx.kernel_stats(q) for k, q in kinds.items()}
    ctx.set_profiling(False)
    info = ctx.info()
    tuning = ctx.tuning()
    counts = ctx.row_counts()
    ctx.close()
    mean = {"core": float(counts[0].mean()), "shell": float(counts[1].mean()),
            "full": float(counts[2].mean())}
    res = {
        "name": name, "precision": precision, "P": P, "full": use_full,
        "ms_per_step": 1e3 * elapsed / steps,
        "atom_steps_per_s": N * steps / elapsed,
        "status": int(status),
        "kernels_ms": {k: {"launches": s[0], "total_ms": s[1],
                           "avg_us": 1e3 * s[1] / s[0] if s[0] else 0.0} for k, s in stats.items()},
        "mean_row": mean,
        "caps": info,
        "tuning": tuning,
    }
    log(f"[bench] {name}: {res['ms_per_step']:.4f} ms/step, {res['atom_steps_per_s']:.3e} atom-steps/s")
    return res


def force_error_vs_oracle(x0, box, torch, rows):
    """Relative L2 error of the raw RBL force (P = 10, no mean subtraction)
    against the FP64 CPU oracle on sampled rows, for both precisions."""
    import oracle
    from paper_2105_04884_amd import Context
    pos = x0.cpu().numpy()
    L = oracle.System(pos, box, RS, RC, SKIN).lists(rows=rows, kinds=("core", "shell"))
    fo, _, _ = oracle.rbl_forces(pos, box, RS, RC, L, 10, 1, 0)
    out = {}
    for precision in ("fp64", "mixed"):
        with Context(N, precision=precision, momentum_fix=False) as ctx:
            ctx.build(x0, box, RS, RC)
            f = ctx.forces(10, seed=1, step=0, pos=x0).cpu().numpy()[:, rows]
        out[precision] = float(np.linalg.norm(f - fo) / np.linalg.norm(fo))
    return out


def cpu_baseline(st, rows_n):
    """The CPU oracle (single thread, FP64, as it stands) on a bounded sample
    of the workload: one list build and K_REBUILD RBL force evaluations for
    `rows_n` rows of the N = 1M state, plus the integrator over all N; the
    per-row cost is scaled to atom-steps/s of the full system."""
    import oracle
    rows = np.arange(0, N, max(1, N // rows_n), dtype=np.int64)[:rows_n]
    t0 = time.perf_counter()
    sysm = oracle.System(st.pos, st.box, RS, RC, SKIN)
    L = sysm.lists(rows=rows, kinds=("core", "shell"))
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    for s in range(K_REBUILD):
        oracle.rbl_forces(st.pos, st.box, RS, RC, L, 10, 1, s)
    t_force = (time.perf_counter() - t0) / K_REBUILD
    per_row_step = t_build / K_REBUILD / len(rows) + t_force / len(rows)
    value = 1.0 / per_row_step
    return {
        "value": value,
        "unit": "atom-steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{len(rows)} of the {N} rows of the density-0.8442 fluid: one core+shell "
                   f"list build ({t_build:.1f} s) and {K_REBUILD} RBL force evaluations at P=10 "
                   f"({t_force * K_REBUILD:.1f} s), scaled per atom-step with lists rebuilt "
                   f"every {K_REBUILD} steps; single-threaded FP64 C"),
        "seconds": t_build + K_REBUILD * t_force,
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (this build has no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.steps % K_REBUILD or args.warmup % K_REBUILD:
        print("--steps and --warmup must be multiples of 10 (the list lifetime)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2105_04884_amd import inputs

    if args.calib_copy_mb > 0:
        src = torch.empty(args.calib_copy_mb * 2**20 // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {args.calib_copy_mb} MiB read + {args.calib_copy_mb} MiB written, 3 launches")
        del src, dst
    log("[bench] generating the N=1M fluid")
    st = inputs.million_fluid(seed=1)
    x0 = torch.from_numpy(st.pos).cuda()
    v0 = torch.from_numpy(st.vel).cuda()
    variants = [
        ("rbl_mixed_p10", "mixed", 10, False),
        ("rbl_fp64_p10", "fp64", 10, False),
        ("full_mixed", "mixed", 10, True),
        ("full_fp64", "fp64", 10, True),
        ("rbl_mixed_p5", "mixed", 5, False),
        ("rbl_mixed_p20", "mixed", 20, False),
    ]
    if args.variants != "all":
        keep = set(args.variants.split(","))
        variants = [v for v in variants if v[0] in keep]
    results = {}
    for name, prec, P, full in variants:
        log(f"[bench] variant {name}")
        results[name] = run_variant(name, x0, v0, st.box, prec, P, full, args.steps,
                                    args.warmup, torch)
    head = results.get("rbl_mixed_p10") or next(iter(results.values()))

    log("[bench] force error vs the FP64 oracle (sampled rows)")
    rows = np.random.default_rng(0).choice(N, size=2000, replace=False)
    errs = force_error_vs_oracle(x0, st.box, torch, rows)

    # roofline of the dominant kernel of the headline variant
    km = head["kernels_ms"]
    dom = max(km, key=lambda k: km[k]["total_ms"])
    fk = "force_full" if head["full"] else "force_rbl"
    f_avg_s = km[fk]["avg_us"] * 1e-6
    f_bytes = force_algorithmic_bytes(None, N, head["P"], head["mean_row"]["core"])
    roof = {
        "kernel": "k_forces (RBL, pre-drawn batches, mixed)",
        "bound": "hbm",
        "achieved": f_bytes / f_avg_s / 1e9 if f_avg_s > 0 else None,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": (f_bytes / f_avg_s / 1e9) / HBM_PEAK_GBS if f_avg_s > 0 else None,
        "traffic": None,
        "bytes_per_launch": f_bytes,
        "avg_launch_us": km[fk]["avg_us"],
        "dominant_kernel_class": dom,
    }

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(st, args.cpu_rows)

    def speed(name):
        r = results.get(name)
        return r["atom_steps_per_s"] if r else None

    line = {
        "metric": "atom-steps/s RBL vs full Verlet list at N=1M LJ; force RMS err vs FP64 oracle",
        "value": head["atom_steps_per_s"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair + f64 classify/accumulate" if head["precision"] == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "LJ fluid N=1,000,000 rho=0.8442 T=1.0, r_s=1.5 r_c=3.5 skin=0.3, "
                               "P=10, rebuild every 10 steps, dt=0.005, velocity Verlet NVE",
                   "n_particles": N, "P": head["P"], "precision": head["precision"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": {k: {"atom_steps_per_s": r["atom_steps_per_s"], "ms_per_step": r["ms_per_step"],
                         "kernels_avg_us": {q: round(s["avg_us"], 2) for q, s in r["kernels_ms"].items()
                                            if s["launches"]},
                         "kernels_total_ms": {q: round(s["total_ms"], 3) for q, s in r["kernels_ms"].items()
                                              if s["launches"]},
                         "mean_row": r["mean_row"], "tuning": r["tuning"]}
                     for k, r in results.items()},
        "speedup_rbl_mixed_vs_full_fp64": (speed("rbl_mixed_p10") / speed("full_fp64")
                                           if speed("rbl_mixed_p10") and speed("full_fp64") else None),
        "speedup_rbl_mixed_vs_full_mixed": (speed("rbl_mixed_p10") / speed("full_mixed")
                                            if speed("rbl_mixed_p10") and speed("full_mixed") else None),
        "speedup_rbl_mixed_vs_rbl_fp64": (speed("rbl_mixed_p10") / speed("rbl_fp64_p10")
                                          if speed("rbl_mixed_p10") and speed("rbl_fp64_p10") else None),
        "force_rel_l2_err_vs_fp64_oracle": errs,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
