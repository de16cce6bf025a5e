#!/usr/bin/env python3
"""Throughput of the RBL force path on one MI355X.

Workload: N = 1,000,000 LJ particles, density 0.8442, T = 1.0 (FCC lattice +
0.05 sigma jitter, Maxwell-Boltzmann velocities; synthetic, seeded), core
radius r_s = 1.5, cut-off r_c = 3.5, skin 0.3, lists rebuilt every 10 steps,
velocity Verlet at dt = 0.005.  One step = one pass of the whole path:
kick/drift, (every 10th step) binning + list build + batch draw, the force
and the mean-force reduction.

Variants timed back to back on the same GPU: RBL in the mixed form (FP32
pair arithmetic, FP64 classification and accumulation; the headline
``value``), RBL in FP64, and the full Verlet list (direct truncation at r_c)
in both precisions; batch sizes P = 5, 10, 20 for the mixed RBL.

Lists are rebuilt when some particle has moved more than half the skin since
the last build (checked on the device at every step; skin 0.5 and at most 13
steps per list for RBL, skin 0.3 and at most 10 for the full list), so every
pair within the radii is in the lists at every step.  Variants with a fixed
10-step lifetime and no check are timed beside them for comparison.

Timing: the step counts are taken in whole blocks of 10 steps.  Each
variant runs the warm-up (--warmup rounded up to blocks, at least one; the
first run also autotunes the force kernel) from the initial arrays, then
--repeats timed runs of --steps steps (rounded up to blocks, at least 200:
rebuilds fall every ~12 steps, so shorter runs would hold a varying count),
each continuing the state held on the GPU (rbl_continue: every block a
replay of a captured graph, no list build from host arrays) between device
synchronisations.  ``ms_per_step`` is the median run's time per step.  With
the defaults the five timed runs are the 1000 steps of the N = 1e6
workload.  RBL runs without a thermostat heat up slowly (the batch noise,
Sec. II), so their lists are rebuilt more often as a run goes on; timing
the configured length keeps that effect at the workload's size.  The other
workloads time five runs that together make their configured lengths
(2^24 fluid: 200 steps; ensemble and slab: 500).

The CPU oracle baseline runs first, before the GPU is touched, on one core
and on all host cores the process may use (at most 16).

Prints one JSON line (rank 0, N = 1 GPU).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

RS, RC, SKIN, DT, K_REBUILD = 1.5, 3.5, 0.3, 0.005, 10
# Lists rebuilt on displacement (a rebuild at the first step some particle is
# more than skin/2 from where the last build left it, or after the longest
# lifetime): skin and longest lifetime of the RBL form and of the full list,
# each the fastest of a sweep at N = 1e6 (skin 0.3 ... 0.6, lifetimes 10 ... 16).
SKIN_RBL, LIFE_RBL = 0.5, 13
SKIN_FULL, LIFE_FULL = 0.3, 10
# core rows filtered to r_s + skin/2 in the runs with rebuilds on
# displacement where the library's timing finds it pays (rbl_config.core_filter
# = 2); --no-core-filter turns it off
CORE_FILTER = "auto"
N, RHO, TEMP = 1_000_000, 0.8442, 1.0
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200,
                    help="steps per timed run (rounded up to whole 10-step blocks, at least 200)")
    ap.add_argument("--warmup", type=int, default=100,
                    help="warm-up steps (rounded up to whole list lifetimes, at least one)")
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed blocks per variant; the median is reported")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=100_000,
                    help="rows of the N = 1M state the single-core CPU oracle leg processes "
                         "(the all-core leg takes every row)")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes of the all-core CPU oracle leg (0: the usable host cores, "
                         "at most 16)")
    ap.add_argument("--variants", default="all", help="comma list or 'all'")
    ap.add_argument("--table1-equil", type=int, default=200_000,
                    help="equilibration steps of the table1 workload")
    ap.add_argument("--table1-prod", type=int, default=100_000,
                    help="production steps of the table1 workload")
    ap.add_argument("--workloads", default="ensemble,large,slab,mixture",
                    help="further workloads reported beside the headline: comma list of "
                         "'ensemble' (512 replicas), 'large' (N = 2^24), 'slab' (charged "
                         "slab, N = 2M, LJ + erfc), 'mixture' (binary mixture with per-type "
                         "cut-offs, N = 1M), 'table1' (the Sec. III coexistence study: minutes "
                         "of GPU time, not in the default), or 'none'")
    ap.add_argument("--summarize-requests", nargs=2, metavar=("READ_DIR", "WRITE_DIR"),
                    help="write profiles/request_sizes_n1m.txt from two rocprofv3 --pmc runs "
                         "of the request counters (see REQUEST_COUNTERS)")
    ap.add_argument("--summarize", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="instead of running: write the profiles/ summaries from the output "
                         "folders of a rocprofv3 --kernel-trace --stats run and two --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) of this script")
    ap.add_argument("--valu-dir", default=None,
                    help="with --summarize: the output folder of a rocprofv3 --pmc run of the "
                         "VALU counters (writes profiles/valu_n1m.txt)")
    ap.add_argument("--profile-command", default="",
                    help="with --summarize: the bench.py arguments the profiled runs used")
    ap.add_argument("--no-core-filter", action="store_true",
                    help="keep the force kernel on the built core rows (rbl_config.core_filter = 0) "
                         "instead of the rows filtered to r_s + skin/2")
    ap.add_argument("--pin-launch", action="store_true",
                    help="N = 1e6 variants: fix the force kernels' lanes per particle, launch "
                         "mode and core-row filter to the automatic choice there (RBL 1 lane mixed "
                         "with the filter, 2 FP64, full list 4, one block per tile) instead of "
                         "timing them; for profiler runs, whose per-dispatch overhead distorts "
                         "those timings")
    ap.add_argument("--skin", type=float, default=None,
                    help="Verlet skin of the N = 1e6 variants (default: the workload's)")
    ap.add_argument("--max-lifetime", type=int, default=None,
                    help="N = 1e6 variants: longest list lifetime in steps with rebuilds on "
                         "displacement (default: the fixed lifetime, 10)")
    ap.add_argument("--calib-copy-mb", type=int, default=1024,
                    help="size of the plain device copy timed first: the attainable HBM "
                         "bandwidth, and the reference for the byte counters of a profiler run")
    return ap.parse_args(argv)


def plan(args):
    """Checks the arguments and turns the step counts into whole list
    lifetimes: returns (warm-up steps, steps per timed block).  Exits with
    status 2 and a message on arguments this bench cannot run."""
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (the library has no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0 or args.repeats < 1:
        print("--steps and --repeats must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    return lifetimes(args.warmup), max(MIN_TIMED_STEPS, lifetimes(args.steps))


# shortest timed run: about 16 list rebuilds of the N = 1e6 workload
MIN_TIMED_STEPS = 200


def lifetimes(n, K=K_REBUILD):
    """n steps rounded up to whole list lifetimes, at least one."""
    return max(K, -(-int(n) // K) * K)


FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
BUILD_FLOPS_PER_CANDIDATE = 11   # per stencil candidate: image-shifted displacement (2 per
                                 # axis) and r^2 as one multiply and two FMAs
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ("paper_2105_04884_amd/csrc/device.h", "paper_2105_04884_amd/csrc/kernels.h",
                  "paper_2105_04884_amd/csrc/rbl.hip")


def force_algorithmic_bytes(n, P, mean_core):
    """Algorithmic HBM bytes of one pre-drawn RBL force launch: per particle
    the own position (double4, 32 B), core row length (4 B) and entries
    (4 B each), shell length (4 B), P batch entries (4 B each) and the force
    written (3 x 8 B).  Neighbour positions are gathered from cache."""
    return n * (32 + 4 + 4 * mean_core + 4 + 4 * P + 24)


def full_force_algorithmic_bytes(n, mean_full):
    """Same for the full-list force: own position, row length and entries,
    force written."""
    return n * (32 + 4 + 4 * mean_full + 24)


def stencil_candidates(ncell, counts):
    """Candidate pairs the list build tests: for every cell, its population
    times the population of its 5 x 5 x 5 periodic stencil (each cell once
    when an axis has fewer than 5 cells), summed over cells."""
    nz, ny, nx = int(ncell[2]), int(ncell[1]), int(ncell[0])
    grid = counts.reshape(nz, ny, nx).astype(np.int64)
    offs = [sorted({d % m for d in range(-2, 3)}) for m in (nz, ny, nx)]
    acc = np.zeros_like(grid)
    for oz in offs[0]:
        for oy in offs[1]:
            for ox in offs[2]:
                acc += np.roll(grid, shift=(oz, oy, ox), axis=(0, 1, 2))
    return int((grid * acc).sum())


def code_tokens(text):
    """C/C++ source with its comments removed and every run of whitespace
    made one space: what the compiler sees of the code, so that a change
    to comments alone keeps a recorded profile valid."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":  # string or character literal, kept whole
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash():
    """SHA-256 over the code of the kernel sources (comments and layout
    excluded)."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(code_tokens(f.read()).encode())
        h.update(b"\0")
    return h.hexdigest()


def recorded_traffic(key):
    """HBM bytes per launch of kernel class `key` from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE runs, each scaled by the
    factor a plain copy of known size gives), or None when that summary is
    missing or was taken from other kernel sources."""
    path = os.path.join(PROFILES, "hbm_traffic_n1m.txt")
    if not os.path.exists(path):
        return None
    src_hash, found = None, None
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) >= 2 and parts[0] == "source_sha256":
                src_hash = parts[1]
            if len(parts) >= 4 and parts[0] == "traffic" and parts[1] == key:
                found = float(parts[3])
    if src_hash != kernel_source_hash():
        return None
    return found


def recorded_valu(key):
    """VALU counters per launch of kernel class `key` from the committed
    rocprofv3 summary (profiles/valu_n1m.txt), or None when it is missing or
    was taken from other kernel sources."""
    path = os.path.join(PROFILES, "valu_n1m.txt")
    if not os.path.exists(path):
        return None
    src_hash, found = None, None
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) >= 2 and parts[0] == "source_sha256":
                src_hash = parts[1]
            if len(parts) >= 3 and parts[0] == "valu" and parts[1] == key:
                found = json.loads(line.split(None, 2)[2])
    if src_hash != kernel_source_hash():
        return None
    return found


def copy_bandwidth(torch, mib):
    """Attainable HBM bandwidth of a plain device-to-device copy of `mib`
    MiB (read + write bytes over the event-timed duration, best of 5)."""
    if mib <= 0:
        return None
    src = torch.empty(mib * 2**20 // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    best = None
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    gbs = 2 * mib * 2**20 / (best * 1e-3) / 1e9
    log(f"[bench] device copy of {mib} MiB: {gbs:.0f} GB/s (read + write)")
    return gbs


def build_roofline(res):
    """Fused list build + batch draw: bound by FP64 vector arithmetic (the
    stencil candidate tests), priced at the FP64 vector peak."""
    km = res["kernels_ms"]["build"]
    avg_s = km["avg_us_per_build"] * 1e-6
    flops = res["build_candidates"] * BUILD_FLOPS_PER_CANDIDATE
    ach = flops / avg_s / 1e12 if avg_s > 0 else None
    return {
        "kernel": "k_build_draw (cell-stencil core list + shell count + batch draw for 10 steps)",
        "bound": "alu",
        "achieved": ach,
        "peak": FP64_VECTOR_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": ach / FP64_VECTOR_PEAK_TFLOPS if ach else None,
        "traffic": recorded_traffic("build"),
        "flops_per_launch": flops,
        "candidates_per_launch": res["build_candidates"],
        "avg_launch_us": km["avg_us_per_build"],
    }


def force_roofline(res, fk):
    km = res["kernels_ms"][fk]
    avg_s = km["avg_us"] * 1e-6
    if res["full"]:
        nbytes = full_force_algorithmic_bytes(N, res["mean_row"]["full"])
        name = "k_forces (full list)"
    else:
        # with filtered core rows, the rows read on the steps between
        # filterings (the filtering steps read the built rows: an undercount)
        filt = res.get("core_filter") or {}
        core = filt["mean_kept"] if filt.get("used") and filt.get("mean_kept") else res["mean_row"]["core"]
        nbytes = force_algorithmic_bytes(N, res["P"], core)
        name = ("k_forces (RBL, pre-drawn batches, filtered core rows)" if filt.get("used")
                else "k_forces (RBL, pre-drawn batches)")
    ach = nbytes / avg_s / 1e9 if avg_s > 0 else None
    key = f"force_{'full' if res['full'] else 'rbl'}_{res['precision']}_p{res['P']}"
    return {
        "kernel": f"{name}, {res['precision']}",
        "bound": "hbm",
        "achieved": ach,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": ach / HBM_PEAK_GBS if ach else None,
        "traffic": recorded_traffic(key),
        "bytes_per_launch": nbytes,
        "avg_launch_us": km["avg_us"],
    }


KINDS = ("force_rbl", "force_full", "build", "binning", "integrate", "reduce", "predraw")


def timed_blocks(ctx, x, v, torch, P, warmup, steps, repeats, use_full=False, K=None):
    """Warm-up run of `warmup` steps from the arrays x, v (rbl_step; the first
    run of a context autotunes the force kernel), then `repeats` blocks of
    `steps` steps that continue the state held on the GPU (rbl_continue:
    whole captured lifetimes replayed), each timed between device
    synchronisations, then one more block with per-kernel HIP events on the
    context's stream.  All blocks start at a list build (step counts are
    whole lifetimes)."""
    from paper_2105_04884_amd import (KIND_FORCE_RBL, KIND_FORCE_FULL, KIND_BUILD, KIND_BIN,
                                      KIND_INTEGRATE, KIND_REDUCE, KIND_PREDRAW)
    st0, _ = ctx.step(x, v, nsteps=warmup, dt=DT, P=P, seed=1, step0=0,
                      rebuild_every=K or K_REBUILD, use_full=use_full)
    times, statuses, attempts, builds = [], [int(st0)], [], 0
    for r in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, _ = ctx.cont(steps)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        statuses.append(int(st))
        info = ctx.last_run()
        attempts.append(info["attempts"])
        builds += info["builds"]
        log(f"[bench]   run {r + 1}/{repeats}: {steps} steps in {times[-1]:.4f} s, {info['builds']} builds")
    ctx.set_profiling(True)
    st, _ = ctx.cont(steps)
    statuses.append(int(st))
    prof_builds = ctx.last_run()["builds"]
    kinds = dict(zip(KINDS, (KIND_FORCE_RBL, KIND_FORCE_FULL, KIND_BUILD, KIND_BIN, KIND_INTEGRATE,
                             KIND_REDUCE, KIND_PREDRAW)))
    stats = {k: ctx.kernel_stats(q) for k, q in kinds.items()}
    ctx.set_profiling(False)
    med = float(np.median(times))
    km = {k: {"launches": s_[0], "total_ms": s_[1],
              "avg_us": 1e3 * s_[1] / s_[0] if s_[0] else 0.0} for k, s_ in stats.items()}
    # with rebuilds on displacement the build kernel is launched every step
    # and returns at once unless a rebuild is due: its duration per list
    # build is the summed time over the builds that ran
    km["build"]["builds"] = prof_builds
    km["build"]["avg_us_per_build"] = 1e3 * km["build"]["total_ms"] / prof_builds if prof_builds else 0.0
    return {
        "median_s": med,
        "block_seconds": [round(t, 6) for t in times],
        # RBL_OK 0 / RBL_W_SKIN 1 over the warm-up, timed and profiled blocks
        "status": max(statuses),
        "attempts_max": max(attempts),
        "steps_per_build": repeats * steps / builds if builds else None,
        "kernels_ms": km,
    }


def run_variant(name, x0, v0, box, precision, P, use_full, warmup, steps, repeats, torch,
                source="shell", pin=False, check=True, skin=SKIN, max_life=K_REBUILD):
    from paper_2105_04884_amd import Context
    lists = ("full",) if use_full else ("core", "shell")
    x = x0.clone()
    v = v0.clone()
    pinned_lanes = 4 if use_full else (1 if precision == "mixed" else 2)
    launch = {"lanes": pinned_lanes, "persistent": 1} if pin else {}
    if pin:
        # the automatic core-row filter times the kernels, which a profiler
        # distorts: fixed to its usual choice (on at one lane per particle)
        launch["core_filter"] = bool(pinned_lanes == 1 and source != "paper")
    ctx = Context(N, precision=precision, lists=lists, skin=skin, shell_source=source, rebuild_check=check,
                  core_filter=launch.pop("core_filter", CORE_FILTER),
                  **launch)
    ctx.build(x, box, RS, RC)
    K = max_life if check else K_REBUILD
    tb = timed_blocks(ctx, x, v, torch, P, warmup, steps, repeats, use_full, K)
    info = ctx.info()
    tuning = ctx.tuning()
    cfilt = ctx.core_filter()
    counts = ctx.row_counts()
    ncell, _, cell_counts = ctx.export_binning(with_counts=True)
    candidates = stencil_candidates(ncell[0], cell_counts)
    ctx.close()
    mean = {"core": float(counts[0].mean()), "shell": float(counts[1].mean()),
            "full": float(counts[2].mean())}
    res = {
        "name": name, "precision": precision, "P": P, "full": use_full, "shell_source": source,
        "rebuild": (f"displacement (skin/2), at most every {K} steps" if check
                    else f"every {K} steps"),
        "skin": skin,
        "steps_per_build": tb["steps_per_build"],
        "ms_per_step": 1e3 * tb["median_s"] / steps,
        "atom_steps_per_s": N * steps / tb["median_s"],
        "block_seconds": tb["block_seconds"],
        "status": tb["status"],
        "attempts_max": tb["attempts_max"],
        "kernels_ms": tb["kernels_ms"],
        "mean_row": mean,
        "caps": info,
        "tuning": tuning,
        "core_filter": cfilt,
        "build_candidates": candidates,
    }
    log(f"[bench] {name}: {res['ms_per_step']:.4f} ms/step, {res['atom_steps_per_s']:.3e} atom-steps/s "
        f"(blocks {tb['block_seconds']} s, status {tb['status']}, {tb['steps_per_build']} steps per build)")
    return res


def kernels_avg_us(tb):
    return {k: round(v["avg_us"], 2) for k, v in tb["kernels_ms"].items() if v["launches"]}


def run_slab(torch, warmup, steps, repeats, P=20):
    """Charged liquid slab in vapour, N = 2,000,000, LJ + real-space Ewald
    (alpha 0.3), r_s = 1.5, r_c = 5.0, P = 20, mixed precision."""
    from paper_2105_04884_amd import Context, inputs
    st = inputs.slab(seed=1)
    n = st.n
    x, v = torch.from_numpy(st.pos).cuda(), torch.from_numpy(st.vel).cuda()
    q = torch.from_numpy(st.charges).cuda()
    with Context(n, precision="mixed", skin=SKIN_RBL, pair="lj_erfc", alpha=0.3, charges=q, core_filter=CORE_FILTER,
                 rebuild_check=True) as ctx:
        ctx.build(x, st.box, 1.5, 5.0)
        tb = timed_blocks(ctx, x, v, torch, P, warmup, steps, repeats, K=LIFE_RBL)
        cfilt = ctx.core_filter()
    el = tb["median_s"]
    log(f"[bench] slab: {1e3 * el / steps:.3f} ms/step, {n * steps / el:.3e} atom-steps/s")
    return {"workload": "charged LJ slab N=2,000,000, box L x L x 3L (L=133.5), liquid rho=0.8 in the "
                        "middle third, vapour rho=0.02, charges +-1, T=0.9; LJ + erfc(alpha r)/r with "
                        "alpha=0.3, r_s=1.5 r_c=5.0 skin=0.5, P=20, lists rebuilt on displacement "
                        "(skin/2, at most every 13 steps), dt=0.005, mixed",
            "n_particles": n, "steps": steps, "repeats": repeats, "atom_steps_per_s": n * steps / el,
            "ms_per_step": 1e3 * el / steps, "status": tb["status"], "attempts_max": tb["attempts_max"],
            "steps_per_build": tb["steps_per_build"],
            "kernels_avg_us": kernels_avg_us(tb), "core_filter": cfilt}


# binary mixture of the per-type cut-off workload: epsilon 1 for every pair,
# sigma 1 (small), 1.4 (large) and 1.2 between them
MIXTURE_TABLE = np.array([[[1.0, 1.0], [1.0, 1.2]], [[1.0, 1.2], [1.0, 1.4]]])


def run_mixture(torch, warmup, steps, repeats, P=10):
    """Binary LJ mixture, N = 1,000,000 (80% sigma 1, 20% sigma 1.4,
    density 0.5, T = 1): pair radii r_s sigma_ab, r_c sigma_ab, cells from
    the smallest cut-off and one stencil per type (Sec. II).  RBL (P = 10)
    and the typed direct truncation, both mixed, lists rebuilt on
    displacement."""
    from paper_2105_04884_amd import Context, inputs
    st = inputs.binary_mixture(1_000_000, seed=1)
    n = st.n
    out = {"workload": "binary LJ mixture N=1,000,000 (80% sigma=1, 20% sigma=1.4, sigma_AB=1.2, "
                       "epsilon=1), density 0.5, T=1.0, pair radii r_s sigma_ab and r_c sigma_ab "
                       "(r_s=1.5, r_c=3.5), cells from the smallest cut-off, one stencil per type, "
                       "P=10, dt=0.005, mixed, lists rebuilt on displacement",
           "n_particles": n, "steps": steps, "repeats": repeats}
    for name, full, skin, life in (("rbl", False, SKIN_RBL, LIFE_RBL), ("full_list", True, SKIN_FULL, LIFE_FULL)):
        x, v = torch.from_numpy(st.pos).cuda(), torch.from_numpy(st.vel).cuda()
        lists = ("full",) if full else ("core", "shell")
        with Context(n, precision="mixed", lists=lists, skin=skin, rebuild_check=True, types=st.types,
                     eps_sig=MIXTURE_TABLE, core_filter=CORE_FILTER) as ctx:
            ctx.build(x, st.box, RS, RC)
            tb = timed_blocks(ctx, x, v, torch, P, warmup, steps, repeats, full, K=life)
            cfilt = ctx.core_filter()
        el = tb["median_s"]
        log(f"[bench] mixture {name}: {1e3 * el / steps:.3f} ms/step, {n * steps / el:.3e} atom-steps/s")
        out[name] = {"skin": skin, "atom_steps_per_s": n * steps / el, "ms_per_step": 1e3 * el / steps,
                     "status": tb["status"], "attempts_max": tb["attempts_max"],
                     "steps_per_build": tb["steps_per_build"], "kernels_avg_us": kernels_avg_us(tb),
                     "build_us_per_build": round(tb["kernels_ms"]["build"]["avg_us_per_build"], 1),
                     "core_filter": cfilt}
    if "rbl" in out and "full_list" in out:
        out["rbl_speedup_vs_full_list"] = out["rbl"]["atom_steps_per_s"] / out["full_list"]["atom_steps_per_s"]
    return out


def run_ensemble(torch, warmup, steps, repeats, seq_replicas=16):
    """512 independent replicas (N log-uniform in [2000, 65536], density
    uniform in [0.6, 0.9], T uniform in [0.8, 1.5]) advanced together, one
    launch per kernel per step, against the same replicas one context each."""
    from paper_2105_04884_amd import Context, inputs
    ens = inputs.ensemble(512, seed=1)
    pos, vel, boxes, off = ens.concat()
    n = int(off[-1])
    out = {"workload": "512 LJ replicas, N log-uniform in [2000, 65536] (sum %d), density U[0.6, 0.9], "
                       "T U[0.8, 1.5], r_s=1.5 r_c=3.5 skin=0.5, P=10, lists rebuilt on displacement "
                       "(skin/2, at most every 13 steps), dt=0.005" % n,
           "replicas": 512, "n_total": n, "steps": steps, "repeats": repeats}
    for precision in ("mixed", "fp64"):
        x, v = torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()
        with Context(n, precision=precision, replica_offsets=off, skin=SKIN_RBL, rebuild_check=True,
                     core_filter=CORE_FILTER) as ctx:
            ctx.build(x, boxes, RS, RC)
            tb = timed_blocks(ctx, x, v, torch, 10, warmup, steps, repeats, K=LIFE_RBL)
            cfilt = ctx.core_filter()
        el = tb["median_s"]
        out[precision] = {"atom_steps_per_s": n * steps / el, "ms_per_step": 1e3 * el / steps,
                          "status": tb["status"], "attempts_max": tb["attempts_max"],
                          "steps_per_build": tb["steps_per_build"],
                          "kernels_avg_us": kernels_avg_us(tb), "core_filter": cfilt}
        log(f"[bench] ensemble {precision}: {1e3 * el / steps:.3f} ms/step, {n * steps / el:.3e} atom-steps/s")
    # the same replicas one context each, on a sample of them
    picks = np.linspace(0, 511, seq_replicas).astype(int)
    tot_atoms, tot_s = 0, 0.0
    for r in picks:
        s_ = ens.states[r]
        x, v = torch.from_numpy(s_.pos).cuda(), torch.from_numpy(s_.vel).cuda()
        with Context(s_.n, precision="mixed", skin=SKIN_RBL, rebuild_check=True, core_filter=CORE_FILTER) as ctx:
            ctx.build(x, s_.box, RS, RC)
            tb = timed_blocks(ctx, x, v, torch, 10, warmup, steps, 1, K=LIFE_RBL)
        tot_atoms += s_.n * steps
        tot_s += tb["median_s"]
    out["sequential_mixed"] = {"atom_steps_per_s": tot_atoms / tot_s,
                               "sample": f"{seq_replicas} of the 512 replicas, one context each, "
                                         f"{steps} steps each"}
    out["speedup_batched_vs_sequential"] = out["mixed"]["atom_steps_per_s"] / (tot_atoms / tot_s)
    log(f"[bench] ensemble sequential: {tot_atoms / tot_s:.3e} atom-steps/s")
    return out


def run_large(torch, warmup, steps, repeats):
    """N = 2^24 LJ fluid, density 0.8, T = 1.2, r_s = 1.3, r_c = 4.0, P = 10,
    mixed precision, lists every 10 steps."""
    from paper_2105_04884_amd import Context, inputs
    st = inputs.large_fluid(seed=1)
    n = st.n
    x, v = torch.from_numpy(st.pos).cuda(), torch.from_numpy(st.vel).cuda()
    with Context(n, precision="mixed", skin=SKIN_RBL, rebuild_check=True, core_filter=CORE_FILTER) as ctx:
        ctx.build(x, st.box, 1.3, 4.0)
        tb = timed_blocks(ctx, x, v, torch, 10, warmup, steps, repeats, K=LIFE_RBL)
        tuning = ctx.tuning()
        cfilt = ctx.core_filter()
    el = tb["median_s"]
    log(f"[bench] large: {1e3 * el / steps:.3f} ms/step, {n * steps / el:.3e} atom-steps/s")
    return {"workload": "LJ fluid N=16,777,216 rho=0.8 T=1.2, r_s=1.3 r_c=4.0 skin=0.5, P=10, "
                        "lists rebuilt on displacement (skin/2, at most every 13 steps), dt=0.005, "
                        "mixed",
            "n_particles": n, "steps": steps, "repeats": repeats, "atom_steps_per_s": n * steps / el,
            "ms_per_step": 1e3 * el / steps, "status": tb["status"], "attempts_max": tb["attempts_max"],
            "steps_per_build": tb["steps_per_build"],
            "kernels_avg_us": kernels_avg_us(tb),
            # the autotuner's launch-mode choice and times (one block per tile
            # against the persistent grid) and lanes per particle
            "force_launch": {"persistent": tuning["persistent_rbl"],
                             "us_tile_grid_vs_persistent": tuning["rbl_grid_vs_persistent_us"],
                             "lanes": tuning["lpp_rbl"]},
            "core_filter": cfilt}


def rdf_from_counts(counts, frames, n, volume, dr):
    """g(r) of Sec. III from ordered-pair counts per bin of width dr summed
    over `frames` frames: counts / (frames N rho 4/3 pi ((k+1)^3 - k^3) dr^3),
    rho = N / V.  Returns (bin centres, g)."""
    counts = np.asarray(counts, dtype=np.float64)
    nb = counts.shape[-1]
    edges = np.arange(nb + 1) * dr
    shell = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    rho = n / volume
    return 0.5 * (edges[1:] + edges[:-1]), counts / (frames * n * rho * shell)


def msd_slope(times, msd, lo=0.2, hi=1.0):
    """Least-squares slope of msd(t) over lo*t_max <= t <= hi*t_max, t_max
    the longest lag: the long-time limit eta(t)/t of Sec. III (Table I)."""
    times = np.asarray(times, dtype=np.float64)
    msd = np.asarray(msd, dtype=np.float64)
    tmax = times.max()
    sel = (times >= lo * tmax) & (times <= hi * tmax)
    A = np.vstack([times[sel], np.ones(sel.sum())]).T
    return float(np.linalg.lstsq(A, msd[sel], rcond=None)[0][0])


def run_table1(torch, equil=200_000, prod=100_000, every=1000, runs=10):
    """The gas-liquid coexistence study of Sec. III (Table I): N = 2000,
    density 0.2, T = 0.9, Langevin friction 1, dt = 0.002; direct truncation
    at r_c = 6, 3, 2, and RBL with r_s = 2, r_c = 6 and P = 10, 20, 50, 100.
    `runs` independent replicas (seeds 1..runs) per setting run in one
    context.  After `equil` steps, `prod` steps are sampled every `every`
    steps: g(r) (pair histogram, bins of 0.01 up to r = 2), the continuous
    trajectory for the MSD, and u, P with tail corrections.  Reports, averaged
    over the replicas, the first peak of g(r), the MSD slope lim eta(t)/t
    (lags up to half the production run), u and P."""
    from paper_2105_04884_amd import Context, inputs
    n1, rho, kT, dt, gamma = 2000, 0.2, 0.9, 0.002, 1.0
    states = [inputs.lj_fluid(n1, rho, kT, seed=s + 1) for s in range(runs)]
    pos = np.concatenate([s.pos for s in states], axis=1)
    vel = np.concatenate([s.vel for s in states], axis=1)
    boxes = np.stack([s.box for s in states])
    off = np.arange(runs + 1, dtype=np.int64) * n1
    n = runs * n1
    volume = float(np.prod(states[0].box))
    r_max, nbins = 2.0, 200
    dr = r_max / nbins
    settings = [("DT r_c=6", True, 1.0, 6.0, 10), ("DT r_c=3", True, 1.0, 3.0, 10),
                ("DT r_c=2", True, 1.0, 2.0, 10)]
    settings += [(f"RBL r_s=2 r_c=6 P={P}", False, 2.0, 6.0, P) for P in (10, 20, 50, 100)]
    frames = prod // every
    out = {"workload": f"Sec. III gas-liquid coexistence: {runs} replicas of N={n1}, rho={rho}, "
                       f"T={kT}, Langevin gamma={gamma}, dt={dt}, {equil} equilibration + {prod} "
                       f"production steps, samples every {every}, lists every 10 steps, FP64",
           "settings": {}}
    for name, full, rs, rc, P in settings:
        x, v = torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda()
        lists = ("full",) if full else ("core", "shell")
        t0 = time.perf_counter()
        with Context(n, replica_offsets=off, lists=lists, shift=False, skin=SKIN) as ctx:
            ctx.set_thermostat(gamma, kT)
            ctx.build(x, boxes, rs, rc)
            s = 0
            chunk = 20_000
            while s < equil:
                m = min(chunk, equil - s)
                ctx.step(x, v, nsteps=m, dt=dt, P=P, seed=1, step0=s, rebuild_every=10, use_full=full)
                s += m
            log(f"[bench] table1 {name}: equilibrated ({equil} steps)")
            counts = torch.zeros((runs, nbins), dtype=torch.int64, device="cuda")
            snaps, us, ps, tks = [], [], [], []
            for f in range(frames):
                _, ev = ctx.step(x, v, nsteps=every, dt=dt, P=P, seed=1, step0=s, rebuild_every=10,
                                 use_full=full, want_ev=True)
                s += every
                ctx.rdf(x, r_max, nbins, counts)
                snaps.append(ctx.unwrap(x))
                th = ctx.thermo(ev, v)
                us.append(th[:, 0])
                ps.append(th[:, 1])
                tks.append(th[:, 2])
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            lags = np.arange(1, frames // 2 + 1)
            msd = np.zeros((len(lags), runs))
            for k, lag in enumerate(lags):
                acc = torch.zeros(runs, dtype=torch.float64, device="cuda")
                for t in range(frames - lag):
                    acc += ctx.msd(snaps[t + lag], snaps[t])
                msd[k] = (acc / (frames - lag)).cpu().numpy()
        _, g = rdf_from_counts(counts.cpu().numpy(), frames, n1, volume, dr)
        times = lags * every * dt
        peaks = g.max(axis=1)
        slopes = np.array([msd_slope(times, msd[:, r], lo=0.2, hi=1.0) for r in range(runs)])
        res = {"peak_g": float(peaks.mean()), "peak_g_sem": float(peaks.std(ddof=1) / np.sqrt(runs)),
               "msd_slope": float(slopes.mean()), "msd_slope_sem": float(slopes.std(ddof=1) / np.sqrt(runs)),
               "u_per_particle": float(np.mean(us)), "pressure": float(np.mean(ps)),
               "kinetic_T": float(np.mean(tks)), "seconds": el,
               "atom_steps_per_s": n * (equil + prod) / el}
        out["settings"][name] = res
        log(f"[bench] table1 {name}: peak g {res['peak_g']:.3f}, MSD slope {res['msd_slope']:.3f}, "
            f"u {res['u_per_particle']:.4f}, P {res['pressure']:.4f} ({el:.1f} s)")
    return out


def force_error_vs_oracle(x0, box, torch, rows):
    """Relative L2 error of the raw RBL force (P = 10, no mean subtraction)
    against the FP64 CPU oracle on sampled rows, for both precisions and
    the three draw populations (keys "stencil_*": the stencil cells of the
    search grid, "paper_*": those of the paper's own grid)."""
    import oracle
    from paper_2105_04884_amd import Context
    pos = x0.cpu().numpy()
    sysm = oracle.System(pos, box, RS, RC, SKIN)
    out = {}
    for source, prefix in (("shell", ""), ("stencil", "stencil_"), ("paper", "paper_")):
        L = (sysm.lists(rows=rows, kinds=("core", "shell")) if source == "shell"
             else sysm.stencil_lists(rows=rows) if source == "stencil"
             else sysm.paper_stencil_lists(rows=rows))
        fo, _, _ = oracle.rbl_forces(pos, box, RS, RC, L, 10, 1, 0)
        for precision in ("fp64", "mixed"):
            with Context(N, precision=precision, momentum_fix=False, shell_source=source) as ctx:
                ctx.build(x0, box, RS, RC)
                f = ctx.forces(10, seed=1, step=0, pos=x0).cpu().numpy()[:, rows]
            out[prefix + precision] = float(np.linalg.norm(f - fo) / np.linalg.norm(fo))
    return out


# State the CPU oracle workers read (set before the pool forks, so the
# children share the parent's arrays instead of receiving copies).
_CPU_STATE = {}


def _oracle_rows_job(job):
    """One worker of the CPU oracle leg: one list build for `rows` and
    K_REBUILD force evaluations there (RBL at P = 10, or the full list);
    returns (seconds of the build, seconds of the forces)."""
    import oracle
    rows, full = job
    pos, box = _CPU_STATE["pos"], _CPU_STATE["box"]
    t0 = time.perf_counter()
    L = oracle.System(pos, box, RS, RC, SKIN).lists(rows=rows, kinds=("full",) if full else ("core", "shell"))
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    for s_ in range(K_REBUILD):
        if full:
            oracle.full_forces(pos, box, RC, L)
        else:
            oracle.rbl_forces(pos, box, RS, RC, L, 10, 1, s_)
    return t_build, time.perf_counter() - t0


def usable_cores(limit=16):
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(limit, n))


def cpu_oracle(st, rows_1core, workers, full=False):
    """The CPU oracle as it stands (single-threaded FP64 C) on the N = 1M
    state: one list build and K_REBUILD force evaluations (RBL at P = 10, or
    the full list) for a sample of rows, scaled to atom-steps/s with lists
    rebuilt every K_REBUILD steps.  Run on one core for `rows_1core` rows,
    then on `workers` processes, each a contiguous share of every row
    (wall-clock time of the whole pool)."""
    import multiprocessing as mp
    _CPU_STATE["pos"], _CPU_STATE["box"] = st.pos, st.box
    rows1 = np.arange(0, N, max(1, N // rows_1core), dtype=np.int64)[:rows_1core]
    tb, tf = _oracle_rows_job((rows1, full))
    one = len(rows1) * K_REBUILD / (tb + tf)
    what = "full-list" if full else "core+shell list"
    force = "full-list force evaluations" if full else "RBL force evaluations at P=10"
    out = {
        "value": one, "unit": "atom-steps/s", "cores": 1, "kind": "oracle",
        "sample": (f"{len(rows1)} of the {N} rows of the density-0.8442 fluid: one {what} build "
                   f"({tb:.1f} s) and {K_REBUILD} {force} ({tf:.1f} s), scaled per atom-step with "
                   f"lists rebuilt every {K_REBUILD} steps; single-threaded FP64 C"),
        "seconds": tb + tf,
    }
    if workers > 1:
        rows_all = np.arange(N, dtype=np.int64)
        if full:
            rows_all = rows_all[: N // 4]
        jobs = [(c, full) for c in np.array_split(rows_all, workers)]
        ctx = mp.get_context("fork")
        t0 = time.perf_counter()
        with ctx.Pool(workers) as pool:
            parts = pool.map(_oracle_rows_job, jobs, chunksize=1)
        wall = time.perf_counter() - t0
        out["all_cores"] = {
            "value": len(rows_all) * K_REBUILD / wall, "unit": "atom-steps/s", "cores": workers,
            "kind": "oracle",
            "sample": (f"{len(rows_all)} rows split over {workers} processes of the same single-threaded "
                       f"oracle (one {what} build and {K_REBUILD} {force} each), wall-clock of the "
                       f"pool {wall:.1f} s"),
            "seconds": wall,
            "max_worker_seconds": max(a + b for a, b in parts),
        }
    _CPU_STATE.clear()
    return out


def method_error(x0, box, rs=RS, rc=RC, Ps=(5, 10, 20)):
    """Relative L2 distance of the RBL force from the full-list force at the
    same state (mean force subtracted, as in the MD loop) for each batch
    size: the statistical error of the method itself, not an error of the
    implementation.  Keys "stencil_P" draw from the stencil cells of the
    search grid, "paper_P" from those of the paper's own grid, instead of
    the shell rows; "population" holds the mean draw population (n_i, or
    N_I) of each."""
    from paper_2105_04884_amd import Context
    out = {"population": {}}
    for source, prefix in (("shell", ""), ("stencil", "stencil_"), ("paper", "paper_")):
        lists = ("core", "shell", "full") if source == "shell" else ("core", "full")
        with Context(N, precision="fp64", lists=lists, shell_source=source) as ctx:
            ctx.build(x0, box, rs, rc)
            ff = ctx.full_forces(x0)
            for P in Ps:
                f = ctx.forces(P, seed=1, step=0, pos=x0)
                out[prefix + str(P)] = float((f - ff).norm() / ff.norm())
            out["population"][source] = float(ctx.row_counts()[1].mean())
    return out


def _read_csv(folder, suffix):
    import csv
    import glob
    paths = sorted(glob.glob(os.path.join(folder, "**", "*" + suffix), recursive=True))
    if not paths:
        raise SystemExit(f"no *{suffix} under {folder}")
    with open(paths[0]) as f:
        return list(csv.DictReader(f))


def kernel_class(name, P):
    """Kernel class key of a kernel instantiation name (see KERNEL_SOURCES)."""
    if "k_build_draw<" in name:
        return "build"
    for tmpl in ("k_forces_lpp<", "k_forces<"):
        if tmpl in name:
            args = name.split(tmpl, 1)[1].split(">", 1)[0].split(",")
            prec = "mixed" if args[0].strip() == "1" else "fp64"
            kind = {"0": "full", "1": "rbl_inline", "2": "rbl"}[args[1].strip()]
            return f"force_{kind}_{prec}_p{P}"
    return None


# A kernel that is launched every step but works only at some (the list
# build with rebuilds on displacement returns at once while its gate is
# clear) is summarised over its working dispatches: those whose primary
# measure (duration, or the counter of the run) reaches ACTIVE_FRACTION of
# the kernel's largest.
ACTIVE_FRACTION = 0.05


def active_mean(values):
    """(count, mean) over the working dispatches of one kernel (see
    ACTIVE_FRACTION); all of them when none stands out."""
    v = np.asarray(values, dtype=float)
    if v.size == 0:
        return 0, 0.0
    keep = v[v >= ACTIVE_FRACTION * v.max()] if v.max() > 0 else v
    return int(keep.size), float(keep.mean())


def trace_durations(trace_dir):
    """Per kernel name, the list of dispatch durations (ns) of a rocprofv3
    kernel trace."""
    rows = _read_csv(trace_dir, "kernel_trace.csv")
    out = {}
    for r in rows:
        out.setdefault(r["Kernel_Name"], []).append(float(r["End_Timestamp"]) - float(r["Start_Timestamp"]))
    return out


def summarize(trace_dir, fetch_dir, write_dir, command, calib_mib, P=10):
    """Writes profiles/kernel_trace_n1m.txt (per-kernel launch statistics)
    and profiles/hbm_traffic_n1m.txt (HBM bytes per launch of each kernel
    class: FETCH_SIZE and WRITE_SIZE averaged over its dispatches, each
    scaled by expected / measured for the plain copy of calib_mib MiB)."""
    os.makedirs(PROFILES, exist_ok=True)
    stats = _read_csv(trace_dir, "kernel_stats.csv")
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# rocprofv3 kernel trace, N = 1,000,000 LJ fluid (density 0.8442), RBL mixed P = 10",
             "# and full list FP64 variants of bench.py",
             f"# command: rocprofv3 --kernel-trace --stats -d <dir> -o bench --output-format csv "
             f"-- python3 bench.py {command}",
             "# columns: calls, total ms, average us, min us, max us, share %, kernel", ""]
    for r in stats:
        lines.append(f"{int(r['Calls']):7d} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                     f"{float(r['AverageNs']) / 1e3:10.2f} {float(r['MinNs']) / 1e3:10.2f} "
                     f"{float(r['MaxNs']) / 1e3:10.2f} {float(r['Percentage']):6.2f}  {r['Name']}")
    durs = trace_durations(trace_dir)
    lines += ["", "# working dispatches (duration >= 5% of the kernel's longest) of kernels",
              "# that also return at once: calls, average us, kernel"]
    for name, v in sorted(durs.items()):
        n_act, mean = active_mean(v)
        if n_act < len(v):
            lines.append(f"active {n_act:7d} {mean / 1e3:10.2f}  {name}")
    # a force step with filtered core rows queues two instances (one returns
    # at once): the class's time per step sums them, as the bench's own
    # events around the step's force launches do
    per_class = {}
    for name, v in durs.items():
        cls = kernel_class(name, P)
        if cls:
            tot, steps = per_class.get(cls, (0.0, 0))
            per_class[cls] = (tot + sum(v), max(steps, len(v)))
    lines += ["", "# per kernel class: force steps, microseconds per step (all instances)"]
    for cls, (tot, steps) in sorted(per_class.items()):
        lines.append(f"step {cls} {steps:7d} {tot / steps / 1e3:10.2f}")
    with open(os.path.join(PROFILES, "kernel_trace_n1m.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")

    expected_kib = calib_mib * 1024.0
    per = {}
    factors = {}
    for tag, folder in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _read_csv(folder, "counter_collection.csv")
        copies = [float(r["Counter_Value"]) for r in rows
                  if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == tag
                  and float(r["Counter_Value"]) >= 0.25 * expected_kib]
        if not copies:
            raise SystemExit(f"{tag}: no dispatch of the {calib_mib} MiB calibration copy found")
        factors[tag] = expected_kib / float(np.median(copies))
        agg = {}
        for r in rows:
            if r["Counter_Name"] != tag:
                continue
            agg.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        for name, vals in agg.items():
            per.setdefault(name, {})[tag] = active_mean(vals)
    lines = ["# HBM traffic per kernel launch from two rocprofv3 counter runs of bench.py,",
             "# N = 1,000,000 LJ fluid (density 0.8442)",
             f"# command 1: rocprofv3 --pmc FETCH_SIZE -d <dir> -o bench --output-format csv "
             f"-- python3 bench.py {command}",
             f"# command 2: rocprofv3 --pmc WRITE_SIZE -d <dir> -o bench --output-format csv "
             f"-- python3 bench.py {command}",
             f"# calibration: a plain {calib_mib} MiB device copy (expected {expected_kib:.0f} KiB "
             f"read and written) reads FETCH_SIZE x{factors['FETCH_SIZE']:.4f} and "
             f"WRITE_SIZE x{factors['WRITE_SIZE']:.4f} of that",
             f"calibration fetch_factor {factors['FETCH_SIZE']:.6f} write_factor {factors['WRITE_SIZE']:.6f}",
             f"source_sha256 {kernel_source_hash()}",
             "# per kernel: working dispatches (counter >= 5% of its largest), mean FETCH_SIZE KiB,",
             "# mean WRITE_SIZE KiB (raw), name", ""]
    classes = {}
    for name, d in sorted(per.items(), key=lambda kv: -kv[1].get("FETCH_SIZE", (0, 0))[1]):
        nf, fk = d.get("FETCH_SIZE", (0, 0.0))
        nw, wk = d.get("WRITE_SIZE", (0, 0.0))
        lines.append(f"kernel {nf:6d} {fk:14.1f} {wk:14.1f}  {name}")
        cls = kernel_class(name, P)
        if cls and (cls not in classes or nf > classes[cls][0]):
            scaled = (fk * factors["FETCH_SIZE"] + wk * factors["WRITE_SIZE"]) * 1024.0
            classes[cls] = (nf, scaled, name)
    lines.append("")
    lines.append("# scaled HBM bytes per launch of each kernel class (the instantiation with")
    lines.append("# the most dispatches): traffic <class> bytes_per_launch <bytes> <name>")
    for cls, (nf, scaled, name) in sorted(classes.items()):
        lines.append(f"traffic {cls} bytes_per_launch {scaled:.0f}  {name}")
    with open(os.path.join(PROFILES, "hbm_traffic_n1m.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


VALU_COUNTERS = ["SQ_INSTS_VALU", "SQ_INSTS_VALU_FLOPS_FP32", "SQ_INSTS_VALU_FLOPS_FP64",
                 "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
                 "SQ_ACTIVE_INST_VALU", "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE"]


def summarize_valu(valu_dir, trace_dir, command, P=10):
    """Writes profiles/valu_n1m.txt: per kernel class (the instantiation with
    the most dispatches), the mean per launch of the VALU counters of one
    rocprofv3 --pmc run, the launch duration of the kernel trace, and from
    them the achieved FP64 and FP32 rates against the vector peaks (78.6 and
    157.3 TFLOP/s) and the VALU busy fraction
    SQ_ACTIVE_INST_VALU * 4 / (SIMDs * GRBM_GUI_ACTIVE per XCD)."""
    rows = _read_csv(valu_dir, "counter_collection.csv")
    stats = {name: active_mean(v)[1] for name, v in trace_durations(trace_dir).items()}
    by_dispatch = {}
    for r in rows:
        by_dispatch.setdefault((r["Kernel_Name"], r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
    per = {}
    for (name, _), d in by_dispatch.items():
        per.setdefault(name, []).append(d)
    for name, ds in per.items():
        top = max(d.get("SQ_INSTS_VALU", 0.0) for d in ds)
        work = [d for d in ds if d.get("SQ_INSTS_VALU", 0.0) >= ACTIVE_FRACTION * top] if top > 0 else ds
        merged = {}
        for d in work:
            for k, v in d.items():
                merged.setdefault(k, []).append(v)
        per[name] = merged
    simds, xcds = 256 * 4, 8
    classes = {}
    for name, d in per.items():
        cls = kernel_class(name, P)
        n = len(d.get("SQ_INSTS_VALU", []))
        if cls and name in stats and (cls not in classes or n > classes[cls][0]):
            m = {k: float(np.mean(v)) for k, v in d.items()}
            us = stats[name] / 1e3
            # the FLOPS counters count per wavefront instruction (an FMA two):
            # x 64 lanes; for FP64 equal to 64 (ADD + MUL + 2 FMA) instructions
            f64 = 64.0 * m.get("SQ_INSTS_VALU_FLOPS_FP64", 0.0)
            f32 = 64.0 * m.get("SQ_INSTS_VALU_FLOPS_FP32", 0.0)
            gui = m.get("GRBM_GUI_ACTIVE", 0.0) / xcds
            busy = m.get("SQ_ACTIVE_INST_VALU", 0.0) * 4.0 / (simds * gui) if gui > 0 else None
            classes[cls] = (n, {"kernel": name, "dispatches": n, "avg_launch_us": us,
                                "counters_per_launch": m,
                                "fp64_flops_per_launch": f64, "fp32_flops_per_launch": f32,
                                "fp64_tflops": f64 / (us * 1e-6) / 1e12,
                                "fp64_frac_of_78.6": f64 / (us * 1e-6) / 78.6e12,
                                "fp32_tflops": f32 / (us * 1e-6) / 1e12,
                                "fp32_frac_of_157.3": f32 / (us * 1e-6) / 157.3e12,
                                "valu_busy": busy})
    lines = ["# VALU counters per kernel launch from one rocprofv3 counter run of bench.py,",
             "# N = 1,000,000 LJ fluid (density 0.8442)",
             f"# command: rocprofv3 --pmc {' '.join(VALU_COUNTERS)} -d <dir> -o bench "
             f"--output-format csv -- python3 bench.py {command}",
             "# durations and counters over working dispatches (see kernel_trace_n1m.txt); the FLOPS counters "
             "count per wavefront instruction (an FMA counts two), so flops = 64 x counter",
             f"source_sha256 {kernel_source_hash()}",
             "# valu <class> <json>", ""]
    for cls, (_, d) in sorted(classes.items()):
        lines.append(f"valu {cls} {json.dumps(d)}")
    with open(os.path.join(PROFILES, "valu_n1m.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


REQUEST_COUNTERS = (["TCC_EA0_RDREQ_DRAM_32B", "TCC_EA0_RDREQ", "TCC_EA0_RDREQ_32B", "TCC_BUBBLE"],
                    ["TCC_EA0_WRREQ", "TCC_EA0_WRREQ_64B", "TCC_EA0_WRREQ_DRAM"])


def summarize_requests(rd_dir, wr_dir, command, P=10):
    """Writes profiles/request_sizes_n1m.txt: per kernel class, the L2-to-memory
    read and write requests by size over the working dispatches, the bytes
    they imply (TCC_EA0_RDREQ_DRAM_32B counts a request in 32-byte units),
    and what FETCH_SIZE's formula makes of the same requests, so that the
    copy calibration of the traffic figures can be checked kernel by kernel."""
    per = {}
    for tag, folder, key in (("rd", rd_dir, "TCC_EA0_RDREQ"), ("wr", wr_dir, "TCC_EA0_WRREQ")):
        by = {}
        for r in _read_csv(folder, "counter_collection.csv"):
            by.setdefault((r["Kernel_Name"], r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
        names = {}
        for (name, _), d in by.items():
            names.setdefault(name, []).append(d)
        for name, ds in names.items():
            top = max(d.get(key, 0.0) for d in ds)
            work = [d for d in ds if d.get(key, 0.0) >= ACTIVE_FRACTION * top] if top > 0 else ds
            m = {c: float(np.mean([d.get(c, 0.0) for d in work])) for c in work[0]}
            per.setdefault(name, {}).update(m)
    lines = ["# L2-to-memory requests by size per kernel launch (working dispatches), two rocprofv3",
             "# counter runs of bench.py, N = 1,000,000 LJ fluid (density 0.8442)",
             f"# command 1: rocprofv3 --pmc {' '.join(REQUEST_COUNTERS[0])} -d <dir> -o bench "
             f"--output-format csv -- python3 bench.py {command}",
             f"# command 2: rocprofv3 --pmc {' '.join(REQUEST_COUNTERS[1])} -d <dir> -o bench "
             f"--output-format csv -- python3 bench.py {command}",
             "# read bytes = 32 x TCC_EA0_RDREQ_DRAM_32B (a request counted in 32-byte units);",
             "# FETCH_SIZE's formula on this architecture: 128 BUBBLE + 64 (RDREQ - BUBBLE - RDREQ_32B)",
             "# + 32 RDREQ_32B bytes; write bytes = 64 WRREQ_64B + 32 (WRREQ - WRREQ_64B)",
             f"source_sha256 {kernel_source_hash()}",
             "# columns: RDREQ, RDREQ_32B, BUBBLE, RDREQ_DRAM_32B, read MB, FETCH_SIZE formula MB,",
             "# bytes per read request, WRREQ, WRREQ_64B, write MB, kernel", ""]
    shown = [(n, m) for n, m in per.items() if kernel_class(n, P) or "copyBuffer" in n]
    for name, m in sorted(shown, key=lambda kv: -kv[1].get("TCC_EA0_RDREQ", 0.0)):
        rq, r32, bub = m.get("TCC_EA0_RDREQ", 0.0), m.get("TCC_EA0_RDREQ_32B", 0.0), m.get("TCC_BUBBLE", 0.0)
        dram = m.get("TCC_EA0_RDREQ_DRAM_32B", 0.0)
        fetch = bub * 128 + (rq - bub - r32) * 64 + r32 * 32
        wq, w64 = m.get("TCC_EA0_WRREQ", 0.0), m.get("TCC_EA0_WRREQ_64B", 0.0)
        lines.append(f"{rq:11.4e} {r32:10.3e} {bub:10.3e} {dram:11.4e} {32 * dram / 1e6:9.1f} {fetch / 1e6:9.1f} "
                     f"{32 * dram / rq if rq else 0.0:6.1f} {wq:11.4e} {w64:11.4e} "
                     f"{(w64 * 64 + (wq - w64) * 32) / 1e6:9.1f}  {name}")
    with open(os.path.join(PROFILES, "request_sizes_n1m.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def guarded(name, fn, *a, **kw):
    """Runs an optional part of the bench; a failure is logged and recorded
    instead of ending the run before the JSON line."""
    try:
        return fn(*a, **kw)
    except Exception as e:  # noqa: BLE001 -- the line is still printed
        log(f"[bench] {name} failed: {type(e).__name__}: {e}")
        return {"error": f"{type(e).__name__}: {e}"}


def main(argv=None):
    global CORE_FILTER
    args = parse(argv)
    CORE_FILTER = False if args.no_core_filter else "auto"
    if args.summarize_requests:
        summarize_requests(*args.summarize_requests, args.profile_command)
        return
    if args.summarize:
        summarize(*args.summarize, args.profile_command, args.calib_copy_mb)
        if args.valu_dir:
            summarize_valu(args.valu_dir, args.summarize[0], args.profile_command)
        return
    warmup, steps = plan(args)
    from paper_2105_04884_amd import inputs

    log("[bench] generating the N=1M fluid")
    st = inputs.million_fluid(seed=1)
    # the CPU oracle first, before anything touches the GPU
    cpu = cpu_full = None
    if not args.no_cpu_baseline:
        workers = args.cpu_workers or usable_cores()
        log(f"[bench] CPU oracle baseline (1 core, then {workers} processes)")
        cpu = guarded("cpu baseline", cpu_oracle, st, args.cpu_rows, workers)
        cpu_full = guarded("cpu baseline (full list)", cpu_oracle, st, max(1, args.cpu_rows // 4),
                           workers, full=True)
        log(f"[bench] CPU oracle: {cpu.get('value', 0):.3e} atom-steps/s on 1 core, "
            f"{cpu.get('all_cores', {}).get('value', 0):.3e} on {workers}")

    import torch
    copy_gbs = copy_bandwidth(torch, args.calib_copy_mb)
    x0 = torch.from_numpy(st.pos).cuda()
    v0 = torch.from_numpy(st.vel).cuda()
    # (name, precision, P, full list, draw population, rebuild on displacement)
    variants = [
        ("rbl_mixed_p10", "mixed", 10, False, "shell", True),
        ("rbl_fp64_p10", "fp64", 10, False, "shell", True),
        ("full_mixed", "mixed", 10, True, "shell", True),
        ("full_fp64", "fp64", 10, True, "shell", True),
        ("rbl_mixed_p5", "mixed", 5, False, "shell", True),
        ("rbl_mixed_p20", "mixed", 20, False, "shell", True),
        ("rbl_stencil_mixed_p10", "mixed", 10, False, "stencil", True),
        # the paper's own grid at skin 0.3 (cells of 1.8, 7^3 of them): at
        # skin 0.5 its cells of 2.0 would coincide with the search grid's
        ("rbl_paper_mixed_p10", "mixed", 10, False, "paper", True),
        # fixed 10-step lifetimes at skin 0.3 (no displacement check: some
        # particles pass skin/2 within a lifetime, status RBL_W_SKIN)
        ("rbl_mixed_p10_fixed10", "mixed", 10, False, "shell", False),
        ("full_fp64_fixed10", "fp64", 10, True, "shell", False),
    ]
    if args.variants != "all":
        keep = set(args.variants.split(","))
        variants = [v for v in variants if v[0] in keep]
    log(f"[bench] {warmup} warm-up steps, {args.repeats} timed blocks of {steps} steps per variant")
    results = {}
    for name, prec, P, full, source, check in variants:
        log(f"[bench] variant {name}")
        if not check:
            skin, life = SKIN, K_REBUILD
        else:
            skin, life = (SKIN_FULL, LIFE_FULL) if full or source == "paper" else (SKIN_RBL, LIFE_RBL)
            skin = args.skin if args.skin is not None else skin
            life = args.max_lifetime if args.max_lifetime is not None else life
        results[name] = run_variant(name, x0, v0, st.box, prec, P, full, warmup, steps, args.repeats,
                                    torch, source, args.pin_launch, check, skin, life)
    head = results.get("rbl_mixed_p10") or next(iter(results.values()))

    # roofline of the dominant kernel of the headline variant (largest
    # share of the event-timed block), and of the force kernel beside it
    km = head["kernels_ms"]
    dom = max(km, key=lambda k: km[k]["total_ms"])
    fk = "force_full" if head["full"] else "force_rbl"
    force_roof = force_roofline(head, fk)
    if dom == "build":
        roof = build_roofline(head)
        roof["secondary"] = force_roof
    else:
        roof = force_roof
        roof["secondary"] = build_roofline(head)
    roof["dominant_kernel_class"] = dom

    def valu_key(kind):
        if kind == "build":
            return "build"
        return f"force_{'full' if head['full'] else 'rbl'}_{head['precision']}_p{head['P']}"
    roof["valu_counters"] = recorded_valu(valu_key(dom))
    roof["secondary"]["valu_counters"] = recorded_valu(valu_key("force" if dom == "build" else "build"))
    roof["share_of_step"] = km[dom]["total_ms"] / sum(k["total_ms"] for k in km.values())
    roof["hbm_copy_GBs"] = copy_gbs

    log("[bench] force error vs the FP64 oracle (sampled rows)")
    rows = np.random.default_rng(0).choice(N, size=2000, replace=False)
    errs = guarded("force error", force_error_vs_oracle, x0, st.box, torch, rows)
    log("[bench] method error of RBL against the full list")
    merr = guarded("method error", method_error, x0, st.box)
    log("[bench] method error at the Sec. III radii (r_s = 2, r_c = 6)")
    merr_wide = guarded("method error (r_s = 2, r_c = 6)", method_error, x0, st.box, 2.0, 6.0, (10, 20, 50))

    extra = {}
    wl = [w for w in args.workloads.split(",") if w and w != "none"]
    if "ensemble" in wl:
        log("[bench] workload: 512-replica ensemble")
        extra["ensemble"] = guarded("ensemble", run_ensemble, torch, 10, lifetimes(500 // args.repeats),
                                    args.repeats)
    if "large" in wl:
        log("[bench] workload: N = 2^24")
        extra["large"] = guarded("large", run_large, torch, 10, lifetimes(200 // args.repeats), args.repeats)
    if "mixture" in wl:
        log("[bench] workload: binary mixture with per-type cut-offs")
        extra["mixture"] = guarded("mixture", run_mixture, torch, 10, lifetimes(500 // args.repeats),
                                   args.repeats)
    if "slab" in wl:
        log("[bench] workload: charged slab")
        extra["slab"] = guarded("slab", run_slab, torch, 10, lifetimes(500 // args.repeats), args.repeats)
    if "table1" in wl:
        log("[bench] workload: Sec. III gas-liquid coexistence (Table I)")
        extra["table1"] = guarded("table1", run_table1, torch, args.table1_equil, args.table1_prod)

    def speed(name):
        r = results.get(name)
        return r["atom_steps_per_s"] if r else None

    line = {
        "metric": "atom-steps/s RBL vs full Verlet list at N=1M LJ; force RMS err vs FP64 oracle",
        "value": head["atom_steps_per_s"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "repeats": args.repeats,
        "timing": ("median over the repeats of one block of `steps` steps (captured graphs of 10 "
                   "steps replayed, continuing the GPU-resident state after `warmup` steps), between "
                   "device synchronisations"),
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair + f64 classify/accumulate" if head["precision"] == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "LJ fluid N=1,000,000 rho=0.8442 T=1.0, r_s=1.5 r_c=3.5, P=10, "
                               "dt=0.005, velocity Verlet NVE; lists rebuilt when a particle has moved "
                               "more than skin/2 since the last build (skin 0.5, at most every 13 "
                               "steps; full list: skin 0.3, at most every 10)",
                   "n_particles": N, "P": head["P"], "precision": head["precision"]},
        "status": head["status"],
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": {k: {"atom_steps_per_s": r["atom_steps_per_s"], "ms_per_step": r["ms_per_step"],
                         "block_seconds": r["block_seconds"], "status": r["status"],
                         "attempts_max": r["attempts_max"],
                         "kernels_avg_us": {q: round(s_["avg_us"], 2) for q, s_ in r["kernels_ms"].items()
                                            if s_["launches"]},
                         "kernels_total_ms": {q: round(s_["total_ms"], 3) for q, s_ in r["kernels_ms"].items()
                                              if s_["launches"]},
                         "mean_row": r["mean_row"], "tuning": r["tuning"], "core_filter": r["core_filter"],
                         "caps": r["caps"]}
                     for k, r in results.items()},
        "speedup_rbl_mixed_vs_full_fp64": (speed("rbl_mixed_p10") / speed("full_fp64")
                                           if speed("rbl_mixed_p10") and speed("full_fp64") else None),
        "speedup_rbl_mixed_vs_full_mixed": (speed("rbl_mixed_p10") / speed("full_mixed")
                                            if speed("rbl_mixed_p10") and speed("full_mixed") else None),
        "speedup_rbl_mixed_vs_rbl_fp64": (speed("rbl_mixed_p10") / speed("rbl_fp64_p10")
                                          if speed("rbl_mixed_p10") and speed("rbl_fp64_p10") else None),
        "force_rel_l2_err_vs_fp64_oracle": errs,
        "method_rel_l2_rbl_vs_full_list": merr,
        "method_rel_l2_rbl_vs_full_list_rs2_rc6": merr_wide,
        "cpu_baseline_full_list": cpu_full,
        "workloads": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
