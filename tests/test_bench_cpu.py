"""Host-side helpers of bench.py: the stencil candidate count that prices the
list build, kernel-class names of profiler rows, and the one-GPU guard."""
import itertools
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _brute_candidates(nc, counts):
    nx, ny, nz = nc
    grid = counts.reshape(nz, ny, nx)
    total = 0
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        cells = {((z + dz) % nz, (y + dy) % ny, (x + dx) % nx)
                 for dz in range(-2, 3) for dy in range(-2, 3) for dx in range(-2, 3)}
        total += int(grid[z, y, x]) * sum(int(grid[c]) for c in cells)
    return total


@pytest.mark.parametrize("nc", [(7, 7, 7), (6, 8, 9), (3, 5, 7), (1, 2, 4)])
def test_stencil_candidates_brute_force(nc):
    rng = np.random.default_rng(sum(nc))
    counts = rng.integers(0, 9, size=int(np.prod(nc))).astype(np.int32)
    assert bench.stencil_candidates(np.array(nc), counts) == _brute_candidates(nc, counts)


def test_kernel_class_names():
    assert bench.kernel_class("void rbl::k_build_draw<12, true>(rbl::FusedArgs)", 10) == "build"
    assert bench.kernel_class("void rbl::k_forces_lpp<1, 2, false, false, 2>(rbl::ForceArgs)",
                              10) == "force_rbl_mixed_p10"
    assert bench.kernel_class("void rbl::k_forces_lpp<0, 0, false, false, 4>(rbl::ForceArgs)",
                              10) == "force_full_fp64_p10"
    assert bench.kernel_class("void rbl::k_forces<0, 1, false, false, 16>(rbl::ForceArgs)",
                              5) == "force_rbl_inline_fp64_p5"
    assert bench.kernel_class("rbl::k_integrate<1>(rbl::IntArgs)", 10) is None


def test_recorded_traffic_needs_matching_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    (tmp_path / "hbm_traffic_n1m.txt").write_text(
        f"source_sha256 {bench.kernel_source_hash()}\n"
        "traffic build bytes_per_launch 123456  k_build_draw<12, true>\n")
    assert bench.recorded_traffic("build") == 123456.0
    assert bench.recorded_traffic("force_rbl_mixed_p10") is None
    (tmp_path / "hbm_traffic_n1m.txt").write_text(
        "source_sha256 0000\ntraffic build bytes_per_launch 123456  k\n")
    assert bench.recorded_traffic("build") is None


def test_code_tokens_drop_comments_and_layout_only():
    src = 'int a = 1; // note\nconst char* s = "x // y /* z */";\n/* block\n */ char c = \'/\';  int  b;'
    assert bench.code_tokens(src) == 'int a = 1; const char* s = "x // y /* z */"; char c = \'/\'; int b;'
    # a code change shows, a comment change does not
    assert bench.code_tokens("x = 1; // a") == bench.code_tokens("x  =  1;  /* b */")
    assert bench.code_tokens("x = 1;") != bench.code_tokens("x = 2;")
    assert bench.code_tokens('s = "a\\"b"; // c') == 's = "a\\"b";'


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_rdf_normalisation_of_an_ideal_gas():
    """g(r) from the oracle's pair counts of uniform random points is 1
    within Poisson error away from r = 0."""
    import oracle
    from paper_2105_04884_amd import inputs
    box = np.array([12.0, 12.0, 12.0])
    frames, n, nb, rmax = 3, 1500, 25, 5.0
    counts = np.zeros(nb)
    for f in range(frames):
        st = inputs.random_gas(n, box, seed=20 + f)
        counts += oracle.rdf_counts(st.pos, box, rmax, nb)
    r, g = bench.rdf_from_counts(counts, frames, n, float(box.prod()), rmax / nb)
    assert np.allclose(r[:2], [0.1, 0.3])
    assert abs(g[5:].mean() - 1.0) < 0.02


def test_msd_slope_of_a_line():
    t = np.linspace(0.1, 10.0, 100)
    assert bench.msd_slope(t, 2.5 * t + 0.3) == pytest.approx(2.5, rel=1e-12)
    # a ballistic start is left out of the fit window
    m = np.where(t < 1.0, t * t, 2.0 * t - 1.0)
    assert bench.msd_slope(t, m) == pytest.approx(2.0, rel=1e-12)


def test_short_command_plans_whole_lifetimes():
    """A short command line (any step counts) is accepted; the counts
    become whole 10-step blocks, the warm-up at least one, a timed run at
    least 200 steps."""
    assert bench.plan(bench.parse(["--gpus", "1", "--steps", "20", "--warmup", "5"])) == (10, 200)
    assert bench.plan(bench.parse(["--steps", "205", "--warmup", "0"])) == (10, 210)
    assert bench.plan(bench.parse(["--steps", "1", "--warmup", "11"])) == (20, 200)
    assert bench.plan(bench.parse([])) == (100, 200)


@pytest.mark.parametrize("argv", [["--steps", "0"], ["--warmup", "-1"], ["--repeats", "0"]])
def test_unusable_step_counts_are_refused(argv):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert ">=" in r.stderr


def test_cpu_oracle_leg_on_a_small_sample():
    """The CPU baseline leg as the bench runs it (before any GPU work): one
    core on a row sample, then a process pool over every row; both report
    a positive rate and the core count they used."""
    from paper_2105_04884_amd import inputs
    st = inputs.million_fluid(seed=1)
    orig = bench.N
    try:
        # rows of the first 20k IDs only keep the pool run short
        bench.N = 20_000
        res = bench.cpu_oracle(st, 500, 2)
    finally:
        bench.N = orig
    assert res["cores"] == 1 and res["value"] > 0
    assert res["all_cores"]["cores"] == 2 and res["all_cores"]["value"] > 0
    assert bench.usable_cores() >= 1


def test_msd_of_a_free_langevin_particle():
    """The mean-squared displacement eta(t) of Sec. III, taken as the bench
    takes it (unwrapped positions, average over time origins, least-squares
    slope over the late lags), for free particles under the Langevin
    thermostat: eta(t) = 6 (kT/gamma^2) (gamma t - 1 + exp(-gamma t)) for a
    velocity drawn from the bath, long-time slope 6 kT / gamma.  Oracle
    runs of one particle in an empty box (no pair in range, F = 0), many
    seeds."""
    import math
    import oracle
    box = np.array([8.0, 8.0, 8.0])
    gamma, kT, dt, every, frames = 1.0, 0.9, 0.01, 50, 80
    rng = np.random.default_rng(3)
    runs = 300
    msd = np.zeros(frames // 2)
    for seed in range(runs):
        x = np.array([[4.0], [4.0], [4.0]])
        v = rng.normal(0.0, math.sqrt(kT), size=(3, 1))
        u = x.copy()
        snaps = [u.copy()]
        for f in range(frames):
            x, v, _, _ = oracle.md_run(x, v, box, 1.5, 3.5, 0.3, dt, every, p=10, seed=seed + 1,
                                       step0=f * every, K=10, gamma=gamma, kT=kT, unwrapped=u)
            snaps.append(u.copy())
        snaps = np.array(snaps)[:, :, 0]
        for lag in range(1, frames // 2 + 1):
            d = snaps[lag:] - snaps[:-lag]
            msd[lag - 1] += float((d ** 2).sum(axis=1).mean())
    msd /= runs
    t = np.arange(1, frames // 2 + 1) * every * dt
    exact = 6.0 * kT / gamma ** 2 * (gamma * t - 1.0 + np.exp(-gamma * t))
    assert np.all(np.abs(msd - exact) < 0.08 * exact), (msd[:5], exact[:5])
    slope = bench.msd_slope(t, msd)
    assert abs(slope - 6.0 * kT / gamma) < 0.1 * 6.0 * kT / gamma, slope


def test_active_mean_skips_dispatches_that_return_at_once():
    """A build kernel launched every step that works at one step in ten:
    its summary averages the working dispatches only; a kernel that works at
    every dispatch keeps all of them."""
    gated = [1.2e6] + [3e3] * 9 + [1.25e6] + [2.5e3] * 9
    assert bench.active_mean(gated) == (2, 1.225e6)
    steady = [110.0, 108.0, 112.0]
    assert bench.active_mean(steady) == (3, 110.0)
    assert bench.active_mean([]) == (0, 0.0)
