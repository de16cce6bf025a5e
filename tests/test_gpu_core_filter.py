"""Filtered core rows (rbl_config.core_filter) on the GPU.  In runs with
rebuilds on displacement the force kernel may read core rows cut to the
partners within r_s + skin/2, filtered again at every rebuild and whenever
a particle has moved skin/4 since; every partner that can come within r_s
is kept and a dropped one contributes an exact zero, so a run with the
filter must equal the run without it bit for bit (positions, velocities,
forces, build count), whatever the precision, population, draw and launch
path.  The automatic setting (the default) must report its decision and
times, and equal the unfiltered run too."""
import numpy as np
import pytest

from paper_2105_04884_amd import Context, inputs

from gpu_util import RC, RS, dev, host, torch_cuda

pytestmark = pytest.mark.gpu


def _run(st, core_filter, steps, skin=0.5, K=13, **kw):
    torch = torch_cuda()
    x, v = dev(st.pos), dev(st.vel)
    f = torch.zeros_like(x)
    with Context(st.n, rebuild_check=True, skin=skin, lanes=kw.pop("lanes", 1), core_filter=core_filter,
                 **kw) as ctx:
        ctx.build(x, st.box, RS, RC)
        status, _ = ctx.step(x, v, nsteps=steps, dt=0.005, P=10, seed=3, rebuild_every=K, force=f)
        info = ctx.core_filter()
        builds = ctx.last_run()["builds"]
    assert status == 0
    return host(x), host(v), host(f), builds, info


def _assert_same(a, b):
    assert a[3] == b[3], f"builds {a[3]} against {b[3]}"
    for q, name in enumerate(("positions", "velocities", "forces")):
        assert np.array_equal(a[q], b[q]), f"{name} differ: max {np.abs(a[q] - b[q]).max():.3e}"


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("source,predraw", [("shell", True), ("stencil", True), ("shell", False)])
@pytest.mark.parametrize("graphs", [True, False])
def test_filtered_rows_give_the_unfiltered_run(precision, source, predraw, graphs):
    """A hot fluid (T = 2.5, N = 20,000): 60 steps with several rebuilds and
    refilterings, forced filter against none, bit for bit."""
    st = inputs.lj_fluid(20_000, 0.8442, 2.5, seed=5)
    kw = {"precision": precision, "shell_source": source, "predraw": predraw, "graphs": graphs}
    on = _run(st, 1, 60, **kw)
    off = _run(st, 0, 60, **kw)
    assert on[4]["used"] and not off[4]["used"]
    assert on[3] >= 3
    # the rows at the last filtering hold the partners within r_s + skin/2:
    # about (2.0 / 2.5)^3 of the built rows' r_s + skin, a lattice-free fluid
    assert 0 < on[4]["mean_kept"] < 26
    _assert_same(on, off)


def test_filtered_rows_with_lj_erfc_and_replicas():
    """Two replicas of different density with charges (LJ + erfc): forced
    filter against none, bit for bit."""
    torch = torch_cuda()
    a = inputs.lj_fluid(6000, 0.8, 1.5, seed=7)
    b = inputs.lj_fluid(9000, 0.6, 1.0, seed=8)
    pos = np.ascontiguousarray(np.concatenate([a.pos, b.pos], axis=1))
    vel = np.ascontiguousarray(np.concatenate([a.vel, b.vel], axis=1))
    boxes = np.stack([a.box, b.box])
    off_ = np.array([0, a.n, a.n + b.n], dtype=np.int64)
    n = a.n + b.n
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    out = []
    for cf in (1, 0):
        x, v = dev(pos), dev(vel)
        f = torch.zeros_like(x)
        with Context(n, precision="mixed", rebuild_check=True, skin=0.5, lanes=1, core_filter=cf,
                     replica_offsets=off_, pair="lj_erfc", alpha=0.3, charges=dev(q)) as ctx:
            ctx.build(x, boxes, RS, RC)
            status, _ = ctx.step(x, v, nsteps=40, dt=0.005, P=10, seed=4, rebuild_every=13, force=f)
            used = ctx.core_filter()["used"]
            builds = ctx.last_run()["builds"]
        assert status == 0
        out.append((host(x), host(v), host(f), builds, used))
    assert out[0][4] and not out[1][4]
    _assert_same(out[0], out[1])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("ntypes", [2, 3])
def test_filtered_rows_with_particle_types(precision, ntypes):
    """Particle types (pair radii r_s sigma_ab, r_c sigma_ab; each pair's
    filter radius r_s sigma_ab + skin/2): a hot mixture, forced filter
    against none, bit for bit."""
    torch = torch_cuda()
    if ntypes == 2:
        st = inputs.mixture(16_000, 0.5, 2.0, 11, (0.8, 0.2))
        table = np.array([[[1.0, 1.0], [1.0, 1.2]], [[1.0, 1.2], [1.0, 1.4]]])
    else:
        st = inputs.mixture(12_000, 0.45, 2.0, 12, (0.5, 0.3, 0.2))
        eps = np.array([[1.0, 1.5, 0.7], [1.5, 0.5, 1.2], [0.7, 1.2, 2.0]])
        sig = np.array([[1.0, 0.8, 1.3], [0.8, 0.88, 1.1], [1.3, 1.1, 1.6]])
        table = np.ascontiguousarray(np.stack([eps, sig], axis=-1))
    out = []
    for cf in (1, 0):
        x, v = dev(st.pos), dev(st.vel)
        f = torch.zeros_like(x)
        with Context(st.n, precision=precision, rebuild_check=True, skin=0.5, lanes=1, core_filter=cf,
                     types=st.types, eps_sig=table) as ctx:
            ctx.build(x, st.box, RS, RC)
            status, _ = ctx.step(x, v, nsteps=50, dt=0.004, P=10, seed=2, rebuild_every=13, force=f)
            used = ctx.core_filter()["used"]
            builds = ctx.last_run()["builds"]
        assert status == 0
        out.append((host(x), host(v), host(f), builds, used))
    assert out[0][4] and not out[1][4]
    assert out[0][3] >= 2
    _assert_same(out[0], out[1])


def test_filtered_rows_with_the_langevin_thermostat():
    """BAOAB Langevin steps (gamma = 1, kT = 2.0) move the particles with
    noise between the displacement tests: forced filter against none, bit
    for bit."""
    torch = torch_cuda()
    st = inputs.lj_fluid(12_000, 0.8442, 2.0, seed=9)
    out = []
    for cf in (1, 0):
        x, v = dev(st.pos), dev(st.vel)
        f = torch.zeros_like(x)
        with Context(st.n, precision="mixed", rebuild_check=True, skin=0.5, lanes=1, core_filter=cf) as ctx:
            ctx.set_thermostat(1.0, 2.0)
            ctx.build(x, st.box, RS, RC)
            status, _ = ctx.step(x, v, nsteps=50, dt=0.005, P=10, seed=6, rebuild_every=13, force=f)
            used = ctx.core_filter()["used"]
            builds = ctx.last_run()["builds"]
        assert status == 0
        out.append((host(x), host(v), host(f), builds, used))
    assert out[0][4] and not out[1][4]
    _assert_same(out[0], out[1])


def _two_runs(st, core_filter, **kw):
    """40 steps, then 40 more continued from the state the first left;
    returns the final state and the filter report after each run."""
    torch = torch_cuda()
    x, v = dev(st.pos), dev(st.vel)
    f = torch.zeros_like(x)
    with Context(st.n, rebuild_check=True, skin=0.5, core_filter=core_filter, **kw) as ctx:
        ctx.build(x, st.box, RS, RC)
        s1, _ = ctx.step(x, v, nsteps=40, dt=0.005, P=10, seed=3, rebuild_every=13, force=f)
        first = ctx.core_filter()
        s2, _ = ctx.cont(40, pos=x, vel=v, force=f)
        info = ctx.core_filter()
        builds = ctx.last_run()["builds"]
    assert s1 == 0 and s2 == 0
    return host(x), host(v), host(f), builds, info, first


def test_automatic_filter_at_the_benchmark_size():
    """N = 10^6 in the benchmark's configuration (mixed, one lane per
    particle as the autotuner picks there, autotuned launch mode): the
    automatic setting leaves the first run unfiltered, decides at its end,
    reports its three times and, used or not, gives the unfiltered runs bit
    for bit."""
    st = inputs.million_fluid(seed=1)
    auto = _two_runs(st, "auto", precision="mixed", lanes=1, persistent=0)
    off = _two_runs(st, 0, precision="mixed", lanes=1, persistent=0)
    assert not auto[5]["used"]
    us = auto[4]["force_us"]
    print(f"core filter: used {auto[4]['used']}, unfiltered {us[0]:.1f} us, filtered {us[1]:.1f} us, "
          f"filtering {us[2]:.1f} us")
    if auto[4]["used"]:
        assert all(t > 0 for t in us) and auto[4]["mean_kept"] > 0
    _assert_same(auto, off)
