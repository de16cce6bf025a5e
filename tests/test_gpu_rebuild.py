"""Lists rebuilt on displacement (cfg.rebuild_check) on the GPU against the
oracle: the rebuild schedule of particles in free flight worked out by
hand, trajectories of hot fluids with the oracle's displacement criterion,
captured and step-by-step execution and continued runs bit for bit, and at
the benchmark's sizes lists that hold every core pair at the final state."""
import numpy as np
import pytest

import oracle
from paper_2105_04884_amd import Context, inputs
from paper_2105_04884_amd import _lib

from gpu_util import RC, RS, SKIN, assert_forces_close, dev, host, rel_l2, torch_cuda

pytestmark = pytest.mark.gpu


def _free_flight(speeds, box=20.0):
    n = len(speeds)
    pos = np.zeros((3, n))
    for k in range(n):
        pos[:, k] = [1.0 + 9.0 * (k % 2), 2.0 + 9.0 * ((k // 2) % 2), 3.0 + 9.0 * (k // 4)]
    vel = np.zeros((3, n))
    vel[0] = speeds
    return pos, vel, np.array([box, box, box])


@pytest.mark.parametrize("graphs", [True, False])
@pytest.mark.parametrize("speeds,K,want", [
    ([1.1, 0.0], 100, [0, 28, 56, 84]),
    ([1.1, 0.0], 25, [0, 25, 50, 75, 100]),
    ([0.3, 2.0, 1.1, 0.0], 100, [0, 16, 32, 48, 64, 80, 96]),
    ([0.0, 0.0], 40, [0, 40, 80]),
])
def test_free_flight_rebuild_schedule(speeds, K, want, graphs):
    """The oracle's hand-worked schedule (rebuild at the first step more
    than skin/2 = 0.15 from the last build, or K steps after it): same
    number of builds and same last build on the GPU, also when the run is
    split with rbl_continue."""
    torch_cuda()
    pos, vel, box = _free_flight(speeds)
    for chunks in ((100,), (37, 63)):
        x, v = dev(pos), dev(vel)
        builds = 0
        with Context(len(speeds), rebuild_check=True, graphs=graphs, lanes=1) as ctx:
            ctx.build(x, box, RS, RC)
            st, _ = ctx.step(x, v, nsteps=chunks[0], dt=0.005, P=10, seed=1, rebuild_every=K)
            builds += ctx.last_run()["builds"]
            for c in chunks[1:]:
                st, _ = ctx.cont(c, pos=x, vel=v)
                builds += ctx.last_run()["builds"]
            info = ctx.last_run()
        assert st == _lib.RBL_OK
        assert builds == len(want), (chunks, builds, want)
        assert info["build_step"] == want[-1]
        assert np.allclose(host(v), vel)


# the full list has no draw population, so it runs once
@pytest.mark.parametrize("source,use_full", [("shell", False), ("stencil", False), ("shell", True)])
def test_hot_fluid_trajectory_matches_oracle(source, use_full):
    """N = 1000 at T = 3 with a 40-step longest lifetime, rebuilds decided
    by displacement: 60 steps (FP64, one lane per particle) against the
    oracle's run with the same criterion; same number of builds."""
    torch_cuda()
    st = inputs.lj_fluid(1000, 0.8, 3.0, seed=21)
    x, v = dev(st.pos), dev(st.vel)
    lists = ("full",) if use_full else ("core", "shell")
    with Context(st.n, rebuild_check=True, lanes=1, lists=lists, shell_source=source) as ctx:
        ctx.build(x, st.box, RS, RC)
        status, _ = ctx.step(x, v, nsteps=60, dt=0.005, P=10, seed=7, rebuild_every=40, use_full=use_full)
        info = ctx.last_run()
    assert status == _lib.RBL_OK
    builds = []
    xo, vo, _, _ = oracle.md_run(st.pos, st.vel, st.box, RS, RC, SKIN, 0.005, 60, p=10, seed=7, K=40,
                                 use_full=use_full, shell_source=source, check=True, builds=builds)
    assert info["builds"] == len(builds) and info["build_step"] == builds[-1], (info, builds)
    assert len(builds) > 5
    assert rel_l2(host(x), xo) < 1e-12
    assert rel_l2(host(v), vo) < 1e-9


@pytest.mark.parametrize("chunks", [(60,), (25, 35), (7, 1, 52)])
def test_gated_runs_identical_across_execution_modes(chunks):
    """Captured blocks of gated steps, the same steps queued one by one, and
    runs continued in pieces give the same trajectory bit for bit."""
    torch_cuda()
    st = inputs.lj_fluid(1000, 0.8, 2.0, seed=22)
    out = []
    for graphs in (True, False):
        x, v = dev(st.pos), dev(st.vel)
        with Context(st.n, rebuild_check=True, lanes=1, graphs=graphs) as ctx:
            ctx.build(x, st.box, RS, RC)
            ctx.step(x, v, nsteps=chunks[0], dt=0.005, P=10, seed=3, rebuild_every=10)
            for c in chunks[1:]:
                ctx.cont(c, pos=x, vel=v)
        out.append((host(x), host(v)))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
    ref = oracle.md_run(st.pos, st.vel, st.box, RS, RC, SKIN, 0.005, 60, p=10, seed=3, K=10, check=True)
    assert rel_l2(out[0][0], ref[0]) < 1e-12


def _core_rows_hold_current_pairs(ctx, xg, box, rs, rows):
    """Every pair closer than r_s at the final positions is in the row the
    last build left (the force then misses no core pair)."""
    got = ctx.export_lists(rows=rows, kinds=("core",))
    cur = oracle.System(xg, box, rs, rs + 1e-9, 0.0).lists(rows=rows, kinds=("core",))
    for k in range(len(rows)):
        have = set(got["core_idx"][got["core_off"][k]:got["core_off"][k + 1]].tolist())
        need = cur.row("core", k)
        d = xg[:, need] - xg[:, [rows[k]]]
        d -= box[:, None] * np.rint(d / box[:, None])
        need = need[(d ** 2).sum(axis=0) < rs * rs]
        assert set(need.tolist()) <= have, rows[k]


@pytest.mark.parametrize("name", ["million", "large", "slab"])
def test_bench_workloads_with_displacement_rebuilds(name):
    """The benchmark's single-system workloads with rebuilds on displacement
    (mixed precision, autotuned launch): RBL_OK, more builds than a 10-step
    lifetime would take when the fluid is hot enough, and at the final state
    every current core pair of sampled particles in its row."""
    torch_cuda()
    kw = {}
    if name == "million":
        st, rs, rc, P = inputs.million_fluid(seed=1), RS, RC, 10
    elif name == "large":
        st, rs, rc, P = inputs.large_fluid(seed=1), 1.3, 4.0, 10
    else:
        st, rs, rc, P = inputs.slab(seed=1), RS, 5.0, 20
        kw = {"pair": "lj_erfc", "alpha": 0.3, "charges": dev(st.charges)}
    x, v = dev(st.pos), dev(st.vel)
    with Context(st.n, precision="mixed", rebuild_check=True, **kw) as ctx:
        ctx.build(x, st.box, rs, rc)
        status, _ = ctx.step(x, v, nsteps=30, dt=0.005, P=P, seed=1, rebuild_every=10)
        info = ctx.last_run()
        assert status == _lib.RBL_OK
        assert info["builds"] >= 4, info
        rows = np.random.default_rng(6).choice(st.n, size=200, replace=False)
        _core_rows_hold_current_pairs(ctx, host(x), st.box, rs, rows)
