"""Langevin thermostat and the observables of Sec. III on the GPU against
the oracle: BAOAB trajectories (the thermostat noise goes through each
side's own log/cos/sin, so states match to rounding, not bit for bit), the
continuous trajectory behind the mean-squared displacement, the RDF pair
histogram (bit-exact integer counts) and the tail-corrected energy and
pressure.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2105_04884_amd import Context, RblError, inputs
from paper_2105_04884_amd import _lib

from gpu_util import RC, RS, SKIN, assert_forces_close, dev, host, rel_l2, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("use_full", [False, True])
def test_langevin_trajectory_matches_oracle(use_full):
    """100 BAOAB steps (gamma = 1, kT = 0.9) of the N = 1000 fluid; captured
    and step-by-step execution agree bit for bit."""
    torch = torch_cuda()
    st = inputs.small_fluid(seed=1)
    runs = []
    for graphs in (True, False):
        x, v = dev(st.pos), dev(st.vel)
        f = torch.zeros_like(x)
        lists = ("full",) if use_full else ("core", "shell")
        with Context(st.n, lanes=1, graphs=graphs, lists=lists) as ctx:
            ctx.set_thermostat(1.0, 0.9)
            ctx.build(x, st.box, RS, RC)
            ctx.step(x, v, nsteps=100, dt=0.005, P=10, seed=3, rebuild_every=10, use_full=use_full,
                     force=f)
        runs.append((host(x), host(v), host(f)))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])
    xo, vo, fo, _ = oracle.md_run(st.pos, st.vel, st.box, RS, RC, SKIN, 0.005, 100, p=10, seed=3,
                                  K=10, use_full=use_full, gamma=1.0, kT=0.9)
    x, v, f = runs[0]
    assert rel_l2(x, xo) < 1e-11
    assert rel_l2(v, vo) < 1e-8
    assert_forces_close(f, fo, 1e-7)
    # the thermostat acted: NVE from the same start ends elsewhere
    xn, _, _, _ = oracle.md_run(st.pos, st.vel, st.box, RS, RC, SKIN, 0.005, 100, p=10, seed=3,
                                K=10, use_full=use_full)
    assert rel_l2(x, xn) > 1e-6


def test_langevin_ensemble_per_replica_temperatures():
    """Replicas with their own bath temperatures, each against its oracle
    run with the replica index in the noise counter."""
    torch_cuda()
    specs = [(600, 0.8, 1.0, 1), (900, 0.6, 1.4, 2), (300, 0.3, 0.7, 3)]
    kts = [0.8, 1.5, 0.6]
    states = [inputs.lj_fluid(*s) for s in specs]
    pos = np.concatenate([s.pos for s in states], axis=1)
    vel = np.concatenate([s.vel for s in states], axis=1)
    boxes = np.stack([s.box for s in states])
    off = np.zeros(len(states) + 1, dtype=np.int64)
    off[1:] = np.cumsum([s.n for s in states])
    x, v = dev(pos), dev(vel)
    with Context(int(off[-1]), replica_offsets=off, lanes=1) as ctx:
        ctx.set_thermostat(0.5, kts)
        ctx.build(x, boxes, RS, RC)
        ctx.step(x, v, nsteps=40, dt=0.005, P=10, seed=4, rebuild_every=10)
    xg, vg = host(x), host(v)
    for r, s in enumerate(states):
        xo, vo, _, _ = oracle.md_run(s.pos, s.vel, s.box, RS, RC, SKIN, 0.005, 40, p=10, seed=4,
                                     K=10, replica=r, gamma=0.5, kT=kts[r])
        sl = slice(off[r], off[r + 1])
        assert rel_l2(xg[:, sl], xo) < 1e-11, r
        assert rel_l2(vg[:, sl], vo) < 1e-8, r


def test_unwrapped_trajectory_matches_oracle():
    """A hot, dilute fluid whose particles cross the box: positions plus the
    counted wraps equal the oracle's never-wrapped trajectory, across two
    rbl_step calls; the mean-squared displacement is the plain mean."""
    torch = torch_cuda()
    st = inputs.lj_fluid(500, 0.3, 3.0, seed=6)
    x, v = dev(st.pos), dev(st.vel)
    x0 = dev(st.pos)
    with Context(st.n, lanes=1) as ctx:
        ctx.set_thermostat(1.0, 3.0)
        ctx.build(x, st.box, RS, RC)
        u0 = ctx.unwrap(x0)                      # no wraps counted yet: the input
        assert torch.equal(u0, x0)
        ctx.step(x, v, nsteps=200, dt=0.005, P=10, seed=5, rebuild_every=10)
        ctx.step(x, v, nsteps=200, dt=0.005, P=10, seed=5, step0=200, rebuild_every=10)
        u = ctx.unwrap(x)
        msd = host(ctx.msd(u, x0))[0]
    uo = st.pos.copy()
    oracle.md_run(st.pos, st.vel, st.box, RS, RC, SKIN, 0.005, 200, p=10, seed=5, K=10,
                  gamma=1.0, kT=3.0, unwrapped=uo)
    # the oracle's second call starts from its own wrapped state; carry on
    # the unwrapped array from there
    xo1, vo1, _, _ = oracle.md_run(st.pos, st.vel, st.box, RS, RC, SKIN, 0.005, 200, p=10,
                                   seed=5, K=10, gamma=1.0, kT=3.0)
    oracle.md_run(xo1, vo1, st.box, RS, RC, SKIN, 0.005, 200, p=10, seed=5, step0=200, K=10,
                  gamma=1.0, kT=3.0, unwrapped=uo)
    ug = host(u)
    assert np.max(np.abs(ug - host(x))) > st.box[0] * 0.9   # some particle crossed the box
    assert rel_l2(ug, uo) < 1e-10
    d = ug - st.pos
    assert msd == pytest.approx(float((d * d).sum(axis=0).mean()), rel=1e-12)


def test_unwrap_counts_a_repeated_run_once():
    """A run repeated after a capacity overflow adds its wraps once."""
    torch_cuda()
    st = inputs.lj_fluid(500, 0.3, 3.0, seed=7)
    outs = []
    for factor in (0.5, 3.0):
        x, v = dev(st.pos), dev(st.vel)
        with Context(st.n, capacity_factor=factor, lanes=1) as ctx:
            ctx.build(x, st.box, RS, RC)
            ctx.step(x, v, nsteps=300, dt=0.005, P=10, seed=2, rebuild_every=10)
            outs.append(host(ctx.unwrap(x)))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("case", ["fluid1000", "fcc", "ensemble"])
def test_rdf_counts_match_oracle(case):
    """Ordered-pair histograms bit for bit; two frames accumulate."""
    torch_cuda()
    if case == "fluid1000":
        states = [inputs.small_fluid(seed=1)]
    elif case == "fcc":
        states = [inputs.perfect_fcc(5, 0.9)]
    else:
        states = [inputs.lj_fluid(*s) for s in [(700, 0.8, 1.0, 1), (1300, 0.4, 1.2, 2)]]
    pos = np.concatenate([s.pos for s in states], axis=1)
    boxes = np.stack([s.box for s in states])
    off = np.zeros(len(states) + 1, dtype=np.int64)
    off[1:] = np.cumsum([s.n for s in states])
    kw = {"replica_offsets": off} if len(states) > 1 else {}
    r_max, nbins = 3.5, 350
    with Context(int(off[-1]), **kw) as ctx:
        ctx.build(dev(pos), boxes if len(states) > 1 else states[0].box, RS, RC)
        counts = ctx.rdf(dev(pos), r_max, nbins)
        ctx.rdf(dev(pos), r_max, nbins, counts)
        got = host(counts).astype(np.uint64)
    for r, s in enumerate(states):
        ref = oracle.rdf_counts(s.pos, s.box, r_max, nbins)
        assert np.array_equal(got[r], 2 * ref), (case, r)


def test_thermo_energy_and_pressure_with_tails():
    """u = U/N + u_tail and P = rho T + W/(3V) + p_tail from a force call's
    [U, W] against the oracle's unshifted pair sums and tail formulas."""
    torch_cuda()
    st = inputs.small_fluid(seed=1)
    L = oracle.System(st.pos, st.box, RS, RC, SKIN).lists(kinds=("full",))
    with Context(st.n, lists=("full",), shift=False) as ctx:
        ctx.set_thermostat(1.0, 0.9)
        ctx.build(dev(st.pos), st.box, RS, RC)
        _, ev = ctx.full_forces(dev(st.pos), want_ev=True)
        out = ctx.thermo(ev, dev(st.vel))[0]
    _, e, w = oracle.full_forces(st.pos, st.box, RC, L, shift=False)
    V = float(np.prod(st.box))
    rho = st.n / V
    ut, pt = oracle.tail(rho, RC)
    tk = float((st.vel ** 2).sum()) / (3 * st.n - 3)
    assert out[0] == pytest.approx(e.sum() / st.n + ut, rel=1e-12)
    assert out[1] == pytest.approx(rho * 0.9 + w.sum() / (3 * V) + pt, rel=1e-12)
    assert out[2] == pytest.approx(tk, rel=1e-12)
    assert out[3] == pytest.approx(rho * tk + w.sum() / (3 * V) + pt, rel=1e-12)
    with Context(st.n, lists=("full",)) as ctx:           # shifted pair: refused
        ctx.build(dev(st.pos), st.box, RS, RC)
        _, ev = ctx.full_forces(dev(st.pos), want_ev=True)
        with pytest.raises(RblError):
            ctx.thermo(ev)


def test_thermostat_argument_checks():
    torch_cuda()
    with Context(10) as ctx:
        with pytest.raises(RblError):
            ctx.set_thermostat(-1.0, 1.0)
        with pytest.raises(RblError):
            ctx.set_thermostat(1.0, None)
        with pytest.raises(RblError):
            ctx.set_thermostat(1.0, -0.5)
        ctx.set_thermostat(0.0)


def test_observable_argument_checks_and_missing_values():
    """rbl_rdf refuses r_max beyond r_c and empty histograms; without a
    thermostat the bath-temperature pressure is NaN and without velocities
    the kinetic columns are NaN; unwrap and msd need the boxes of a build."""
    torch = torch_cuda()
    st = inputs.small_fluid(seed=1)
    with Context(st.n, lists=("full",), shift=False) as ctx:
        with pytest.raises(RblError):
            ctx.unwrap(dev(st.pos))
        ctx.build(dev(st.pos), st.box, RS, RC)
        with pytest.raises(RblError):
            ctx.rdf(dev(st.pos), RC + 0.1, 10)
        with pytest.raises(RblError):
            ctx.rdf(dev(st.pos), 2.0, 0, counts=torch.zeros((1, 0), dtype=torch.int64, device="cuda"))
        _, ev = ctx.full_forces(dev(st.pos), want_ev=True)
        out = ctx.thermo(ev)[0]
        assert np.isfinite(out[0]) and np.isnan(out[1]) and np.isnan(out[2]) and np.isnan(out[3])
        u = ctx.unwrap(dev(st.pos))
        assert torch.equal(u, dev(st.pos))
        assert host(ctx.msd(u, u))[0] == 0.0


def test_langevin_with_the_stencil_population():
    """The thermostat and the stencil draw population together: 60 BAOAB
    steps of an N = 8000 fluid against the oracle's run."""
    torch_cuda()
    st = inputs.lj_fluid(8000, 0.8442, 1.0, seed=21)
    x, v = dev(st.pos), dev(st.vel)
    with Context(st.n, lanes=1, shell_source="stencil") as ctx:
        ctx.set_thermostat(1.0, 1.2)
        ctx.build(x, st.box, RS, RC)
        ctx.step(x, v, nsteps=60, dt=0.005, P=10, seed=6, rebuild_every=10)
    xo, vo, _, _ = oracle.md_run(st.pos, st.vel, st.box, RS, RC, SKIN, 0.005, 60, p=10, seed=6,
                                 K=10, gamma=1.0, kT=1.2, shell_source="stencil")
    assert rel_l2(host(x), xo) < 1e-11
    assert rel_l2(host(v), vo) < 1e-8
