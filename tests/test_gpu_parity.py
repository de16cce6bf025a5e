"""GPU path (librbl through its C-ABI) against the CPU oracle.

Integer and index work (cell binning, neighbour lists, batches) must match
bit for bit; forces match within 1e-12 relative L2 in FP64 and 2e-5 in the
mixed FP32-pair / FP64-accumulate form, always at identical states.
"""
import numpy as np
import pytest

import oracle
from paper_2105_04884_amd import Context, RblError, inputs
from paper_2105_04884_amd import _lib

from gpu_util import (FP64_TOL, MIXED_TOL, RC, RS, SKIN, assert_forces_close, assert_lists_equal, dev,
                      host, oracle_rbl_total, rel_l2, torch_cuda)

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "fluid1000":
        st = inputs.small_fluid(seed=1)
        return st.pos, st.box
    if name == "gas_small_box":
        box = np.array([9.1, 9.1, 9.1])
        return inputs.random_gas(300, box, seed=5).pos, box
    if name == "elongated":
        box = np.array([8.2, 9.5, 24.0])
        return inputs.random_gas(900, box, seed=6).pos, box
    if name == "tiny_grid":
        box = np.array([7.7, 7.9, 12.0])
        return inputs.random_gas(250, box, seed=8).pos, box
    if name == "ragged_65":
        box = np.array([8.0, 8.0, 8.0])
        return inputs.random_gas(65, box, seed=9, min_dist=0.9).pos, box
    if name == "single":
        return np.array([[1.0], [2.0], [3.0]]), np.array([8.0, 8.0, 8.0])
    if name == "vapour":
        st = inputs.lj_fluid(3000, 0.02, 1.0, seed=4)
        return st.pos, st.box
    if name == "unwrapped":
        st = inputs.small_fluid(seed=2)
        shift = np.array([[2.0], [-3.0], [1.0]]) * st.box[:, None]
        return st.pos + shift, st.box
    raise KeyError(name)


CASES = ["fluid1000", "gas_small_box", "elongated", "tiny_grid", "ragged_65", "single",
         "vapour", "unwrapped"]


@pytest.mark.parametrize("case", CASES)
def test_binning_matches_oracle(case):
    torch_cuda()
    pos, box = _case(case)
    n = pos.shape[1]
    with Context(n, lists=("core", "shell", "full")) as ctx:
        ctx.build(dev(pos), box, RS, RC)
        ncell, slot, cnt = ctx.export_binning(with_counts=True)
    onc, _, oslot, ocs = oracle.System(pos, box, RS, RC, SKIN).binning()
    assert np.array_equal(ncell[0], onc)
    assert np.array_equal(slot, oslot)
    assert np.array_equal(cnt, np.diff(ocs))


@pytest.mark.parametrize("case", CASES)
def test_lists_match_oracle(case):
    torch_cuda()
    pos, box = _case(case)
    n = pos.shape[1]
    with Context(n, lists=("core", "shell", "full")) as ctx:
        ctx.build(dev(pos), box, RS, RC)
        got = ctx.export_lists()
    ref = oracle.System(pos, box, RS, RC, SKIN).lists(method="cells")
    assert_lists_equal(got, ref)


@pytest.mark.parametrize("P", [1, 3, 10, 20, 33, 64, 128])
def test_batches_match_oracle(P):
    torch_cuda()
    pos, box = _case("fluid1000")
    n = pos.shape[1]
    rows = np.arange(n)
    L = oracle.System(pos, box, RS, RC, SKIN).lists(kinds=("shell",))
    with Context(n) as ctx:
        ctx.build(dev(pos), box, RS, RC)
        for seed, step in ((1, 0), (7, 12345), (2**40 + 3, 2**32 + 5)):
            batch, count = ctx.export_batches(P, seed, step, rows)
            for i in range(n):
                sh = L.row("shell", i)
                kpos = oracle.batch_positions(seed, i, step, 0, P, len(sh))
                assert count[i] == len(kpos)
                assert np.array_equal(batch[i, :count[i]], sh[kpos]), (seed, step, i)
                assert np.all(batch[i, count[i]:] == -1)


def _draw_rows(pos, box, source, rows, rc=RC):
    """Oracle draw population per row (positions k of a batch index it):
    the shell row, or the stencil row of the paper's form."""
    sysm = oracle.System(pos, box, RS, rc, SKIN)
    if source == "shell":
        L = sysm.lists(rows=rows, kinds=("shell",))
        return [L.row("shell", k) for k in range(len(rows))]
    off, idx = sysm.stencil_rows(rows)
    return [idx[off[k]:off[k + 1]] for k in range(len(rows))]


def _check_drawn(batch, count, step0, popl, rows, P, seed, replica=0, pid=None):
    """Every stored batch against the oracle's Floyd draw, entry by entry."""
    nsteps = batch.shape[0]
    for k, i in enumerate(rows):
        pop = popl[k]
        assert count[k] == min(len(pop), P), (i, count[k], len(pop))
        for r in range(nsteps):
            kpos = oracle.batch_positions(seed, int(i if pid is None else pid[k]), step0 + r, replica,
                                          P, len(pop))
            assert np.array_equal(batch[r, k, :count[k]], pop[kpos]), (i, step0 + r)
            assert np.all(batch[r, k, count[k]:] == -1)


@pytest.mark.parametrize("source", ["shell", "stencil"])
@pytest.mark.parametrize("P", [1, 10, 33, 128])
def test_fused_build_batches_match_oracle(source, P):
    """The batches the fused build + draw kernel stores for a list lifetime
    (the ones the MD loop's force kernel reads), exported and compared bit
    for bit with the oracle's Floyd draw on the oracle's own rows: for every
    particle and every step of the lifetime.  Entry builds at a lifetime
    start, inside a lifetime and past 2^32 steps, then a build inside a
    captured lifetime (graph replay, device step counter)."""
    torch = torch_cuda()
    st = inputs.small_fluid(seed=1)
    n = st.n
    rows = np.arange(n)
    x0 = dev(st.pos)
    with Context(n, lanes=1, shell_source=source) as ctx:
        ctx.build(x0, st.box, RS, RC)
        for seed, step0 in ((1, 0), (7, 13), (2**40 + 3, 2**32 + 5)):
            x, v = dev(st.pos), dev(st.vel)
            ctx.step(x, v, nsteps=0, dt=0.005, P=P, seed=seed, step0=step0, rebuild_every=10)
            batch, count, s0 = ctx.export_drawn_batches(rows)
            assert s0 == step0 and batch.shape == (10 - step0 % 10, n, P)
            _check_drawn(batch, count, s0, _draw_rows(st.pos, st.box, source, rows), rows, P, seed)
        # 20 steps: the second lifetime's build runs inside the captured graph
        x, v = dev(st.pos), dev(st.vel)
        ctx.step(x, v, nsteps=20, dt=0.005, P=P, seed=3, step0=0, rebuild_every=10)
        batch, count, s0 = ctx.export_drawn_batches(rows)
        assert s0 == 20 and batch.shape[0] == 10
        # the final positions are those of the build at step 20
        _check_drawn(batch, count, s0, _draw_rows(host(x), st.box, source, rows), rows, P, 3)


def test_fused_build_batches_million_sampled():
    """The stored batches of the N = 1M fluid (mixed precision, autotuned
    lanes: the bench's configuration) on 300 sampled rows, all 10 steps of
    the lifetime, for both draw populations."""
    torch = torch_cuda()
    st = inputs.million_fluid(seed=1)
    rows = np.random.default_rng(5).choice(st.n, size=300, replace=False)
    for source in ("shell", "stencil"):
        x, v = dev(st.pos), dev(st.vel)
        with Context(st.n, precision="mixed", shell_source=source) as ctx:
            ctx.build(x, st.box, RS, RC)
            ctx.step(x, v, nsteps=20, dt=0.005, P=10, seed=1, step0=0, rebuild_every=10)
            batch, count, s0 = ctx.export_drawn_batches(rows)
        assert s0 == 20 and batch.shape == (10, 300, 10)
        _check_drawn(batch, count, s0, _draw_rows(host(x), st.box, source, rows), rows, 10, 1)


def _displaced(pos, amount, seed):
    rng = np.random.default_rng(seed)
    return pos + rng.uniform(-amount, amount, size=pos.shape)


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
@pytest.mark.parametrize("P", [5, 10, 20, 64])
def test_rbl_forces_match_oracle(precision, tol, P):
    """Force at the build state and at displaced positions (classification
    by current distance), with mean-force subtraction; energy and virial."""
    torch_cuda()
    pos, box = _case("fluid1000")
    n = pos.shape[1]
    L = oracle.System(pos, box, RS, RC, SKIN).lists()
    with Context(n, precision=precision) as ctx:
        ctx.build(dev(pos), box, RS, RC)
        for k, p in enumerate((pos, _displaced(pos, 0.1, 3))):
            f, ev = ctx.forces(P, seed=11 + k, step=3 * k, pos=dev(p), want_ev=True)
            fo, eo, wo = oracle_rbl_total(p, box, L, P, 11 + k, 3 * k)
            assert_forces_close(host(f), fo, tol)
            U, W = host(ev)
            assert abs(U - eo) <= tol * max(1.0, abs(eo)) * 10
            assert abs(W - wo) <= tol * max(1.0, abs(wo)) * 10


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", MIXED_TOL)])
def test_full_forces_match_oracle(precision, tol):
    torch_cuda()
    for case in ("fluid1000", "elongated", "vapour"):
        pos, box = _case(case)
        n = pos.shape[1]
        L = oracle.System(pos, box, RS, RC, SKIN).lists()
        with Context(n, precision=precision, lists=("full",)) as ctx:
            ctx.build(dev(pos), box, RS, RC)
            p = _displaced(pos, 0.05, 1)
            f, ev = ctx.full_forces(dev(p), want_ev=True)
            fo, eo, wo = oracle.full_forces(p, box, RC, L)
            assert_forces_close(host(f), fo, tol, case)
            U, W = host(ev)
            assert abs(U - eo.sum()) <= 10 * tol * abs(eo.sum())
            assert abs(W - wo.sum()) <= 10 * tol * abs(wo.sum())


def test_rbl_forces_edge_cases():
    """Empty shells (vapour), n_i <= P (taken whole), one particle, ragged N."""
    torch_cuda()
    for case in ("vapour", "single", "ragged_65", "tiny_grid"):
        pos, box = _case(case)
        n = pos.shape[1]
        L = oracle.System(pos, box, RS, RC, SKIN).lists()
        with Context(n) as ctx:
            ctx.build(dev(pos), box, RS, RC)
            for P in (1, 10):
                f = ctx.forces(P, seed=5, step=1, pos=dev(pos))
                fo, _, _ = oracle_rbl_total(pos, box, L, P, 5, 1)
                if np.linalg.norm(fo) == 0:
                    assert np.abs(host(f)).max() == 0.0
                else:
                    assert_forces_close(host(f), fo, FP64_TOL, (case, P))


def test_trajectory_matches_oracle():
    """100 velocity-Verlet steps of the N = 1000 fluid (P = 10, lists every
    10 steps): final state, force and energy against the oracle run; the
    lists of the final build bit-exact at the GPU's own final state."""
    torch = torch_cuda()
    st = inputs.small_fluid(seed=1)
    n = st.n
    x = dev(st.pos)
    v = dev(st.vel)
    f = torch.zeros_like(x)
    with Context(n, lists=("core", "shell")) as ctx:
        ctx.build(x, st.box, RS, RC)
        status, ev = ctx.step(x, v, nsteps=100, dt=0.005, P=10, seed=1, step0=0,
                              rebuild_every=10, force=f, want_ev=True)
        # the loop's fused build keeps shell rows in LDS only: core rows and
        # shell counts are exported
        got_lists = ctx.export_lists(kinds=("core",))
        got_counts = ctx.row_counts()
    xo, vo, fo, evo = oracle.md_run(st.pos, st.vel, st.box, RS, RC, SKIN, 0.005, 100, p=10,
                                    seed=1, K=10, want_ev=True)
    assert rel_l2(host(x), xo) < 1e-12
    assert rel_l2(host(v), vo) < 1e-9
    assert_forces_close(host(f), fo, 1e-9)
    assert abs(host(ev)[0] - evo[-1, 0]) < 1e-9 * abs(evo[-1, 0])
    xg = host(x)
    ref = oracle.System(xg, st.box, RS, RC, SKIN).lists(kinds=("core", "shell"))
    assert_lists_equal(got_lists, ref, kinds=("core",))
    assert np.array_equal(got_counts[1], np.diff(ref.shell_off))


@pytest.mark.parametrize("predraw", [True, False])
def test_step_restart_and_determinism(predraw):
    """40 steps straight equal 20 + 20 resumed at a rebuild boundary, bit for
    bit; pre-drawn and inline batches, and captured-graph and step-by-step
    execution, give the same trajectory (one lane per particle, the layout
    the inline-draw kernel has)."""
    torch_cuda()
    st = inputs.small_fluid(seed=3)
    n = st.n
    runs = []
    for chunks in ((40,), (20, 20)):
        x, v = dev(st.pos), dev(st.vel)
        with Context(n, predraw=predraw, lanes=1) as ctx:
            ctx.build(x, st.box, RS, RC)
            s0 = 0
            for c in chunks:
                ctx.step(x, v, nsteps=c, dt=0.005, P=10, seed=9, step0=s0, rebuild_every=10)
                s0 += c
        runs.append((host(x), host(v)))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])
    for kw in ({"predraw": not predraw}, {"predraw": predraw, "graphs": False}):
        x2, v2 = dev(st.pos), dev(st.vel)
        with Context(n, lanes=1, **kw) as ctx:
            ctx.build(x2, st.box, RS, RC)
            ctx.step(x2, v2, nsteps=40, dt=0.005, P=10, seed=9, step0=0, rebuild_every=10)
        assert np.array_equal(runs[0][0], host(x2)), kw
        assert np.array_equal(runs[0][1], host(v2)), kw


@pytest.mark.parametrize("use_full", [False, True])
@pytest.mark.parametrize("graphs", [True, False])
@pytest.mark.parametrize("chunks", [(20, 20), (15, 25), (7, 13, 1, 19)])
def test_continue_equals_one_run(chunks, graphs, use_full):
    """rbl_step over the first chunk followed by rbl_continue over the rest
    (state kept on the GPU, outputs written only by the last call) equals
    one rbl_step over all 40 steps bit for bit, whether the chunks end on a
    list rebuild or inside a list lifetime."""
    torch = torch_cuda()
    st = inputs.small_fluid(seed=5)
    lists = ("full",) if use_full else ("core", "shell")
    x, v = dev(st.pos), dev(st.vel)
    f = torch.zeros_like(x)
    with Context(st.n, lanes=1, graphs=graphs, lists=lists) as ctx:
        ctx.build(x, st.box, RS, RC)
        ctx.step(x, v, nsteps=40, dt=0.005, P=10, seed=4, step0=0, rebuild_every=10,
                 use_full=use_full, force=f)
    ref = (host(x), host(v), host(f))
    x, v = dev(st.pos), dev(st.vel)
    f = torch.zeros_like(x)
    with Context(st.n, lanes=1, graphs=graphs, lists=lists) as ctx:
        ctx.build(x, st.box, RS, RC)
        ctx.step(x, v, nsteps=chunks[0], dt=0.005, P=10, seed=4, step0=0, rebuild_every=10,
                 use_full=use_full)
        for k, c in enumerate(chunks[1:]):
            lastc = k == len(chunks) - 2
            ctx.cont(c, pos=x if lastc else None, vel=v if lastc else None, force=f if lastc else None)
        info = ctx.last_run()
    assert (info["attempts"], info["end_step"], info["resumable"]) == (1, 40, True)
    # fixed lifetimes: the run's last build is the one at step 40
    assert info["build_step"] == 40
    for a, b in zip((host(x), host(v), host(f)), ref):
        assert np.array_equal(a, b)


def test_continue_needs_an_unchanged_run():
    torch_cuda()
    st = inputs.small_fluid(seed=5)
    x, v = dev(st.pos), dev(st.vel)
    with Context(st.n) as ctx:
        ctx.build(x, st.box, RS, RC)
        with pytest.raises(RblError, match="RBL_E_STATE"):
            ctx.cont(10)
        ctx.step(x, v, nsteps=10, dt=0.005, P=10, seed=1)
        with pytest.raises(RblError, match="RBL_E_ARG"):
            ctx.cont(0)
        ctx.cont(10)
        assert ctx.last_run()["end_step"] == 20
        ctx.rdf(x, 2.0, 10)                       # loads the caller's positions
        assert not ctx.last_run()["resumable"]
        with pytest.raises(RblError, match="RBL_E_STATE"):
            ctx.cont(10)
        ctx.step(x, v, nsteps=10, dt=0.005, P=10, seed=1, step0=20)
        ctx.build(x, st.box, RS, RC)              # a new build
        with pytest.raises(RblError, match="RBL_E_STATE"):
            ctx.cont(10)


def test_continue_overflow_repeats_from_its_start():
    """Rows sized tightly at the lattice start overflow once the fluid
    melts during a continued run; the call is repeated from its starting
    state (a list rebuild there, at a lifetime boundary) and matches a run
    that never overflowed, bit for bit; the repeat is counted.  (With
    capacity factor 1 the fused build's shell room is 192 entries for a
    longest first shell row of 178; the oracle's run of this fluid first
    exceeds it at step 170, with 196.)"""
    torch_cuda()
    st = inputs.small_fluid(seed=4)
    runs, attempts = [], []
    for factor in (1.0, 3.0):
        x, v = dev(st.pos), dev(st.vel)
        with Context(st.n, capacity_factor=factor, lists=("core",), lanes=4) as ctx:
            ctx.build(x, st.box, RS, RC)
            # the first force only: the rows grow while the continued run melts the lattice
            ctx.step(x, v, nsteps=0, dt=0.005, P=10, seed=2, rebuild_every=10)
            ctx.cont(200, pos=x, vel=v)
            attempts.append(ctx.last_run()["attempts"])
        runs.append((host(x), host(v)))
    assert attempts == [2, 1], attempts
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])


@pytest.mark.parametrize("n,rc,steps", [
    (6400, 5.0, 20),   # ~1860 stencil candidates: one centre particle per LDS group
    (4666, 6.5, 10),   # ~4700 candidates, beyond the fused kernel's LDS lists
])
def test_large_stencils_match_oracle(n, rc, steps):
    """Fused build + draw with stencils far above the N = 1M fluid's (751
    candidates per cell): the LDS shell lists then take one centre particle
    per group, and past their budget the run falls back to explicit rows
    with inline draws.  Trajectory against the oracle (FP64, one lane per
    particle), core rows and shell counts bit-exact at the final state."""
    torch_cuda()
    st = inputs.lj_fluid(n, 0.8, 1.0, seed=11)
    x, v = dev(st.pos), dev(st.vel)
    with Context(n, lanes=1) as ctx:
        ctx.build(x, st.box, RS, rc)
        status, _ = ctx.step(x, v, nsteps=steps, dt=0.002, P=10, seed=3, rebuild_every=10)
        got_lists = ctx.export_lists(kinds=("core",))
        got_counts = ctx.row_counts()
    assert status in (0, _lib.RBL_W_SKIN)
    xo, vo, _, _ = oracle.md_run(st.pos, st.vel, st.box, RS, rc, SKIN, 0.002, steps, p=10,
                                 seed=3, K=10)
    assert rel_l2(host(x), xo) < 1e-13
    assert rel_l2(host(v), vo) < 1e-11
    ref = oracle.System(host(x), st.box, RS, rc, SKIN).lists(kinds=("core", "shell"))
    assert_lists_equal(got_lists, ref, kinds=("core",))
    assert np.array_equal(got_counts[1], np.diff(ref.shell_off))


def test_step_overflow_restart():
    """Rows sized tightly at a lattice-like first build overflow once the
    fluid melts; the run is repeated from the caller's arrays with larger
    rows and matches a run that never overflowed, bit for bit."""
    torch_cuda()
    st = inputs.small_fluid(seed=4)
    runs, caps = [], []
    for factor in (0.5, 3.0):
        x, v = dev(st.pos), dev(st.vel)
        with Context(st.n, capacity_factor=factor, lists=("core",), lanes=4) as ctx:
            ctx.build(x, st.box, RS, RC)
            cap0 = ctx.info()["cap_core"]
            ctx.step(x, v, nsteps=200, dt=0.005, P=10, seed=2, rebuild_every=10)
            caps.append((cap0, ctx.info()["cap_core"]))
        runs.append((host(x), host(v)))
    assert caps[0][1] > caps[0][0], caps          # the tight context regrew its rows
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1])


def test_full_list_nve_energy():
    """NVE with the direct-truncation force conserves energy on the GPU."""
    torch = torch_cuda()
    st = inputs.small_fluid(seed=1)
    x, v = dev(st.pos), dev(st.vel)
    with Context(st.n, lists=("full",)) as ctx:
        ctx.build(x, st.box, RS, RC)
        _, ev0 = ctx.step(x, v, nsteps=0, dt=0.004, use_full=True, want_ev=True)
        e0 = host(ev0)[0] + 0.5 * float((v * v).sum())
        _, ev1 = ctx.step(x, v, nsteps=200, dt=0.004, use_full=True, want_ev=True)
        e1 = host(ev1)[0] + 0.5 * float((v * v).sum())
    assert abs(e1 - e0) / abs(e0) < 2e-4


def test_ensemble_matches_oracle_per_replica():
    torch = torch_cuda()
    specs = [(500, 0.8, 1.0, 1), (777, 0.6, 1.2, 2), (1200, 0.9, 0.8, 3), (300, 0.3, 1.0, 4)]
    states = [inputs.lj_fluid(*s) for s in specs]
    pos = np.concatenate([s.pos for s in states], axis=1)
    boxes = np.stack([s.box for s in states])
    off = np.zeros(len(states) + 1, dtype=np.int64)
    off[1:] = np.cumsum([s.n for s in states])
    n = int(off[-1])
    with Context(n, replica_offsets=off, lists=("core", "shell", "full")) as ctx:
        ctx.build(dev(pos), boxes, RS, RC)
        got = ctx.export_lists()
        f = ctx.forces(10, seed=3, step=7, pos=dev(pos))
        ff = ctx.full_forces(dev(pos))
    f, ff = host(f), host(ff)
    for r, s in enumerate(states):
        L = oracle.System(s.pos, s.box, RS, RC, SKIN).lists()
        sl = slice(off[r], off[r + 1])
        for kind in ("core", "shell", "full"):
            go = got[kind + "_off"][off[r]:off[r + 1] + 1]
            gi = got[kind + "_idx"][go[0]:go[-1]] - off[r]
            assert np.array_equal(go - go[0], getattr(L, kind + "_off"))
            assert np.array_equal(gi, getattr(L, kind + "_idx"))
        fo, _, _ = oracle_rbl_total(s.pos, s.box, L, 10, 3, 7, replica=r)
        assert_forces_close(f[:, sl], fo, FP64_TOL)
        fu, _, _ = oracle.full_forces(s.pos, s.box, RC, L)
        assert_forces_close(ff[:, sl], fu, FP64_TOL)


def test_million_particle_sampled_parity():
    """N = 1,000,000 LJ fluid at density 0.8442 (the benchmark workload):
    sampled rows' lists and batches bit-exact, sampled raw forces (no mean
    subtraction) within tolerance in both precisions."""
    torch_cuda()
    st = inputs.million_fluid(seed=1)
    n = st.n
    rows = np.random.default_rng(0).choice(n, size=400, replace=False)
    rows = np.concatenate([rows, [0, n - 1]])
    L = oracle.System(st.pos, st.box, RS, RC, SKIN).lists(rows=rows)
    x = dev(st.pos)
    for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
        with Context(n, precision=precision, momentum_fix=False,
                     lists=("core", "shell", "full")) as ctx:
            ctx.build(x, st.box, RS, RC)
            if precision == "fp64":
                got = ctx.export_lists(rows=rows)
                assert_lists_equal(got, L)
                batch, count = ctx.export_batches(10, 1, 0, rows)
                for k, i in enumerate(rows):
                    sh = L.row("shell", k)
                    kp = oracle.batch_positions(1, int(i), 0, 0, 10, len(sh))
                    assert np.array_equal(batch[k, :count[k]], sh[kp])
            f = host(ctx.forces(10, seed=1, step=0, pos=x))[:, rows]
            fo, _, _ = oracle.rbl_forces(st.pos, st.box, RS, RC, L, 10, 1, 0)
            assert_forces_close(f, fo, tol)
            ff = host(ctx.full_forces(x))[:, rows]
            ffo, _, _ = oracle.full_forces(st.pos, st.box, RC, L)
            assert_forces_close(ff, ffo, tol)


def test_large_fluid_sampled_parity():
    """N = 2^24 LJ fluid at density 0.8 with r_s = 1.3, r_c = 4.0 (the large
    single-system workload): explicit rows, batches and raw forces of
    sampled particles against the oracle, then 10 fused MD steps and the
    sampled core rows and shell counts at the GPU's final state."""
    torch_cuda()
    rs, rc = 1.3, 4.0
    st = inputs.large_fluid(seed=1)
    n = st.n
    rows = np.random.default_rng(1).choice(n, size=300, replace=False)
    rows = np.concatenate([rows, [0, n - 1]])
    L = oracle.System(st.pos, st.box, rs, rc, SKIN).lists(rows=rows, kinds=("core", "shell"))
    x = dev(st.pos)
    with Context(n, precision="fp64", momentum_fix=False, lanes=1) as ctx:
        ctx.build(x, st.box, rs, rc)
        got = ctx.export_lists(rows=rows, kinds=("core", "shell"))
        assert_lists_equal(got, L, kinds=("core", "shell"))
        batch, count = ctx.export_batches(10, 1, 0, rows)
        for k, i in enumerate(rows):
            sh = L.row("shell", k)
            kp = oracle.batch_positions(1, int(i), 0, 0, 10, len(sh))
            assert np.array_equal(batch[k, :count[k]], sh[kp])
        f = host(ctx.forces(10, seed=1, step=0, pos=x))[:, rows]
        fo, _, _ = oracle.rbl_forces(st.pos, st.box, rs, rc, L, 10, 1, 0)
        assert_forces_close(f, fo, FP64_TOL)
        v = dev(st.vel)
        status, _ = ctx.step(x, v, nsteps=10, dt=0.005, P=10, seed=1, rebuild_every=10)
        assert status in (0, _lib.RBL_W_SKIN)
        got = ctx.export_lists(rows=rows, kinds=("core",))
        counts = ctx.row_counts(rows)
    L2 = oracle.System(host(x), st.box, rs, rc, SKIN).lists(rows=rows, kinds=("core", "shell"))
    assert_lists_equal(got, L2, kinds=("core",))
    assert np.array_equal(counts[1], np.diff(L2.shell_off))


def test_ensemble_512_sampled_replicas_md():
    """The 512-replica ensemble (N log-uniform in [2000, 65536], densities
    and temperatures uniform) advanced together, 20 FP64 steps with lists
    every 10: eight sampled replicas against the oracle's run of each alone
    (replica index in the Philox counter)."""
    torch_cuda()
    ens = inputs.ensemble(512, seed=1)
    pos, vel, boxes, off = ens.concat()
    n = int(off[-1])
    x, v = dev(pos), dev(vel)
    with Context(n, replica_offsets=off, lanes=1) as ctx:
        ctx.build(x, boxes, RS, RC)
        status, _ = ctx.step(x, v, nsteps=20, dt=0.005, P=10, seed=5, rebuild_every=10)
    assert status in (0, _lib.RBL_W_SKIN)
    xg, vg = host(x), host(v)
    for r in np.linspace(0, 511, 8).astype(int):
        s = ens.states[r]
        sl = slice(off[r], off[r + 1])
        xo, vo, _, _ = oracle.md_run(s.pos, s.vel, s.box, RS, RC, SKIN, 0.005, 20, p=10, seed=5, K=10,
                                     replica=int(r))
        assert rel_l2(xg[:, sl], xo) < 1e-13, r
        assert rel_l2(vg[:, sl], vo) < 1e-11, r


ALPHA = 0.3  # real-space Ewald screening of the charged slab


def test_charged_slab_forces_match_oracle():
    """LJ + real-space Ewald pair (alpha 0.3, r_c = 5.0, P = 20) on a small
    charged liquid slab in vapour: lists bit-exact, RBL and full forces and
    the energy within tolerance in both precisions."""
    torch_cuda()
    rc, P = 5.0, 20
    st = inputs.slab(6000, seed=2)
    L = oracle.System(st.pos, st.box, RS, rc, SKIN).lists()
    x, q = dev(st.pos), dev(st.charges)
    fo, eo, _ = oracle.rbl_forces(st.pos, st.box, RS, rc, L, P, 4, 3, charges=st.charges, alpha=ALPHA)
    ffo, efo, _ = oracle.full_forces(st.pos, st.box, rc, L, charges=st.charges, alpha=ALPHA)
    for precision, tol in (("fp64", FP64_TOL), ("mixed", MIXED_TOL)):
        with Context(st.n, precision=precision, momentum_fix=False, pair="lj_erfc", alpha=ALPHA,
                     charges=q, lists=("core", "shell", "full")) as ctx:
            ctx.build(x, st.box, RS, rc)
            if precision == "fp64":
                assert_lists_equal(ctx.export_lists(), L)
            f, ev = ctx.forces(P, seed=4, step=3, pos=x, want_ev=True)
            assert_forces_close(host(f), fo, tol)
            assert abs(host(ev)[0] - eo.sum()) < 10 * tol * abs(eo.sum())
            ff, evf = ctx.full_forces(x, want_ev=True)
            assert_forces_close(host(ff), ffo, tol)
            assert abs(host(evf)[0] - efo.sum()) < 10 * tol * abs(efo.sum())


def test_charged_slab_trajectory_matches_oracle():
    """20 FP64 steps of the charged slab (lists every 10, fused build and
    draw) against the oracle's run."""
    torch_cuda()
    rc, P = 5.0, 20
    st = inputs.slab(6000, seed=3)
    x, v, q = dev(st.pos), dev(st.vel), dev(st.charges)
    with Context(st.n, pair="lj_erfc", alpha=ALPHA, charges=q, lanes=1) as ctx:
        ctx.build(x, st.box, RS, rc)
        status, _ = ctx.step(x, v, nsteps=20, dt=0.004, P=P, seed=6, rebuild_every=10)
    assert status in (0, _lib.RBL_W_SKIN)
    xo, vo, _, _ = oracle.md_run(st.pos, st.vel, st.box, RS, rc, SKIN, 0.004, 20, p=P, seed=6, K=10,
                                 charges=st.charges, alpha=ALPHA)
    assert rel_l2(host(x), xo) < 1e-12
    assert rel_l2(host(v), vo) < 1e-9


def test_slab_two_million_sampled_parity():
    """The N = 2,000,000 charged slab (box L x L x 3L, liquid at 0.8 in the
    middle third, vapour at 0.02 around it; r_c = 5.0, P = 20): sampled
    rows' lists, batches and forces, then 10 fused MD steps and the sampled
    core rows and shell counts at the final state."""
    torch_cuda()
    rc, P = 5.0, 20
    st = inputs.slab(seed=1)
    n = st.n
    rows = np.random.default_rng(3).choice(n, size=300, replace=False)
    rows = np.concatenate([rows, [0, n - 1]])
    L = oracle.System(st.pos, st.box, RS, rc, SKIN).lists(rows=rows, kinds=("core", "shell"))
    x, q = dev(st.pos), dev(st.charges)
    with Context(n, precision="fp64", momentum_fix=False, pair="lj_erfc", alpha=ALPHA, charges=q,
                 lanes=1) as ctx:
        ctx.build(x, st.box, RS, rc)
        assert_lists_equal(ctx.export_lists(rows=rows, kinds=("core", "shell")), L,
                           kinds=("core", "shell"))
        batch, count = ctx.export_batches(P, 1, 0, rows)
        for k, i in enumerate(rows):
            sh = L.row("shell", k)
            kp = oracle.batch_positions(1, int(i), 0, 0, P, len(sh))
            assert np.array_equal(batch[k, :count[k]], sh[kp])
        f = host(ctx.forces(P, seed=1, step=0, pos=x))[:, rows]
        fo, _, _ = oracle.rbl_forces(st.pos, st.box, RS, rc, L, P, 1, 0, charges=st.charges, alpha=ALPHA)
        assert_forces_close(f, fo, FP64_TOL)
        v = dev(st.vel)
        status, _ = ctx.step(x, v, nsteps=10, dt=0.004, P=P, seed=1, rebuild_every=10)
        assert status in (0, _lib.RBL_W_SKIN)
        got = ctx.export_lists(rows=rows, kinds=("core",))
        counts = ctx.row_counts(rows)
    L2 = oracle.System(host(x), st.box, RS, rc, SKIN).lists(rows=rows, kinds=("core", "shell"))
    assert_lists_equal(got, L2, kinds=("core",))
    assert np.array_equal(counts[1], np.diff(L2.shell_off))


def test_persistent_force_grid_matches_tile_grid():
    """The persistent force grid (resident blocks walking the work tiles)
    and one block per tile give the same forces and trajectory bit for bit
    at N = 10^6, where the persistent blocks take several tiles each."""
    torch_cuda()
    st = inputs.million_fluid(seed=2)
    out = []
    for persistent in (1, 2):
        x, v = dev(st.pos), dev(st.vel)
        with Context(st.n, precision="mixed", lanes=2, persistent=persistent) as ctx:
            ctx.build(x, st.box, RS, RC)
            f = host(ctx.forces(10, seed=1, step=0, pos=x))
            ctx.step(x, v, nsteps=20, dt=0.005, P=10, seed=1, rebuild_every=10)
            assert ctx.tuning()["persistent_rbl"] == persistent - 1
        out.append((f, host(x), host(v)))
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_error_paths():
    torch = torch_cuda()
    pos, box = _case("fluid1000")
    n = pos.shape[1]
    x = dev(pos)
    with Context(n) as ctx:
        with pytest.raises(RblError) as e:
            ctx.forces(10, 1, 0, x)
        assert e.value.status == _lib.RBL_E_STATE
        with pytest.raises(RblError) as e:
            ctx.build(x, np.array([7.0, 7.0, 7.0]), RS, RC)
        assert e.value.status == _lib.RBL_E_BOX
        with pytest.raises(RblError) as e:
            ctx.build(x, box, 2.0, 1.0)
        assert e.value.status == _lib.RBL_E_ARG
        ctx.build(x, box, RS, RC)
        for P in (0, _lib.MAX_P + 1):
            with pytest.raises(RblError) as e:
                ctx.forces(P, 1, 0, x)
            assert e.value.status == _lib.RBL_E_ARG
        with pytest.raises(RblError) as e:
            ctx.full_forces(x)
        assert e.value.status == _lib.RBL_E_STATE
        bad = pos.copy()
        bad[0, 5] = np.nan
        with pytest.raises(RblError) as e:
            ctx.build(dev(bad), box, RS, RC)
        assert e.value.status == _lib.RBL_E_NONFINITE


def test_skin_warning_on_large_displacement():
    """A particle that moves more than skin/2 in one list lifetime makes
    rbl_step return the skin warning."""
    torch_cuda()
    box = np.array([20.0, 20.0, 20.0])
    pos = np.array([[2.0, 12.0], [2.0, 12.0], [2.0, 12.0]])
    vel = np.array([[40.0, 0.0], [0.0, 0.0], [0.0, 0.0]])
    x, v = dev(pos), dev(vel)
    with Context(2) as ctx:
        ctx.build(x, box, RS, RC)
        status, _ = ctx.step(x, v, nsteps=10, dt=0.005, P=10, seed=1, rebuild_every=10)
        assert status == _lib.RBL_W_SKIN
        x, v = dev(pos), dev(np.zeros((3, 2)))
        status, _ = ctx.step(x, v, nsteps=10, dt=0.005, P=10, seed=1, rebuild_every=10)
        assert status == _lib.RBL_OK


@pytest.mark.parametrize("lanes", [1, 2, 4])
def test_lanes_per_particle_variants_match_oracle(lanes):
    """Every lanes-per-particle layout of the pre-drawn RBL and full-list
    kernels stays within tolerance of the oracle along a trajectory."""
    torch_cuda()
    st = inputs.small_fluid(seed=1)
    for use_full in (False, True):
        x, v = dev(st.pos), dev(st.vel)
        lists = ("full",) if use_full else ("core", "shell")
        with Context(st.n, lanes=lanes, lists=lists) as ctx:
            ctx.build(x, st.box, RS, RC)
            ctx.step(x, v, nsteps=30, dt=0.005, P=10, seed=1, rebuild_every=10, use_full=use_full)
            assert ctx.tuning()["lpp_rbl"] == lanes
        xo, vo, _, _ = oracle.md_run(st.pos, st.vel, st.box, RS, RC, SKIN, 0.005, 30, p=10, seed=1,
                                     K=10, use_full=use_full)
        assert rel_l2(host(x), xo) < 1e-12
        assert rel_l2(host(v), vo) < 1e-9


def test_autotuner_picks_a_measured_layout():
    torch_cuda()
    st = inputs.small_fluid(seed=1)
    x, v = dev(st.pos), dev(st.vel)
    with Context(st.n) as ctx:
        ctx.build(x, st.box, RS, RC)
        ctx.step(x, v, nsteps=20, dt=0.005, P=10, seed=1, rebuild_every=10)
        t = ctx.tuning()
    assert t["lpp_rbl"] in (1, 2, 4)
    assert all(u > 0 for u in t["rbl_us"])
    assert t["rbl_us"][(1, 2, 4).index(t["lpp_rbl"])] == min(t["rbl_us"])


@pytest.mark.parametrize("lanes", [2, 4])
def test_mixed_classification_at_thresholds_matches_fp64(lanes):
    """Pairs planted within 1e-7 of r_s and r_c: the mixed kernels classify
    them on FP64 r^2 as the oracle does, so full-list and RBL forces (the
    multi-lane kernels) match the FP64 oracle within the mixed tolerance, at
    the build state and after a displacement, and the planted particles'
    forces show no pair on the wrong side of a threshold."""
    torch_cuda()
    rng = np.random.default_rng(12)
    box = np.array([16.0, 16.0, 16.0])
    st = inputs.random_gas(1500, box, seed=13, min_dist=0.85)
    pos = st.pos.copy()
    # plant pairs at the thresholds: particle 2k+1 placed at distance r from 2k
    for k, r in enumerate([RS * (1 - 1e-7), RS * (1 + 1e-7), RC * (1 - 1e-7), RC * (1 + 1e-7), RS, RC]):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        pos[:, 2 * k + 1] = pos[:, 2 * k] + r * u
    pos = pos % box[:, None]
    Lf = oracle.System(pos, box, RS, RC, SKIN).lists(kinds=("core", "shell", "full"))
    with Context(pos.shape[1], precision="mixed", lanes=lanes, lists=("core", "shell", "full")) as ctx:
        ctx.build(dev(pos), box, RS, RC)
        planted = np.arange(12)
        for p in (pos, pos + rng.uniform(-0.05, 0.05, size=pos.shape)):
            ff = host(ctx.full_forces(dev(p)))
            fo, _, _ = oracle.full_forces(p, box, RC, Lf)
            assert_forces_close(ff, fo, MIXED_TOL)
            # a pair classified on the wrong side of r_c would move its
            # particles' force by |f(r_c)| ~ 4e-3, of r_s by ~1
            err = np.linalg.norm(ff[:, planted] - fo[:, planted], axis=0)
            assert np.all(err <= 1e-5 * np.maximum(np.linalg.norm(fo[:, planted], axis=0), 1.0))
            f = host(ctx.forces(64, seed=5, step=1, pos=dev(p)))
            fr, _, _ = oracle_rbl_total(p, box, Lf, 64, 5, 1)
            assert_forces_close(f, fr, MIXED_TOL)


@pytest.mark.parametrize("source", ["shell", "stencil"])
def test_million_particle_md_in_the_bench_configuration(source):
    """N = 10^6 in the configuration the benchmark times (mixed precision,
    fused build + draw, autotuned lanes and launch mode, captured list
    lifetimes): after 20 steps (the last force evaluation right after a
    rebuild), the raw force of sampled rows equals the oracle's RBL force at
    the GPU's final positions (lists built there, Philox step 20)."""
    torch = torch_cuda()
    st = inputs.million_fluid(seed=1)
    n = st.n
    x, v = dev(st.pos), dev(st.vel)
    f = torch.zeros_like(x)
    with Context(n, precision="mixed", momentum_fix=False, shell_source=source) as ctx:
        ctx.build(x, st.box, RS, RC)
        status, _ = ctx.step(x, v, nsteps=20, dt=0.005, P=10, seed=1, rebuild_every=10, force=f)
        tuning = ctx.tuning()
    assert status in (0, _lib.RBL_W_SKIN)
    assert tuning["lpp_rbl"] in (1, 2, 4)
    xg = host(x)
    rows = np.random.default_rng(1).choice(n, size=300, replace=False)
    sysm = oracle.System(xg, st.box, RS, RC, SKIN)
    L = sysm.lists(rows=rows, kinds=("core", "shell")) if source == "shell" else sysm.stencil_lists(rows=rows)
    fo, _, _ = oracle.rbl_forces(xg, st.box, RS, RC, L, 10, 1, 20)
    assert_forces_close(host(f)[:, rows], fo, MIXED_TOL)


def _bench_config_md(st, rs, rc, P, charges=None, steps=20):
    """`steps` MD steps in the benchmark's configuration (mixed precision,
    fused build + draw, autotuned lanes and launch mode, captured list
    lifetimes, no mean subtraction so the force is the raw estimate); returns
    the final positions and the force of the last evaluation (step `steps`,
    right after a rebuild)."""
    torch = torch_cuda()
    x, v = dev(st.pos), dev(st.vel)
    f = torch.zeros_like(x)
    kw = {}
    if charges is not None:
        kw = {"pair": "lj_erfc", "alpha": ALPHA, "charges": dev(charges)}
    with Context(st.n, precision="mixed", momentum_fix=False, **kw) as ctx:
        ctx.build(x, st.box, rs, rc)
        status, _ = ctx.step(x, v, nsteps=steps, dt=0.005, P=P, seed=1, rebuild_every=10, force=f)
        assert ctx.last_run()["attempts"] >= 1
    assert status in (0, _lib.RBL_W_SKIN)
    return host(x), host(f)


def test_large_fluid_mixed_in_the_bench_configuration():
    """N = 2^24 (r_s = 1.3, r_c = 4.0, P = 10) as the benchmark runs it:
    sampled raw forces after 20 steps against the FP64 oracle at the GPU's
    final positions, within the mixed tolerance (error reported)."""
    st = inputs.large_fluid(seed=1)
    xg, f = _bench_config_md(st, 1.3, 4.0, 10)
    rows = np.random.default_rng(2).choice(st.n, size=300, replace=False)
    L = oracle.System(xg, st.box, 1.3, 4.0, SKIN).lists(rows=rows, kinds=("core", "shell"))
    fo, _, _ = oracle.rbl_forces(xg, st.box, 1.3, 4.0, L, 10, 1, 20)
    e, m = assert_forces_close(f[:, rows], fo, MIXED_TOL)
    print(f"2^24 mixed: relative L2 {e:.2e}, worst row {m:.2e}")


def test_slab_mixed_in_the_bench_configuration():
    """The N = 2M charged slab (LJ + erfc, r_c = 5.0, P = 20) as the
    benchmark runs it, sampled raw forces after 20 steps against the FP64
    oracle."""
    st = inputs.slab(seed=1)
    xg, f = _bench_config_md(st, RS, 5.0, 20, charges=st.charges)
    rows = np.random.default_rng(4).choice(st.n, size=300, replace=False)
    L = oracle.System(xg, st.box, RS, 5.0, SKIN).lists(rows=rows, kinds=("core", "shell"))
    fo, _, _ = oracle.rbl_forces(xg, st.box, RS, 5.0, L, 20, 1, 20, charges=st.charges, alpha=ALPHA)
    e, m = assert_forces_close(f[:, rows], fo, MIXED_TOL)
    print(f"slab mixed: relative L2 {e:.2e}, worst row {m:.2e}")


def test_ensemble_512_mixed_in_the_bench_configuration():
    """The 512-replica ensemble advanced together as the benchmark runs it
    (mixed, autotuned lanes and launch mode on the uneven 64-slot replica
    slices): on eight sampled replicas every raw force after 20 steps
    against the FP64 oracle of that replica alone (replica index in the
    Philox counter)."""
    torch = torch_cuda()
    ens = inputs.ensemble(512, seed=1)
    pos, vel, boxes, off = ens.concat()
    n = int(off[-1])
    x, v = dev(pos), dev(vel)
    f = torch.zeros_like(x)
    with Context(n, precision="mixed", momentum_fix=False, replica_offsets=off) as ctx:
        ctx.build(x, boxes, RS, RC)
        status, _ = ctx.step(x, v, nsteps=20, dt=0.005, P=10, seed=5, rebuild_every=10, force=f)
    assert status in (0, _lib.RBL_W_SKIN)
    xg, fg = host(x), host(f)
    for r in np.linspace(0, 511, 8).astype(int):
        sl = slice(off[r], off[r + 1])
        xr = np.ascontiguousarray(xg[:, sl])
        L = oracle.System(xr, boxes[r], RS, RC, SKIN).lists(kinds=("core", "shell"))
        fo, _, _ = oracle.rbl_forces(xr, boxes[r], RS, RC, L, 10, 5, 20, replica=int(r))
        e, m = assert_forces_close(fg[:, sl], fo, MIXED_TOL, f"replica {r}")
        print(f"ensemble mixed replica {r}: relative L2 {e:.2e}, worst row {m:.2e}")


@pytest.mark.parametrize("P", [1, 33, 128])
def test_fused_draw_at_extreme_batch_sizes(P):
    """The fused build + draw at P = 1, 33 (first unrolled-loop-free Floyd
    instance) and RBL_MAX_P = 128: a 20-step trajectory of the N = 1000
    fluid against the oracle's (FP64, one lane per particle)."""
    torch_cuda()
    st = inputs.small_fluid(seed=5)
    x, v = dev(st.pos), dev(st.vel)
    with Context(st.n, lanes=1) as ctx:
        ctx.build(x, st.box, RS, RC)
        ctx.step(x, v, nsteps=20, dt=0.005, P=P, seed=3, rebuild_every=10)
    xo, vo, _, _ = oracle.md_run(st.pos, st.vel, st.box, RS, RC, SKIN, 0.005, 20, p=P, seed=3, K=10)
    assert rel_l2(host(x), xo) < 1e-13
    assert rel_l2(host(v), vo) < 1e-11


def test_fused_build_on_a_lattice_with_exact_ties():
    """A simple cubic lattice of spacing 1 with r_c + skin = 2.7 + 0.3 = 3
    exactly: every (3,0,0) and (2,2,1) neighbour sits at r^2 = 9, on the
    outer threshold, and must stay out of the shell as in the oracle.  The
    fused build (with its bounding-box skip of far candidates) at the
    lattice state gives the oracle's core rows and shell counts bit for bit,
    and a 20-step run from there follows the oracle's trajectory."""
    torch_cuda()
    rc = 2.7
    assert rc + SKIN == 3.0
    g = (np.arange(12) + 0.25).astype(np.float64)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()])
    box = np.array([12.0, 12.0, 12.0])
    n = pos.shape[1]
    rng = np.random.default_rng(4)
    vel = rng.normal(size=(3, n))
    vel -= vel.mean(axis=1, keepdims=True)
    ref = oracle.System(pos, box, RS, rc, SKIN).lists(kinds=("core", "shell"))
    shell_len = np.diff(ref.shell_off)
    assert shell_len.min() == shell_len.max()  # every site sees the same shell
    with Context(n, lanes=1) as ctx:
        xg, vg = dev(pos), dev(np.zeros_like(pos))
        ctx.build(xg, box, RS, rc)
        ctx.step(xg, vg, nsteps=0, dt=0.005, P=10, seed=3, rebuild_every=10)
        got = ctx.export_lists(kinds=("core",))
        counts = ctx.row_counts()
    assert_lists_equal(got, ref, kinds=("core",))
    assert np.array_equal(counts[1], shell_len)
    with Context(n, lanes=1) as ctx:
        xg, vg = dev(pos), dev(vel)
        ctx.build(xg, box, RS, rc)
        ctx.step(xg, vg, nsteps=20, dt=0.005, P=10, seed=3, rebuild_every=10)
    xo, vo, _, _ = oracle.md_run(pos, vel, box, RS, rc, SKIN, 0.005, 20, p=10, seed=3, K=10)
    assert rel_l2(host(xg), xo) < 1e-13
    assert rel_l2(host(vg), vo) < 1e-11


@pytest.mark.parametrize("case", ["gas_small_box", "elongated", "tiny_grid", "ragged_65", "vapour",
                                  "unwrapped"])
def test_fused_build_on_odd_geometries(case):
    """The fused build (bounding-box skip, ring of kept candidates, lists in
    LDS) on small and elongated grids where the stencil wraps onto itself,
    on sparse and ragged populations and on unwrapped coordinates: core
    rows and shell counts at the build state bit-exact, then 20 steps from
    rest against the oracle's trajectory.  The uniform gases hold pairs
    closer than 0.25 sigma, whose forces fling particles across the box in
    one step, so their runs start from a gas of the same size and box with
    no pair closer than 0.9."""
    torch = torch_cuda()
    pos, box = _case(case)
    n = pos.shape[1]
    ref = oracle.System(pos, box, RS, RC, SKIN).lists(kinds=("core", "shell"))
    with Context(n, lanes=1) as ctx:
        x, v = dev(pos), torch.zeros((3, n), dtype=torch.float64, device="cuda")
        ctx.build(x, box, RS, RC)
        ctx.step(x, v, nsteps=0, dt=0.005, P=10, seed=9, rebuild_every=10)
        got = ctx.export_lists(kinds=("core",))
        counts = ctx.row_counts()
    assert_lists_equal(got, ref, kinds=("core",))
    assert np.array_equal(counts[1], np.diff(ref.shell_off))
    if case in ("gas_small_box", "elongated", "tiny_grid"):
        pos = inputs.random_gas(n, box, seed=17, min_dist=0.9).pos
    with Context(n, lanes=1) as ctx:
        x, v = dev(pos), torch.zeros((3, n), dtype=torch.float64, device="cuda")
        ctx.build(x, box, RS, RC)
        ctx.step(x, v, nsteps=20, dt=0.005, P=10, seed=9, rebuild_every=10)
    xo, vo, _, _ = oracle.md_run(pos, np.zeros_like(pos), box, RS, RC, SKIN, 0.005, 20, p=10, seed=9, K=10)
    assert rel_l2(host(x), xo) < 1e-12
    assert rel_l2(host(v), vo) < 1e-9
