"""rbl_forces_noalloc (scratch in a static device array) against rbl_forces
through the C-ABI: bit-identical forces and energy/virial on two calls in a
row, the second with a smaller system, for the shell-row draw (inline), the
stencil population and P > 32 (batches in the scratch array), and the
size limit."""
import numpy as np
import pytest

from paper_2105_04884_amd import Context, RblError, inputs
from paper_2105_04884_amd import _lib

from gpu_util import RC, RS, dev, host, torch_cuda

pytestmark = pytest.mark.gpu


def _pair(torch, ctx, n, pos, P, seed, step, R=1):
    f_ref, ev_ref = ctx.forces(P, seed=seed, step=step, pos=pos, want_ev=True)
    f = torch.full((3, n), np.nan, dtype=torch.float64, device="cuda")
    ev = torch.full((2 * R,), np.nan, dtype=torch.float64, device="cuda")
    ctx.forces_noalloc(P, seed, step, pos, f, ev)
    return (host(f_ref), host(ev_ref)), (host(f), host(ev))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("source,P", [("shell", 10), ("stencil", 10), ("shell", 64)])
def test_noalloc_forces_equal_rbl_forces(source, P, precision):
    torch = torch_cuda()
    big = inputs.small_fluid(seed=1)
    small = inputs.random_gas(300, np.array([9.0, 9.0, 9.0]), seed=2, min_dist=0.9)
    for st, box in ((big, big.box), (small, np.array([9.0, 9.0, 9.0]))):
        x = dev(st.pos)
        with Context(st.n, precision=precision, shell_source=source) as ctx:
            ctx.build(x, box, RS, RC)
            for seed, step in ((3, 0), (5, 17)):
                ref, got = _pair(torch, ctx, st.n, x, P, seed, step)
                assert np.array_equal(ref[0], got[0]), (st.n, seed, step)
                assert np.array_equal(ref[1], got[1]), (st.n, seed, step)


def test_noalloc_leaves_stored_batches_and_state():
    """The context's own buffers are untouched: its stored batches and a
    following rbl_forces give what they gave before."""
    torch = torch_cuda()
    st = inputs.small_fluid(seed=2)
    x = dev(st.pos)
    with Context(st.n, shell_source="stencil") as ctx:
        ctx.build(x, st.box, RS, RC)
        f0 = host(ctx.forces(12, seed=1, step=4, pos=x))
        b0, c0, s0 = ctx.export_drawn_batches(np.arange(st.n))
        f = torch.empty((3, st.n), dtype=torch.float64, device="cuda")
        ctx.forces_noalloc(40, 9, 1, x, f)
        b1, c1, s1 = ctx.export_drawn_batches(np.arange(st.n))
        assert s0 == s1 and np.array_equal(b0, b1) and np.array_equal(c0, c1)
        assert np.array_equal(f0, host(ctx.forces(12, seed=1, step=4, pos=x)))


def test_noalloc_rejects_sizes_beyond_its_array():
    """Stencil draws of P = 128 for 2^17 + slots need more than 64 MiB:
    RBL_E_CAPACITY with the sizes in the message, and nothing is written."""
    torch = torch_cuda()
    st = inputs.lj_fluid(140_000, 0.8, 1.0, seed=3)
    x = dev(st.pos)
    with Context(st.n, shell_source="stencil") as ctx:
        ctx.build(x, st.box, RS, RC)
        f = torch.zeros((3, st.n), dtype=torch.float64, device="cuda")
        with pytest.raises(RblError) as e:
            ctx.forces_noalloc(128, 1, 0, x, f)
        assert e.value.status == _lib.RBL_E_CAPACITY and "bytes" in str(e.value)
        assert float(f.abs().max()) == 0.0
        # within the limit at a small P
        ref = host(ctx.forces(10, seed=1, step=0, pos=x))
        ctx.forces_noalloc(10, 1, 0, x, f)
        assert np.array_equal(ref, host(f))
