"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import numpy as np
import pytest

import oracle

RS, RC, SKIN = 1.5, 3.5, 0.3
FP64_TOL = 1e-12     # relative L2 force error, FP64 path
MIXED_TOL = 2e-5     # relative L2 force error, FP32-pair / FP64-accumulate path


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(a):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b))) / (nb if nb > 0 else 1.0)


def max_row_err(a, b):
    """max_i |a_i - b_i| / rms_i |b_i| over the particles (columns) of two
    [3][n] force arrays: one bad row shows here even when it hides in the
    relative L2 error of all rows."""
    a, b = np.asarray(a), np.asarray(b)
    d = np.sqrt(((a - b) ** 2).sum(axis=0))
    rms = float(np.sqrt((b ** 2).sum(axis=0).mean()))
    return float(d.max()) / (rms if rms > 0 else 1.0) if d.size else 0.0


def assert_forces_close(got, ref, tol, what=""):
    """Relative L2 error below tol over all rows, and no single row off by
    more than 10 tol relative to the rms force."""
    e = rel_l2(got, ref)
    m = max_row_err(got, ref)
    assert e < tol, f"{what} relative L2 {e:.3e} >= {tol:.1e}"
    assert m < 10 * tol, f"{what} worst row {m:.3e} (relative to the rms force) >= {10 * tol:.1e}"
    return e, m


def assert_lists_equal(gpu, orc, kinds=("core", "shell", "full")):
    for kind in kinds:
        go, gi = gpu[kind + "_off"], gpu[kind + "_idx"]
        oo, oi = getattr(orc, kind + "_off"), getattr(orc, kind + "_idx")
        if not np.array_equal(go, oo):
            bad = np.nonzero(np.diff(go) != np.diff(oo))[0][:5]
            raise AssertionError(f"{kind} row lengths differ at rows {bad}: "
                                 f"gpu {np.diff(go)[bad]} oracle {np.diff(oo)[bad]}")
        if not np.array_equal(gi, oi):
            first = int(np.nonzero(gi != oi)[0][0])
            row = int(np.searchsorted(oo, first, side="right") - 1)
            raise AssertionError(f"{kind} entries differ in row {row}")


def oracle_rbl_total(pos, box, lists, P, seed, step, replica=0, momentum_fix=True, pid=None):
    f, e, w = oracle.rbl_forces(pos, box, RS, RC, lists, P, seed, step, replica=replica, pid=pid)
    if momentum_fix:
        f, _ = oracle.mean_subtract(f)
    return f, float(e.sum()), float(w.sum())
