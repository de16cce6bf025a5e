"""ctypes wrapper of the plain FP64 CPU oracle (``oracle/rbl_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product package.

The shared library is compiled by ``oracle/build.py`` (gcc, -O2,
-ffp-contract=off); ``load()`` compiles it on first use when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def _ptr_or_null(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def load():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.library_path()
    if not os.path.exists(path) or _build.stale():
        _build.build()
    lib = C.CDLL(path)
    lib.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    lib.orc_floyd_choices.argtypes = [C.c_int, C.c_int, _u32p, _i32p]
    lib.orc_floyd_choices.restype = C.c_int
    lib.orc_batch_positions.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32,
                                        C.c_int, C.c_int, _i32p]
    lib.orc_batch_positions.restype = C.c_int
    lib.orc_lj.argtypes = [C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.orc_wrap.argtypes = [C.c_int64, _f64p, _f64p]
    lib.orc_cell_grid.argtypes = [_f64p, C.c_double, C.c_double, _i32p]
    lib.orc_sys_new.argtypes = [C.c_int64, _f64p, _f64p, C.c_double, C.c_double, C.c_double]
    lib.orc_sys_new.restype = C.c_void_p
    lib.orc_sys_new_typed.argtypes = [C.c_int64, _f64p, _f64p, C.c_double, C.c_double, C.c_double,
                                      C.c_int, C.c_void_p, C.c_void_p]
    lib.orc_sys_new_typed.restype = C.c_void_p
    lib.orc_sys_stencil.argtypes = [C.c_void_p, C.c_int, _i32p]
    lib.orc_sys_stencil.restype = C.c_int
    lib.orc_lj_typed.argtypes = [C.c_double, C.c_double, C.c_double,
                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.orc_sys_free.argtypes = [C.c_void_p]
    lib.orc_sys_ncells.argtypes = [C.c_void_p]
    lib.orc_sys_ncells.restype = C.c_int64
    lib.orc_sys_info.argtypes = [C.c_void_p, _i32p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.orc_list_counts.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.c_void_p, _i64p]
    lib.orc_list_counts.restype = C.c_int
    lib.orc_list_fill.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p]
    lib.orc_list_fill.restype = C.c_int
    lib.orc_forces_rbl.argtypes = [C.c_int64, _f64p, _f64p, C.c_double, C.c_double, C.c_int,
                                   C.c_int64, C.c_void_p, _i64p, _i32p, _i64p, _i32p,
                                   C.c_int, C.c_uint64, C.c_uint64, C.c_uint32, C.c_void_p,
                                   C.c_void_p, C.c_double, _f64p, _f64p, _f64p,
                                   C.c_int, C.c_void_p, C.c_void_p]
    lib.orc_forces_rbl.restype = C.c_int
    lib.orc_forces_full.argtypes = [C.c_int64, _f64p, _f64p, C.c_double, C.c_int,
                                    C.c_int64, C.c_void_p, _i64p, _i32p, C.c_void_p, C.c_double,
                                    _f64p, _f64p, _f64p, C.c_int, C.c_void_p, C.c_void_p]
    lib.orc_forces_full.restype = C.c_int
    lib.orc_mean_subtract.argtypes = [C.c_int64, _f64p, _f64p]
    lib.orc_stencil_rows.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.orc_stencil_rows.restype = C.c_int
    lib.orc_erfc_pair.argtypes = [C.c_double, C.c_double, C.c_double,
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.orc_md_run.argtypes = [C.c_int64, _f64p, _f64p, _f64p, C.c_double, C.c_double,
                               C.c_double, C.c_double, C.c_int64, C.c_int, C.c_uint64,
                               C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint32,
                               C.c_void_p, C.c_double, C.c_int, C.c_double, C.c_double,
                               C.c_void_p, _f64p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                               C.c_int, C.c_void_p, C.c_void_p]
    lib.orc_paper_stencil_rows.argtypes = [C.c_int64, _f64p, _f64p, C.c_double, C.c_double, C.c_double,
                                           C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p]
    lib.orc_paper_stencil_rows.restype = C.c_int
    lib.orc_md_run.restype = C.c_int
    lib.orc_langevin_noise.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, _f64p]
    lib.orc_rdf.argtypes = [C.c_int64, _f64p, _f64p, C.c_double, C.c_int, C.c_void_p]
    lib.orc_rdf.restype = C.c_int
    lib.orc_tail.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    _lib = lib
    return lib


# ---------------------------------------------------------------------------
# random numbers and the batch draw

def philox4x32_10(counter, key) -> np.ndarray:
    lib = load()
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(np.asarray(counter, dtype=np.uint32),
                          np.asarray(key, dtype=np.uint32), out)
    return out


def floyd_choices(p: int, n: int, choices) -> np.ndarray:
    lib = load()
    out = np.zeros(max(p, 1), dtype=np.int32)
    r = lib.orc_floyd_choices(p, n, np.asarray(choices, dtype=np.uint32), out)
    if r < 0:
        raise ValueError(f"invalid Floyd choices (code {r})")
    return out[:p]


def batch_positions(seed: int, pid: int, step: int, replica: int, p: int, n: int) -> np.ndarray:
    lib = load()
    out = np.zeros(max(p, n, 1), dtype=np.int32)
    cnt = lib.orc_batch_positions(seed, pid, step, replica, p, n, out)
    return out[:cnt].copy()


def lj(r2: float):
    """(fmag, u): force factor multiplying (x_i - x_j) and unshifted energy."""
    lib = load()
    f = C.c_double()
    u = C.c_double()
    lib.orc_lj(float(r2), C.byref(f), C.byref(u))
    return f.value, u.value


def lj_typed(r2: float, eps: float, sig: float):
    """(fmag, u) of the LJ pair with its own epsilon and sigma (unshifted)."""
    lib = load()
    f = C.c_double()
    u = C.c_double()
    lib.orc_lj_typed(float(r2), float(eps), float(sig), C.byref(f), C.byref(u))
    return f.value, u.value


def _types(types, eps_sig, n):
    """(nt, type array, table) for the C calls: nt = 0 without types."""
    if types is None:
        if eps_sig is not None:
            raise ValueError("eps_sig needs types")
        return 0, None, None
    t = np.ascontiguousarray(types, dtype=np.int32)
    es = np.ascontiguousarray(eps_sig, dtype=np.float64)
    if t.shape != (n,):
        raise ValueError("types must have one entry per particle")
    if es.ndim != 3 or es.shape[0] != es.shape[1] or es.shape[2] != 2:
        raise ValueError("eps_sig must be shaped (n_types, n_types, 2)")
    return int(es.shape[0]), t, es


def erfc_pair(r2: float, qq: float, alpha: float):
    """(fmag, u) of the real-space Ewald term qq erfc(alpha r)/r (unshifted)."""
    lib = load()
    f = C.c_double()
    u = C.c_double()
    lib.orc_erfc_pair(float(r2), float(qq), float(alpha), C.byref(f), C.byref(u))
    return f.value, u.value


def wrap(pos: np.ndarray, box) -> np.ndarray:
    lib = load()
    p = np.ascontiguousarray(pos, dtype=np.float64).copy()
    lib.orc_wrap(p.shape[1], p, np.asarray(box, dtype=np.float64))
    return p


def cell_grid(box, rc: float, skin: float) -> np.ndarray:
    lib = load()
    out = np.zeros(3, dtype=np.int32)
    lib.orc_cell_grid(np.asarray(box, dtype=np.float64), rc, skin, out)
    return out


# ---------------------------------------------------------------------------
# neighbour lists

@dataclass
class Lists:
    rows: np.ndarray       # particle IDs of the rows
    core_off: np.ndarray
    core_idx: np.ndarray
    shell_off: np.ndarray
    shell_idx: np.ndarray
    full_off: np.ndarray
    full_idx: np.ndarray

    def row(self, kind: str, k: int) -> np.ndarray:
        off = getattr(self, kind + "_off")
        idx = getattr(self, kind + "_idx")
        return idx[off[k]:off[k + 1]]


class System:
    """Positions at a list build: wrapped copy, canonical cell binning, and
    neighbour lists for any subset of rows."""

    def __init__(self, pos, box, rs: float, rc: float, skin: float, types=None, eps_sig=None):
        """``types`` (one per particle) and ``eps_sig`` ((n_types, n_types, 2)
        table of epsilon_ab, sigma_ab): a system of several particle types,
        pair radii rs sigma_ab and rc sigma_ab, cells sized by the smallest
        cut-off and one stencil per type."""
        lib = load()
        self._lib = lib
        self._h = None
        self.pos = np.ascontiguousarray(pos, dtype=np.float64)
        self.box = np.ascontiguousarray(box, dtype=np.float64)
        self.n = int(self.pos.shape[1])
        self.rs, self.rc, self.skin = float(rs), float(rc), float(skin)
        self.nt, self.types, self.eps_sig = _types(types, eps_sig, self.n)
        h = lib.orc_sys_new_typed(self.n, self.pos, self.box, rs, rc, skin, self.nt,
                                  _ptr_or_null(self.types), _ptr_or_null(self.eps_sig))
        if not h:
            raise ValueError("invalid type table")
        self._h = h

    def type_stencil(self, a: int) -> np.ndarray:
        """Stencil half-widths (3,) of centre type a (typed systems)."""
        out = np.zeros(3, dtype=np.int32)
        if self._lib.orc_sys_stencil(self._h, int(a), out):
            raise ValueError("untyped system or bad type")
        return out

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.orc_sys_free(self._h)
            self._h = None

    def binning(self):
        """(ncell (3,), wrapped positions (3, n), slot_of_id (n,), cell_start)"""
        nc = self._lib.orc_sys_ncells(self._h)
        ncell = np.zeros(3, dtype=np.int32)
        wpos = np.zeros((3, self.n))
        slot = np.zeros(self.n, dtype=np.int64)
        cs = np.zeros(nc + 1, dtype=np.int64)
        self._lib.orc_sys_info(self._h, ncell, wpos.ctypes.data_as(C.c_void_p),
                               slot.ctypes.data_as(C.c_void_p), cs.ctypes.data_as(C.c_void_p))
        return ncell, wpos, slot, cs

    def lists(self, rows=None, method: str = "cells", kinds=("core", "shell", "full")) -> Lists:
        m = {"cells": 0, "brute": 1}[method]
        if rows is None:
            rows_arr = np.arange(self.n, dtype=np.int64)
        else:
            rows_arr = np.ascontiguousarray(rows, dtype=np.int64)
        nrows = rows_arr.shape[0]
        counts = np.zeros(3 * nrows, dtype=np.int64)
        r = self._lib.orc_list_counts(self._h, m, nrows, rows_arr.ctypes.data_as(C.c_void_p), counts)
        if r:
            raise ValueError("bad row index")
        counts = counts.reshape(3, nrows)
        offs, idxs = [], []
        for q, kind in enumerate(("core", "shell", "full")):
            off = np.zeros(nrows + 1, dtype=np.int64)
            off[1:] = np.cumsum(counts[q])
            offs.append(off)
            idxs.append(np.zeros(int(off[-1]), dtype=np.int32) if kind in kinds else None)
        r = self._lib.orc_list_fill(
            self._h, m, nrows, rows_arr.ctypes.data_as(C.c_void_p),
            offs[0].ctypes.data_as(C.c_void_p), _ptr_or_null(idxs[0]),
            offs[1].ctypes.data_as(C.c_void_p), _ptr_or_null(idxs[1]),
            offs[2].ctypes.data_as(C.c_void_p), _ptr_or_null(idxs[2]))
        if r:
            raise RuntimeError(f"orc_list_fill failed ({r})")
        empty = np.zeros(0, dtype=np.int32)
        return Lists(rows_arr, offs[0], idxs[0] if idxs[0] is not None else empty,
                     offs[1], idxs[1] if idxs[1] is not None else empty,
                     offs[2], idxs[2] if idxs[2] is not None else empty)

    def stencil_rows(self, rows=None):
        """(off, idx): for each row all particles of the stencil cells around
        its cell, itself included, in slot order (the paper's draw
        population I, of size N_I)."""
        rows_arr = (np.arange(self.n, dtype=np.int64) if rows is None
                    else np.ascontiguousarray(rows, dtype=np.int64))
        nrows = rows_arr.shape[0]
        cnt = np.zeros(max(nrows, 1), dtype=np.int64)
        rp = rows_arr.ctypes.data_as(C.c_void_p)
        if self._lib.orc_stencil_rows(self._h, nrows, rp, cnt.ctypes.data_as(C.c_void_p), None):
            raise ValueError("bad row index")
        off = np.zeros(nrows + 1, dtype=np.int64)
        off[1:] = np.cumsum(cnt[:nrows])
        idx = np.zeros(int(off[-1]), dtype=np.int32)
        r = self._lib.orc_stencil_rows(self._h, nrows, rp, off.ctypes.data_as(C.c_void_p),
                                       idx.ctypes.data_as(C.c_void_p))
        if r:
            raise RuntimeError(f"orc_stencil_rows failed ({r})")
        return off, idx

    def paper_stencil_rows(self, rows=None):
        """(off, idx, ncell, h): the stencil population on the paper's own
        grid (cells of edge rs + skin, (2h+1)^3 cells around i's cell with
        h = floor((rc + skin)/w) + 1), members in that grid's slot order."""
        lib = self._lib
        rows_arr = (np.arange(self.n, dtype=np.int64) if rows is None
                    else np.ascontiguousarray(rows, dtype=np.int64))
        nrows = rows_arr.shape[0]
        cnt = np.zeros(max(nrows, 1), dtype=np.int64)
        nc = np.zeros(3, dtype=np.int32)
        h = np.zeros(1, dtype=np.int32)
        rp = rows_arr.ctypes.data_as(C.c_void_p)
        args = (self.n, self.pos, self.box, self.rs, self.rc, self.skin, nrows, rp)
        if lib.orc_paper_stencil_rows(*args, cnt.ctypes.data_as(C.c_void_p), None,
                                      nc.ctypes.data_as(C.c_void_p), h.ctypes.data_as(C.c_void_p)):
            raise ValueError("bad row index or stencil too large")
        off = np.zeros(nrows + 1, dtype=np.int64)
        off[1:] = np.cumsum(cnt[:nrows])
        idx = np.zeros(int(off[-1]), dtype=np.int32)
        if lib.orc_paper_stencil_rows(*args, off.ctypes.data_as(C.c_void_p), idx.ctypes.data_as(C.c_void_p),
                                      None, None):
            raise RuntimeError("orc_paper_stencil_rows failed")
        return off, idx, nc, int(h[0])

    def paper_stencil_lists(self, rows=None) -> Lists:
        """Core rows as in lists(), shell rows replaced by the paper-grid
        stencil population."""
        L = self.lists(rows=rows, kinds=("core",))
        off, idx, _, _ = self.paper_stencil_rows(rows)
        return Lists(L.rows, L.core_off, L.core_idx, off, idx, L.full_off, L.full_idx)

    def stencil_lists(self, rows=None) -> Lists:
        """Core rows as in lists(), shell rows replaced by the stencil rows:
        the draw population of the paper's own form of eq. (4)."""
        L = self.lists(rows=rows, kinds=("core",))
        off, idx = self.stencil_rows(rows)
        return Lists(L.rows, L.core_off, L.core_idx, off, idx, L.full_off, L.full_idx)


# ---------------------------------------------------------------------------
# forces and dynamics

def _charges(charges, n):
    if charges is None:
        return None
    q = np.ascontiguousarray(charges, dtype=np.float64)
    if q.shape != (n,):
        raise ValueError("charges must have one entry per particle")
    return q


def rbl_forces(pos, box, rs, rc, lists: Lists, p: int, seed: int, step: int,
               replica: int = 0, shift: bool = True, pid=None, charges=None, alpha: float = 0.0,
               types=None, eps_sig=None):
    """Raw RBL force (before mean subtraction) for the rows of ``lists``.
    With ``charges`` the real-space Ewald term (screening ``alpha``) is added
    to the LJ pair; with ``types``/``eps_sig`` each pair takes its own LJ
    parameters and radii.  Returns (f (3, nrows), e (nrows,), w (nrows,))."""
    lib = load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    nrows = lists.rows.shape[0]
    f = np.zeros((3, nrows))
    e = np.zeros(nrows)
    w = np.zeros(nrows)
    pid_arr = None if pid is None else np.ascontiguousarray(pid, dtype=np.int64)
    q = _charges(charges, pos.shape[1])
    nt, t, es = _types(types, eps_sig, pos.shape[1])
    r = lib.orc_forces_rbl(pos.shape[1], pos, np.asarray(box, dtype=np.float64), rs, rc, int(shift),
                           nrows, lists.rows.ctypes.data_as(C.c_void_p),
                           lists.core_off, lists.core_idx, lists.shell_off, lists.shell_idx,
                           p, seed, step, replica, _ptr_or_null(pid_arr), _ptr_or_null(q), float(alpha),
                           f, e, w, nt, _ptr_or_null(t), _ptr_or_null(es))
    if r:
        raise ValueError(f"orc_forces_rbl failed ({r})")
    return f, e, w


def full_forces(pos, box, rc, lists: Lists, shift: bool = True, charges=None, alpha: float = 0.0,
                types=None, eps_sig=None):
    lib = load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    q = _charges(charges, pos.shape[1])
    nt, t, es = _types(types, eps_sig, pos.shape[1])
    nrows = lists.rows.shape[0]
    f = np.zeros((3, nrows))
    e = np.zeros(nrows)
    w = np.zeros(nrows)
    r = lib.orc_forces_full(pos.shape[1], pos, np.asarray(box, dtype=np.float64), rc, int(shift),
                            nrows, lists.rows.ctypes.data_as(C.c_void_p),
                            lists.full_off, lists.full_idx, _ptr_or_null(q), float(alpha), f, e, w,
                            nt, _ptr_or_null(t), _ptr_or_null(es))
    if r:
        raise ValueError(f"orc_forces_full failed ({r})")
    return f, e, w


def mean_subtract(f: np.ndarray):
    lib = load()
    g = np.ascontiguousarray(f, dtype=np.float64).copy()
    mean = np.zeros(3)
    lib.orc_mean_subtract(g.shape[1], g, mean)
    return g, mean


def md_run(pos, vel, box, rs, rc, skin, dt, nsteps, p=10, seed=1, step0=0, K=10,
           use_full=False, shift=True, momentum_fix=True, replica=0, want_ev=False,
           charges=None, alpha: float = 0.0, shell_source: str = "shell",
           gamma: float = 0.0, kT: float = 1.0, unwrapped=None, check: bool = False,
           builds=None, types=None, eps_sig=None):
    """Run of Algorithm 1: velocity Verlet (NVE) for gamma = 0, Langevin
    (BAOAB, friction gamma, bath temperature kT) otherwise.  Returns (pos,
    vel, force, ev) with ev of shape (nsteps+1, 2) = (U, W) per force
    evaluation or None.  ``unwrapped`` (float64 array shaped like pos,
    updated in place) follows the positions without wrapping.  Lists are
    rebuilt before every evaluation s with s % K == 0, or with ``check``
    when some particle has moved more than skin/2 since the last build or K
    steps have passed; ``builds`` (a list) receives the steps of the
    builds.  ``types``/``eps_sig``: particle types (see System)."""
    lib = load()
    x = np.ascontiguousarray(pos, dtype=np.float64).copy()
    v = np.ascontiguousarray(vel, dtype=np.float64).copy()
    f = np.zeros_like(x)
    ev = np.zeros((nsteps + 1, 2)) if want_ev else None
    q = _charges(charges, x.shape[1])
    nt, t, es = _types(types, eps_sig, x.shape[1])
    if unwrapped is not None:
        if (not isinstance(unwrapped, np.ndarray) or unwrapped.dtype != np.float64
                or unwrapped.shape != x.shape or not unwrapped.flags.c_contiguous):
            raise ValueError("unwrapped must be a contiguous float64 array shaped like pos")
    bsteps = np.zeros(nsteps + 1, dtype=np.int64)
    nb = np.zeros(1, dtype=np.int64)
    r = lib.orc_md_run(x.shape[1], x, v, np.asarray(box, dtype=np.float64), rs, rc, skin, dt,
                       nsteps, p, seed, step0, K, int(use_full), int(shift), int(momentum_fix),
                       replica, _ptr_or_null(q), float(alpha),
                       {"shell": 0, "stencil": 1, "paper": 2}[shell_source], float(gamma), float(kT),
                       _ptr_or_null(unwrapped), f, _ptr_or_null(ev), int(bool(check)),
                       bsteps.ctypes.data_as(C.c_void_p), nb.ctypes.data_as(C.c_void_p),
                       nt, _ptr_or_null(t), _ptr_or_null(es))
    if r:
        raise RuntimeError(f"orc_md_run failed ({r})")
    if builds is not None:
        builds.extend(int(b) for b in bsteps[:int(nb[0])])
    return x, v, f, ev


# ---------------------------------------------------------------------------
# thermostat noise and observables (Sec. III)

def langevin_noise(seed: int, pid: int, step: int, replica: int = 0) -> np.ndarray:
    """The three standard normal numbers of particle pid's Ornstein-Uhlenbeck
    step at force evaluation ``step``."""
    lib = load()
    g = np.zeros(3)
    lib.orc_langevin_noise(seed, pid, step, replica, g)
    return g


def rdf_counts(pos, box, r_max: float, nbins: int) -> np.ndarray:
    """Ordered-pair distance histogram (uint64 per bin of width r_max/nbins)."""
    lib = load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    counts = np.zeros(nbins, dtype=np.uint64)
    r = lib.orc_rdf(pos.shape[1], pos, np.asarray(box, dtype=np.float64), float(r_max), int(nbins),
                    counts.ctypes.data_as(C.c_void_p))
    if r:
        raise ValueError("invalid RDF arguments")
    return counts


def tail(rho: float, rc: float):
    """(energy per particle, pressure) tail corrections beyond rc."""
    lib = load()
    u = C.c_double()
    p = C.c_double()
    lib.orc_tail(float(rho), float(rc), C.byref(u), C.byref(p))
    return u.value, p.value
