"""Random-batch list (RBL) short-range force path for LJ molecular dynamics on
AMD Instinct MI355X (gfx950), after Liang, Xu & Zhao (arXiv:2105.04884).

The compute path is librbl.so (hand-written HIP kernels behind a C-ABI,
``include/rbl.h``).  This module marshals arguments only: PyTorch supplies
device memory (``tensor.data_ptr()``) and the HIP stream.

    ctx = Context(n, lists=("core", "shell"))
    ctx.build(pos, box, r_s=1.5, r_c=3.5)          # pos: cuda float64 (3, n)
    f = ctx.forces(P=10, seed=1, step=0, pos=pos)   # RBL force, eqs. (3)+(4)
    ctx.step(pos, vel, nsteps=100, dt=0.005, P=10, seed=1)
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (KIND_BIN, KIND_BUILD, KIND_FORCE_FULL, KIND_FORCE_RBL, KIND_INTEGRATE,
                   KIND_PREDRAW, KIND_REDUCE, MAX_P, RBL_W_SKIN, STATUS_NAMES, LibraryMissing)

__all__ = ["Context", "RblError", "SkinWarning", "MAX_P", "LibraryMissing", "version"]


class RblError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class SkinWarning(UserWarning):
    pass


def _check(status: int):
    if status < 0:
        msg = _lib.load().rbl_last_error().decode(errors="replace")
        raise RblError(status, msg)
    return status


def version() -> str:
    return _lib.load().rbl_version().decode()


def _torch():
    import torch
    return torch


def _dev_ptr(t, shape=None, name="tensor"):
    """Device pointer of a contiguous float64 CUDA tensor."""
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def _i64(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _i32(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class Context:
    """One RBL context: owns the cell-sorted state and neighbour lists of
    ``n`` particles (one system, or ``replica_offsets`` for an ensemble)."""

    def __init__(self, n: int, *, precision: str = "fp64", lists=("core", "shell"),
                 skin: float = 0.3, shift: bool = True, momentum_fix: bool = True,
                 predraw: bool = True, graphs: bool = True, lanes: int = 0, persistent: int = 0,
                 capacity_factor: float = 1.25,
                 replica_offsets=None,
                 pair: str = "lj", alpha: float = 0.0, charges=None, shell_source: str = "shell",
                 rebuild_check: bool = False, core_filter="auto", types=None, eps_sig=None,
                 stream=None):
        """``types`` (n ints) and ``eps_sig`` ((n_types, n_types, 2) table of
        epsilon_ab, sigma_ab): particle types with per-pair LJ parameters and
        radii r_s sigma_ab, r_c sigma_ab (rbl_config.n_types)."""
        torch = _torch()
        lib = _lib.load()
        cfg = _lib.Config()
        lib.rbl_config_init(C.byref(cfg), int(n))
        cfg.precision = {"fp64": _lib.PREC_FP64, "mixed": _lib.PREC_MIXED}[precision]
        cfg.pair = {"lj": _lib.PAIR_LJ, "lj_erfc": _lib.PAIR_LJ_ERFC}[pair]
        mask = 0
        for k in lists:
            mask |= {"core": _lib.LIST_CORE, "shell": _lib.LIST_SHELL, "full": _lib.LIST_FULL}[k]
        cfg.lists = mask
        cfg.skin = float(skin)
        cfg.alpha = float(alpha)
        cfg.shift = int(bool(shift))
        cfg.momentum_fix = int(bool(momentum_fix))
        cfg.predraw = int(bool(predraw))
        cfg.graphs = int(bool(graphs))
        cfg.lanes = int(lanes)
        cfg.persistent = int(persistent)
        cfg.capacity_factor = float(capacity_factor)
        cfg.shell_source = {"shell": _lib.SHELL_LIST, "stencil": _lib.SHELL_STENCIL,
                            "paper": _lib.SHELL_PAPER}[shell_source]
        cfg.rebuild_check = int(bool(rebuild_check))
        cfg.core_filter = 2 if core_filter == "auto" else int(bool(core_filter))
        self._offsets = None
        if replica_offsets is not None:
            self._offsets = np.ascontiguousarray(replica_offsets, dtype=np.int64)
            cfg.n_replicas = len(self._offsets) - 1
            cfg.replica_offsets = _i64(self._offsets)
        self._charges = charges
        if charges is not None:
            cfg.charges = _dev_ptr(charges, (n,), "charges").value
        if types is not None or eps_sig is not None:
            if types is None or eps_sig is None:
                raise ValueError("types and eps_sig go together")
            self._types = np.ascontiguousarray(types, dtype=np.int32).reshape(-1)
            self._eps_sig = np.ascontiguousarray(eps_sig, dtype=np.float64)
            if self._types.shape != (int(n),):
                raise ValueError("types needs one entry per particle")
            if (self._eps_sig.ndim != 3 or self._eps_sig.shape[0] != self._eps_sig.shape[1]
                    or self._eps_sig.shape[2] != 2):
                raise ValueError("eps_sig must be shaped (n_types, n_types, 2)")
            cfg.n_types = int(self._eps_sig.shape[0])
            cfg.types = _i32(self._types)
            cfg.pair_coeffs = self._eps_sig.ctypes.data_as(C.POINTER(C.c_double))
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.n = int(n)
        self.n_replicas = int(cfg.n_replicas)
        handle = C.c_void_p()
        _check(lib.rbl_create(C.byref(cfg), C.c_void_p(stream.cuda_stream), C.byref(handle)))
        self._h = handle
        self._lib = lib

    # -- lifecycle --------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.rbl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- the path -----------------------------------------------------------
    def build(self, pos, box, r_s: float, r_c: float):
        box_arr = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(-1))
        if box_arr.size != 3 * self.n_replicas:
            raise ValueError("box needs 3 edges per replica")
        _check(self._lib.rbl_build(self._h, _dev_ptr(pos, (3, self.n), "pos"),
                                   box_arr.ctypes.data_as(C.POINTER(C.c_double)),
                                   float(r_s), float(r_c)))

    def _ev(self, want_ev):
        if not want_ev:
            return None
        torch = _torch()
        return torch.zeros(2 * self.n_replicas, dtype=torch.float64, device="cuda")

    def forces(self, P: int, seed: int, step: int, pos, force=None, want_ev: bool = False):
        torch = _torch()
        if force is None:
            force = torch.empty((3, self.n), dtype=torch.float64, device="cuda")
        ev = self._ev(want_ev)
        _check(self._lib.rbl_forces(self._h, int(P), int(seed), int(step),
                                    _dev_ptr(pos, (3, self.n), "pos"),
                                    _dev_ptr(force, (3, self.n), "force"), _dev_ptr(ev)))
        return (force, ev) if want_ev else force

    def forces_noalloc(self, P: int, seed: int, step: int, pos, force, ev=None):
        """rbl_forces_noalloc: the RBL force into the given ``force`` (and
        ``ev``, 2 doubles per replica, if given) with no device allocation
        (the caller supplies every output)."""
        _check(self._lib.rbl_forces_noalloc(self._h, int(P), int(seed), int(step),
                                            _dev_ptr(pos, (3, self.n), "pos"),
                                            _dev_ptr(force, (3, self.n), "force"),
                                            _dev_ptr(ev, (2 * self.n_replicas,), "ev")))
        return force

    def full_forces(self, pos, force=None, want_ev: bool = False):
        torch = _torch()
        if force is None:
            force = torch.empty((3, self.n), dtype=torch.float64, device="cuda")
        ev = self._ev(want_ev)
        _check(self._lib.rbl_full_forces(self._h, _dev_ptr(pos, (3, self.n), "pos"),
                                         _dev_ptr(force, (3, self.n), "force"), _dev_ptr(ev)))
        return (force, ev) if want_ev else force

    def step(self, pos, vel, nsteps: int, dt: float, P: int = 10, seed: int = 1, step0: int = 0,
             rebuild_every: int = 10, use_full: bool = False, force=None, want_ev: bool = False):
        """Velocity-Verlet run in place on pos/vel.  Returns (status, ev)."""
        ev = self._ev(want_ev)
        st = _check(self._lib.rbl_step(self._h, _dev_ptr(pos, (3, self.n), "pos"),
                                       _dev_ptr(vel, (3, self.n), "vel"),
                                       _dev_ptr(force, (3, self.n), "force"),
                                       int(nsteps), float(dt), int(P), int(seed), int(step0),
                                       int(rebuild_every), int(bool(use_full)), _dev_ptr(ev)))
        return st, ev

    def cont(self, nsteps: int, pos=None, vel=None, force=None, want_ev: bool = False):
        """Continues the last ``step``/``cont`` run for ``nsteps`` steps from
        the state held in the context (rbl_continue); writes the final state
        into whichever of pos, vel, force are given.  Returns (status, ev)."""
        ev = self._ev(want_ev)
        st = _check(self._lib.rbl_continue(self._h, _dev_ptr(pos, (3, self.n), "pos"),
                                           _dev_ptr(vel, (3, self.n), "vel"),
                                           _dev_ptr(force, (3, self.n), "force"),
                                           int(nsteps), _dev_ptr(ev)))
        return st, ev

    def last_run(self):
        """Passes the last run took, its last force-evaluation index, whether
        ``cont`` may follow, its list builds and the step of the last one."""
        a, r = C.c_int32(), C.c_int32()
        e, nb, bs = C.c_int64(), C.c_int64(), C.c_int64()
        _check(self._lib.rbl_last_run(self._h, C.byref(a), C.byref(e), C.byref(r), C.byref(nb), C.byref(bs)))
        return {"attempts": a.value, "end_step": e.value, "resumable": bool(r.value),
                "builds": nb.value, "build_step": bs.value}

    # -- thermostat and observables ----------------------------------------
    def set_thermostat(self, gamma: float, kT=None):
        """Langevin friction ``gamma`` (0: NVE) and bath temperature ``kT``
        (a number or one per replica) for later ``step`` calls."""
        kt = None
        if kT is not None:
            kt = np.ascontiguousarray(np.broadcast_to(np.asarray(kT, dtype=np.float64),
                                                      (self.n_replicas,)))
        _check(self._lib.rbl_set_thermostat(
            self._h, float(gamma), None if kt is None else kt.ctypes.data_as(C.POINTER(C.c_double))))

    def unwrap(self, pos, out=None):
        """Positions without the wraps of the list builds (continuous
        trajectory), as a new tensor or in ``out``."""
        torch = _torch()
        if out is None:
            out = torch.empty((3, self.n), dtype=torch.float64, device="cuda")
        _check(self._lib.rbl_unwrap(self._h, _dev_ptr(pos, (3, self.n), "pos"),
                                    _dev_ptr(out, (3, self.n), "out")))
        return out

    def msd(self, a, b):
        """Per-replica mean of |a_i - b_i|^2 (device tensor)."""
        torch = _torch()
        out = torch.empty(self.n_replicas, dtype=torch.float64, device="cuda")
        _check(self._lib.rbl_msd(self._h, _dev_ptr(a, (3, self.n), "a"), _dev_ptr(b, (3, self.n), "b"),
                                 _dev_ptr(out)))
        return out

    def rdf(self, pos, r_max: float, nbins: int, counts=None):
        """Adds the ordered-pair distance histogram at ``pos`` to ``counts``
        (int64 tensor [n_replicas, nbins] holding the uint64 counts; a zeroed
        one is made if None) and returns it."""
        torch = _torch()
        if counts is None:
            counts = torch.zeros((self.n_replicas, int(nbins)), dtype=torch.int64, device="cuda")
        if (not isinstance(counts, torch.Tensor) or not counts.is_cuda or counts.dtype != torch.int64
                or not counts.is_contiguous() or tuple(counts.shape) != (self.n_replicas, int(nbins))):
            raise ValueError("counts must be a contiguous int64 CUDA tensor [n_replicas, nbins]")
        _check(self._lib.rbl_rdf(self._h, _dev_ptr(pos, (3, self.n), "pos"), float(r_max), int(nbins),
                                 C.c_void_p(counts.data_ptr())))
        return counts

    def thermo(self, ev, vel=None) -> np.ndarray:
        """[n_replicas, 4]: energy per particle and pressure with tail
        corrections (pressure at the bath kT, kinetic temperature, pressure
        at the kinetic temperature); see rbl_thermo."""
        out = np.zeros((self.n_replicas, 4))
        _check(self._lib.rbl_thermo(self._h, _dev_ptr(vel, (3, self.n), "vel"),
                                    _dev_ptr(ev, (2 * self.n_replicas,), "ev"),
                                    out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    # -- parity exports ----------------------------------------------------
    def row_counts(self, rows=None):
        rows_arr = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
        nrows = self.n if rows_arr is None else rows_arr.shape[0]
        counts = np.zeros(3 * nrows, dtype=np.int64)
        _check(self._lib.rbl_row_counts(self._h, nrows,
                                        None if rows_arr is None else _i64(rows_arr), _i64(counts)))
        return counts.reshape(3, nrows)

    def export_lists(self, rows=None, kinds=("core", "shell", "full")):
        rows_arr = (np.arange(self.n, dtype=np.int64) if rows is None
                    else np.ascontiguousarray(rows, dtype=np.int64))
        counts = self.row_counts(rows_arr)
        out = {"rows": rows_arr}
        ptrs = []
        for q, kind in enumerate(("core", "shell", "full")):
            off = np.zeros(rows_arr.shape[0] + 1, dtype=np.int64)
            off[1:] = np.cumsum(counts[q])
            idx = np.zeros(int(off[-1]), dtype=np.int32) if kind in kinds else None
            out[kind + "_off"] = off
            out[kind + "_idx"] = idx
            ptrs += [_i64(off), None if idx is None else _i32(idx)]
        _check(self._lib.rbl_export_lists(self._h, rows_arr.shape[0], _i64(rows_arr), *ptrs))
        return out

    def export_batches(self, P: int, seed: int, step: int, rows):
        rows_arr = np.ascontiguousarray(rows, dtype=np.int64)
        batch = np.zeros((rows_arr.shape[0], P), dtype=np.int32)
        count = np.zeros(rows_arr.shape[0], dtype=np.int32)
        _check(self._lib.rbl_export_batches(self._h, int(P), int(seed), int(step), rows_arr.shape[0],
                                            _i64(rows_arr), _i32(batch), _i32(count)))
        return batch, count

    def export_drawn_batches(self, rows):
        """The batches stored on the device (rbl_export_drawn_batches):
        returns (batch [nsteps][len(rows)][P] of partner IDs, -1 padded;
        count [len(rows)]; first step)."""
        rows_arr = np.ascontiguousarray(rows, dtype=np.int64)
        ns, p = C.c_int32(), C.c_int32()
        s0 = C.c_int64()
        _check(self._lib.rbl_export_drawn_batches(self._h, 0, None, None, None, C.byref(ns), C.byref(p),
                                                  C.byref(s0)))
        batch = np.zeros((ns.value, rows_arr.shape[0], max(p.value, 1)), dtype=np.int32)
        count = np.zeros(rows_arr.shape[0], dtype=np.int32)
        _check(self._lib.rbl_export_drawn_batches(self._h, rows_arr.shape[0], _i64(rows_arr), _i32(batch),
                                                  _i32(count), None, None, None))
        return batch, count, s0.value

    def export_binning(self, with_counts: bool = False):
        ncell = np.zeros(3 * self.n_replicas, dtype=np.int32)
        slot = np.zeros(self.n, dtype=np.int64)
        cnt = None
        if with_counts:
            # total cells over replicas is known only after the build
            ncell_probe = np.zeros(3 * self.n_replicas, dtype=np.int32)
            _check(self._lib.rbl_export_binning(self._h, _i32(ncell_probe), _i64(slot), None))
            total = int(np.prod(ncell_probe.reshape(-1, 3), axis=1).sum())
            cnt = np.zeros(total, dtype=np.int32)
        _check(self._lib.rbl_export_binning(self._h, _i32(ncell), _i64(slot),
                                            None if cnt is None else _i32(cnt)))
        return ncell.reshape(-1, 3), slot, cnt

    # -- control -----------------------------------------------------------
    def sync(self) -> int:
        return _check(self._lib.rbl_sync(self._h))

    def set_profiling(self, on: bool):
        _check(self._lib.rbl_set_profiling(self._h, int(bool(on))))

    def kernel_stats(self, kind: int):
        launches = C.c_int64()
        ms = C.c_double()
        _check(self._lib.rbl_kernel_stats(self._h, int(kind), C.byref(launches), C.byref(ms)))
        return launches.value, ms.value

    def tuning(self):
        a, b = C.c_int32(), C.c_int32()
        us = (C.c_double * 6)()
        _check(self._lib.rbl_tuning(self._h, C.byref(a), C.byref(b), us))
        pr, pf = C.c_int32(), C.c_int32()
        pus = (C.c_double * 4)()
        _check(self._lib.rbl_launch_modes(self._h, C.byref(pr), C.byref(pf), pus))
        return {"lpp_rbl": a.value, "lpp_full": b.value,
                "rbl_us": list(us[0:3]), "full_us": list(us[3:6]),
                "persistent_rbl": pr.value, "persistent_full": pf.value,
                "rbl_grid_vs_persistent_us": list(pus[0:2]),
                "full_grid_vs_persistent_us": list(pus[2:4])}

    def core_filter(self):
        """Whether the last run read filtered core rows, the times of the
        automatic decision (unfiltered, filtered and filtering launch, us)
        and the mean filtered row length at the last filtering."""
        used = C.c_int32()
        us = (C.c_double * 3)()
        kept = C.c_double()
        _check(self._lib.rbl_core_filter(self._h, C.byref(used), us, C.byref(kept)))
        return {"used": bool(used.value), "force_us": list(us), "mean_kept": kept.value}

    def info(self):
        ns = C.c_int64()
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        _check(self._lib.rbl_info(self._h, C.byref(ns), C.byref(a), C.byref(b), C.byref(c)))
        return {"n_slots": ns.value, "cap_core": a.value, "cap_shell": b.value, "cap_full": c.value}
