"""Seeded synthetic Lennard-Jones workloads (initial states only).

This module holds no arithmetic of the random-batch list method itself: it
only lays particles on a lattice, jitters them and draws Maxwell-Boltzmann
velocities, with numpy's own PCG64 generator.  Both the CPU oracle tests and
the GPU path take their inputs from here.

The paper's experiments are synthetic LJ fluids in reduced units
(sigma = epsilon = m = 1) in a periodic cube (Sec. III); the workloads below
follow that recipe at the sizes the benchmark and the parity tests use.

Layout of every returned array: positions and velocities are float64 numpy
arrays of shape (3, N) (structure of arrays: x row, y row, z row), box is a
float64 array (Lx, Ly, Lz).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

_FCC_BASIS = np.array(
    [[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]]
)


@dataclass
class State:
    pos: np.ndarray  # (3, N) float64
    vel: np.ndarray  # (3, N) float64
    box: np.ndarray  # (3,) float64
    charges: Optional[np.ndarray] = None  # (N,) float64, charged systems only
    types: Optional[np.ndarray] = None    # (N,) int32, multi-type systems only

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])


def fcc_sites(n: int, box: np.ndarray) -> np.ndarray:
    """Positions of n particles on an FCC lattice filling ``box``.

    With m = ceil((n/4)^(1/3)) unit cells per edge there are M = 4 m^3 >= n
    sites; particle k takes site floor(k*M/n), so sites are spread evenly
    when n is not of the form 4 m^3.  Sites are offset by a quarter lattice
    constant so that none sits on a box face.
    """
    m = max(1, int(math.ceil((n / 4.0) ** (1.0 / 3.0) - 1e-9)))
    while 4 * m**3 < n:
        m += 1
    sites = 4 * m**3
    k = np.arange(n, dtype=np.int64)
    site = (k * sites) // n
    cell = site // 4
    b = site % 4
    ix = cell % m
    iy = (cell // m) % m
    iz = cell // (m * m)
    frac = np.stack([ix, iy, iz]).astype(np.float64) + _FCC_BASIS[b].T + 0.25
    return frac * (np.asarray(box, dtype=np.float64)[:, None] / m)


def maxwell_boltzmann(rng: np.random.Generator, n: int, temperature: float) -> np.ndarray:
    """Gaussian velocities with zero net momentum, rescaled to exactly T
    with 3N-3 degrees of freedom (unit mass)."""
    v = rng.standard_normal((3, n)) * math.sqrt(temperature)
    if n > 1:
        v -= v.mean(axis=1, keepdims=True)
        ke2 = float(np.sum(v * v))
        dof = 3 * n - 3
        if ke2 > 0:
            v *= math.sqrt(temperature * dof / ke2)
    return v


def lj_fluid(n: int, density: float, temperature: float, seed: int,
             jitter: float = 0.05) -> State:
    """Cubic periodic LJ fluid: FCC lattice + uniform jitter of +-``jitter``
    per component + Maxwell-Boltzmann velocities at ``temperature``."""
    L = (n / density) ** (1.0 / 3.0)
    box = np.array([L, L, L], dtype=np.float64)
    rng = np.random.default_rng(seed)
    pos = fcc_sites(n, box)
    pos += rng.uniform(-jitter, jitter, size=(3, n))
    vel = maxwell_boltzmann(rng, n, temperature)
    return State(np.ascontiguousarray(pos), np.ascontiguousarray(vel), box)


def mixture(n: int, density: float, temperature: float, seed: int, fractions,
            jitter: float = 0.05) -> State:
    """Multi-type LJ fluid: the lattice, jitter and velocities of
    ``lj_fluid``, and each particle of type t with probability
    ``fractions[t]`` (independent draws from a second PCG64 stream)."""
    st = lj_fluid(n, density, temperature, seed, jitter)
    p = np.asarray(fractions, dtype=np.float64)
    rng = np.random.default_rng([seed, 2])
    st.types = rng.choice(p.shape[0], size=n, p=p / p.sum()).astype(np.int32)
    return st


def perfect_fcc(cells: int, density: float) -> State:
    """Perfect FCC crystal of 4*cells^3 particles, no jitter, zero velocity."""
    n = 4 * cells**3
    L = (n / density) ** (1.0 / 3.0)
    box = np.array([L, L, L], dtype=np.float64)
    return State(fcc_sites(n, box), np.zeros((3, n)), box)


def random_gas(n: int, box, seed: int, min_dist: float = 0.0) -> State:
    """Uniformly random positions in ``box`` (optionally rejecting overlaps
    closer than ``min_dist``; meant for small n only)."""
    box = np.asarray(box, dtype=np.float64)
    rng = np.random.default_rng(seed)
    if min_dist <= 0.0:
        pos = rng.uniform(0.0, 1.0, size=(3, n)) * box[:, None]
    else:
        pts = []
        while len(pts) < n:
            p = rng.uniform(0.0, 1.0, size=3) * box
            ok = True
            for q in pts:
                d = p - q
                d -= box * np.rint(d / box)
                if float(d @ d) < min_dist * min_dist:
                    ok = False
                    break
            if ok:
                pts.append(p)
        pos = np.array(pts).T.copy()
    vel = maxwell_boltzmann(rng, n, 1.0)
    return State(np.ascontiguousarray(pos), vel, box)


# ---------------------------------------------------------------------------
# Named workloads (reduced LJ units).

def small_fluid(seed: int = 1) -> State:
    """N = 1000, density 0.8, T = 1.0: the small trajectory-parity case."""
    return lj_fluid(1000, 0.8, 1.0, seed)


def million_fluid(seed: int = 1) -> State:
    """N = 1,000,000, density 0.8442, T = 1.0: the headline throughput case."""
    return lj_fluid(1_000_000, 0.8442, 1.0, seed)


def binary_mixture(n: int = 1_000_000, seed: int = 1) -> State:
    """Binary LJ mixture for the per-type cut-off path: 80% small (type 0)
    and 20% large (type 1) particles on the lattice of a density-0.5 fluid,
    T = 1.0."""
    return mixture(n, 0.5, 1.0, seed, (0.8, 0.2))


def large_fluid(seed: int = 1) -> State:
    """N = 16,777,216, density 0.8, T = 1.2: the large single-system case."""
    return lj_fluid(16_777_216, 0.8, 1.2, seed)


def slab(n: int = 2_000_000, rho_liquid: float = 0.8, rho_vapour: float = 0.02,
         temperature: float = 0.9, seed: int = 1, jitter: float = 0.05) -> State:
    """Charged liquid slab in vapour.  Box (L, L, 3L) with
    L = (n / (rho_liquid + 2 rho_vapour))^(1/3); the liquid (FCC + jitter at
    rho_liquid, round(rho_liquid L^3) particles) fills the middle third
    L <= z < 2L, the rest is vapour, split evenly over the two outer thirds
    (FCC + jitter, about rho_vapour each).  Charges +1 and -1, n/2 of each
    (n odd: one more +1), assigned by a random permutation; Maxwell-Boltzmann
    velocities at ``temperature``."""
    L = (n / (rho_liquid + 2.0 * rho_vapour)) ** (1.0 / 3.0)
    cube = np.array([L, L, L], dtype=np.float64)
    n_l = min(n, int(round(rho_liquid * L**3)))
    n_v = n - n_l
    n_v1 = n_v // 2
    rng = np.random.default_rng(seed)
    parts = []
    for count, z0 in ((n_v1, 0.0), (n_l, L), (n_v - n_v1, 2.0 * L)):
        if count == 0:
            continue
        p = fcc_sites(count, cube)
        p += rng.uniform(-jitter, jitter, size=(3, count))
        p[2] += z0
        parts.append(p)
    pos = np.concatenate(parts, axis=1)
    vel = maxwell_boltzmann(rng, n, temperature)
    order = rng.permutation(n)
    charges = np.where(order < (n + 1) // 2, 1.0, -1.0)
    box = np.array([L, L, 3.0 * L], dtype=np.float64)
    return State(np.ascontiguousarray(pos), np.ascontiguousarray(vel), box, charges)


@dataclass
class Ensemble:
    states: list  # list[State]
    densities: np.ndarray
    temperatures: np.ndarray

    @property
    def sizes(self) -> np.ndarray:
        return np.array([s.n for s in self.states], dtype=np.int64)

    def concat(self):
        """(pos (3, sum N), vel (3, sum N), boxes (R, 3), offsets (R+1,))"""
        pos = np.concatenate([s.pos for s in self.states], axis=1)
        vel = np.concatenate([s.vel for s in self.states], axis=1)
        boxes = np.stack([s.box for s in self.states])
        off = np.zeros(len(self.states) + 1, dtype=np.int64)
        off[1:] = np.cumsum(self.sizes)
        return np.ascontiguousarray(pos), np.ascontiguousarray(vel), boxes, off


def ensemble(replicas: int = 512, n_min: int = 2000, n_max: int = 65536,
             rho=(0.6, 0.9), temp=(0.8, 1.5), seed: int = 1) -> Ensemble:
    """Independent LJ replicas: N log-uniform in [n_min, n_max], density and
    temperature uniform in the given ranges, replica r seeded with r + 1."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, size=(replicas, 3))
    sizes = np.rint(n_min * (n_max / n_min) ** u[:, 0]).astype(np.int64)
    dens = rho[0] + (rho[1] - rho[0]) * u[:, 1]
    temps = temp[0] + (temp[1] - temp[0]) * u[:, 2]
    states = [lj_fluid(int(sizes[r]), float(dens[r]), float(temps[r]), r + 1)
              for r in range(replicas)]
    return Ensemble(states, dens, temps)
