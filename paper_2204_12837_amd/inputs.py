"""Seeded synthetic workloads for the PIC macro-particle operators.

This module only draws random numbers and lays them out; it holds none of
the method's arithmetic (no shape functions, no push, no deposit).  It is the
one piece of code shared by the CPU oracle's tests and the HIP path, so that
both see the same bytes.

Workload shapes follow the paper's set-ups: a 2D uniform plasma with
regularly loaded cells (section "Basic performance benchmarks", first case),
a density profile varying along x only that loads patches unevenly (the
radiation-pressure slab of the same section and the 3D plasma expansion of
section "Plasma expansion benchmark"), and 3D patches of 8^3 cells with two
species (electrons and cold ions), also from the plasma-expansion set-up.

Units are normalised (c = 1, charges in e, masses in m_e); momenta are
u = p / (m c) in each species' own mass.

Recipe (seed = 1000 + workload number):
  1. positions: cells in x-fastest order, ``ppc(cell)`` particles per cell,
     each coordinate ``(i + U) * d`` with ``U ~ U[0, 1)``; all x draws first,
     then all y draws (then z);
  2. momenta: u_x, u_y, u_z arrays, each ``N(0, sigma^2)`` of the species;
  3. a random permutation of the particle order (a PIC code's particle order
     inside a patch is arbitrary; generation order would put every particle
     of a cell next to each other); ids are the positions after it.  Option
     order="cell_interleaved" then reorders the particles stably by (patch,
     rank of the particle among its cell's, cell inside the patch), so that
     64 consecutive particles of a patch sit in 64 different cells (a layout
     experiment; the default is the random order);
  4. fields Ex, Ey, Ez, Bx, By, Bz: i.i.d. ``U(-A, A)`` per node, then a
     uniform background added to Bz;
  5. W (the adjoint workload's loss weights): ``N(0, 1)`` per node per J
     component.
Species are drawn one after the other in steps 1-3, each with its own child
generator spawned from the workload seed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class SpeciesSpec:
    name: str
    q: float
    m: float
    sigma: float
    # particles per cell as a function of the cell's x index (numpy int array)
    ppc: Callable[[np.ndarray], np.ndarray]
    w: float


@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    n: tuple  # cells per axis (nx, ny, nz); nz = 1 in 2D
    d: tuple  # cell sizes
    dt: float
    patch: tuple  # patch size in cells per axis (pz = 1 in 2D)
    species: List[SpeciesSpec]
    field_amp: float
    bz0: float
    steps: int
    seed: int
    ckpt: int = 0
    # particle boundary per axis: 0 periodic, 1 reflecting walls at 0 and L,
    # 2 removing walls (particles leaving [0, L) are deleted)
    particle_bc: tuple = (0, 0, 0)

    @property
    def n_patches(self) -> int:
        return int(np.prod([self.n[a] // self.patch[a] for a in range(self.dim)]))

    @property
    def n_cells(self) -> int:
        return int(np.prod(self.n[: self.dim]))


def cfl_dt(d: Sequence[float], dim: int, frac: float = 0.95) -> float:
    """Time step as a fraction of the Yee-grid Courant limit (c = 1)."""
    return frac / math.sqrt(sum(1.0 / (d[a] * d[a]) for a in range(dim)))


def _const(k):
    return lambda ix: np.full(ix.shape, k, dtype=np.int64)


def _bump_profile(ix: np.ndarray) -> np.ndarray:
    # empty for x < 1024 cells, then a 4 ppc background plus a Gaussian bump
    # (sigma 64 cells) centred at x = 1536 cells, peaking at 64 ppc
    xc = ix.astype(np.float64) + 0.5
    v = np.rint(4.0 + 60.0 * np.exp(-((xc - 1536.0) ** 2) / (2.0 * 64.0 ** 2)))
    return np.where(ix < 1024, 0, v).astype(np.int64)


def _ramp_profile(nx: int, peak: int):
    def f(ix):
        return np.rint(peak * (ix.astype(np.float64) + 0.5) / nx).astype(np.int64)
    return f


def workload(name: str, **over) -> Workload:
    """The named synthetic workloads.

    uniform64     2D3V, 64x64 cells, 16 ppc e-, sigma 0.01, fields +-0.01 and
                  Bz += 1, 8x8 patches, 10 steps (small parity case)
    uniform1024   2D3V, 1024x1024 cells, 32 ppc e- (33.5M), sigma 0.05,
                  fields +-0.01, 16x16 patches, 100 steps
    imbalanced    2D3V, 2048x512 cells, x-profile (empty half, Gaussian bump
                  to 64 ppc), 16x16 patches: patches hold 0 .. 16k particles
    expansion3d   3D3V, 256x128x128 cells, e- and p+ (m = 1836), each with
                  a linear count ramp 0 -> 8 ppc along x, 8^3 patches
    adjoint256    2D3V, 256x256 cells, 16 ppc e-, 20 steps, checkpoint 5
    """
    d2 = (0.1, 0.1, 0.1)
    dt2 = cfl_dt(d2, 2)
    dt3 = cfl_dt(d2, 3)
    e = lambda sigma, ppc, w: SpeciesSpec("electron", -1.0, 1.0, sigma, ppc, w)
    if name == "uniform64":
        wl = Workload(name, 2, (64, 64, 1), d2, dt2, (8, 8, 1),
                      [e(0.01, _const(16), 1.0 / 16)], 0.01, 1.0, 10, 1001)
    elif name == "uniform1024":
        wl = Workload(name, 2, (1024, 1024, 1), d2, dt2, (16, 16, 1),
                      [e(0.05, _const(32), 1.0 / 32)], 0.01, 0.0, 100, 1002)
    elif name == "imbalanced":
        wl = Workload(name, 2, (2048, 512, 1), d2, dt2, (16, 16, 1),
                      [e(0.05, _bump_profile, 1.0 / 64)], 0.01, 0.0, 100, 1003)
    elif name == "expansion3d":
        wl = Workload(name, 3, (256, 128, 128), d2, dt3, (8, 8, 8),
                      [e(0.02, _ramp_profile(256, 8), 1.0 / 8),
                       SpeciesSpec("proton", 1.0, 1836.0, 0.0, _ramp_profile(256, 8), 1.0 / 8)],
                      0.01, 0.0, 50, 1004)
    elif name == "adjoint256":
        wl = Workload(name, 2, (256, 256, 1), d2, dt2, (16, 16, 1),
                      [e(0.01, _const(16), 1.0 / 16)], 0.01, 1.0, 20, 1005, ckpt=5)
    else:
        raise KeyError(name)
    return dataclasses.replace(wl, **over) if over else wl


def custom(dim, n, patch, ppc, sigma=0.01, field_amp=0.01, bz0=1.0, d=0.1,
           steps=1, seed=7, n_species=1, dt=None) -> Workload:
    """A small workload for parity sweeps (constant ppc)."""
    n = tuple(n) + (1,) * (3 - len(n))
    patch = tuple(patch) + (1,) * (3 - len(patch))
    dd = (d, d, d)
    sp = [SpeciesSpec("electron", -1.0, 1.0, sigma, _const(ppc), 1.0 / max(ppc, 1))]
    if n_species > 1:
        sp.append(SpeciesSpec("proton", 1.0, 1836.0, sigma / 10, _const(ppc), 1.0 / max(ppc, 1)))
    return Workload("custom", dim, n, dd, dt if dt is not None else cfl_dt(dd, dim),
                    patch, sp, field_amp, bz0, steps, seed)


@dataclasses.dataclass
class ParticleSet:
    q: float
    m: float
    w: float
    x: np.ndarray  # (dim, N) float64
    u: np.ndarray  # (3, N) float64
    wt: np.ndarray  # (N,) float64 weights
    id: np.ndarray  # (N,) int64


@dataclasses.dataclass
class Inputs:
    wl: Workload
    species: List[ParticleSet]
    E: np.ndarray  # (3, nz, ny, nx) float64, x fastest
    B: np.ndarray
    W: Optional[np.ndarray]  # (3, nz, ny, nx) float64 or None


def _interleave(wl: Workload, cell: np.ndarray) -> np.ndarray:
    """Stable order of particles (given their generation cells, x fastest) by
    patch, then by their rank among their cell's particles, then by cell
    inside the patch."""
    nx, ny = wl.n[0], wl.n[1]
    cx, rest = cell % nx, cell // nx
    cy, cz = rest % ny, rest // ny
    px, py, pz = wl.patch
    npx, npy = nx // px, ny // py
    patch = (cx // px) + npx * ((cy // py) + npy * (cz // pz))
    local = (cx % px) + px * ((cy % py) + py * (cz % pz))
    key = patch * (px * py * pz) + local
    o = np.argsort(key, kind="stable")
    ks = key[o]
    rank = np.empty_like(key)
    rank[o] = np.arange(key.size) - np.searchsorted(ks, ks, side="left")
    return np.lexsort((local, rank, patch))


def _draw_species(rng: np.random.Generator, wl: Workload, sp: SpeciesSpec,
                  order: str = "random") -> ParticleSet:
    nx, ny, nz = wl.n
    dim = wl.dim
    ix = np.arange(nx)
    ppc_x = sp.ppc(ix)
    ncol = ny * (nz if dim == 3 else 1)
    counts = np.tile(ppc_x, ncol)  # per cell, x fastest
    N = int(counts.sum())
    cell = np.repeat(np.arange(counts.size, dtype=np.int64), counts)
    cx = cell % nx
    rest = cell // nx
    cy = rest % ny
    cz = rest // ny
    idx = [cx, cy, cz]
    x = np.empty((dim, N), dtype=np.float64)
    for a in range(dim):
        U = rng.random(N)
        x[a] = (idx[a].astype(np.float64) + U) * wl.d[a]
    del cx, cy, cz, rest, idx
    u = np.empty((3, N), dtype=np.float64)
    for a in range(3):
        u[a] = rng.normal(0.0, sp.sigma, N) if sp.sigma > 0 else 0.0
    perm = rng.permutation(N)
    if order == "cell_interleaved":
        perm = perm[_interleave(wl, cell[perm])]
    elif order != "random":
        raise ValueError(f"unknown particle order {order!r}")
    del cell
    x = np.ascontiguousarray(x[:, perm])
    u = np.ascontiguousarray(u[:, perm])
    wt = np.full(N, sp.w, dtype=np.float64)
    pid = np.arange(N, dtype=np.int64)
    return ParticleSet(sp.q, sp.m, sp.w, x, u, wt, pid)


def generate(wl: Workload, with_W: Optional[bool] = None, order: str = "random") -> Inputs:
    """Draw one workload's particles, fields and (optionally) loss weights;
    order: "random" or "cell_interleaved" (step 3 of the recipe)."""
    root = np.random.default_rng(wl.seed)
    children = root.spawn(len(wl.species) + 1)
    species = [_draw_species(children[s], wl, sp, order) for s, sp in enumerate(wl.species)]
    frng = children[-1]
    nx, ny, nz = wl.n
    shape = (nz if wl.dim == 3 else 1, ny, nx)
    E = np.empty((3,) + shape)
    B = np.empty((3,) + shape)
    for c in range(3):
        E[c] = frng.uniform(-wl.field_amp, wl.field_amp, shape)
    for c in range(3):
        B[c] = frng.uniform(-wl.field_amp, wl.field_amp, shape)
    B[2] += wl.bz0
    W = None
    if with_W or (with_W is None and wl.ckpt):
        W = frng.normal(0.0, 1.0, (3,) + shape)
    return Inputs(wl, species, E, B, W)
