"""Windows of patches that the oracle reproduces exactly from a subset of
the particles (used at sizes where the oracle cannot step every particle).

With the fields given, the particles of a step do not interact, and none
moves faster than light: in k steps a particle crosses fewer than k dt / d
cells of an axis, and the deposit of a step reaches at most three cells from
the particle.  The particles that can end k steps inside a window, or
deposit onto its nodes in the last step, therefore start within
margin_cells(wl, k) cells of it."""
import math

import numpy as np

import oracle as O
from paper_2204_12837_amd import inputs as I


def margin_cells(wl, steps):
    return math.ceil(steps * wl.dt / min(wl.d[:wl.dim])) + 3


def subset(inp, keep):
    """The inputs restricted to the particles keep[s] of each species."""
    sps = [I.ParticleSet(s.q, s.m, s.w, s.x[:, k], s.u[:, k], s.wt[k], s.id[k])
           for s, k in zip(inp.species, keep)]
    return I.Inputs(inp.wl, sps, inp.E, inp.B, inp.W)


def near(x, d, n, a0, length, margin):
    """Particles whose cell lies in [a0 - margin, a0 + length + margin) of a
    periodic axis of n cells."""
    if length + 2 * margin >= n:
        return np.ones(x.shape, dtype=bool)
    c = np.floor(x / d).astype(np.int64)
    return np.mod(c - (a0 - margin), n) < length + 2 * margin


def window_patches(wl, a0, npw):
    """Patch keys (x fastest) of the window of npw[a] patches from cell a0[a]."""
    npa = [wl.n[a] // wl.patch[a] for a in range(3)]
    idx = [np.mod(a0[a] // wl.patch[a] + np.arange(npw[a]), npa[a]) for a in range(3)]
    pz, py, px = np.meshgrid(idx[2], idx[1], idx[0], indexing="ij")
    return (px + npa[0] * (py + npa[1] * pz)).ravel()


def window_nodes(wl, a0, npw):
    """Index arrays (z, y, x) of the window's nodes in a (nz, ny, nx) field."""
    sl = [np.mod(a0[a] + np.arange(npw[a] * wl.patch[a]), wl.n[a]) for a in range(3)]
    return np.ix_(sl[2], sl[1], sl[0])


def oracle_window(wl, inp, steps, a0, npw, margin):
    keep = []
    for s in inp.species:
        k = np.ones(s.id.size, dtype=bool)
        for a in range(wl.dim):
            k &= near(s.x[a], wl.d[a], wl.n[a], a0[a], npw[a] * wl.patch[a], margin)
        keep.append(k)
    sub = subset(inp, keep)
    sps = O.species_from(sub)
    for s in sps:
        O.bin(wl, s)
    J = A = None
    for _ in range(steps):
        J, A = O.step(wl, sps, inp.E, inp.B, with_abs=True)
    return sps, J, A
