"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg import this
package; the HIP library and its Python binding never do.  Arrays are numpy
float64 / int64, C-contiguous; the oracle works on host copies.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

from . import build as _build

_DP = C.POINTER(C.c_double)
_I64P = C.POINTER(C.c_int64)


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("d", C.c_double * 3),
                ("dt", C.c_double), ("patch", C.c_int32 * 3), ("bc", C.c_int32 * 3)]


class Species(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double), ("n", C.c_int64), ("x", _DP * 3),
                ("u", _DP * 3), ("w", _DP), ("id", _I64P), ("off", _I64P)]


_libs = {}


def _lib(name: str = "liborc.so"):
    if name not in _libs:
        path = _build.lib_path(name)
        if not os.path.exists(path):
            _build.build(force=False)
        lib = C.CDLL(path)
        lib.orc_shape.argtypes = [C.c_double, C.c_int32, _I64P, _DP]
        lib.orc_interp.argtypes = [C.POINTER(Grid), _DP * 3, _DP * 3, C.c_int64, _DP * 3, _DP * 6]
        lib.orc_boris_traj.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int32, _DP, _DP,
                                       _DP, _DP, C.c_int64, _DP, _DP]
        lib.orc_deposit.argtypes = [C.POINTER(Grid), C.c_double, C.c_double, _DP, _DP, C.c_double,
                                    _DP * 3, C.c_void_p]
        lib.orc_bin.argtypes = [C.POINTER(Grid), C.POINTER(Species)]
        lib.orc_step.argtypes = [C.POINTER(Grid), C.POINTER(Species), C.c_int32, _DP * 3, _DP * 3,
                                 _DP * 3, C.c_void_p]
        lib.orc_rho.argtypes = [C.POINTER(Grid), C.c_double, C.c_int64, _DP * 3, _DP, _DP]
        lib.orc_jvp.argtypes = [C.POINTER(Grid), C.c_double, C.c_double, C.c_int64, _DP * 3,
                                _DP * 3, _DP, _DP * 3, _DP * 3, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_int64, _DP * 3, _DP * 3]
        lib.orc_fd.argtypes = [C.POINTER(Grid), C.c_double, C.c_double, C.c_int64, _DP * 3,
                               _DP * 3, _DP, _DP * 3, _DP * 3, _DP * 3, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_int64, C.c_double, _DP, _DP]
        lib.orc_maxwell.argtypes = [C.POINTER(Grid), _DP * 3, _DP * 3, _DP * 3, C.c_int64]
        lib.orc_maxwell.restype = None
        lib.orc_maxwell_adjoint.argtypes = [C.POINTER(Grid), _DP * 3, _DP * 3, _DP * 3, C.c_int64]
        lib.orc_maxwell_adjoint.restype = None
        lib.orc_real_size.restype = C.c_int32
        _libs[name] = lib
    return _libs[name]


class OracleError(RuntimeError):
    pass


_ERRS = {1: "CFL: a particle moved more than one node", 2: "position outside the periodic box",
         3: "bad argument"}


def _check(rc: int):
    if rc:
        raise OracleError(_ERRS.get(rc, f"error {rc}"))


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


def _arr3(arrs: Sequence[Optional[np.ndarray]]):
    out = (_DP * 3)()
    for k, a in enumerate(arrs):
        out[k] = _p(a) if a is not None else _DP()
    return out


def grid(wl) -> Grid:
    """Grid struct from a workload (anything with dim, n, d, dt, patch)."""
    g = Grid()
    g.dim = wl.dim
    for a in range(3):
        g.n[a] = int(wl.n[a]) if a < wl.dim else 1
        g.d[a] = float(wl.d[a])
        g.patch[a] = int(wl.patch[a]) if a < wl.dim else 1
        g.bc[a] = int(getattr(wl, "particle_bc", (0, 0, 0))[a]) if a < wl.dim else 0
    g.dt = float(wl.dt)
    return g


def shape(xi: float, s: int):
    i = C.c_int64()
    S = (C.c_double * 3)()
    _lib().orc_shape(xi, s, C.byref(i), S)
    return i.value, np.array(S[:])


def interp(wl, E: np.ndarray, B: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Fields (6, n) at positions x (dim, n)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[1]
    out = np.zeros((6, n))
    E = np.ascontiguousarray(E.reshape(3, -1))
    B = np.ascontiguousarray(B.reshape(3, -1))
    outs = (_DP * 6)(*[_p(out[c]) for c in range(6)])
    _lib().orc_interp(C.byref(grid(wl)), _arr3(E), _arr3(B), n,
                      _arr3([x[a] for a in range(x.shape[0])]), outs)
    return out


def boris_traj(q, m, dt, dim, E, B, x0, u0, nsteps, lib="liborc.so"):
    xs = np.zeros((nsteps + 1, 3))
    us = np.zeros((nsteps + 1, 3))
    f = lambda v: np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(3))
    E, B, x0, u0 = f(E), f(B), f(x0), f(u0)
    _lib(lib).orc_boris_traj(q, m, dt, dim, _p(E), _p(B), _p(x0), _p(u0), nsteps, _p(xs), _p(us))
    return xs, us


def deposit(wl, q, w, x0, x1, vz, J: np.ndarray, A: Optional[np.ndarray] = None):
    """J (3, ...) += one particle's Esirkepov deposit."""
    f = lambda v: np.ascontiguousarray(np.asarray(list(v) + [0.0] * (3 - len(v)), dtype=np.float64))
    a0, a1 = f(x0), f(x1)
    Jf = J.reshape(3, -1)
    assert np.shares_memory(Jf, J)
    Ap = None
    if A is not None:
        Af = A.reshape(3, -1)
        assert np.shares_memory(Af, A)
        keep = _arr3(Af)
        Ap = C.cast(C.pointer(keep), C.c_void_p)
    _check(_lib().orc_deposit(C.byref(grid(wl)), q, w, _p(a0), _p(a1), vz, _arr3(Jf), Ap))


class OSpecies:
    """Host particle arrays of one species in the oracle's layout."""

    def __init__(self, q, m, x, u, w, pid, n_patches):
        self.q, self.m = float(q), float(m)
        self.x = np.ascontiguousarray(x, dtype=np.float64).copy()
        self.u = np.ascontiguousarray(u, dtype=np.float64).copy()
        self.w = np.ascontiguousarray(w, dtype=np.float64).copy()
        self.id = np.ascontiguousarray(pid, dtype=np.int64).copy()
        self.off = np.zeros(n_patches + 1, dtype=np.int64)

    @property
    def n(self):
        return self.id.size

    def cstruct(self) -> Species:
        s = Species()
        s.q, s.m, s.n = self.q, self.m, self.n
        for a in range(3):
            s.x[a] = _p(self.x[a]) if a < self.x.shape[0] else _DP()
            s.u[a] = _p(self.u[a])
        s.w = _p(self.w)
        s.id = self.id.ctypes.data_as(_I64P)
        s.off = self.off.ctypes.data_as(_I64P)
        return s

    def follow(self, s: Species):
        """Keep the first s.n particles (the oracle deletes particles at
        removing walls, compacting the survivors to the front)."""
        n = int(s.n)
        if n != self.n:
            self.x = self.x[:, :n].copy()
            self.u = self.u[:, :n].copy()
            self.w = self.w[:n].copy()
            self.id = self.id[:n].copy()


def species_from(inputs) -> List[OSpecies]:
    npch = inputs.wl.n_patches
    return [OSpecies(s.q, s.m, s.x, s.u, s.wt, s.id, npch) for s in inputs.species]


def bin(wl, sp: OSpecies):
    s = sp.cstruct()
    rc = _lib().orc_bin(C.byref(grid(wl)), C.byref(s))
    sp.follow(s)
    _check(rc)


def step(wl, sps: List[OSpecies], E, B, with_abs=False):
    """One step for species already sorted by patch.  Returns J (3, nz, ny, nx)
    and, if asked, A (per-node sum of |contributions|)."""
    shp = E.shape
    J = np.zeros(shp)
    A = np.zeros(shp) if with_abs else None
    arr = (Species * len(sps))(*[s.cstruct() for s in sps])
    Ef = np.ascontiguousarray(E.reshape(3, -1))
    Bf = np.ascontiguousarray(B.reshape(3, -1))
    Jf = J.reshape(3, -1)
    Ap = None
    keep = None
    if with_abs:
        keep = _arr3(A.reshape(3, -1))
        Ap = C.cast(C.pointer(keep), C.c_void_p)
    rc = _lib().orc_step(C.byref(grid(wl)), arr, len(sps), _arr3(Ef), _arr3(Bf), _arr3(Jf), Ap)
    for sp, cs in zip(sps, arr):
        sp.follow(cs)
    _check(rc)
    return (J, A) if with_abs else J


def rho(wl, q, x, w) -> np.ndarray:
    nz = wl.n[2] if wl.dim == 3 else 1
    r = np.zeros((nz, wl.n[1], wl.n[0]))
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    _lib().orc_rho(C.byref(grid(wl)), q, x.shape[1], _arr3([x[a] for a in range(x.shape[0])]),
                   _p(w), _p(r.reshape(-1)))
    return r


def maxwell(wl, E, B, J, nsteps: int = 1, lib="liborc.so"):
    """nsteps Yee updates (Ampere, then Faraday) of copies of E and B with the
    current J; returns the new (E, B), each (3, nz, ny, nx)."""
    E = np.array(E, dtype=np.float64, order="C", copy=True)
    B = np.array(B, dtype=np.float64, order="C", copy=True)
    Jc = np.ascontiguousarray(J, dtype=np.float64)
    Ef, Bf, Jf = E.reshape(3, -1), B.reshape(3, -1), Jc.reshape(3, -1)
    _lib(lib).orc_maxwell(C.byref(grid(wl)), _arr3(Ef), _arr3(Bf), _arr3(Jf), int(nsteps))
    return E, B


def maxwell_adjoint(wl, Eb, Bb, nsteps: int = 1, Jb=None, lib="liborc.so"):
    """Reverse mode of maxwell(): cotangents (Eb, Bb) of the fields after
    nsteps steps -> cotangents of the fields before and of the current
    (added to Jb, zeros if None).  Returns (Eb, Bb, Jb) as new arrays."""
    Eb = np.array(Eb, dtype=np.float64, order="C", copy=True)
    Bb = np.array(Bb, dtype=np.float64, order="C", copy=True)
    Jb = np.zeros_like(Eb) if Jb is None else np.array(Jb, dtype=np.float64, order="C", copy=True)
    _lib(lib).orc_maxwell_adjoint(C.byref(grid(wl)), _arr3(Eb.reshape(3, -1)),
                                  _arr3(Bb.reshape(3, -1)), _arr3(Jb.reshape(3, -1)), int(nsteps))
    return Eb, Bb, Jb


def _opt3(a: Optional[np.ndarray], keep: list):
    if a is None:
        return None
    a = np.ascontiguousarray(a.reshape(3, -1), dtype=np.float64)
    arr = _arr3(a)
    keep.append((a, arr))
    return C.cast(C.pointer(arr), C.c_void_p)


def jvp(wl, q, m, x, u, w, E, B, du=None, dE=None, dB=None, nsteps=None):
    """Forward-mode derivative: returns (J_final, dJ_final) along (du, dE, dB)."""
    nsteps = wl.steps if nsteps is None else nsteps
    shp = E.shape
    J = np.zeros(shp)
    dJ = np.zeros(shp)
    keep: list = []
    x = np.ascontiguousarray(x)
    u = np.ascontiguousarray(u)
    w = np.ascontiguousarray(w)
    Ef = np.ascontiguousarray(E.reshape(3, -1))
    Bf = np.ascontiguousarray(B.reshape(3, -1))
    rc = _lib().orc_jvp(C.byref(grid(wl)), q, m, x.shape[1], _arr3([x[0], x[1]]), _arr3(u), _p(w),
                        _arr3(Ef), _arr3(Bf), _opt3(du, keep), _opt3(dE, keep), _opt3(dB, keep),
                        nsteps, _arr3(J.reshape(3, -1)), _arr3(dJ.reshape(3, -1)))
    _check(rc)
    return J, dJ


def fd(wl, q, m, x, u, w, E, B, W, du=None, dE=None, dB=None, h=1e-6, nsteps=None,
       extended=True, quad=False):
    """Central difference of L = sum W.J_final along (du, dE, dB), computed
    in binary128 (quad=True), x87 long double (extended=True) or double.
    Returns (fd, L0)."""
    nsteps = wl.steps if nsteps is None else nsteps
    keep: list = []
    x = np.ascontiguousarray(x)
    u = np.ascontiguousarray(u)
    w = np.ascontiguousarray(w)
    Ef = np.ascontiguousarray(E.reshape(3, -1))
    Bf = np.ascontiguousarray(B.reshape(3, -1))
    Wf = np.ascontiguousarray(W.reshape(3, -1))
    out, L0 = C.c_double(), C.c_double()
    lib = _lib("liborc_q.so" if quad else "liborc_ld.so" if extended else "liborc.so")
    rc = lib.orc_fd(C.byref(grid(wl)), q, m, x.shape[1], _arr3([x[0], x[1]]), _arr3(u), _p(w),
                    _arr3(Ef), _arr3(Bf), _arr3(Wf), _opt3(du, keep), _opt3(dE, keep),
                    _opt3(dB, keep), nsteps, h, C.byref(out), C.byref(L0))
    _check(rc)
    return out.value, L0.value


def real_size(extended=False, quad=False) -> int:
    return _lib("liborc_q.so" if quad else "liborc_ld.so" if extended else "liborc.so").orc_real_size()
