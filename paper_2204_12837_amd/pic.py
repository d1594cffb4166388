"""Python binding of the C ABI in include/pic.h (ctypes).

Argument marshalling only: every operation on particles and fields runs in
the HIP kernels of ``libpic.so``.  PyTorch provides device memory and the
stream.  If the library is not built, every entry point raises ``PicError``;
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

(PIC_OK, PIC_ERR_ARG, PIC_ERR_HIP, PIC_ERR_CAPACITY, PIC_ERR_CFL, PIC_ERR_POS, PIC_ERR_STATE,
 PIC_ERR_UNSORTED) = range(8)
STATUS_NAMES = {0: "PIC_OK", 1: "PIC_ERR_ARG", 2: "PIC_ERR_HIP", 3: "PIC_ERR_CAPACITY",
                4: "PIC_ERR_CFL", 5: "PIC_ERR_POS", 6: "PIC_ERR_STATE", 7: "PIC_ERR_UNSORTED"}
BC_PERIODIC, BC_REFLECT, BC_REMOVE = 0, 1, 2
MODE_PER_PATCH, MODE_PERSISTENT = 0, 1
FLAG_CHECK, FLAG_GRAPH, FLAG_TRACE, FLAG_DETERMINISTIC, FLAG_RESIDENT = 1, 2, 4, 8, 16

_DP = C.POINTER(C.c_double)
_I64P = C.POINTER(C.c_int64)


class PicError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ConfigC(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("d", C.c_double * 3), ("dt", C.c_double),
                ("patch", C.c_int32 * 3), ("shape_order", C.c_int32), ("mode", C.c_int32),
                ("chunk", C.c_int32), ("wg_size", C.c_int32), ("flags", C.c_uint32),
                ("bin_x", C.c_int32), ("particle_bc", C.c_int32 * 3)]


class SpeciesC(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double), ("n", C.c_int64), ("capacity", C.c_int64),
                ("x", C.c_void_p * 3), ("u", C.c_void_p * 3), ("w", C.c_void_p), ("id", C.c_void_p),
                ("x_alt", C.c_void_p * 3), ("u_alt", C.c_void_p * 3), ("w_alt", C.c_void_p),
                ("id_alt", C.c_void_p), ("offset", C.c_void_p)]


class FieldsC(C.Structure):
    _fields_ = [("e", C.c_void_p * 3), ("b", C.c_void_p * 3), ("j", C.c_void_p * 3)]


class TraceRecordC(C.Structure):
    _fields_ = [("patch", C.c_int32), ("unit", C.c_int32), ("block", C.c_int32),
                ("species", C.c_int32), ("t0", C.c_uint64), ("t1", C.c_uint64)]


class CotangentC(C.Structure):
    _fields_ = [("x", C.c_void_p * 3), ("u", C.c_void_p * 3), ("n", C.c_int64)]


ENTRY_POINTS = ("pic_validate_config", "pic_num_patches", "pic_bin_width", "pic_init", "pic_free",
                "pic_bin",
                "pic_interp_push", "pic_project", "pic_step", "pic_check", "pic_last_error",
                "pic_timing_enable", "pic_timing_read", "pic_adjoint", "pic_maxwell",
                "pic_maxwell_adjoint", "pic_rho", "pic_cycle", "pic_step_noalloc", "pic_trace_read",
                "pic_sync")
KERNELS = {"zero": 0, "ipp": 1, "rebin": 2, "interp_push": 3, "project": 4, "tag": 5, "sort": 6,
           "adjoint": 7, "exchange": 8, "slab": 9, "maxwell": 10, "rho": 11}

_lib_handle = None


def lib():
    """Load libpic.so (raises PicError if it is not built)."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise PicError(PIC_ERR_STATE, f"{LIB_PATH} is not built "
                           "(python -m paper_2204_12837_amd.build)")
        L = C.CDLL(LIB_PATH)
        L.pic_validate_config.argtypes = [C.POINTER(ConfigC), C.c_char_p, C.c_size_t]
        L.pic_validate_config.restype = C.c_int
        L.pic_num_patches.argtypes = [C.POINTER(ConfigC)]
        L.pic_num_patches.restype = C.c_int64
        L.pic_bin_width.argtypes = [C.POINTER(ConfigC)]
        L.pic_bin_width.restype = C.c_int32
        L.pic_init.argtypes = [C.POINTER(ConfigC), C.c_int32, C.POINTER(C.c_void_p)]
        L.pic_init.restype = C.c_int
        L.pic_free.argtypes = [C.c_void_p]
        L.pic_free.restype = None
        for name in ("pic_bin", "pic_interp_push"):
            getattr(L, name).restype = C.c_int
        L.pic_bin.argtypes = [C.c_void_p, C.POINTER(SpeciesC), C.c_int32, C.c_void_p]
        L.pic_interp_push.argtypes = [C.c_void_p, C.POINTER(SpeciesC), C.c_int32,
                                      C.POINTER(FieldsC), C.c_void_p]
        L.pic_project.argtypes = [C.c_void_p, C.POINTER(SpeciesC), C.c_int32, C.POINTER(FieldsC),
                                  C.c_void_p]
        L.pic_project.restype = C.c_int
        L.pic_step.argtypes = [C.c_void_p, C.POINTER(SpeciesC), C.c_int32, C.POINTER(FieldsC),
                               C.c_int32, C.c_void_p]
        L.pic_step.restype = C.c_int
        L.pic_step_noalloc.argtypes = L.pic_step.argtypes
        L.pic_step_noalloc.restype = C.c_int
        L.pic_check.argtypes = [C.c_void_p, C.c_void_p]
        L.pic_check.restype = C.c_int
        L.pic_sync.argtypes = [C.c_void_p, C.c_void_p]
        L.pic_sync.restype = C.c_int
        L.pic_timing_enable.argtypes = [C.c_void_p, C.c_int32]
        L.pic_timing_enable.restype = C.c_int
        L.pic_timing_read.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                                      C.POINTER(C.c_int64)]
        L.pic_timing_read.restype = C.c_int
        L.pic_adjoint.argtypes = [C.c_void_p, C.POINTER(SpeciesC), C.c_int32, C.POINTER(FieldsC),
                                  C.c_void_p * 3, C.c_int32, C.c_int32, C.POINTER(CotangentC),
                                  C.c_void_p * 3, C.c_void_p * 3, C.c_void_p]
        L.pic_adjoint.restype = C.c_int
        L.pic_maxwell.argtypes = [C.c_void_p, C.c_void_p * 3, C.c_void_p * 3, C.c_void_p * 3,
                                  C.c_int32, C.c_void_p]
        L.pic_maxwell.restype = C.c_int
        L.pic_maxwell_adjoint.argtypes = L.pic_maxwell.argtypes
        L.pic_maxwell_adjoint.restype = C.c_int
        L.pic_rho.argtypes = [C.c_void_p, C.POINTER(SpeciesC), C.c_int32, C.c_void_p, C.c_void_p]
        L.pic_rho.restype = C.c_int
        L.pic_cycle.argtypes = [C.c_void_p, C.POINTER(SpeciesC), C.c_int32, C.c_void_p * 3,
                                C.c_void_p * 3, C.c_void_p * 3, C.c_int32, C.c_void_p]
        L.pic_cycle.restype = C.c_int
        L.pic_trace_read.argtypes = [C.c_void_p, C.POINTER(TraceRecordC), C.c_int64,
                                     C.POINTER(C.c_int64)]
        L.pic_trace_read.restype = C.c_int
        L.pic_last_error.argtypes = [C.c_void_p]
        L.pic_last_error.restype = C.c_char_p
        _lib_handle = L
    return _lib_handle


def make_config(wl, mode=MODE_PER_PATCH, chunk=0, wg_size=0, flags=0, bin_x=0) -> ConfigC:
    """Config struct from a workload description (dim, n, d, dt, patch and,
    if it has one, particle_bc: per-axis particle boundaries, BC_*); bin_x =
    0 lets the library choose the x-bin width."""
    c = ConfigC()
    c.dim = wl.dim
    for a in range(3):
        c.n[a] = int(wl.n[a]) if a < wl.dim else 1
        c.d[a] = float(wl.d[a])
        c.patch[a] = int(wl.patch[a]) if a < wl.dim else 1
    c.dt = float(wl.dt)
    c.shape_order = 2
    c.mode, c.chunk, c.wg_size, c.flags = mode, chunk, wg_size, flags
    c.bin_x = bin_x
    bc = getattr(wl, "particle_bc", (0, 0, 0))
    for a in range(wl.dim):
        c.particle_bc[a] = int(bc[a])
    return c


def validate(cfg: ConfigC):
    buf = C.create_string_buffer(256)
    rc = lib().pic_validate_config(C.byref(cfg), buf, 256)
    return rc, buf.value.decode()


def _ptr(t: Optional[torch.Tensor]):
    return t.data_ptr() if t is not None else None


def slab_capacity(n: int, n_patches: int) -> int:
    """Buffer length with which pic_step keeps every patch's particles in a
    slab with room for arrivals: n + n/8 + 80 per patch."""
    return n + n // 8 + 80 * n_patches


class Species:
    """One species' device arrays: two buffer sets (the sort ping-pongs
    between them; pic_step keeps its per-patch slabs in the second) and the
    patch offsets.  The default capacity is slab_capacity(n, n_patches)."""

    def __init__(self, q: float, m: float, x: torch.Tensor, u: torch.Tensor, w: torch.Tensor,
                 pid: torch.Tensor, n_patches: int, capacity: Optional[int] = None):
        dev = x.device
        n = x.shape[1]
        cap = max(slab_capacity(n, n_patches) if capacity is None else int(capacity), 1)
        self.q, self.m, self.n, self.capacity = float(q), float(m), n, cap
        self.dim = x.shape[0]
        f64 = dict(dtype=torch.float64, device=dev)

        def buf(src, rows):
            t = torch.zeros((rows, cap), **f64) if rows else torch.zeros(cap, **f64)
            if src is not None:
                (t[:, :n] if rows else t[:n]).copy_(src)
            return t

        self.x, self.u, self.w = buf(x, self.dim), buf(u, 3), buf(w, 0)
        self.id = torch.zeros(cap, dtype=torch.int64, device=dev)
        self.id[:n].copy_(pid)
        self.x_alt, self.u_alt, self.w_alt = buf(None, self.dim), buf(None, 3), buf(None, 0)
        self.id_alt = torch.zeros(cap, dtype=torch.int64, device=dev)
        self.offset = torch.zeros(n_patches + 1, dtype=torch.int64, device=dev)

    def cstruct(self) -> SpeciesC:
        s = SpeciesC()
        s.q, s.m, s.n, s.capacity = self.q, self.m, self.n, self.capacity
        for a in range(3):
            s.x[a] = self.x[a].data_ptr() if a < self.dim else None
            s.x_alt[a] = self.x_alt[a].data_ptr() if a < self.dim else None
            s.u[a] = self.u[a].data_ptr()
            s.u_alt[a] = self.u_alt[a].data_ptr()
        s.w, s.w_alt = self.w.data_ptr(), self.w_alt.data_ptr()
        s.id, s.id_alt = self.id.data_ptr(), self.id_alt.data_ptr()
        s.offset = self.offset.data_ptr()
        return s

    def adopt(self, s: SpeciesC):
        """Follow the buffer swap the library made in the struct, and the
        particle count (removing walls delete particles)."""
        self.n = int(s.n)
        if s.w != self.w.data_ptr():
            assert s.w == self.w_alt.data_ptr()
            self.x, self.x_alt = self.x_alt, self.x
            self.u, self.u_alt = self.u_alt, self.u
            self.w, self.w_alt = self.w_alt, self.w
            self.id, self.id_alt = self.id_alt, self.id

    # views of the live particles
    @property
    def xs(self):
        return self.x[:, :self.n]

    @property
    def us(self):
        return self.u[:, :self.n]

    @property
    def ws(self):
        return self.w[:self.n]

    @property
    def ids(self):
        return self.id[:self.n]


class Cotangent:
    """Cotangents of one species' positions and momenta, indexed by particle id."""

    def __init__(self, n_ids: int, dim: int = 2, device="cuda"):
        self.x = torch.zeros((dim, max(n_ids, 1)), dtype=torch.float64, device=device)
        self.u = torch.zeros((3, max(n_ids, 1)), dtype=torch.float64, device=device)
        self.n = n_ids

    def cstruct(self) -> CotangentC:
        c = CotangentC()
        for a in range(3):
            c.x[a] = self.x[a].data_ptr() if a < self.x.shape[0] else None
            c.u[a] = self.u[a].data_ptr()
        c.n = self.n
        return c


def fields_struct(E=None, B=None, J=None) -> FieldsC:
    f = FieldsC()
    for c in range(3):
        f.e[c] = E[c].data_ptr() if E is not None else None
        f.b[c] = B[c].data_ptr() if B is not None else None
        f.j[c] = J[c].data_ptr() if J is not None else None
    return f


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """A library context (pic_init / pic_free) for the workload's grid,
    patches and particle boundaries (wl.particle_bc, BC_* per axis; with
    BC_REMOVE the calls that delete particles update each Species.n).
    resident=True (PIC_FLAG_RESIDENT): step() leaves the particles in the
    slab layout between calls; sync() (or any other call that takes the
    particles) writes the dense layout back before the arrays are read."""

    def __init__(self, wl, device: int = 0, mode=MODE_PER_PATCH, chunk=0, wg_size=0,
                 check=False, graph=False, bin_x=0, trace=False, deterministic=False,
                 resident=False):
        self.wl = wl
        flags = ((FLAG_CHECK if check else 0) | (FLAG_GRAPH if graph else 0)
                 | (FLAG_TRACE if trace else 0) | (FLAG_DETERMINISTIC if deterministic else 0)
                 | (FLAG_RESIDENT if resident else 0))
        self.cfg = make_config(wl, mode, chunk, wg_size, flags, bin_x)
        rc, msg = validate(self.cfg)
        if rc:
            raise PicError(rc, msg)
        self.n_patches = int(lib().pic_num_patches(C.byref(self.cfg)))
        self.bin_width = int(lib().pic_bin_width(C.byref(self.cfg)))
        # slabs of pic_step's slab layout: one per x-bin
        self.n_slabs = self.n_patches * (int(self.cfg.patch[0]) // self.bin_width)
        h = C.c_void_p()
        rc = lib().pic_init(C.byref(self.cfg), device, C.byref(h))
        if rc:
            raise PicError(rc, "pic_init failed")
        self._h = h
        self.device = torch.device("cuda", device)

    def close(self):
        if getattr(self, "_h", None):
            lib().pic_free(self._h)
            self._h = None

    __del__ = close

    def _raise(self, rc):
        if rc:
            raise PicError(rc, lib().pic_last_error(self._h).decode())

    def _call_sp(self, fn, species: Sequence[Species], *args):
        arr = (SpeciesC * len(species))(*[s.cstruct() for s in species])
        rc = fn(self._h, arr, len(species), *args)
        for s, cs in zip(species, arr):
            s.adopt(cs)
        self._raise(rc)

    def bin(self, species: Sequence[Species]):
        self._call_sp(lib().pic_bin, species, _stream())

    def interp_push(self, species: Sequence[Species], E, B):
        f = fields_struct(E, B, None)
        self._call_sp(lib().pic_interp_push, species, C.byref(f), _stream())

    def project(self, species: Sequence[Species], J):
        f = fields_struct(None, None, J)
        self._call_sp(lib().pic_project, species, C.byref(f), _stream())

    def step(self, species: Sequence[Species], E, B, J, nsteps: int = 1):
        f = fields_struct(E, B, J)
        self._call_sp(lib().pic_step, species, C.byref(f), int(nsteps), _stream())

    def step_noalloc(self, species: Sequence[Species], E, B, J, nsteps: int = 1):
        """pic_step_noalloc: pic_step in the dense layout with the library's
        static device scratch (no allocation)."""
        f = fields_struct(E, B, J)
        self._call_sp(lib().pic_step_noalloc, species, C.byref(f), int(nsteps), _stream())

    def check(self):
        self._raise(lib().pic_check(self._h, _stream()))

    def sync(self):
        """pic_sync: the particles that resident steps left in their slabs
        back to the dense layout (first buffer set, offsets)."""
        self._raise(lib().pic_sync(self._h, _stream()))

    def maxwell(self, E, B, J, nsteps: int = 1):
        """pic_maxwell: nsteps Yee updates of E and B (in place) with current J
        (tensors of shape (3, nz, ny, nx), float64, contiguous, on the device)."""
        self._yee(lib().pic_maxwell, E, B, J, nsteps)

    def cycle(self, species: Sequence[Species], E, B, J, nsteps: int = 1):
        """pic_cycle: nsteps of {particle step, field step}; E and B evolve in
        place, J holds the last step's current."""
        for t in (E, B, J):
            if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.device:
                raise PicError(PIC_ERR_ARG, "fields must be contiguous float64 on the device")
        ptr = lambda t: (C.c_void_p * 3)(*[t[c].data_ptr() for c in range(3)])
        self._call_sp(lib().pic_cycle, species, ptr(E), ptr(B), ptr(J), int(nsteps), _stream())

    def rho(self, species: Sequence[Species], rho):
        """pic_rho: rho += charge density of the (patch-sorted) species; rho a
        contiguous float64 tensor of shape (nz, ny, nx) on the device."""
        if rho.dtype != torch.float64 or not rho.is_contiguous() or rho.device != self.device:
            raise PicError(PIC_ERR_ARG, "rho must be contiguous float64 on the device")
        arr = (SpeciesC * len(species))(*[s.cstruct() for s in species])
        self._raise(lib().pic_rho(self._h, arr, len(species), rho.data_ptr(), _stream()))

    def maxwell_adjoint(self, Eb, Bb, Jb, nsteps: int = 1):
        """pic_maxwell_adjoint: cotangents of the fields after nsteps steps ->
        before (in place); the current's cotangent is added to Jb."""
        self._yee(lib().pic_maxwell_adjoint, Eb, Bb, Jb, nsteps)

    def _yee(self, fn, E, B, J, nsteps):
        for t in (E, B, J):
            if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.device:
                raise PicError(PIC_ERR_ARG, "fields must be contiguous float64 on the device")
        ptr = lambda t: (C.c_void_p * 3)(*[t[c].data_ptr() for c in range(3)])
        self._raise(fn(self._h, ptr(E), ptr(B), ptr(J), int(nsteps), _stream()))

    def adjoint(self, ckpt: Sequence["Species"], E, B, Jbar, nsteps: int, with_deposit,
                cot: Sequence["Cotangent"], Ebar, Bbar):
        """pic_adjoint on one segment (see include/pic.h); with_deposit is
        0/False, 1/True or 2."""
        arr = (SpeciesC * len(ckpt))(*[s.cstruct() for s in ckpt])
        f = fields_struct(E, B, None)
        jb = (C.c_void_p * 3)(*[Jbar[c].data_ptr() for c in range(3)]) if Jbar is not None \
            else (C.c_void_p * 3)()
        cs = (CotangentC * len(cot))(*[c.cstruct() for c in cot])
        eb = (C.c_void_p * 3)(*[Ebar[c].data_ptr() for c in range(3)])
        bb = (C.c_void_p * 3)(*[Bbar[c].data_ptr() for c in range(3)])
        rc = lib().pic_adjoint(self._h, arr, len(ckpt), C.byref(f), jb, int(nsteps),
                               int(with_deposit), cs, eb, bb, _stream())
        self._raise(rc)

    def trace_read(self):
        """Records of the last traced fused-kernel launch (PIC_FLAG_TRACE) as
        a list of (patch, unit, block, species, t0, t1) tuples; t0, t1 in
        ticks of the device's 100 MHz clock."""
        n = C.c_int64()
        self._raise(lib().pic_trace_read(self._h, None, 0, C.byref(n)))
        buf = (TraceRecordC * max(n.value, 1))()
        self._raise(lib().pic_trace_read(self._h, buf, n.value, C.byref(n)))
        return [(r.patch, r.unit, r.block, r.species, r.t0, r.t1) for r in buf[:n.value]]

    def timing(self, on: bool = True):
        self._raise(lib().pic_timing_enable(self._h, 1 if on else 0))

    def timing_read(self):
        """{kernel class: (total ms, launches)} since timing was enabled."""
        out = {}
        for name, k in KERNELS.items():
            ms, n = C.c_double(), C.c_int64()
            self._raise(lib().pic_timing_read(self._h, k, C.byref(ms), C.byref(n)))
            out[name] = (ms.value, n.value)
        return out


def upload(inputs, device="cuda", capacity_factor: Optional[float] = None,
           n_slabs: Optional[int] = None) -> List[Species]:
    """Device species from generated inputs (a list of ParticleSet); buffers
    of capacity_factor * n particles, or slab_capacity(n, n_slabs) (n_slabs:
    Context.n_slabs, by default the number of patches)."""
    out = []
    npch = inputs.wl.n_patches
    ns = npch if n_slabs is None else int(n_slabs)
    for s in inputs.species:
        t = lambda a: torch.from_numpy(a).to(device)
        n = s.x.shape[1]
        cap = slab_capacity(n, ns) if capacity_factor is None else int(n * capacity_factor)
        out.append(Species(s.q, s.m, t(s.x), t(s.u), t(s.wt), t(s.id), npch, capacity=cap))
    return out


def upload_fields(inputs, device="cuda"):
    E = torch.from_numpy(inputs.E).to(device).contiguous()
    B = torch.from_numpy(inputs.B).to(device).contiguous()
    J = torch.zeros_like(E)
    return E, B, J
