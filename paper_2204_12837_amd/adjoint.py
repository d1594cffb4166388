"""Gradients of L = <Jbar, J_final> with respect to the initial momenta and
the (static) fields, through the library's hand-written adjoint, with step
checkpointing: the forward keeps the particle state every `every` steps, and
the backward walks the segments from the last to the first, recomputing each
segment from its checkpoint on the GPU (pic_adjoint).

`PicSteps` wraps this as a torch.autograd.Function: J = PicSteps.apply(u0,
E, B, run) with `run` a StepRun holding everything that is not
differentiated (positions, weights, ids, charge, mass, workload, steps).

`PicCycle` differentiates the self-consistent loop (pic_cycle: particle
step, then field step with its current): (J, E_N, B_N) =
PicCycle.apply(u0, E0, B0, run).  The forward keeps the particle state and
the fields before every step; the backward reverses each step as the field
solver's reverse mode (which yields the current's cotangent) followed by
the particle adjoint seeded with that cotangent and with the later state's.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import torch

from . import pic


@dataclasses.dataclass
class StepRun:
    wl: object              # workload description (dim, n, d, dt, patch)
    x0: torch.Tensor        # (2, n) initial positions (device)
    w: torch.Tensor         # (n,) weights
    ids: torch.Tensor       # (n,) int64 ids in [0, n)
    q: float
    m: float
    nsteps: int
    every: int = 5          # checkpoint interval (steps per recomputed segment)
    mode: int = pic.MODE_PER_PATCH
    ctx: Optional[pic.Context] = None


def _clone_live(s: pic.Species) -> pic.Species:
    """A checkpoint: an independent copy of the live particles (buffers of
    exactly n particles: pic_adjoint only reads them)."""
    c = pic.Species(s.q, s.m, s.xs, s.us, s.ws, s.ids, s.offset.numel() - 1, capacity=s.n)
    c.offset.copy_(s.offset)
    return c


def forward(run: StepRun, u0: torch.Tensor, E: torch.Tensor, B: torch.Tensor):
    """nsteps steps from (x0, u0); returns (J_final, checkpoints) where the
    checkpoints are the particle states at steps 0, every, 2*every, ..."""
    ctx = run.ctx or pic.Context(run.wl, mode=run.mode, graph=True)
    run.ctx = ctx
    sp = pic.Species(run.q, run.m, run.x0, u0.detach(), run.w, run.ids,
                     ctx.n_patches)
    J = torch.zeros_like(E)
    ctx.bin([sp])
    ckpts: List[pic.Species] = []
    k = 0
    while k < run.nsteps:
        ckpts.append(_clone_live(sp))
        kk = min(run.every, run.nsteps - k)
        ctx.step([sp], E, B, J, nsteps=kk)
        k += kk
    return J, ckpts


def backward(run: StepRun, ckpts: List[pic.Species], E, B, Jbar):
    """Gradients (du0, dE, dB) of <Jbar, J_final>."""
    ctx = run.ctx
    n = run.ids.numel()
    cot = pic.Cotangent(n, 2, E.device)
    Eb = torch.zeros_like(E)
    Bb = torch.zeros_like(B)
    Jb = Jbar.contiguous()
    starts = list(range(0, run.nsteps, run.every))
    for seg in range(len(starts) - 1, -1, -1):
        k0 = starts[seg]
        kk = min(run.every, run.nsteps - k0)
        ctx.adjoint([ckpts[seg]], E, B, Jb, kk, seg == len(starts) - 1, [cot], Eb, Bb)
    return cot.u[:, run.ids], Eb, Bb


class PicSteps(torch.autograd.Function):
    """J_final = PicSteps.apply(u0, E, B, run); backward gives d/d u0, E, B."""

    @staticmethod
    def forward(fctx, u0, E, B, run: StepRun):
        E = E.detach().contiguous()
        B = B.detach().contiguous()
        J, ckpts = forward(run, u0, E, B)
        fctx.run = run
        fctx.ckpts = ckpts
        fctx.save_for_backward(E, B)
        return J

    @staticmethod
    def backward(fctx, gJ):
        E, B = fctx.saved_tensors
        du, dE, dB = backward(fctx.run, fctx.ckpts, E, B, gJ)
        return du.clone(), dE, dB, None


class YeeSteps(torch.autograd.Function):
    """(E1, B1) = YeeSteps.apply(E, B, J, ctx, nsteps): nsteps field-solver
    steps (pic_maxwell) on copies of E and B, with the current J; the
    backward is the hand-written reverse mode (pic_maxwell_adjoint), which
    returns the cotangents of E, B and J.  The map is linear, so nothing is
    kept but the context."""

    @staticmethod
    def forward(fctx, E, B, J, ctx: pic.Context, nsteps: int):
        E1, B1 = E.detach().clone(), B.detach().clone()
        ctx.maxwell(E1, B1, J.detach().contiguous(), nsteps)
        fctx.lib_ctx, fctx.nsteps = ctx, nsteps
        return E1, B1

    @staticmethod
    def backward(fctx, gE, gB):
        Eb = (gE if gE is not None else torch.zeros_like(gB)).detach().clone().contiguous()
        Bb = (gB if gB is not None else torch.zeros_like(gE)).detach().clone().contiguous()
        Jb = torch.zeros_like(Eb)
        fctx.lib_ctx.maxwell_adjoint(Eb, Bb, Jb, fctx.nsteps)
        return Eb, Bb, Jb, None, None


@dataclasses.dataclass
class CycleRun:
    wl: object              # workload description (dim, n, d, dt, patch)
    x0: torch.Tensor        # (2, n) initial positions (device)
    w: torch.Tensor         # (n,) weights
    ids: torch.Tensor       # (n,) int64 ids in [0, n)
    q: float
    m: float
    nsteps: int
    ctx: Optional[pic.Context] = None


def cycle_forward(run: CycleRun, u0: torch.Tensor, E0: torch.Tensor, B0: torch.Tensor):
    """nsteps steps of {particle step; field step} from (x0, u0, E0, B0).
    Returns (J of the last step, E_N, B_N, states) with the particle state
    and the fields before every step."""
    ctx = run.ctx or pic.Context(run.wl)
    run.ctx = ctx
    sp = pic.Species(run.q, run.m, run.x0, u0.detach(), run.w, run.ids, ctx.n_patches)
    E, B = E0.detach().clone().contiguous(), B0.detach().clone().contiguous()
    J = torch.zeros_like(E)
    ctx.bin([sp])
    states = []
    for _ in range(run.nsteps):
        states.append((_clone_live(sp), E.clone(), B.clone()))
        ctx.cycle([sp], E, B, J, nsteps=1)
    return J, E, B, states


def cycle_backward(run: CycleRun, states, Jbar, Ebar, Bbar):
    """Gradients (du0, dE0, dB0) of <Jbar, J_last> + <Ebar, E_N> + <Bbar, B_N>."""
    ctx = run.ctx
    dev = states[0][1].device
    cot = pic.Cotangent(run.ids.numel(), 2, dev)
    Eb = Ebar.detach().clone().contiguous()
    Bb = Bbar.detach().clone().contiguous()
    for k in range(run.nsteps - 1, -1, -1):
        sp, Ek, Bk = states[k]
        last = k == run.nsteps - 1
        Jb = Jbar.detach().clone().contiguous() if last else torch.zeros_like(Eb)
        # field step k: cotangents of the fields the particle step used, and
        # of the current it deposited
        ctx.maxwell_adjoint(Eb, Bb, Jb, 1)
        # particle step k: seeded by the current's cotangent and (except for
        # the last step) by the cotangents of the state after it
        ctx.adjoint([sp], Ek, Bk, Jb, 1, 1 if last else 2, [cot], Eb, Bb)
    return cot.u[:, run.ids], Eb, Bb


class PicCycle(torch.autograd.Function):
    """(J, E_N, B_N) = PicCycle.apply(u0, E0, B0, run); backward gives the
    gradients with respect to u0, E0 and B0."""

    @staticmethod
    def forward(fctx, u0, E0, B0, run: CycleRun):
        J, E, B, states = cycle_forward(run, u0, E0, B0)
        fctx.run, fctx.states = run, states
        return J, E, B

    @staticmethod
    def backward(fctx, gJ, gE, gB):
        z = fctx.states[0][1]
        gJ = torch.zeros_like(z) if gJ is None else gJ
        gE = torch.zeros_like(z) if gE is None else gE
        gB = torch.zeros_like(z) if gB is None else gB
        du, dE, dB = cycle_backward(fctx.run, fctx.states, gJ, gE, gB)
        return du.clone(), dE, dB, None
