"""Gradients of L = <Jbar, J_final> with respect to the initial momenta and
the (static) fields, through the library's hand-written adjoint, with step
checkpointing: the forward keeps the particle state every `every` steps, and
the backward walks the segments from the last to the first, recomputing each
segment from its checkpoint on the GPU (pic_adjoint).

`PicSteps` wraps this as a torch.autograd.Function: J = PicSteps.apply(u0,
E, B, run) with `run` a StepRun holding everything that is not
differentiated (positions, weights, ids, charge, mass, workload, steps).
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
