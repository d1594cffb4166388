"""The HIP adjoint (reverse mode, hand-written) against the oracle's
forward-mode derivative and extended-precision finite differences.

L = sum W . J_final; gradients with respect to the initial momenta u0 and the
static fields E, B, through torch.autograd (PicSteps) with step
checkpointing."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2204_12837_amd import adjoint as ADJ
from paper_2204_12837_amd import inputs as I

from _parity import say

pytestmark = pytest.mark.gpu


def _setup(wl, inp):
    s = inp.species[0]
    L = np.array([wl.n[0] * wl.d[0], wl.n[1] * wl.d[1]])
    x = np.mod(s.x, L[:, None])
    x = np.where(x >= L[:, None], 0.0, x)
    return s, x


def _gpu_grads(wl, inp, x, every):
    s = inp.species[0]
    dev = "cuda:0"
    run = ADJ.StepRun(wl, torch.from_numpy(x).to(dev), torch.from_numpy(s.wt).to(dev),
                      torch.from_numpy(s.id).to(dev), s.q, s.m, wl.steps, every)
    u0 = torch.from_numpy(s.u).to(dev).requires_grad_(True)
    E = torch.from_numpy(inp.E).to(dev).requires_grad_(True)
    B = torch.from_numpy(inp.B).to(dev).requires_grad_(True)
    W = torch.from_numpy(inp.W).to(dev)
    J = ADJ.PicSteps.apply(u0, E, B, run)
    L = (W * J).sum()
    L.backward()
    torch.cuda.synchronize()
    run.ctx.check()
    return (J.detach().cpu().numpy(), u0.grad.cpu().numpy(), E.grad.cpu().numpy(),
            B.grad.cpu().numpy())


def _dot(g, v):
    return math.fsum((g * v).ravel()), math.fsum(np.abs(g * v).ravel())


@pytest.mark.parametrize("every", [3, 5])
def test_adjoint_matches_oracle_jvp(every):
    wl = I.custom(2, (32, 32), (8, 8), ppc=4, seed=401, sigma=0.05, bz0=1.0, steps=7)
    inp = I.generate(wl, with_W=True)
    s, x = _setup(wl, inp)
    say(f"case adjoint small every={every}")
    J, gu, gE, gB = _gpu_grads(wl, inp, x, every)
    rng = np.random.default_rng(402)
    for kind in ("u", "E", "B", "all"):
        du = rng.normal(size=s.u.shape) if kind in ("u", "all") else None
        dE = rng.normal(size=inp.E.shape) if kind in ("E", "all") else None
        dB = rng.normal(size=inp.B.shape) if kind in ("B", "all") else None
        Jo, dJ = O.jvp(wl, s.q, s.m, x, s.u, s.wt, inp.E, inp.B, du, dE, dB)
        ref = math.fsum((inp.W * dJ).ravel())
        got, scale = 0.0, 0.0
        for g, v in ((gu, du), (gE, dE), (gB, dB)):
            if v is not None:
                a, b = _dot(g, v)
                got += a
                scale += b
        assert abs(got - ref) <= 1e-11 * scale, (kind, got, ref, scale)
    # the forward J is the oracle's
    assert np.max(np.abs(J - Jo)) <= 1e-12 * np.abs(Jo).max()


def test_adjoint_matches_extended_precision_fd():
    """The criterion of the adjoint: central differences (h = 1e-6) of the
    loss computed in x87 extended precision, relative error <= 1e-7."""
    wl = I.custom(2, (64, 64), (16, 16), ppc=8, seed=403, sigma=0.01, bz0=1.0, steps=20)
    inp = I.generate(wl, with_W=True)
    s, x = _setup(wl, inp)
    say("case adjoint fd 64x64 20 steps every 5")
    J, gu, gE, gB = _gpu_grads(wl, inp, x, 5)
    rng = np.random.default_rng(404)
    for kind in ("u", "EB"):
        du = rng.normal(size=s.u.shape) if kind == "u" else None
        dE = rng.normal(size=inp.E.shape) * 0.01 if kind == "EB" else None
        dB = rng.normal(size=inp.B.shape) * 0.01 if kind == "EB" else None
        fd, _ = O.fd(wl, s.q, s.m, x, s.u, s.wt, inp.E, inp.B, inp.W, du, dE, dB, h=1e-6)
        got = 0.0
        for g, v in ((gu, du), (gE, dE), (gB, dB)):
            if v is not None:
                got += _dot(g, v)[0]
        assert abs(got - fd) <= 1e-7 * abs(fd), (kind, got, fd)


def test_adjoint_full_size_sampled():
    """The adjoint workload at full size (256x256 cells, 16 ppc = 1,048,576
    particles, 20 steps, checkpoint every 5): per-particle momentum
    gradients of sampled particles, each from the oracle's derivative of that
    particle alone (particles do not interact), and one direction over all
    momenta and fields from the oracle's forward-mode derivative."""
    wl = I.workload("adjoint256")
    inp = I.generate(wl)
    s, x = _setup(wl, inp)
    say("case adjoint256 full size")
    J, gu, gE, gB = _gpu_grads(wl, inp, x, wl.ckpt)
    rng = np.random.default_rng(405)
    scale = np.abs(gu).max()
    for p in rng.choice(s.u.shape[1], 12, replace=False):
        xs = np.ascontiguousarray(x[:, p:p + 1])
        us = np.ascontiguousarray(s.u[:, p:p + 1])
        ws = np.ascontiguousarray(s.wt[p:p + 1])
        for c in range(3):
            du = np.zeros((3, 1))
            du[c, 0] = 1.0
            _, dJ = O.jvp(wl, s.q, s.m, xs, us, ws, inp.E, inp.B, du, None, None)
            ref = math.fsum((inp.W * dJ).ravel())
            assert abs(gu[c, p] - ref) <= 1e-10 * scale + 1e-11 * abs(ref), (p, c, gu[c, p], ref)
    du = rng.normal(size=s.u.shape)
    dE = rng.normal(size=inp.E.shape) * 0.01
    dB = rng.normal(size=inp.B.shape) * 0.01
    _, dJ = O.jvp(wl, s.q, s.m, x, s.u, s.wt, inp.E, inp.B, du, dE, dB)
    ref = math.fsum((inp.W * dJ).ravel())
    got, sc = 0.0, 0.0
    for g, v in ((gu, du), (gE, dE), (gB, dB)):
        a, b = _dot(g, v)
        got += a
        sc += b
    assert abs(got - ref) <= 1e-11 * sc, (got, ref, sc)


def test_adjoint256_finite_differences():
    """The adjoint's criterion at its workload (256x256 cells, 16 ppc =
    1,048,576 particles, 20 steps, checkpoint every 5): along 4 random unit
    directions in u and 4 in (E, B), and on 32 sampled scalars each of
    dL/du, dL/dE and dL/dB, the GPU gradient equals the oracle's central
    difference of L in binary128 (h = 1e-6) to 1e-7 relative
    (scalars where |FD| > 1e-3 of the largest sampled one), and the oracle's
    forward-mode derivative to rounding.  The oracle's values were written
    by tests/golden/make_adjoint256_fd.py."""
    import json
    import os
    import sys

    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, os.path.join(here, "golden"))
    import make_adjoint256_fd as G

    with open(os.path.join(here, "golden", "adjoint256_fd.json")) as fh:
        gold = json.load(fh)
    wl, inp, x = G.setup()
    assert G.inputs_sha(inp, x) == gold["inputs_sha256"], "the generated inputs changed"
    s = inp.species[0]
    say("case adjoint256 finite differences (directions and sampled scalars)")
    J, gu, gE, gB = _gpu_grads(wl, inp, x, wl.ckpt)
    for d in gold["directions"]:
        if d["kind"] == "u":
            vs = G.unit_direction(d["seed"], [s.u.shape])
            gs = [gu]
        else:
            vs = G.unit_direction(d["seed"], [inp.E.shape, inp.B.shape])
            gs = [gE, gB]
        got = math.fsum(_dot(g, v)[0] for g, v in zip(gs, vs))
        scale = math.fsum(_dot(g, v)[1] for g, v in zip(gs, vs))
        assert abs(got - d["fd"]) <= 1e-7 * abs(d["fd"]), (d, got)
        assert abs(got - d["jvp"]) <= 1e-11 * scale, (d, got, scale)
    grads = {"u": gu, "E": gE.reshape(3, -1), "B": gB.reshape(3, -1)}
    for kind, g in grads.items():
        sc = [e for e in gold["scalars"] if e["kind"] == kind]
        assert len(sc) == 32
        top = max(abs(e["fd"]) for e in sc)
        big = np.abs(g).max()
        checked = 0
        for e in sc:
            got = g[e["component"], e["index"]]
            assert abs(got - e["jvp"]) <= 1e-10 * big + 1e-11 * abs(e["jvp"]), (e, got)
            if abs(e["fd"]) > 1e-3 * top:
                assert abs(got - e["fd"]) <= 1e-7 * abs(e["fd"]), (e, got)
                checked += 1
        assert checked >= 24, (kind, checked)


def test_checkpoint_interval_does_not_change_gradients():
    wl = I.custom(2, (32, 32), (8, 8), ppc=4, seed=406, sigma=0.05, bz0=1.0, steps=8)
    inp = I.generate(wl, with_W=True)
    s, x = _setup(wl, inp)
    say("case adjoint checkpoint intervals")
    ref = _gpu_grads(wl, inp, x, 8)
    for every in (1, 2, 3):
        got = _gpu_grads(wl, inp, x, every)
        for a, b in zip(ref[1:], got[1:]):
            assert np.max(np.abs(a - b)) <= 1e-12 * np.abs(a).max()


def test_tiled_adjoint_falls_back_outside_its_tile():
    """The tiled backward kernel keeps every stencil that leaves its patch's
    tile on the global path: with checkpoint offsets that put every particle
    in patch 0, almost all stencils lie outside patch 0's tile, and the
    gradients still equal the ones of the correctly sorted checkpoints."""
    wl = I.custom(2, (48, 48), (8, 8), ppc=3, seed=420, sigma=0.05, bz0=1.0, steps=6)
    inp = I.generate(wl, with_W=True)
    s, x = _setup(wl, inp)
    dev = "cuda:0"
    run = ADJ.StepRun(wl, torch.from_numpy(x).to(dev), torch.from_numpy(s.wt).to(dev),
                      torch.from_numpy(s.id).to(dev), s.q, s.m, wl.steps, 3)
    u0 = torch.from_numpy(s.u).to(dev)
    E = torch.from_numpy(inp.E).to(dev).contiguous()
    B = torch.from_numpy(inp.B).to(dev).contiguous()
    W = torch.from_numpy(inp.W).to(dev).contiguous()
    J, ckpts = ADJ.forward(run, u0, E, B)
    say("case tiled adjoint fallback")
    du, dE, dB = ADJ.backward(run, ckpts, E, B, W)
    for c in ckpts:
        c.offset[1:] = c.n  # every particle claimed by patch 0
    du2, dE2, dB2 = ADJ.backward(run, ckpts, E, B, W)
    torch.cuda.synchronize()
    run.ctx.check()
    for a, b in ((du, du2), (dE, dE2), (dB, dB2)):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.max(np.abs(a - b)) <= 1e-12 * max(np.abs(a).max(), 1e-300)


@pytest.mark.parametrize("walls", [None, (1, 1, 0), (2, 1, 0)])
def test_self_consistent_loop_gradient_matches_oracle_fd(walls):
    """Gradient through the self-consistent loop (PicCycle: particle step,
    then field step with its current, 5 times) of
    L = <W, J_last> + <V, E_5> + <U, B_5>: its directional derivative along a
    random (du0, dE0, dB0) equals the central difference of the oracle's own
    loop (h = 1e-5; the difference converges to 1e-9 between h = 1e-4 and
    1e-5 on the periodic case).  Also with reflecting walls on both axes and
    fast particles, so that the gradient passes through many mirrors, and
    with removing walls along x (deleted particles contribute nothing)."""
    import copy
    import dataclasses

    wl = I.custom(2, (32, 32), (8, 8), ppc=4, seed=430, sigma=0.3 if walls else 0.05, bz0=1.0,
                  field_amp=0.05, steps=5)
    if walls:
        wl = dataclasses.replace(wl, particle_bc=walls)
    inp = I.generate(wl, with_W=True)
    rng = np.random.default_rng(431)
    V = rng.standard_normal(inp.E.shape)
    U = rng.standard_normal(inp.B.shape)
    s, x = _setup(wl, inp)
    du = rng.standard_normal(s.u.shape) * 0.01
    dE = rng.standard_normal(inp.E.shape) * 0.01
    dB = rng.standard_normal(inp.B.shape) * 0.01
    say("case self-consistent loop gradient")

    def oracle_loss(t):
        inp2 = copy.deepcopy(inp)
        inp2.species[0].u = s.u + t * du
        E, B = inp.E + t * dE, inp.B + t * dB
        sps = O.species_from(inp2)
        for sp in sps:
            O.bin(wl, sp)
        J = None
        for _ in range(wl.steps):
            J = O.step(wl, sps, E, B)
            E, B = O.maxwell(wl, E, B, J, 1)
        return (inp.W * J).sum() + (V * E).sum() + (U * B).sum()

    if walls:  # the walls are met: momenta mirrored, particles deleted
        sps = O.species_from(inp)
        O.bin(wl, sps[0])
        E, B = inp.E, inp.B
        for _ in range(wl.steps):
            E, B = O.maxwell(wl, E, B, O.step(wl, sps, E, B), 1)
        if 2 in walls:
            assert s.id.size - sps[0].n > 20
        else:
            o0, o1 = np.argsort(s.id), np.argsort(sps[0].id)
            flips = (np.sign(s.u[:2, o0]) != np.sign(sps[0].u[:2, o1])).sum()
            assert flips > 50, flips
    h = 1e-5
    fd = (oracle_loss(h) - oracle_loss(-h)) / (2 * h)
    dev = "cuda:0"
    run = ADJ.CycleRun(wl, torch.from_numpy(x).to(dev), torch.from_numpy(s.wt).to(dev),
                       torch.from_numpy(s.id).to(dev), s.q, s.m, wl.steps)
    u0 = torch.from_numpy(s.u).to(dev).requires_grad_(True)
    E0 = torch.from_numpy(inp.E).to(dev).contiguous().requires_grad_(True)
    B0 = torch.from_numpy(inp.B).to(dev).contiguous().requires_grad_(True)
    J, E, B = ADJ.PicCycle.apply(u0, E0, B0, run)
    t = lambda a: torch.from_numpy(a).to(dev)
    L = (t(inp.W) * J).sum() + (t(V) * E).sum() + (t(U) * B).sum()
    L.backward()
    torch.cuda.synchronize()
    run.ctx.check()
    g = (math.fsum((u0.grad.cpu().numpy() * du).ravel()) + math.fsum((E0.grad.cpu().numpy() * dE).ravel())
         + math.fsum((B0.grad.cpu().numpy() * dB).ravel()))
    assert abs(g - fd) <= 1e-6 * abs(fd), (g, fd)
    # the forward value matches the oracle's loss at t = 0
    assert abs(L.item() - oracle_loss(0.0)) <= 1e-9 * abs(oracle_loss(0.0))
