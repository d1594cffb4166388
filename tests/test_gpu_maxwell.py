"""The HIP field solver (pic_maxwell) against the oracle's Yee update, and
the self-consistent loop {pic_step; pic_maxwell} against the oracle's.

The field update repeats the oracle's operation order without contraction,
so E and B are compared bit for bit, at small sizes and at the benchmark
workloads' grid sizes.  In the closed loop the fields depend on J, which
matches the oracle only to rounding (the order of the float64 atomic
additions), so there the bar is a relative 1e-9 after five cycles, and
Gauss's law (div E - rho constant) is checked on the GPU's own output."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2204_12837_amd import inputs as I
from paper_2204_12837_amd import pic

from _parity import say

pytestmark = pytest.mark.gpu


def _fields(wl, seed):
    rng = np.random.default_rng(seed)
    shp = (3, wl.n[2] if wl.dim == 3 else 1, wl.n[1], wl.n[0])
    return rng.standard_normal(shp), rng.standard_normal(shp), 0.1 * rng.standard_normal(shp)


def _gpu(wl, E, B, J, steps):
    ctx = pic.Context(wl, check=True)
    t = lambda a: torch.from_numpy(a).to("cuda:0").contiguous()
    Eg, Bg, Jg = t(E), t(B), t(J)
    ctx.maxwell(Eg, Bg, Jg, steps)
    torch.cuda.synchronize()
    ctx.close()
    return Eg.cpu().numpy(), Bg.cpu().numpy()


CASES = [
    # dim, n, d, steps
    (2, (24, 20), (0.1, 0.13), 5),
    (2, (300, 7), (0.1, 0.1), 3),           # a row longer than one workgroup, ragged tail
    (3, (12, 10, 8), (0.1, 0.12, 0.09), 5),
    (3, (6, 6, 6), (0.1, 0.1, 0.1), 2),
]


@pytest.mark.parametrize("case", CASES)
def test_yee_bitwise(case):
    dim, n, d, steps = case
    dd = tuple(d) + (0.1,) * (3 - len(d))
    wl = I.custom(dim, n, n, ppc=0, dt=0.9 * I.cfl_dt(dd, dim))
    wl.d = dd
    E, B, J = _fields(wl, 600 + sum(n))
    say(f"case yee {case}")
    Eo, Bo = O.maxwell(wl, E, B, J, steps)
    Eg, Bg = _gpu(wl, E, B, J, steps)
    assert np.array_equal(Eg, Eo), np.abs(Eg - Eo).max()
    assert np.array_equal(Bg, Bo), np.abs(Bg - Bo).max()


@pytest.mark.parametrize("name", ["uniform1024", "expansion3d"])
def test_yee_bitwise_full_grid(name):
    """The benchmark workloads' grids (1024^2 and 256x128x128 cells)."""
    wl = I.workload(name)
    E, B, J = _fields(wl, 610)
    say(f"case yee full grid {name}")
    Eo, Bo = O.maxwell(wl, E, B, J, 2)
    Eg, Bg = _gpu(wl, E, B, J, 2)
    assert np.array_equal(Eg, Eo)
    assert np.array_equal(Bg, Bo)


def test_yee_zero_steps_leave_fields():
    wl = I.custom(2, (16, 16), (8, 8), ppc=0)
    E, B, J = _fields(wl, 620)
    Eg, Bg = _gpu(wl, E, B, J, 0)
    assert np.array_equal(Eg, E) and np.array_equal(Bg, B)


def _div(wl, F):
    out = np.zeros(F.shape[1:])
    for a in range(wl.dim):
        out += (F[a] - np.roll(F[a], 1, axis=2 - a)) / wl.d[a]
    return out


def test_self_consistent_loop_matches_oracle():
    """Five cycles of {one particle step (J), one field step with that J}:
    particles and fields follow the oracle's loop, and Gauss's law holds on
    the GPU's output (div E - rho unchanged)."""
    wl = I.workload("uniform64")
    inp = I.generate(wl)
    cycles = 5
    say("case self-consistent loop uniform64")
    sps = O.species_from(inp)
    for s in sps:
        O.bin(wl, s)
    Eo, Bo = inp.E.copy(), inp.B.copy()
    for _ in range(cycles):
        Jo = O.step(wl, sps, Eo, Bo)
        Eo, Bo = O.maxwell(wl, Eo, Bo, Jo, 1)
    ctx = pic.Context(wl, check=True)
    sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    rho = lambda: sum(O.rho(wl, s.q, s.xs.cpu().numpy(), s.ws.cpu().numpy()) for s in sp)
    gauss0 = _div(wl, E.cpu().numpy()) - rho()
    for _ in range(cycles):
        ctx.step(sp, E, B, J, nsteps=1)
        ctx.maxwell(E, B, J, 1)
    torch.cuda.synchronize()
    ctx.check()
    gauss1 = _div(wl, E.cpu().numpy()) - rho()
    scale = max(np.abs(gauss0).max(), 1.0)
    assert np.abs(gauss1 - gauss0).max() <= 1e-11 * scale
    Eg, Bg = E.cpu().numpy(), B.cpu().numpy()
    assert np.abs(Eg - Eo).max() <= 1e-9 * np.abs(Eo).max()
    assert np.abs(Bg - Bo).max() <= 1e-9 * np.abs(Bo).max()
    assert np.abs(Eg - inp.E).max() > 1e-6  # the fields evolved
    s, o = sp[0], sps[0]
    assert np.array_equal(s.offset.cpu().numpy(), o.off)
    gi, oi = np.argsort(s.ids.cpu().numpy()), np.argsort(o.id)
    assert np.abs(s.xs.cpu().numpy()[:, gi] - o.x[:, oi]).max() <= 1e-9
    assert np.abs(s.us.cpu().numpy()[:, gi] - o.u[:, oi]).max() <= 1e-9 * np.abs(o.u).max()


@pytest.mark.parametrize("case", CASES)
def test_yee_adjoint_bitwise(case):
    """pic_maxwell_adjoint equals the oracle's reverse mode bit for bit (the
    GPU evaluates the transposed formulas through the forward kernels with
    negated coefficients, which is exact)."""
    dim, n, d, steps = case
    dd = tuple(d) + (0.1,) * (3 - len(d))
    wl = I.custom(dim, n, n, ppc=0, dt=0.9 * I.cfl_dt(dd, dim))
    wl.d = dd
    Eb, Bb, Jb0 = _fields(wl, 700 + sum(n))
    say(f"case yee adjoint {case}")
    Eo, Bo, Jo = O.maxwell_adjoint(wl, Eb, Bb, steps, Jb=Jb0)
    ctx = pic.Context(wl, check=True)
    t = lambda a: torch.from_numpy(a).to("cuda:0").contiguous()
    Eg, Bg, Jg = t(Eb), t(Bb), t(Jb0)
    ctx.maxwell_adjoint(Eg, Bg, Jg, steps)
    torch.cuda.synchronize()
    ctx.close()
    assert np.array_equal(Eg.cpu().numpy(), Eo)
    assert np.array_equal(Bg.cpu().numpy(), Bo)
    assert np.array_equal(Jg.cpu().numpy(), Jo)


def test_yee_autograd_gradcheck():
    """torch.autograd.gradcheck of YeeSteps (finite differences of the
    linear map against the hand-written reverse mode) on a small 2D grid."""
    from paper_2204_12837_amd import adjoint as ADJ

    wl = I.custom(2, (6, 6), (6, 6), ppc=0)
    ctx = pic.Context(wl, check=True)
    rng = np.random.default_rng(710)
    shp = (3, 1, 6, 6)
    E, B, J = (torch.from_numpy(rng.standard_normal(shp)).to("cuda:0").requires_grad_(True)
               for _ in range(3))
    say("case yee gradcheck")
    assert torch.autograd.gradcheck(lambda e, b, j: ADJ.YeeSteps.apply(e, b, j, ctx, 3),
                                    (E, B, J), eps=1e-6, atol=1e-8, rtol=1e-6)
    ctx.close()


def _oracle_loop(wl, inp, cycles):
    sps = O.species_from(inp)
    for s in sps:
        O.bin(wl, s)
    Eo, Bo = inp.E.copy(), inp.B.copy()
    for _ in range(cycles):
        Jo = O.step(wl, sps, Eo, Bo)
        Eo, Bo = O.maxwell(wl, Eo, Bo, Jo, 1)
    return sps, Eo, Bo


@pytest.mark.parametrize("mode", [0, 1])
def test_resident_cycle_calls(mode):
    """pic_cycle with PIC_FLAG_RESIDENT: one-step calls that continue in the
    slabs (with the field step of every call), then pic_sync, follow the
    oracle's loop to 1e-9."""
    wl = I.custom(2, (64, 32), (8, 8), ppc=4, seed=950 + mode, sigma=0.2, field_amp=0.05)
    inp = I.generate(wl)
    say(f"case resident cycle mode={mode}")
    cycles = 5
    sps, Eo, Bo = _oracle_loop(wl, inp, cycles)
    ctx = pic.Context(wl, check=True, mode=mode, chunk=512, resident=True)
    sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    for k in (1, 1, 2, 1):
        ctx.cycle(sp, E, B, J, k)
    ctx.sync()
    torch.cuda.synchronize()
    ctx.check()
    Eg, Bg = E.cpu().numpy(), B.cpu().numpy()
    assert np.abs(Eg - Eo).max() <= 1e-9 * np.abs(Eo).max()
    assert np.abs(Bg - Bo).max() <= 1e-9 * np.abs(Bo).max()
    for s, o in zip(sp, sps):
        assert np.array_equal(s.offset.cpu().numpy(), o.off)
        gi, oi = np.argsort(s.ids.cpu().numpy()), np.argsort(o.id)
        assert np.abs(s.xs.cpu().numpy()[:, gi] - o.x[:, oi]).max() <= 1e-9
        assert np.abs(s.us.cpu().numpy()[:, gi] - o.u[:, oi]).max() <= 1e-9 * max(np.abs(o.u).max(), 1e-3)
    ctx.close()


CYCLE_CASES = [
    # workload args, cycles, mode, chunk, graph, capacity_factor
    ((2, (64, 32), (8, 8), 4, 1, 0.2), 6, 0, 0, False, None),
    ((2, (64, 32), (8, 8), 4, 1, 0.2), 6, 1, 512, True, None),
    ((2, (48, 24), (8, 8), 3, 1, 0.2), 4, 0, 0, True, 1.0),    # dense layout, paired graphs
    ((3, (16, 16, 8), (8, 8, 8), 2, 2, 0.2), 4, 1, 256, False, None),
]


@pytest.mark.parametrize("case", CYCLE_CASES)
def test_cycle_matches_oracle_loop(case):
    """pic_cycle (particle step + field step per step, inside one call:
    slab layout, persistent mode, captured graphs) follows the oracle's
    loop to 1e-9, and keeps Gauss's law on its own output."""
    (dim, n, patch, ppc, nsp, sigma), cycles, mode, chunk, graph, cap = case
    wl = I.custom(dim, n, patch, ppc=ppc, seed=900 + cycles + mode, sigma=sigma, n_species=nsp,
                  field_amp=0.05)
    inp = I.generate(wl)
    say(f"case cycle {case}")
    sps, Eo, Bo = _oracle_loop(wl, inp, cycles)
    ctx = pic.Context(wl, check=True, mode=mode, chunk=chunk, graph=graph)
    sp = pic.upload(inp, "cuda:0", capacity_factor=cap, n_slabs=ctx.n_slabs)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    rho = lambda: sum(O.rho(wl, s.q, s.xs.cpu().numpy(), s.ws.cpu().numpy()) for s in sp)
    gauss0 = _div(wl, E.cpu().numpy()) - rho()
    ctx.cycle(sp, E, B, J, cycles)
    torch.cuda.synchronize()
    ctx.check()
    gauss1 = _div(wl, E.cpu().numpy()) - rho()
    assert np.abs(gauss1 - gauss0).max() <= 1e-11 * max(np.abs(gauss0).max(), 1.0)
    Eg, Bg = E.cpu().numpy(), B.cpu().numpy()
    assert np.abs(Eg - Eo).max() <= 1e-9 * np.abs(Eo).max()
    assert np.abs(Bg - Bo).max() <= 1e-9 * np.abs(Bo).max()
    for s, o in zip(sp, sps):
        assert np.array_equal(s.offset.cpu().numpy(), o.off)
        gi, oi = np.argsort(s.ids.cpu().numpy()), np.argsort(o.id)
        assert np.abs(s.xs.cpu().numpy()[:, gi] - o.x[:, oi]).max() <= 1e-9
        assert np.abs(s.us.cpu().numpy()[:, gi] - o.u[:, oi]).max() <= 1e-9 * max(np.abs(o.u).max(), 1e-3)
    ctx.close()
