"""Reflecting and removing particle walls: the HIP path against the oracle.

Particles fast enough (thermal spread 0.5) that many of them meet a wall in
a few steps, on every launch path: the slab layout per patch and persistent,
the dense layout, the split Interpolation+Push / Projection path, replayed
graphs, x-bins, 3D with two species, the self-consistent loop; the adjoint
through the mirror against the oracle's tangent; pic_bin's error for a
position outside a reflecting axis and its deletion of one outside a
removing axis; the surviving counts handed back.  The bar is the periodic
one: per-patch counts and sets exact, particles bit for bit, J within 1e-12
of the sum of absolute contributions per node."""
import dataclasses
import math

import numpy as np
import pytest

import oracle as O
from paper_2204_12837_amd import inputs as I

from _parity import compare, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu


def _walls(wl, axes):
    return dataclasses.replace(wl, particle_bc=tuple(int(a in axes) for a in range(3)))


def _mirrors(wl, inp, osp):
    """Particles whose momentum along a walled axis changed sign (with the
    fields this weak, only a wall does that in a few steps)."""
    n = 0
    for s0, s in zip(inp.species, osp):
        o0, o1 = np.argsort(s0.id), np.argsort(s.id)
        for a in range(wl.dim):
            if wl.particle_bc[a] == 1:
                n += int((np.sign(s0.u[a, o0]) != np.sign(s.u[a, o1])).sum())
    return n


def _case(wl, steps, **kw):
    inp = I.generate(wl)
    osp, J, A = run_oracle(wl, inp, steps)
    assert _mirrors(wl, inp, osp) > 20, "the case must exercise the walls"
    say(f"case walls {wl.particle_bc} dim={wl.dim} n={wl.n} steps={steps} {kw}")
    gout, Jg = run_gpu(wl, inp, steps, **kw)
    compare(osp, J, A, gout, Jg)


_W2 = dict(sigma=0.5, field_amp=0.01, bz0=0.5)


@pytest.mark.parametrize("axes", [(0,), (1,), (0, 1)])
def test_walls_slab_per_patch(axes):
    wl = _walls(I.custom(2, (48, 40), (8, 8), ppc=6, seed=501, **_W2), axes)
    _case(wl, 6)


@pytest.mark.parametrize("axes", [(0,), (0, 1)])
def test_walls_slab_persistent(axes):
    wl = _walls(I.custom(2, (48, 40), (8, 8), ppc=6, seed=502, **_W2), axes)
    _case(wl, 6, mode=1, chunk=256, wg_size=256)


def test_walls_dense_layout_and_short_calls():
    wl = _walls(I.custom(2, (40, 32), (8, 8), ppc=5, seed=503, **_W2), (0, 1))
    _case(wl, 5, capacity_factor=1.0, step_sizes=[2, 1, 2])


def test_walls_dense_persistent():
    wl = _walls(I.custom(2, (40, 32), (8, 8), ppc=5, seed=504, **_W2), (0,))
    _case(wl, 4, mode=1, chunk=256, capacity_factor=1.0, step_sizes=[2, 2])


def test_walls_split_path():
    wl = _walls(I.custom(2, (40, 32), (8, 8), ppc=5, seed=505, **_W2), (0, 1))
    _case(wl, 4, split=True)


def test_walls_graph_replay():
    wl = _walls(I.custom(2, (48, 32), (8, 8), ppc=5, seed=506, **_W2), (1,))
    _case(wl, 7, graph=True, step_sizes=[4, 3])


def test_walls_with_x_bins():
    """Patches 32 cells wide cut into x-bins of 8."""
    wl = _walls(I.custom(2, (64, 32), (32, 16), ppc=4, seed=507, **_W2), (0,))
    _case(wl, 5, bin_x=8)


@pytest.mark.parametrize("mode", [0, 1])
def test_walls_3d_two_species(mode):
    wl = _walls(I.custom(3, (24, 16, 16), (8, 8, 8), ppc=2, seed=508, n_species=2, sigma=0.5,
                         field_amp=0.01, bz0=0.5), (0, 2))
    kw = dict(mode=1, chunk=512, wg_size=256) if mode else {}
    _case(wl, 4, **kw)


def test_walls_bin_rejects_a_position_outside_the_box():
    import torch

    from paper_2204_12837_amd import pic

    wl = _walls(I.custom(2, (16, 16), (8, 8), ppc=2, seed=509), (0,))
    inp = I.generate(wl)
    inp.species[0].x[0, 5] = -1e-3  # outside a walled axis: not wrapped
    ctx = pic.Context(wl, device=0, check=True)
    sp = pic.upload(inp, "cuda:0")
    with pytest.raises(pic.PicError) as e:
        ctx.bin(sp)
        torch.cuda.synchronize()
        ctx.check()
    assert e.value.status == pic.PIC_ERR_POS
    ctx.close()
    # on the periodic axis the same offset wraps
    inp = I.generate(wl)
    inp.species[0].x[1, 5] = -1e-3
    ctx = pic.Context(wl, device=0, check=True)
    sp = pic.upload(inp, "cuda:0")
    ctx.bin(sp)
    torch.cuda.synchronize()
    ctx.check()
    ctx.close()


def test_walls_adjoint_matches_oracle_jvp():
    """Reverse mode through the mirror: <grad, d> equals the oracle's
    tangent (which the CPU pins tie to extended-precision differences)."""
    import torch

    from paper_2204_12837_amd import adjoint as ADJ

    wl = _walls(I.custom(2, (32, 32), (8, 8), ppc=4, seed=510, sigma=0.5, bz0=1.0, steps=7),
                (0, 1))
    inp = I.generate(wl, with_W=True)
    s = inp.species[0]
    x = s.x.copy()
    dev = "cuda:0"
    run = ADJ.StepRun(wl, torch.from_numpy(x).to(dev), torch.from_numpy(s.wt).to(dev),
                      torch.from_numpy(s.id).to(dev), s.q, s.m, wl.steps, 3)
    u0 = torch.from_numpy(s.u).to(dev).requires_grad_(True)
    E = torch.from_numpy(inp.E).to(dev).requires_grad_(True)
    B = torch.from_numpy(inp.B).to(dev).requires_grad_(True)
    W = torch.from_numpy(inp.W).to(dev)
    say("case walls adjoint")
    J = ADJ.PicSteps.apply(u0, E, B, run)
    (W * J).sum().backward()
    torch.cuda.synchronize()
    run.ctx.check()
    gu, gE, gB = u0.grad.cpu().numpy(), E.grad.cpu().numpy(), B.grad.cpu().numpy()
    rng = np.random.default_rng(511)
    du = rng.normal(size=s.u.shape)
    dE = rng.normal(size=inp.E.shape)
    dB = rng.normal(size=inp.B.shape)
    Jo, dJ = O.jvp(wl, s.q, s.m, x, s.u, s.wt, inp.E, inp.B, du, dE, dB)
    ref = math.fsum((inp.W * dJ).ravel())
    terms = [gu * du, gE * dE, gB * dB]
    got = math.fsum(math.fsum(t.ravel()) for t in terms)
    scale = math.fsum(math.fsum(np.abs(t).ravel()) for t in terms)
    assert abs(got - ref) <= 1e-11 * scale, (got, ref, scale)
    assert np.max(np.abs(J.detach().cpu().numpy() - Jo)) <= 1e-12 * np.abs(Jo).max()
    # the walls matter for this loss: the periodic run's derivative differs
    wp = dataclasses.replace(wl, particle_bc=(0, 0, 0))
    _, dJp = O.jvp(wp, s.q, s.m, x, s.u, s.wt, inp.E, inp.B, du, dE, dB)
    assert abs(math.fsum((inp.W * dJp).ravel()) - ref) > 1e-6 * abs(ref)


# --------------------------------------------------------------------------
# removing walls

def _bcs(wl, bc):
    return dataclasses.replace(wl, particle_bc=tuple(bc) + (0,) * (3 - len(bc)))


def _remove_case(wl, steps, **kw):
    inp = I.generate(wl)
    n0 = [s.id.size for s in inp.species]
    osp, J, A = run_oracle(wl, inp, steps)
    gone = sum(n0) - sum(s.id.size for s in osp)
    assert gone > 20, "the case must delete particles"
    say(f"case remove {wl.particle_bc} dim={wl.dim} n={wl.n} steps={steps} {kw}")
    gout, Jg = run_gpu(wl, inp, steps, **kw)
    compare(osp, J, A, gout, Jg)
    for o, g in zip(osp, gout):
        assert g["id"].size == o.id.size  # the surviving count was handed back


@pytest.mark.parametrize("bc", [(2, 0), (2, 1), (2, 2)])
def test_remove_slab_per_patch(bc):
    wl = _bcs(I.custom(2, (48, 40), (8, 8), ppc=6, seed=521, **_W2), bc)
    _remove_case(wl, 6)


def test_remove_slab_persistent():
    wl = _bcs(I.custom(2, (48, 40), (8, 8), ppc=6, seed=522, **_W2), (1, 2))
    _remove_case(wl, 6, mode=1, chunk=256, wg_size=256)


def test_remove_short_calls_and_graphs():
    """Calls of one and two steps take the slab layout too; graph replays."""
    wl = _bcs(I.custom(2, (40, 32), (8, 8), ppc=5, seed=523, **_W2), (2, 0))
    _remove_case(wl, 6, step_sizes=[1, 2, 3])
    _remove_case(wl, 5, graph=True, step_sizes=[3, 2])


def test_remove_split_path():
    wl = _bcs(I.custom(2, (40, 32), (8, 8), ppc=5, seed=524, **_W2), (2, 1))
    _remove_case(wl, 4, split=True)


def test_remove_with_x_bins():
    wl = _bcs(I.custom(2, (64, 32), (32, 16), ppc=4, seed=525, **_W2), (2, 0))
    _remove_case(wl, 5, bin_x=8)


@pytest.mark.parametrize("mode", [0, 1])
def test_remove_3d_two_species(mode):
    wl = _bcs(I.custom(3, (24, 16, 16), (8, 8, 8), ppc=2, seed=526, n_species=2, sigma=0.5,
                       field_amp=0.01, bz0=0.5), (1, 0, 2))
    kw = dict(mode=1, chunk=512, wg_size=256) if mode else {}
    _remove_case(wl, 4, **kw)


def test_remove_needs_slab_room():
    from paper_2204_12837_amd import pic

    wl = _bcs(I.custom(2, (16, 16), (8, 8), ppc=2, seed=527, steps=2), (2, 0))
    inp = I.generate(wl)
    ctx = pic.Context(wl, device=0, check=True)
    sp = pic.upload(inp, "cuda:0", capacity_factor=1.0)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    with pytest.raises(pic.PicError) as e:
        ctx.step(sp, E, B, J, nsteps=1)
    assert e.value.status == pic.PIC_ERR_CAPACITY
    ctx.close()


@pytest.mark.parametrize("every", [3, 7])
def test_remove_adjoint_matches_oracle_jvp(every):
    """Reverse mode with removing walls: particles deleted inside a segment
    contribute nothing (zero cotangents), the others through every step;
    <grad, d> equals the oracle's tangent, which deletes the same particles
    (checkpoints every 3 steps: deletions inside and across segments)."""
    import torch

    from paper_2204_12837_amd import adjoint as ADJ

    wl = _bcs(I.custom(2, (32, 32), (8, 8), ppc=4, seed=531, sigma=0.5, bz0=1.0, steps=7),
              (2, 1))
    inp = I.generate(wl, with_W=True)
    s = inp.species[0]
    dev = "cuda:0"
    run = ADJ.StepRun(wl, torch.from_numpy(s.x).to(dev), torch.from_numpy(s.wt).to(dev),
                      torch.from_numpy(s.id).to(dev), s.q, s.m, wl.steps, every)
    u0 = torch.from_numpy(s.u).to(dev).requires_grad_(True)
    E = torch.from_numpy(inp.E).to(dev).requires_grad_(True)
    B = torch.from_numpy(inp.B).to(dev).requires_grad_(True)
    W = torch.from_numpy(inp.W).to(dev)
    say(f"case remove adjoint every={every}")
    J = ADJ.PicSteps.apply(u0, E, B, run)
    (W * J).sum().backward()
    torch.cuda.synchronize()
    run.ctx.check()
    gu, gE, gB = u0.grad.cpu().numpy(), E.grad.cpu().numpy(), B.grad.cpu().numpy()
    rng = np.random.default_rng(532)
    du = rng.normal(size=s.u.shape)
    dE = rng.normal(size=inp.E.shape)
    dB = rng.normal(size=inp.B.shape)
    Jo, dJ = O.jvp(wl, s.q, s.m, s.x, s.u, s.wt, inp.E, inp.B, du, dE, dB)
    ref = math.fsum((inp.W * dJ).ravel())
    terms = [gu * du, gE * dE, gB * dB]
    got = math.fsum(math.fsum(t.ravel()) for t in terms)
    scale = math.fsum(math.fsum(np.abs(t).ravel()) for t in terms)
    assert abs(got - ref) <= 1e-11 * scale, (got, ref, scale)
    assert np.max(np.abs(J.detach().cpu().numpy() - Jo)) <= 1e-12 * np.abs(Jo).max()
    # deleted particles have exactly zero momentum gradients, and there are many
    osp = O.species_from(inp)
    O.bin(wl, osp[0])
    for _ in range(wl.steps):
        O.step(wl, osp, inp.E, inp.B)
    gone = ~np.isin(s.id, osp[0].id)
    assert gone.sum() > 20
    assert not gu[:, gone].any() and np.abs(gu[:, ~gone]).max() > 0


def test_remove_bin_deletes_positions_outside_the_box():
    import torch

    from paper_2204_12837_amd import pic

    wl = _bcs(I.custom(2, (16, 16), (8, 8), ppc=3, seed=528), (2, 0))
    inp = I.generate(wl)
    s0 = inp.species[0]
    Lx = wl.n[0] * wl.d[0]
    s0.x[0, [4, 9, 17]] = [-1e-9, Lx, Lx + 0.05]
    s0.x[1, 30] -= wl.n[1] * wl.d[1]  # periodic axis: wrapped
    osp = O.species_from(inp)
    O.bin(wl, osp[0])
    assert osp[0].n == s0.id.size - 3
    ctx = pic.Context(wl, device=0, check=True)
    sp = pic.upload(inp, "cuda:0")
    say("case remove bin")
    ctx.bin(sp)
    torch.cuda.synchronize()
    ctx.check()
    assert sp[0].n == osp[0].n
    assert np.array_equal(sp[0].offset.cpu().numpy(), osp[0].off)
    assert np.array_equal(sp[0].ids.cpu().numpy(), osp[0].id)
    assert np.array_equal(sp[0].xs.cpu().numpy(), osp[0].x)
    ctx.close()


def test_remove_in_the_self_consistent_loop():
    """pic_cycle with removing walls along x follows the oracle's loop of
    {step, Yee step}: the same particles survive, fields to 1e-9."""
    import torch

    from paper_2204_12837_amd import pic

    wl = _bcs(I.custom(2, (48, 32), (8, 8), ppc=4, seed=529, sigma=0.4, field_amp=0.05), (2, 0))
    inp = I.generate(wl)
    sps = O.species_from(inp)
    for s in sps:
        O.bin(wl, s)
    Eo, Bo = inp.E.copy(), inp.B.copy()
    for _ in range(5):
        Jo = O.step(wl, sps, Eo, Bo)
        Eo, Bo = O.maxwell(wl, Eo, Bo, Jo, 1)
    assert sps[0].n < inp.species[0].id.size - 20
    ctx = pic.Context(wl, check=True)
    sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    say("case remove cycle")
    ctx.cycle(sp, E, B, J, 5)
    torch.cuda.synchronize()
    ctx.check()
    assert np.abs(E.cpu().numpy() - Eo).max() <= 1e-9 * np.abs(Eo).max()
    assert np.abs(B.cpu().numpy() - Bo).max() <= 1e-9 * np.abs(Bo).max()
    assert sp[0].n == sps[0].n
    assert np.array_equal(sp[0].offset.cpu().numpy(), sps[0].off)
    assert np.array_equal(np.sort(sp[0].ids.cpu().numpy()), np.sort(sps[0].id))
    ctx.close()


def test_remove_every_particle_then_step_again():
    """Every particle flies at 0.98 c towards a removing wall: after enough
    steps none is left (n = 0, every offset 0, as in the oracle), and a
    further call on the empty species runs and deposits nothing."""
    import torch

    from paper_2204_12837_amd import pic

    wl = _bcs(I.custom(2, (16, 16), (8, 8), ppc=3, seed=530), (2, 0))
    inp = I.generate(wl)
    inp.E[:] = 0
    inp.B[:] = 0
    inp.species[0].u[0] = 5.0
    steps = 30  # 16 cells of 0.1 at 0.98 c and dt 0.067: all gone after 25
    osp, J, A = run_oracle(wl, inp, steps)
    assert osp[0].n == 0 and not osp[0].off.any()
    say("case remove everything")
    ctx = pic.Context(wl, check=True)
    sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    E, B, Jg = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    ctx.step(sp, E, B, Jg, nsteps=steps)
    torch.cuda.synchronize()
    ctx.check()
    assert sp[0].n == 0 and not sp[0].offset.cpu().numpy().any()
    ctx.step(sp, E, B, Jg, nsteps=2)
    torch.cuda.synchronize()
    ctx.check()
    assert sp[0].n == 0 and not Jg.cpu().numpy().any()
    ctx.close()
