"""pic_step_noalloc (the entry point that allocates nothing: its scratch is a
static device array) against pic_step in the dense layout, through the C
ABI, on the GPU.  Two calls in a row on one context, the second with fewer
particles than the first; each against pic_step on the same input and, to
the parity bar, against the CPU oracle: per-patch counts exact, the same
particles in the same (stable) order, positions and momenta bit for bit, J
within 1e-12 of the per-node sum of |terms|.  Also: the capacity limit is
reported before anything is enqueued, and the regular entry points still
work on a context after a pic_step_noalloc call."""
import numpy as np
import pytest

from paper_2204_12837_amd import inputs as I

from _parity import compare, run_oracle, say

pytestmark = pytest.mark.gpu

CASES = {
    # name: (workload of the first call, workload of the second, mode, steps)
    "2d_per_patch": (I.custom(2, (64, 48), (8, 8), ppc=6, seed=71, sigma=0.08),
                     I.custom(2, (64, 48), (8, 8), ppc=2, seed=72, sigma=0.08), 0, 3),
    "2d_persistent": (I.custom(2, (64, 48), (8, 8), ppc=6, seed=73, sigma=0.08),
                      I.custom(2, (64, 48), (8, 8), ppc=3, seed=74, sigma=0.08), 1, 2),
    "3d_two_species": (I.custom(3, (16, 16, 24), (8, 8, 8), ppc=3, seed=75, sigma=0.08,
                                n_species=2),
                       I.custom(3, (16, 16, 24), (8, 8, 8), ppc=1, seed=76, sigma=0.08,
                                n_species=2), 1, 3),
}


def _state(sp, J):
    out = [dict(off=s.offset.cpu().numpy(), id=s.ids.cpu().numpy(), x=s.xs.cpu().numpy(),
                u=s.us.cpu().numpy(), w=s.ws.cpu().numpy()) for s in sp]
    return out, J.cpu().numpy()


def _run(ctx, wl, steps, noalloc):
    import torch

    from paper_2204_12837_amd import pic

    inp = I.generate(wl)
    # buffers of exactly n particles: pic_step keeps the dense layout too
    sp = pic.upload(inp, "cuda:0", capacity_factor=1.0)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    if noalloc:
        ctx.step_noalloc(sp, E, B, J, nsteps=steps)
    else:
        ctx.step(sp, E, B, J, nsteps=steps)
    torch.cuda.synchronize()
    ctx.check()
    return inp, _state(sp, J)


@pytest.mark.parametrize("case", list(CASES))
def test_noalloc_equals_pic_step_twice(case):
    from paper_2204_12837_amd import pic

    wl1, wl2, mode, steps = CASES[case]
    ctx_na = pic.Context(wl1, device=0, mode=mode, check=True)
    ctx_ref = pic.Context(wl1, device=0, mode=mode, check=True)
    try:
        for k, wl in enumerate((wl1, wl2)):
            say(f"case {case}, call {k + 1}: {wl.n[:wl.dim]} cells, ppc "
                f"{wl.species[0].ppc(np.zeros(1, dtype=np.int64))[0]}, {steps} steps")
            inp, (g, Jg) = _run(ctx_na, wl, steps, noalloc=True)
            _, (r, Jr) = _run(ctx_ref, wl, steps, noalloc=False)
            n = sum(s["id"].size for s in g)
            assert n == sum(s.x.shape[1] for s in inp.species)
            for a, b in zip(g, r):
                for key in ("off", "id", "x", "u", "w"):
                    assert np.array_equal(a[key], b[key]), (case, k, key)
            osp, J, A = run_oracle(wl, inp, steps)
            compare(osp, J, A, g, Jg, exact_order=True)
            err = np.abs(Jg - Jr)
            assert np.all(err <= 1e-12 * A + 1e-300), err.max()
    finally:
        ctx_na.close()
        ctx_ref.close()


def test_noalloc_then_regular_calls():
    """After pic_step_noalloc re-sorted the particles with the static
    scratch, pic_step and the split entry points on the same context rebuild
    their own segment starts and still match the oracle."""
    import torch

    from paper_2204_12837_amd import pic

    wl = I.custom(2, (48, 48), (8, 8), ppc=4, seed=77, sigma=0.08)
    inp = I.generate(wl)
    say("case noalloc then pic_step (dense, persistent) and the split path")
    ctx = pic.Context(wl, device=0, mode=1, check=True)
    try:
        sp = pic.upload(inp, "cuda:0", capacity_factor=1.0)
        E, B, J = pic.upload_fields(inp, "cuda:0")
        ctx.bin(sp)
        ctx.step_noalloc(sp, E, B, J, nsteps=2)
        ctx.step(sp, E, B, J, nsteps=2)
        J.zero_()
        ctx.interp_push(sp, E, B)
        ctx.project(sp, J)
        ctx.bin(sp)
        torch.cuda.synchronize()
        ctx.check()
        g, Jg = _state(sp, J)
        osp, Jo, A = run_oracle(wl, inp, 5)
        compare(osp, Jo, A, g, Jg, exact_order=True)
    finally:
        ctx.close()


def test_noalloc_capacity_and_refusals():
    """More particles than the static array can serve: PIC_ERR_CAPACITY,
    nothing enqueued (the particles are unchanged); x-bins and removing
    walls are refused."""
    import dataclasses

    import torch

    from paper_2204_12837_amd import pic

    # 2D, 9.4 M particles: 8 bytes each of tags and permutation alone exceed 64 MiB
    wl = I.custom(2, (512, 512), (16, 16), ppc=36, seed=78, sigma=0.05)
    say("case noalloc capacity: 512x512 cells, 36 ppc")
    inp = I.generate(wl)
    ctx = pic.Context(wl, device=0, check=True)
    try:
        sp = pic.upload(inp, "cuda:0", capacity_factor=1.0)
        E, B, J = pic.upload_fields(inp, "cuda:0")
        ctx.bin(sp)
        torch.cuda.synchronize()
        x0 = sp[0].xs.clone()
        with pytest.raises(pic.PicError) as ei:
            ctx.step_noalloc(sp, E, B, J, nsteps=1)
        assert ei.value.status == pic.PIC_ERR_CAPACITY and "static" in str(ei.value)
        torch.cuda.synchronize()
        assert torch.equal(sp[0].xs, x0)
        # the context is still usable
        ctx.step(sp, E, B, J, nsteps=1)
        torch.cuda.synchronize()
        ctx.check()
    finally:
        ctx.close()
        del sp, E, B, J
        torch.cuda.empty_cache()
    small = I.custom(2, (64, 64), (8, 8), ppc=2, seed=79)
    for wlx, kw in ((dataclasses.replace(small, particle_bc=(2, 0, 0)), {}),
                    (I.custom(2, (64, 64), (16, 8), ppc=2, seed=79), {"bin_x": 8})):
        inp = I.generate(wlx)
        c = pic.Context(wlx, device=0, check=True, **kw)
        try:
            sp = pic.upload(inp, "cuda:0", n_slabs=c.n_slabs)
            E, B, J = pic.upload_fields(inp, "cuda:0")
            c.bin(sp)
            with pytest.raises(pic.PicError) as ei:
                c.step_noalloc(sp, E, B, J, nsteps=1)
            assert ei.value.status == pic.PIC_ERR_ARG
        finally:
            c.close()
