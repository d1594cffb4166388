"""Shared helpers of the GPU parity tests: run the CPU oracle and the HIP
library on the same generated inputs and compare them."""
import sys

import numpy as np

import oracle as O


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_oracle(wl, inp, steps, with_abs=True):
    sps = O.species_from(inp)
    for s in sps:
        O.bin(wl, s)
    J = A = None
    for _ in range(steps):
        J, A = O.step(wl, sps, inp.E, inp.B, with_abs=True)
    return sps, J, A


def run_gpu(wl, inp, steps, mode=0, chunk=0, wg_size=0, split=False, device="cuda:0",
            graph=False, step_sizes=None, capacity_factor=None, bin_x=0, resident=False):
    """capacity_factor None gives the buffers room for pic_step's slab
    layout (used for calls of three steps or more); 1.0 keeps the dense
    layout with the permutation sort.  resident: PIC_FLAG_RESIDENT, the
    dense layout written back by pic_sync after the last call."""
    import torch

    from paper_2204_12837_amd import pic

    ctx = pic.Context(wl, device=0, mode=mode, chunk=chunk, wg_size=wg_size, check=True,
                      graph=graph, bin_x=bin_x, resident=resident)
    sp = pic.upload(inp, device, capacity_factor=capacity_factor, n_slabs=ctx.n_slabs)
    E, B, J = pic.upload_fields(inp, device)
    ctx.bin(sp)
    if split:
        for _ in range(steps):
            J.zero_()
            ctx.interp_push(sp, E, B)
            ctx.project(sp, J)
            ctx.bin(sp)
    elif step_sizes:
        assert sum(step_sizes) == steps
        for k in step_sizes:
            ctx.step(sp, E, B, J, nsteps=k)
            torch.cuda.synchronize()
    else:
        ctx.step(sp, E, B, J, nsteps=steps)
    if resident:
        ctx.sync()
    torch.cuda.synchronize()
    ctx.check()
    out = []
    for s in sp:
        out.append(dict(off=s.offset.cpu().numpy(), id=s.ids.cpu().numpy(),
                        x=s.xs.cpu().numpy(), u=s.us.cpu().numpy(), w=s.ws.cpu().numpy()))
    Jg = J.cpu().numpy() if steps > 0 else None
    ctx.close()
    return out, Jg


def compare(osp, J, A, gout, Jg, exact_particles=True, rel=1e-12, exact_order=False):
    """Per-patch counts exact; inside each patch the same particles (by id),
    in the same order if exact_order (the dense layout's stable sort),
    otherwise in any order (the slab layout); particles bit for bit (or
    within rel); J within rel * (sum of |terms|)."""
    for s, g in zip(osp, gout):
        assert np.array_equal(g["off"], s.off), "per-patch counts differ"
        if exact_order:
            assert np.array_equal(g["id"], s.id), "particle order differs"
            gi = np.arange(s.id.size)
        else:
            # order both sides by id inside each patch
            pat = np.repeat(np.arange(s.off.size - 1), np.diff(s.off))
            oo = np.lexsort((s.id, pat))
            go = np.lexsort((g["id"], pat))
            assert np.array_equal(g["id"][go], s.id[oo]), "per-patch particle sets differ"
            gi = np.empty_like(go)
            gi[oo] = go
        assert np.array_equal(g["w"][gi], s.w)
        gx, gu = g["x"][:, gi], g["u"][:, gi]
        if exact_particles:
            assert np.array_equal(gx, s.x), f"x differs: {np.abs(gx - s.x).max()}"
            assert np.array_equal(gu, s.u), f"u differs: {np.abs(gu - s.u).max()}"
        else:
            L = np.abs(s.x).max()
            assert np.all(np.abs(gx - s.x) <= rel * np.maximum(np.abs(s.x), 1e-3 * L))
            assert np.all(np.abs(gu - s.u) <= rel * np.maximum(np.abs(s.u), 1e-3))
    if J is not None:
        err = np.abs(Jg - J)
        assert np.all(err <= rel * A + 1e-300), f"J differs: max {err.max()}, rel to A {(err / np.maximum(A, 1e-300)).max()}"
        assert err.max() <= rel * max(np.abs(J).max(), 1e-300)
