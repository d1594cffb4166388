"""PIC_FLAG_DETERMINISTIC: pic_step gives the same bits on every run (the
dense layout's stable sort, per-wave J tiles, J summed from the tiles in a
fixed order), and still matches the oracle at the parity bar."""
import dataclasses

import numpy as np
import pytest

from paper_2204_12837_amd import inputs as I

from _parity import compare, run_oracle, say

pytestmark = pytest.mark.gpu

CASES = {
    "2d": (I.custom(2, (64, 48), (8, 8), ppc=5, seed=901, sigma=0.1), 0, 0),
    "2d_persistent_config": (I.custom(2, (64, 48), (8, 8), ppc=5, seed=902, sigma=0.1), 1, 0),
    "2d_x_bins_4": (I.custom(2, (64, 32), (32, 16), ppc=3, seed=903, sigma=0.2), 0, 4),
    "2d_reflecting": (dataclasses.replace(I.custom(2, (48, 48), (8, 8), ppc=4, seed=904,
                                                   sigma=0.4), particle_bc=(1, 1, 0)), 0, 0),
    "3d_two_species": (I.custom(3, (24, 16, 16), (8, 8, 8), ppc=2, seed=905, sigma=0.1,
                                n_species=2), 0, 0),
}


def _run(wl, mode, bin_x, steps):
    import torch

    from paper_2204_12837_amd import pic

    inp = I.generate(wl)
    ctx = pic.Context(wl, device=0, mode=mode, bin_x=bin_x, check=True, deterministic=True)
    sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    ctx.step(sp, E, B, J, nsteps=steps)
    torch.cuda.synchronize()
    ctx.check()
    g = [dict(off=s.offset.cpu().numpy(), id=s.ids.cpu().numpy(), x=s.xs.cpu().numpy(),
              u=s.us.cpu().numpy(), w=s.ws.cpu().numpy()) for s in sp]
    Jg = J.cpu().numpy()
    ctx.close()
    return inp, g, Jg


@pytest.mark.parametrize("case", list(CASES))
def test_deterministic_runs_are_bitwise_equal(case):
    wl, mode, bin_x = CASES[case]
    steps = 5
    say(f"case deterministic {case}")
    inp, g1, J1 = _run(wl, mode, bin_x, steps)
    _, g2, J2 = _run(wl, mode, bin_x, steps)
    assert np.array_equal(J1, J2), "J differs between two runs"
    for a, b in zip(g1, g2):
        for k in ("off", "id", "x", "u", "w"):
            assert np.array_equal(a[k], b[k]), k
    osp, J, A = run_oracle(wl, inp, steps)
    compare(osp, J, A, g1, J1, exact_order=bin_x == 0)
