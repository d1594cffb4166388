"""The HIP charge density (pic_rho) against the oracle's.

Each term q w S is the oracle's product; only the order of the additions
at a node differs, so the bar is the J bar: per node |diff| <= 1e-12 times
the sum of the absolute terms (the density of |q|)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2204_12837_amd import inputs as I
from paper_2204_12837_amd import pic

from _parity import say

pytestmark = pytest.mark.gpu


def _check(wl, inp, **ctx_kw):
    ctx = pic.Context(wl, check=True, **ctx_kw)
    sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    ctx.bin(sp)
    shp = (wl.n[2] if wl.dim == 3 else 1, wl.n[1], wl.n[0])
    rho = torch.zeros(shp, dtype=torch.float64, device="cuda:0")
    ctx.rho(sp, rho)
    torch.cuda.synchronize()
    ctx.check()
    g = rho.cpu().numpy()
    r = np.zeros(shp)
    A = np.zeros(shp)
    for s in inp.species:
        r += O.rho(wl, s.q, s.x, s.wt)
        A += O.rho(wl, abs(s.q), s.x, s.wt)
    ctx.close()
    err = np.abs(g - r)
    assert np.all(err <= 1e-12 * A + 1e-300), err.max()
    assert abs(g.sum() - sum(s.q * s.wt.sum() for s in inp.species)) <= 1e-9 * A.sum()
    return g


CASES = [
    # dim, n, patch, ppc, nspecies, seed
    (2, (32, 24), (8, 6), 5, 1, 801),
    (2, (48, 48), (16, 16), 3, 2, 802),
    (3, (16, 12, 12), (8, 6, 6), 2, 2, 803),
    (2, (256, 128), (128, 128), 1, 1, 804),  # tile above 96 KB: global atomics
    (2, (128, 64), (64, 64), 2, 2, 805),     # patches cut into x-bins by the step kernels
]


@pytest.mark.parametrize("case", CASES)
def test_rho_matches_oracle(case):
    dim, n, patch, ppc, nsp, seed = case
    wl = I.custom(dim, n, patch, ppc=ppc, seed=seed, sigma=0.1, n_species=nsp)
    say(f"case rho {case}")
    _check(wl, I.generate(wl))


@pytest.mark.parametrize("name", ["uniform1024", "expansion3d"])
def test_rho_full_size(name):
    wl = I.workload(name)
    say(f"case rho full size {name}")
    _check(wl, I.generate(wl))


def test_rho_after_steps_and_empty_patches():
    """After pic_step (slab layout) on the imbalanced profile's shape, and
    with no particles at all."""
    wl = I.custom(2, (48, 24), (8, 8), ppc=1, seed=810, sigma=0.2)
    wl.species[0].ppc = lambda ix: np.where(ix < 16, 0, np.where(ix < 24, 40, 2)).astype(np.int64)
    inp = I.generate(wl)
    ctx = pic.Context(wl, check=True)
    sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    ctx.step(sp, E, B, J, nsteps=4)
    rho = torch.zeros((1, 24, 48), dtype=torch.float64, device="cuda:0")
    ctx.rho(sp, rho)
    torch.cuda.synchronize()
    ctx.check()
    x, w = sp[0].xs.cpu().numpy(), sp[0].ws.cpu().numpy()
    r = O.rho(wl, -1.0, x, w)
    A = O.rho(wl, 1.0, x, w)
    assert np.all(np.abs(rho.cpu().numpy() - r) <= 1e-12 * A + 1e-300)
    ctx.close()
    wl0 = I.custom(2, (16, 16), (8, 8), ppc=0, seed=811)
    g = _check(wl0, I.generate(wl0))
    assert np.all(g == 0)


def test_rho_flags_a_particle_outside_its_patch():
    """Offsets that hand patch 0 the particles of patch 1: the kernel's tile
    bounds check reports unsorted input."""
    wl = I.custom(2, (32, 32), (8, 8), ppc=2, seed=812)
    inp = I.generate(wl)
    ctx = pic.Context(wl)
    sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    ctx.bin(sp)
    torch.cuda.synchronize()
    off = sp[0].offset
    off[1] = off[2]  # patch 0 now ends where patch 1 ends
    rho = torch.zeros((1, 32, 32), dtype=torch.float64, device="cuda:0")
    ctx.rho(sp, rho)
    with pytest.raises(pic.PicError) as ei:
        ctx.check()
    assert ei.value.status == pic.PIC_ERR_UNSORTED
    ctx.close()
