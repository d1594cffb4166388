"""PIC_FLAG_TRACE (pic_trace_read): the slab layout's fused kernel records
every work item of its last launch -- a (patch, species) workgroup in
per-patch mode, a popped unit in persistent mode -- with its start and end
times (the GPU counterpart of the paper's per-operation scheduling
diagnostics, section "Task scheduling visualization").  Checked: every
item appears exactly once, ends after it starts, the items cover every
patch that holds particles, the persistent unit list has its documented
order (full units, then remainders by size class), and tracing leaves the
results equal to the oracle's."""
import dataclasses

import numpy as np
import pytest

from paper_2204_12837_amd import inputs as I

from _parity import compare, run_oracle, say

pytestmark = pytest.mark.gpu


def _uneven(dim=2):
    """Patches of very different populations: empty below x = 16 cells, then
    1 to 12 particles per cell depending on x."""
    def ppc(ix):
        return np.where(ix < 16, 0, 1 + (ix * 5) % 12).astype(np.int64)

    if dim == 2:
        wl = I.custom(2, (64, 48), (8, 8), ppc=1, seed=801, sigma=0.1)
    else:
        wl = I.custom(3, (32, 16, 16), (8, 8, 8), ppc=1, seed=802, sigma=0.1, n_species=2)
    sp = [dataclasses.replace(s, ppc=ppc) for s in wl.species]
    return dataclasses.replace(wl, species=sp)


def _run(wl, mode, steps=4, chunk=512):
    import torch

    from paper_2204_12837_amd import pic

    inp = I.generate(wl)
    ctx = pic.Context(wl, device=0, mode=mode, chunk=chunk, check=True, trace=True)
    assert ctx.trace_read() == []  # nothing traced yet
    sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    ctx.step(sp, E, B, J, nsteps=steps)
    torch.cuda.synchronize()
    ctx.check()
    rec = ctx.trace_read()
    g = [dict(off=s.offset.cpu().numpy(), id=s.ids.cpu().numpy(), x=s.xs.cpu().numpy(),
              u=s.us.cpu().numpy(), w=s.ws.cpu().numpy()) for s in sp]
    out = (inp, rec, g, J.cpu().numpy(), ctx.n_patches)
    ctx.close()
    return out


@pytest.mark.parametrize("mode", [0, 1])
def test_trace_covers_every_work_item(mode):
    wl = _uneven()
    say(f"case trace 2D mode={mode}")
    steps = 4
    inp, rec, g, Jg, npatch = _run(wl, mode, steps)
    assert rec, "no records"
    patch = np.array([r[0] for r in rec])
    unit = np.array([r[1] for r in rec])
    t0 = np.array([r[4] for r in rec], dtype=np.uint64)
    t1 = np.array([r[5] for r in rec], dtype=np.uint64)
    assert np.all(t1 >= t0) and np.all(t0 > 0)
    assert (t1.max() - t0.min()) < 100_000_000  # under a second of the 100 MHz clock
    osp, J, A = run_oracle(wl, inp, steps)
    compare(osp, J, A, g, Jg, exact_order=False)  # tracing changes nothing
    # the particles at the start of the last step sit in these patches
    osp_prev, _, _ = run_oracle(wl, inp, steps - 1)
    full = set(np.nonzero(np.diff(osp_prev[0].off))[0].tolist())
    if mode == 0:
        assert len(rec) == npatch  # one workgroup per (patch, species)
        assert sorted(patch.tolist()) == list(range(npatch))
        assert np.all(unit == 0)  # the species
    else:
        assert sorted(unit.tolist()) == list(range(len(rec)))  # each unit once
        assert set(patch.tolist()) == full
        assert len(rec) >= len(full)
        # the list's order: every patch's full units in patch order, then
        # the remainders from the largest to the smallest in eight size
        # classes, each class in patch order
        chunk = 512
        counts = np.diff(osp_prev[0].off)
        want = [P for P, c in enumerate(counts) for _ in range(c // chunk)]
        rems = [(((chunk - c % chunk) * 8 - 1) // chunk, P) for P, c in enumerate(counts) if c % chunk]
        want += [P for _, P in sorted(rems)]
        assert patch[np.argsort(unit)].tolist() == want


def test_trace_units_span_species():
    """3D with two species, persistent: one unit list over both species of
    a patch (species -1 in the records)."""
    wl = _uneven(3)
    say("case trace 3D two species persistent")
    inp, rec, g, Jg, npatch = _run(wl, 1, steps=3, chunk=256)
    assert rec and all(r[3] == -1 for r in rec)
    unit = sorted(r[1] for r in rec)
    assert unit == list(range(len(rec)))
    osp, J, A = run_oracle(wl, inp, 3)
    compare(osp, J, A, g, Jg, exact_order=False)
