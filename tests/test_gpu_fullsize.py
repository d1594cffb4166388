"""Parity at the full workload sizes, in the launch configurations the
benchmark times, on windows of patches that the oracle reproduces exactly.

With the fields given, the particles of a step do not interact, and none
moves faster than light: in k steps a particle crosses fewer than k dt / d
cells of an axis.  Every particle that can end a call of k steps inside a
window of patches, or deposit current onto one of its nodes in the last
step (the deposit reaches at most three cells from the particle), starts
within margin = ceil(k dt / d) + 3 cells of the window.  The oracle steps
exactly those particles, taken from the generated inputs, so inside the
window its per-patch counts, its particle sets and values and its J at every
node are those of the full run.  The bar is the small-size bar: counts and
particle sets exact, positions and momenta bit for bit, J within 1e-12 of
the sum of absolute contributions at each node.

The GPU side runs the whole workload (33.5M particles for the uniform plasma)
with the launch mode, chunk and workgroup size that the benchmark times, in
one pic_step call (slab layout)."""
import numpy as np
import pytest

from paper_2204_12837_amd import inputs as I

from _parity import say
from _window import margin_cells, oracle_window, window_nodes, window_patches

pytestmark = pytest.mark.gpu


def _gpu_run(wl, inp, steps, mode, chunk, wg, bin_x=0):
    import torch

    from paper_2204_12837_amd import pic

    ctx = pic.Context(wl, device=0, mode=mode, chunk=chunk, wg_size=wg, check=True, bin_x=bin_x)
    sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    ctx.step(sp, E, B, J, nsteps=steps)
    torch.cuda.synchronize()
    ctx.check()
    ctx.close()
    return sp, J


def _gpu_patches(s, patches):
    """Host copies (off, id, x, u, w) of the GPU species' particles in the
    given patches, patch after patch."""
    import torch

    off = s.offset.cpu().numpy()
    assert off[0] == 0 and off[-1] == s.n and np.all(np.diff(off) >= 0)
    cnt = np.diff(off)[patches]
    idx = np.concatenate([np.arange(off[P], off[P + 1]) for P in patches]) if patches.size else \
        np.zeros(0, np.int64)
    ti = torch.from_numpy(idx).to(s.x.device)
    return (np.concatenate([[0], np.cumsum(cnt)]), s.id.index_select(0, ti).cpu().numpy(),
            s.x.index_select(1, ti).cpu().numpy(), s.u.index_select(1, ti).cpu().numpy(),
            s.w.index_select(0, ti).cpu().numpy())


def _check_window(wl, inp, steps, sp_gpu, Jg, a0, npw):
    a0 = list(a0) + [0] * (3 - len(a0))
    npw = list(npw) + [1] * (3 - len(npw))
    osp, J, A = oracle_window(wl, inp, steps, a0, npw, margin_cells(wl, steps))
    patches = window_patches(wl, a0, npw)
    total = 0
    for o, g in zip(osp, sp_gpu):
        goff, gid, gx, gu, gw = _gpu_patches(g, patches)
        ocnt = np.diff(o.off)[patches]
        assert np.array_equal(np.diff(goff), ocnt), "per-patch counts differ"
        for k, P in enumerate(patches):
            oi = np.arange(o.off[P], o.off[P + 1])
            gi = np.arange(goff[k], goff[k + 1])
            oo, go = oi[np.argsort(o.id[oi])], gi[np.argsort(gid[gi])]
            assert np.array_equal(gid[go], o.id[oo]), f"particle set of patch {P} differs"
            assert np.array_equal(gx[:, go], o.x[:, oo]), f"x differs in patch {P}"
            assert np.array_equal(gu[:, go], o.u[:, oo]), f"u differs in patch {P}"
            assert np.array_equal(gw[go], o.w[oo])
        total += int(ocnt.sum())
    nodes = window_nodes(wl, a0, npw)
    Jgw = np.stack([Jg[c][nodes] for c in range(3)])
    Jw = np.stack([J[c][nodes] for c in range(3)])
    Aw = np.stack([A[c][nodes] for c in range(3)])
    err = np.abs(Jgw - Jw)
    assert np.all(err <= 1e-12 * Aw + 1e-300), f"J differs: max {err.max()}"
    return total


def _run(name, steps, mode, chunk, wg, windows, **over):
    wl = I.workload(name, **over)
    inp = I.generate(wl)
    n = sum(s.id.size for s in inp.species)
    say(f"case {name} {over} full size ({n} particles), {steps} steps, mode={mode} chunk={chunk} "
        f"wg={wg}")
    sp, J = _gpu_run(wl, inp, steps, mode, chunk, wg)
    Jg = J.cpu().numpy()
    for a0, npw in windows:
        say(f"  window from cell {a0}, {npw} patches")
        got = _check_window(wl, inp, steps, sp, Jg, a0, npw)
        say(f"  {got} particles compared")
        assert got > 0


def test_uniform1024_per_patch():
    """The benchmark's headline configuration: per-patch launch, default
    workgroup; a window across the periodic corner and one inside."""
    _run("uniform1024", 10, 0, 0, 0, [((-32, -32), (3, 3)), ((496, 304), (3, 2))])


@pytest.mark.parametrize("mode", [0, 1])
def test_imbalanced(mode):
    """Persistent launch with the chunk and workgroup the autotuner picks on
    this workload, and the per-patch launch: windows at the edge of the
    empty half and on the peak of the bump (16k particles per patch)."""
    chunk, wg = (2048, 256) if mode == 1 else (0, 0)
    _run("imbalanced", 8, mode, chunk, wg, [((1008, 128), (3, 2)), ((1520, 480), (2, 3))])


def test_expansion3d_persistent():
    """3D, two species, persistent launch (chunk 4096, 512 threads)."""
    _run("expansion3d", 5, 1, 4096, 512, [((120, 56, 56), (2, 2, 2)), ((248, 120, 0), (2, 2, 1))])


def test_uniform1024_large_patches():
    """Patches of 64 x 128 cells (automatic 8-cell x-bins), per-patch launch:
    one window across the periodic corner."""
    _run("uniform1024", 10, 0, 0, 0, [((-64, -128), (1, 1)), ((448, 384), (2, 1))],
         patch=(64, 128, 1))


def test_imbalanced_with_x_walls_persistent():
    """The imbalanced workload with reflecting particle walls along x,
    persistent launch: a window on the right wall (the background plasma
    reaches it) and one on the bump."""
    _run("imbalanced", 8, 1, 2048, 256, [((2016, 200), (2, 3)), ((1520, 96), (2, 2))],
         particle_bc=(1, 0, 0))


def test_imbalanced_with_removing_x_walls_persistent():
    """The same with removing walls along x: particles that reach the right
    wall are deleted, on the GPU as in the oracle (window at the wall)."""
    _run("imbalanced", 8, 1, 2048, 256, [((2016, 200), (2, 3))], particle_bc=(2, 0, 0))
