"""Parity of the HIP library with the CPU oracle (needs an MI355X).

The bar: per-patch counts exact; the same particles in every patch, in the
oracle's (stable) order in the dense layout and by id in the slab layout,
where the order inside a patch is arbitrary; particle positions and momenta
bit for bit (the kernels repeat the oracle's operation sequence); J within
1e-12 of the sum of absolute contributions at each node (the only difference
is the order of the float64 atomic additions).

Layouts: calls of three steps or more keep the particles in per-patch slabs
when the buffers have room for them (the default capacity); with buffers of
exactly n particles (capacity factor 1) every call uses the dense layout and
the permutation sort."""
import ctypes as C
import dataclasses

import numpy as np
import pytest

from paper_2204_12837_amd import inputs as I

from _parity import compare, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu

LAYOUTS = {"slab": dict(capacity_factor=None, exact_order=False),
           "dense": dict(capacity_factor=1.0, exact_order=True)}


def run_cmp(wl, inp, steps, layout, osp, J, A, **kw):
    lay = LAYOUTS[layout]
    g, Jg = run_gpu(wl, inp, steps, capacity_factor=lay["capacity_factor"], **kw)
    compare(osp, J, A, g, Jg, exact_order=lay["exact_order"])
    return g, Jg


@pytest.mark.parametrize("layout", list(LAYOUTS))
def test_uniform64_ten_steps(layout):
    wl = I.workload("uniform64")
    inp = I.generate(wl)
    say(f"case uniform64, 10 steps, fused, {layout}")
    osp, J, A = run_oracle(wl, inp, 10)
    run_cmp(wl, inp, 10, layout, osp, J, A)


def test_split_path_equals_oracle():
    wl = I.workload("uniform64")
    inp = I.generate(wl)
    say("case uniform64, 3 steps, split interp_push / project / bin")
    osp, J, A = run_oracle(wl, inp, 3)
    g, Jg = run_gpu(wl, inp, 3, split=True)
    compare(osp, J, A, g, Jg, exact_order=True)


@pytest.mark.parametrize("wg", [64, 128, 192, 512, 1024])
def test_workgroup_sizes(wg):
    wl = I.custom(2, (48, 32), (8, 8), ppc=5, seed=40 + wg, sigma=0.1)
    inp = I.generate(wl)
    say(f"case 48x32 wg={wg}")
    osp, J, A = run_oracle(wl, inp, 3)
    g, Jg = run_gpu(wl, inp, 3, wg_size=wg)
    compare(osp, J, A, g, Jg)


CASES = [
    # dim, n, patch, ppc, nspecies, sigma, steps, seed
    (2, (36, 24), (6, 6), 3, 1, 0.2, 4, 101),
    (2, (30, 42), (10, 7), 2, 2, 0.3, 3, 102),
    (2, (12, 12), (6, 6), 7, 1, 0.5, 5, 103),   # 2x2 patches: neighbours alias
    (2, (8, 16), (8, 8), 4, 1, 0.4, 3, 104),    # one patch along x
    (3, (16, 12, 12), (8, 6, 6), 2, 2, 0.2, 3, 105),
    (3, (12, 12, 12), (6, 6, 6), 1, 1, 0.5, 4, 106),
    (3, (8, 16, 8), (8, 8, 8), 2, 1, 0.3, 2, 107),
]


@pytest.mark.parametrize("layout", list(LAYOUTS))
@pytest.mark.parametrize("case", CASES)
def test_random_small_configs(case, layout):
    dim, n, patch, ppc, nsp, sigma, steps, seed = case
    wl = I.custom(dim, n, patch, ppc=ppc, seed=seed, sigma=sigma, n_species=nsp)
    inp = I.generate(wl)
    say(f"case {case} {layout}")
    osp, J, A = run_oracle(wl, inp, steps)
    run_cmp(wl, inp, steps, layout, osp, J, A)


def test_general_sort_from_any_order():
    """pic_bin on unsorted particles spread over a period around the box."""
    wl = I.custom(2, (32, 24), (8, 6), ppc=3, seed=110)
    inp = I.generate(wl)
    rng = np.random.default_rng(111)
    L = np.array([wl.n[0] * wl.d[0], wl.n[1] * wl.d[1]])
    x = inp.species[0].x
    shift = rng.integers(-1, 2, x.shape)
    x += shift * L[:, None] * 0.999999
    say("case unsorted bin")
    osp, _, _ = run_oracle(wl, inp, 0)
    g, _ = run_gpu(wl, inp, 0)
    compare(osp, None, None, g, None, exact_order=True)


@pytest.mark.parametrize("case", ["two_passes", "three_passes"])
def test_general_sort_many_patches(case):
    """pic_bin's radix sort when the patch keys need more than one 8-bit
    digit: 4,096 patches (two passes) and 65,536 patches plus the key of
    particles deleted at a removing wall (three passes), on particles in
    any order: the oracle's stable order, its offsets and its deletions."""
    if case == "two_passes":
        wl = I.custom(2, (384, 384), (6, 6), ppc=2, seed=114)
    else:
        wl = dataclasses.replace(I.custom(2, (1536, 1536), (6, 6), ppc=1, seed=112),
                                 particle_bc=(2, 0, 0))
    inp = I.generate(wl)
    x = inp.species[0].x
    rng = np.random.default_rng(113)
    L = np.array([wl.n[0] * wl.d[0], wl.n[1] * wl.d[1]])
    if case == "three_passes":
        k = rng.random(x.shape[1]) < 0.01  # outside the removing walls: deleted
        x[0, k] = np.where(rng.random(k.sum()) < 0.5, -0.37, L[0] + 0.25)
        x[1] += rng.integers(-1, 2, x.shape[1]) * L[1] * 0.999999
    else:
        x += rng.integers(-1, 2, x.shape) * L[:, None] * 0.999999
    say(f"case general sort {case}: {wl.n_patches} patches, {x.shape[1]} particles")
    osp, _, _ = run_oracle(wl, inp, 0)
    g, _ = run_gpu(wl, inp, 0)
    compare(osp, None, None, g, None, exact_order=True)


def test_edge_positions():
    """Particles exactly on patch and cell boundaries, on nodes, at the box
    edges and just below L."""
    wl = I.custom(2, (24, 24), (8, 8), ppc=2, seed=120, sigma=0.3)
    inp = I.generate(wl)
    s = inp.species[0]
    d = wl.d[0]
    L = wl.n[0] * d
    vals = np.array([0.0, 8 * d, 16 * d, 0.5 * d, 7.5 * d, np.nextafter(L, 0), np.nextafter(8 * d, 0),
                     np.nextafter(16 * d, 20 * d), 3 * d, 12 * d])
    k = vals.size
    s.x[0, :k] = vals
    s.x[1, :k] = vals[::-1]
    s.x[0, k:2 * k] = vals
    s.x[1, k:2 * k] = 0.0
    s.u[:, :k] = 0.0  # stay on the boundary in a zero-momentum start
    say("case edges")
    osp, J, A = run_oracle(wl, inp, 4)
    for layout in LAYOUTS:
        run_cmp(wl, inp, 4, layout, osp, J, A)


def test_empty_and_crowded_patches():
    """An x-profile with empty patches next to crowded ones (the imbalanced
    workload's shape at small size)."""
    wl = I.custom(2, (48, 24), (8, 8), ppc=1, seed=130, sigma=0.2)
    wl.species[0].ppc = lambda ix: np.where(ix < 16, 0, np.where(ix < 24, 40, 2)).astype(np.int64)
    inp = I.generate(wl)
    say("case empty/crowded patches")
    osp, J, A = run_oracle(wl, inp, 5)
    for layout in LAYOUTS:
        run_cmp(wl, inp, 5, layout, osp, J, A)


def test_zero_steps_and_zero_particles():
    wl = I.custom(2, (16, 16), (8, 8), ppc=0, seed=140)
    inp = I.generate(wl)
    say("case no particles")
    for steps in (2, 4):
        osp, J, A = run_oracle(wl, inp, steps)
        g, Jg = run_gpu(wl, inp, steps)
        compare(osp, J, A, g, Jg)
        assert np.all(Jg == 0)


PERSISTENT_CASES = [
    # dim, n, patch, ppc, nspecies, sigma, steps, seed, chunk, wg
    (2, (48, 24), (8, 8), 6, 1, 0.2, 4, 201, 256, 256),
    (2, (48, 24), (8, 8), 6, 1, 0.2, 4, 202, 512, 128),
    (2, (64, 32), (16, 16), 9, 2, 0.3, 3, 203, 1024, 256),
    (3, (16, 16, 8), (8, 8, 8), 3, 2, 0.2, 3, 204, 256, 256),
    (3, (24, 12, 12), (6, 6, 6), 2, 1, 0.4, 3, 205, 512, 192),
]


@pytest.mark.parametrize("layout", list(LAYOUTS))
@pytest.mark.parametrize("case", PERSISTENT_CASES)
def test_persistent_matches_oracle(case, layout):
    """The persistent work-queue launch (units of `chunk` particles) gives
    the same particles and counts, and J within the bar."""
    dim, n, patch, ppc, nsp, sigma, steps, seed, chunk, wg = case
    wl = I.custom(dim, n, patch, ppc=ppc, seed=seed, sigma=sigma, n_species=nsp)
    inp = I.generate(wl)
    say(f"case persistent {case} {layout}")
    osp, J, A = run_oracle(wl, inp, steps)
    run_cmp(wl, inp, steps, layout, osp, J, A, mode=1, chunk=chunk, wg_size=wg)


def test_persistent_imbalanced_profile():
    """Empty patches next to patches of several thousand particles."""
    wl = I.custom(2, (96, 32), (16, 16), ppc=1, seed=210, sigma=0.2)
    wl.species[0].ppc = lambda ix: np.where(ix < 48, 0, np.where(ix < 64, 24, 3)).astype(np.int64)
    inp = I.generate(wl)
    say("case persistent imbalanced")
    osp, J, A = run_oracle(wl, inp, 4)
    for chunk in (256, 2048):
        for layout in LAYOUTS:
            run_cmp(wl, inp, 4, layout, osp, J, A, mode=1, chunk=chunk)


@pytest.mark.parametrize("layout", list(LAYOUTS))
@pytest.mark.parametrize("mode", [0, 1])
def test_graph_replay_matches_oracle(mode, layout):
    """Steps replayed from captured graphs (runs of eight slab steps and
    single slab steps, or pairs of dense steps), interleaved with eager
    steps and host synchronisations, agree with the oracle after every call
    sequence; the calls of ten steps replay an eight-step graph (the second
    one from the cache)."""
    wl = I.custom(2, (48, 32), (8, 8), ppc=5, seed=300 + mode, sigma=0.2)
    inp = I.generate(wl)
    say(f"case graph mode={mode} {layout}")
    osp, J, A = run_oracle(wl, inp, 27)
    run_cmp(wl, inp, 27, layout, osp, J, A, mode=mode, chunk=512, graph=True,
            step_sizes=[10, 1, 2, 3, 10, 1])


RESIDENT_CASES = [
    # dim, n, patch, bin_x, ppc, nspecies, sigma, seed, call lengths
    (2, (48, 32), (8, 8), 0, 5, 1, 0.2, 350, [1, 1, 2, 1, 3, 1]),
    (2, (96, 48), (48, 24), 8, 3, 2, 0.3, 351, [2, 1, 1, 3]),    # x-bins of 8 cells
    (3, (24, 16, 16), (8, 8, 8), 0, 2, 2, 0.2, 352, [1, 2, 1]),
]


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("case", RESIDENT_CASES)
def test_resident_short_calls(case, mode, graph):
    """PIC_FLAG_RESIDENT: calls of one to three steps that continue in the
    slabs, then pic_sync, give the oracle's particles and current."""
    dim, n, patch, bin_x, ppc, nsp, sigma, seed, sizes = case
    wl = I.custom(dim, n, patch, ppc=ppc, seed=seed + 10 * mode, sigma=sigma, n_species=nsp)
    inp = I.generate(wl)
    steps = sum(sizes)
    say(f"case resident {case} mode={mode} graph={graph}")
    osp, J, A = run_oracle(wl, inp, steps)
    run_cmp(wl, inp, steps, "slab", osp, J, A, mode=mode, chunk=512, graph=graph,
            step_sizes=sizes, bin_x=bin_x, resident=True)


@pytest.mark.parametrize("mode", [0, 1])
def test_resident_then_split_entry_points(mode):
    """Resident calls interleaved with the split entry points, each of which
    writes the resident particles back first: the oracle's particles and
    current after the sequence."""
    import torch

    from paper_2204_12837_amd import pic

    wl = I.custom(2, (48, 32), (8, 8), ppc=4, seed=360 + mode, sigma=0.2)
    inp = I.generate(wl)
    say(f"case resident + split mode={mode}")
    osp, J, A = run_oracle(wl, inp, 6)
    ctx = pic.Context(wl, device=0, mode=mode, chunk=512, check=True, resident=True)
    sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    E, B, Jg = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    ctx.step(sp, E, B, Jg, nsteps=2)      # resident
    Jg.zero_()                            # one split step (the first call writes back)
    ctx.interp_push(sp, E, B)
    ctx.project(sp, Jg)
    ctx.bin(sp)
    ctx.step(sp, E, B, Jg, nsteps=1)      # resident again
    ctx.step(sp, E, B, Jg, nsteps=2)      # continues in the slabs
    ctx.sync()
    torch.cuda.synchronize()
    ctx.check()
    out = [dict(off=s.offset.cpu().numpy(), id=s.ids.cpu().numpy(), x=s.xs.cpu().numpy(),
                u=s.us.cpu().numpy(), w=s.ws.cpu().numpy()) for s in sp]
    compare(osp, J, A, out, Jg.cpu().numpy())
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_resident_alternating_arrays(mode):
    """pic_step on other particle arrays writes the resident ones back first
    (two copies of a plasma stepped alternately on one context in the slab
    layout): each copy ends where the oracle puts it."""
    import torch

    from paper_2204_12837_amd import pic

    wl = I.custom(2, (48, 32), (8, 8), ppc=4, seed=370 + mode, sigma=0.2)
    inp = I.generate(wl)
    say(f"case resident alternating mode={mode}")
    ctx = pic.Context(wl, device=0, mode=mode, chunk=512, check=True, resident=True)
    a = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    b = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    E, B, Jg = pic.upload_fields(inp, "cuda:0")
    ctx.bin(a)
    ctx.bin(b)
    ctx.step(a, E, B, Jg, nsteps=2)   # a resident
    ctx.step(b, E, B, Jg, nsteps=1)   # a written back, b resident
    ctx.step(a, E, B, Jg, nsteps=1)   # b written back, a resident (three steps)
    ctx.sync()
    torch.cuda.synchronize()
    ctx.check()
    for sp, steps in ((a, 3), (b, 1)):
        osp, _, _ = run_oracle(wl, inp, steps)
        out = [dict(off=s.offset.cpu().numpy(), id=s.ids.cpu().numpy(), x=s.xs.cpu().numpy(),
                    u=s.us.cpu().numpy(), w=s.ws.cpu().numpy()) for s in sp]
        compare(osp, None, None, out, None)
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_slab_overflow_replans(mode):
    """A drifting half-box beam floods initially empty patches faster than
    their slab room (64 slots) allows: the device re-plans the slabs inside
    the call and no particle is lost or misplaced."""
    wl = I.custom(2, (64, 32), (8, 8), ppc=1, seed=310 + mode, sigma=0.05, bz0=0.0)
    wl.species[0].ppc = lambda ix: np.where(ix < 32, 16, 0).astype(np.int64)
    inp = I.generate(wl)
    inp.species[0].u[0] += 0.7
    steps = 6
    osp, J, A = run_oracle(wl, inp, steps)
    counts = np.diff(osp[0].off)
    say(f"case slab overflow mode={mode}: max patch count {counts.max()}")
    # patches of the empty half that now hold more than an empty slab's room
    npx = wl.n[0] // wl.patch[0]
    px = np.arange(counts.size) % npx
    assert counts[px >= npx // 2].max() > 64
    run_cmp(wl, inp, steps, "slab", osp, J, A, mode=mode, chunk=256)


@pytest.mark.parametrize("ppc", [72, 280])
@pytest.mark.parametrize("mode", [0, 1])
def test_patch_beyond_the_departure_bitmap(mode, ppc):
    """Patches of more than 16384 particles, whose departures the fused
    kernel leaves to the departures kernel: with 72 ppc its bitmap path,
    with 280 ppc (more than 65536 particles) its tiled large-patch path."""
    wl = I.custom(2, (32, 32), (16, 16), ppc=2, seed=320 + mode, sigma=0.2)
    wl.species[0].ppc = lambda ix: np.where(ix < 16, ppc, 2).astype(np.int64)
    inp = I.generate(wl)
    steps = 4
    osp, J, A = run_oracle(wl, inp, steps)
    counts = np.diff(osp[0].off)
    say(f"case large patches mode={mode} ppc={ppc}: max patch count {counts.max()}")
    assert counts.max() > (16384 if ppc < 100 else 65536)
    run_cmp(wl, inp, steps, "slab", osp, J, A, mode=mode, chunk=2048)


@pytest.mark.parametrize("mode", [0, 1])
def test_many_departures_per_patch(mode):
    """Hot particles in small patches: several hundred departures per patch
    and step, more than one per thread of the departures' and the arrivals'
    workgroups, so each thread takes several departures (and their hole
    fills) in turn and a wave's arrivals spread over every neighbour."""
    wl = I.custom(2, (64, 64), (8, 8), ppc=128, seed=340 + mode, sigma=0.6)
    inp = I.generate(wl)
    # departures of the first step, free streaming (the fields are weak)
    s = inp.species[0]
    v = s.u / np.sqrt(1.0 + (s.u ** 2).sum(0))
    side = wl.patch[0] * wl.d[0]
    p0 = np.floor(s.x[:2] / side).astype(np.int64) % 8
    p1 = np.floor((s.x[:2] + v[:2] * wl.dt) / side).astype(np.int64) % 8
    dep = np.bincount(p0[1] * 8 + p0[0], weights=(p0 != p1).any(0), minlength=64)
    assert dep.min() > 256
    steps = 3
    osp, J, A = run_oracle(wl, inp, steps)
    say(f"case many departures mode={mode}: {int(dep.min())}..{int(dep.max())} per patch")
    run_cmp(wl, inp, steps, "slab", osp, J, A, mode=mode, chunk=2048)


@pytest.mark.parametrize("mode", [0, 1])
def test_3d_patch_beyond_the_departure_bitmap(mode):
    """3D patches of more than 16384 particles: the departures kernel's 3D
    instance (64-thread workgroups, a 16384-slot bitmap) takes them on its
    tiled large-patch path."""
    wl = I.custom(3, (24, 16, 16), (8, 8, 8), ppc=1, seed=330 + mode, sigma=0.2)
    wl.species[0].ppc = lambda ix: np.where(ix < 8, 40, 1).astype(np.int64)
    inp = I.generate(wl)
    steps = 3
    osp, J, A = run_oracle(wl, inp, steps)
    counts = np.diff(osp[0].off)
    say(f"case 3D large patches mode={mode}: max patch count {counts.max()}")
    assert counts.max() > 16384
    run_cmp(wl, inp, steps, "slab", osp, J, A, mode=mode, chunk=4096)


BIN_CASES = [
    # dim, n, patch, bin_x, ppc, nspecies, sigma, steps, seed
    (2, (128, 64), (64, 64), 0, 2, 1, 0.3, 4, 501),        # automatic 16-cell bins
    (2, (96, 48), (48, 24), 8, 3, 2, 0.3, 3, 502),         # bins asked for: 8 cells
    (3, (24, 24, 24), (12, 12, 12), 0, 1, 2, 0.3, 3, 503),  # automatic 4-cell bins
]


@pytest.mark.parametrize("layout", list(LAYOUTS))
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("case", BIN_CASES)
def test_x_bins(case, mode, layout):
    """Patches cut into x-bins: same per-patch counts, particle sets and
    values, and J as the oracle's patch-level run; inside a patch the
    particles are ordered by bin."""
    dim, n, patch, bx, ppc, nsp, sigma, steps, seed = case
    wl = I.custom(dim, n, patch, ppc=ppc, seed=seed, sigma=sigma, n_species=nsp)
    inp = I.generate(wl)
    say(f"case x-bins {case} mode={mode} {layout}")
    osp, J, A = run_oracle(wl, inp, steps)
    g, Jg = run_gpu(wl, inp, steps, mode=mode, chunk=512, bin_x=bx,
                    capacity_factor=LAYOUTS[layout]["capacity_factor"])
    compare(osp, J, A, g, Jg, exact_order=False)


def test_x_bins_split_path_and_general_sort():
    """The split sequence and pic_bin on unsorted input with x-bins."""
    wl = I.custom(2, (128, 64), (64, 64), ppc=2, seed=510, sigma=0.3)
    inp = I.generate(wl)
    say("case x-bins split path")
    osp, J, A = run_oracle(wl, inp, 3)
    g, Jg = run_gpu(wl, inp, 3, split=True)
    compare(osp, J, A, g, Jg, exact_order=False)
    osp, _, _ = run_oracle(wl, inp, 0)
    g, _ = run_gpu(wl, inp, 0)
    compare(osp, None, None, g, None, exact_order=False)


@pytest.mark.parametrize("layout", list(LAYOUTS))
@pytest.mark.parametrize("mode", [0, 1])
def test_x_bins_from_patch_order(mode, layout):
    """Particles sorted by patch but in any order inside it (here: pic_bin
    of a context without bins, which keeps the generation order inside each
    patch) handed to a context with 4-cell x-bins: its calls first put each
    patch's particles into bin order (the per-patch counting sort), and the
    result matches the oracle's patch-level run; also the split path."""
    import torch

    from paper_2204_12837_amd import pic

    wl = I.custom(2, (96, 64), (32, 16), ppc=3, seed=520, sigma=0.3, n_species=2)
    inp = I.generate(wl)
    steps = 3 if layout == "slab" else 2
    say(f"case x-bins from patch order mode={mode} {layout}")
    osp, J, A = run_oracle(wl, inp, steps)
    plain = pic.Context(wl, device=0)
    binned = pic.Context(wl, device=0, mode=mode, chunk=512, bin_x=4, check=True)
    assert plain.n_slabs * 8 == binned.n_slabs
    sp = pic.upload(inp, "cuda:0", capacity_factor=LAYOUTS[layout]["capacity_factor"],
                    n_slabs=binned.n_slabs)
    E, B, Jt = pic.upload_fields(inp, "cuda:0")
    plain.bin(sp)
    torch.cuda.synchronize()
    binned.step(sp, E, B, Jt, nsteps=steps)
    torch.cuda.synchronize()
    binned.check()
    g = [dict(off=s.offset.cpu().numpy(), id=s.ids.cpu().numpy(), x=s.xs.cpu().numpy(),
              u=s.us.cpu().numpy(), w=s.ws.cpu().numpy()) for s in sp]
    compare(osp, J, A, g, Jt.cpu().numpy(), exact_order=False)
    # split path: the bin order happens in pic_interp_push
    sp2 = pic.upload(inp, "cuda:0", capacity_factor=1.0)
    plain.bin(sp2)
    for _ in range(steps):
        Jt.zero_()
        binned.interp_push(sp2, E, B)
        binned.project(sp2, Jt)
        binned.bin(sp2)
    torch.cuda.synchronize()
    binned.check()
    g = [dict(off=s.offset.cpu().numpy(), id=s.ids.cpu().numpy(), x=s.xs.cpu().numpy(),
              u=s.us.cpu().numpy(), w=s.ws.cpu().numpy()) for s in sp2]
    compare(osp, J, A, g, Jt.cpu().numpy(), exact_order=False)
    plain.close()
    binned.close()


@pytest.mark.parametrize("layout", list(LAYOUTS))
def test_particle_outside_its_patch_is_reported(layout):
    """Offsets that hand patch 0 the particles of its x-neighbour: the fused
    kernel's tile bounds check reports PIC_ERR_UNSORTED at the next check, and the
    context then refuses work (PIC_ERR_STATE) until it is freed."""
    import torch

    from paper_2204_12837_amd import pic

    wl = I.custom(2, (32, 32), (8, 8), ppc=2, seed=330)
    inp = I.generate(wl)
    say(f"case position error {layout}")
    ctx = pic.Context(wl)
    sp = pic.upload(inp, "cuda:0", capacity_factor=LAYOUTS[layout]["capacity_factor"],
                    n_slabs=ctx.n_slabs)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    torch.cuda.synchronize()
    off = sp[0].offset
    off[1] = off[2]  # patch 0 now ends where patch 1 ends
    ctx.step(sp, E, B, J, nsteps=3)
    with pytest.raises(pic.PicError) as ei:
        ctx.check()
    assert ei.value.status == pic.PIC_ERR_UNSORTED
    with pytest.raises(pic.PicError) as ei:
        ctx.step(sp, E, B, J, nsteps=1)
    assert ei.value.status == pic.PIC_ERR_STATE
    ctx.close()


def test_call_order_errors():
    """pic_project without pic_interp_push, and pic_step with a sort pending,
    are refused before anything is enqueued."""
    from paper_2204_12837_amd import pic

    wl = I.custom(2, (16, 16), (8, 8), ppc=2, seed=331)
    inp = I.generate(wl)
    ctx = pic.Context(wl, check=True)
    sp = pic.upload(inp, "cuda:0")
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    with pytest.raises(pic.PicError) as ei:
        ctx.project(sp, J)
    assert ei.value.status == pic.PIC_ERR_STATE
    ctx.interp_push(sp, E, B)
    with pytest.raises(pic.PicError) as ei:
        ctx.step(sp, E, B, J, nsteps=1)
    assert ei.value.status == pic.PIC_ERR_STATE
    ctx.project(sp, J)
    ctx.bin(sp)
    ctx.step(sp, E, B, J, nsteps=1)  # usable again
    ctx.check()
    ctx.close()


def _combo(seed):
    """A seeded random combination of the step's options (dimension, sizes,
    x-bins, launch mode, workgroup, chunk, layout, graphs, call lengths,
    particle boundaries: mostly periodic, some reflecting or removing walls;
    removing walls need the slab layout's room, so the dense layout gets
    reflecting ones instead)."""
    rng = np.random.default_rng(seed)
    dim = 3 if seed % 3 == 2 else 2
    if dim == 2:
        patch = (int(rng.choice([6, 8, 12, 16, 24])), int(rng.choice([6, 8, 12])))
        npat = (int(rng.integers(1, 5)), int(rng.integers(1, 5)))
        ppc = int(rng.integers(1, 8))
        wgs = [64, 128, 256, 512, 1024]
    else:
        patch = (int(rng.choice([6, 8, 12])), int(rng.choice([6, 8])), int(rng.choice([6, 8])))
        npat = (int(rng.integers(1, 4)), int(rng.integers(1, 3)), int(rng.integers(1, 3)))
        ppc = int(rng.integers(1, 3))
        wgs = [256, 512, 1024]
    n = tuple(p * k for p, k in zip(patch, npat))
    divs = [b for b in range(1, patch[0] + 1) if patch[0] % b == 0 and b >= 2]
    c = dict(dim=dim, n=n, patch=patch, ppc=ppc, nsp=int(rng.integers(1, 3)),
             sigma=float(rng.choice([0.05, 0.2, 0.4])),
             bin_x=int(rng.choice([0] + divs)), mode=int(rng.integers(0, 2)),
             wg=int(rng.choice(wgs)), chunk=int(rng.choice([256, 512, 2048])),
             layout=str(rng.choice(list(LAYOUTS))), graph=bool(rng.integers(0, 2)),
             sizes=[int(k) for k in rng.integers(1, 5, size=int(rng.integers(1, 4)))])
    bc = [int(v) for v in rng.choice([0, 0, 0, 1, 2], size=dim)]
    if c["layout"] == "dense":
        bc = [1 if v == 2 else v for v in bc]
    c["bc"] = tuple(bc) + (0,) * (3 - dim)
    return c


@pytest.mark.parametrize("seed", range(1000, 1036))
def test_random_option_combinations(seed):
    """Parity with the oracle for random combinations of the step's options
    (the bar of the other parity tests; order inside a patch is compared
    exactly only in the dense layout without x-bins)."""
    from paper_2204_12837_amd import pic

    c = _combo(seed)
    wl = I.custom(c["dim"], c["n"], c["patch"], ppc=c["ppc"], seed=seed, sigma=c["sigma"],
                  n_species=c["nsp"])
    wl = dataclasses.replace(wl, particle_bc=c["bc"])
    cfg = pic.make_config(wl, mode=c["mode"], chunk=c["chunk"], wg_size=c["wg"], bin_x=c["bin_x"])
    if pic.validate(cfg)[0] != pic.PIC_OK:
        pytest.skip(f"configuration not valid: {pic.validate(cfg)[1]}")
    inp = I.generate(wl)
    steps = sum(c["sizes"])
    say(f"case combo {seed}: {c}")
    osp, J, A = run_oracle(wl, inp, steps)
    lay = LAYOUTS[c["layout"]]
    g, Jg = run_gpu(wl, inp, steps, mode=c["mode"], chunk=c["chunk"], wg_size=c["wg"],
                    graph=c["graph"], step_sizes=c["sizes"], capacity_factor=lay["capacity_factor"],
                    bin_x=c["bin_x"])
    exact = (lay["exact_order"] and pic.lib().pic_bin_width(C.byref(cfg)) == c["patch"][0]
             and 2 not in c["bc"])
    compare(osp, J, A, g, Jg, exact_order=exact)
