#!/usr/bin/env python
"""Throughput of the PIC macro-particle step on one MI355X.

One step = J <- 0, the fused Interpolation + Push + pre-BC + Projection of
every particle (in place, in per-patch slabs), and the exchange of the
particles that changed patch (the synchronisation phase); the timed
`pic_step` call of `--steps` steps also includes its one-off copies from the
dense sorted layout into the slabs and back.  Inputs are generated (seeded,
synthetic) and resident in HBM before the timed region starts.

Prints one JSON line: particle-steps/s of the whole call, the roofline of
the dominant kernel (the fused step kernel, HBM-bound by its bytes), the
imbalanced workload next to the uniform one, the 3D two-species workload,
the uniform plasma with patches too large for the LDS (x-bins), the field
solver on the 2D and 3D grids, the charge density, the self-consistent loop
(particles and fields), the adjoint workload, and the CPU oracle timed on a
bounded sample on the host.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (interp+push+project) + % HBM peak; imbalanced vs uniform"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def algorithmic_bytes(wl, n_particles: int) -> int:
    """Bytes the fused step kernel must move once: per particle read x (dim),
    u (3), w and write x (dim), u (3); per cell read E, B (6) and write J (3),
    all float64."""
    dim = wl.dim
    per_particle = 8 * ((dim + 3 + 1) + (dim + 3))
    per_cell = 8 * (6 + 3)
    return per_particle * n_particles + per_cell * wl.n_cells


FUSED_KERNEL = "k_ipp_slab"  # the fused step kernel of a pic_step call of several steps


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("pic_slab.hip", "pic_device.h", "pic_common.h"):
        with open(os.path.join(ROOT, "paper_2204_12837_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{FUSED_KERNEL}_{workload}_traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


FP64_PEAK_TFLOPS = 78.6  # MI355X float64 vector peak


def measured_lds(workload: str):
    """Per-particle LDS instructions and float64 LDS atomics of the 2D fused
    kernel from the committed rocprofv3 counter summary, if it was taken on
    the current kernel source."""
    path = os.path.join(ROOT, "profiles", "k_ipp_slab_uniform1024_lds.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("workload") != workload or t.get("kernel_source_sha") != kernel_source_hash():
        return None
    return t


def measured_valu(workload: str):
    """Per-particle float64 operations and LDS instructions (and the HBM bytes
    per launch) of the 3D persistent fused kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "k_ipp_slab3d_expansion3d_valu.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("workload") != workload or t.get("kernel_source_sha") != kernel_source_hash():
        return None
    return t


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def host_cpu() -> dict:
    """The benchmark host's CPU: model, logical CPUs online (os.cpu_count,
    as nproc), the CPUs this process may run on, and lscpu's topology lines
    when lscpu is there."""
    import shutil
    import subprocess

    info = {"model": cpu_model(), "logical_cpus": os.cpu_count()}
    try:
        info["usable_cpus"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    if shutil.which("lscpu"):
        try:
            out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
            keep = ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core",
                    "CPU max MHz", "L3 cache", "NUMA node(s)")
            for line in out.splitlines():
                k, _, v = line.partition(":")
                if k.strip() in keep:
                    info["lscpu " + k.strip()] = v.strip()
        except (OSError, subprocess.SubprocessError):
            pass
    return info


def run_gpu(wl, steps: int, warmup: int, mode: int = 0, chunk: int = 0, wg: int = 0,
            inp=None, graph: bool = False, bin_x: int = 0, timing: bool = True):
    """Timed pic_step on fresh device copies of the generated inputs.  With
    graph=False and timing the library times each kernel class with HIP
    events on the launch stream; with graph=True steps replay captured graphs
    (no per-kernel timing); timing=False runs the plain eager call."""
    import torch

    from paper_2204_12837_amd import inputs as I
    from paper_2204_12837_amd import pic

    inp = I.generate(wl) if inp is None else inp
    n = sum(s.x.shape[1] for s in inp.species)
    ctx = pic.Context(wl, device=0, mode=mode, chunk=chunk, wg_size=wg, graph=graph, bin_x=bin_x)
    sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    if warmup:
        # at least three steps, so that the slab layout's kernels (which
        # calls of one or two steps do not use) are loaded before the timing;
        # with graphs ten, so that the eight-step and the one-step graph are
        # both captured before it
        ctx.step(sp, E, B, J, nsteps=max(warmup, 10 if graph else 3))
    torch.cuda.synchronize()
    ctx.check()
    timed = timing and not graph
    if timed:
        ctx.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(sp, E, B, J, nsteps=steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.check()
    tim = ctx.timing_read() if timed else {}
    ctx.timing(False)
    ctx.close()
    del sp, E, B, J
    torch.cuda.empty_cache()
    return n, t1 - t0, tim


def tune_persistent(wl, inp):
    """Autotuned (chunk, wg, bin_x) for the persistent launch on these inputs."""
    import torch

    from paper_2204_12837_amd import autotune, pic

    # buffers with slab room for the narrowest x-bins tried
    nb = max([wl.patch[0] // b for b in autotune.bin_candidates(wl) if b > 0] + [1])
    sp = pic.upload(inp, "cuda:0", n_slabs=wl.n_patches * nb)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx = pic.Context(wl)
    ctx.bin(sp)
    ctx.close()
    res = autotune.tune(wl, sp, E, B, J, steps=3, use_cache=False)
    del sp, E, B, J
    torch.cuda.empty_cache()
    return res


def trace_summary(rec):
    """Scheduling of one traced fused-kernel launch: its span, the work
    items' total time over the span (mean concurrency), the peak
    concurrency, their ratio (how busy the workgroups were on average),
    and the part of the span during which fewer than half the peak ran
    (the tail of the longest items)."""
    import numpy as np

    t0 = np.array([r[4] for r in rec], dtype=np.float64)
    t1 = np.array([r[5] for r in rec], dtype=np.float64)
    start, end = t0.min(), t1.max()
    span = end - start
    ev = np.concatenate([np.stack([t0, np.ones_like(t0)], 1), np.stack([t1, -np.ones_like(t1)], 1)])
    ev = ev[np.lexsort((ev[:, 1], ev[:, 0]))]
    active = np.cumsum(ev[:, 1])
    peak = int(active.max())
    dt = np.diff(ev[:, 0])
    low = float(dt[active[:-1] < 0.5 * peak].sum())
    mean = float((t1 - t0).sum() / span) if span > 0 else 0.0
    out = {"items": len(rec), "span_us": span / 100.0, "mean_concurrency": mean,
           "peak_concurrency": peak, "busy_fraction": mean / peak if peak else 0.0,
           "tail_fraction": low / span if span > 0 else 0.0}
    blocks = np.array([r[2] for r in rec])
    if len(np.unique(blocks)) < len(rec):  # persistent: per-worker busy time
        busy = np.bincount(blocks, weights=t1 - t0) / span
        busy = busy[np.unique(blocks)]
        out["workers"] = int(busy.size)
        out["worker_busy_min"] = float(busy.min())
        out["worker_busy_mean"] = float(busy.mean())
    return out


def run_trace(inp=None, chunk=2048, wg=256, steps=5):
    """The imbalanced workload's fused kernel with PIC_FLAG_TRACE, per-patch
    and persistent: how its work items fill the launch."""
    import torch

    from paper_2204_12837_amd import inputs as I
    from paper_2204_12837_amd import pic

    wl = I.workload("imbalanced")
    inp = I.generate(wl) if inp is None else inp
    out = {"workload": "imbalanced", "steps": steps}
    for name, mode in (("per_patch", 0), ("persistent", 1)):
        ctx = pic.Context(wl, device=0, mode=mode, chunk=chunk if mode else 0,
                          wg_size=wg if mode else 0, trace=True)
        sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
        E, B, J = pic.upload_fields(inp, "cuda:0")
        ctx.bin(sp)
        ctx.step(sp, E, B, J, nsteps=steps)
        torch.cuda.synchronize()
        ctx.check()
        out[name] = trace_summary(ctx.trace_read())
        ctx.close()
        del sp, E, B, J
        torch.cuda.empty_cache()
    return out


def run_expansion3d(steps: int, warmup: int):
    """The 3D two-species workload: per-patch launch and the persistent
    launch with an autotuned chunk."""
    from paper_2204_12837_amd import inputs as I

    wl = I.workload("expansion3d")
    inp = I.generate(wl)
    n = sum(s.x.shape[1] for s in inp.species)
    n_pp, s_pp, t_pp = run_gpu(wl, steps, warmup, inp=inp)
    tuned = tune_persistent(wl, inp)
    n_pe, s_pe, t_pe = run_gpu(wl, steps, warmup, mode=1, chunk=tuned["chunk"], wg=tuned["wg"],
                               inp=inp, bin_x=tuned.get("bin_x", 0))
    ipp_pp = t_pp["ipp"][0] / t_pp["ipp"][1]
    ipp_pe = t_pe["ipp"][0] / t_pe["ipp"][1]
    abytes = algorithmic_bytes(wl, n)
    # float64 vector roofline: executed operations per particle (counters)
    # over the faster launch's average fused-kernel duration
    valu = measured_valu("expansion3d")
    alu = None
    if valu:
        tf = valu["fp64_flops_per_particle"] * n / (min(ipp_pp, ipp_pe) * 1e-3) / 1e12
        alu = {"bound": "alu", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
               "frac": tf / FP64_PEAK_TFLOPS,
               "fp64_flops_per_particle": valu["fp64_flops_per_particle"],
               "lds_instructions_per_particle": valu["lds_per_particle"],
               "lds_instructions_per_s": valu["lds_per_particle"] * n / (min(ipp_pp, ipp_pe) * 1e-3),
               # HBM bytes per launch of the persistent kernel from the counters
               # (FETCH_SIZE x 2 + WRITE_SIZE), against the algorithmic bytes
               "traffic": valu.get("hbm_bytes_per_launch"),
               "traffic_over_algorithmic": (valu["hbm_bytes_per_launch"] / abytes
                                            if valu.get("hbm_bytes_per_launch") else None)}
    return {"workload": "expansion3d", "particles": n, "species": 2, "steps": steps, "alu": alu,
            "per_patch": {"ns_per_particle_step": s_pp / (n * steps) * 1e9, "ipp_ms": ipp_pp},
            "persistent": {"ns_per_particle_step": s_pe / (n * steps) * 1e9, "ipp_ms": ipp_pe,
                           "chunk": tuned["chunk"], "wg": tuned["wg"],
                           "bin_x": tuned.get("bin_x", 0),
                           "kernel_ms": {k: round(v[0] / max(v[1], 1), 4)
                                         for k, v in t_pe.items() if v[1]}},
            "ipp_hbm_frac_best": abytes / (min(ipp_pp, ipp_pe) * 1e-3) / 1e9 / HBM_PEAK_GBS}


def run_split(steps: int = 10):
    """The split entry points on the uniform workload: per step J <- 0,
    pic_interp_push, pic_project and pic_bin (the operators one call at a
    time, the sort by neighbour code), timed per kernel class with the
    library's HIP events."""
    import torch

    from paper_2204_12837_amd import inputs as I
    from paper_2204_12837_amd import pic

    wl = I.workload("uniform1024")
    inp = I.generate(wl)
    n = sum(s.x.shape[1] for s in inp.species)
    ctx = pic.Context(wl, device=0)
    sp = pic.upload(inp, "cuda:0", capacity_factor=1.0)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    for _ in range(2):  # warm-up
        J.zero_()
        ctx.interp_push(sp, E, B)
        ctx.project(sp, J)
        ctx.bin(sp)
    torch.cuda.synchronize()
    ctx.timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        J.zero_()
        ctx.interp_push(sp, E, B)
        ctx.project(sp, J)
        ctx.bin(sp)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.check()
    tim = ctx.timing_read()
    ctx.timing(False)
    ctx.close()
    del sp, E, B, J
    torch.cuda.empty_cache()
    return {"workload": "uniform1024", "particles": n, "steps": steps,
            "ms_per_step": (t1 - t0) / steps * 1e3,
            "kernel_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in tim.items() if v[1]}}


def run_short_calls(calls: int = 10, resident: bool = False):
    """pic_step calls of one step each on the uniform workload, as a caller
    that steps one at a time sees it.  Without resident: the dense layout
    (fused kernel writing neighbour-code tags, then the counting sort that
    restores per-patch order).  With resident (PIC_FLAG_RESIDENT): the
    particles stay in the slab layout between calls; the timed region ends
    with the pic_sync that writes the dense layout back."""
    import torch

    from paper_2204_12837_amd import inputs as I
    from paper_2204_12837_amd import pic

    wl = I.workload("uniform1024")
    inp = I.generate(wl)
    n = sum(s.x.shape[1] for s in inp.species)
    ctx = pic.Context(wl, device=0, resident=resident)
    if resident:
        sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    else:
        sp = pic.upload(inp, "cuda:0", capacity_factor=1.0)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    for _ in range(2):
        ctx.step(sp, E, B, J, nsteps=1)
    if resident:
        ctx.sync()
    torch.cuda.synchronize()
    ctx.timing(True)
    t0 = time.perf_counter()
    for _ in range(calls):
        ctx.step(sp, E, B, J, nsteps=1)
    if resident:
        ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.check()
    tim = ctx.timing_read()
    ctx.timing(False)
    ctx.close()
    del sp, E, B, J
    torch.cuda.empty_cache()
    return {"workload": "uniform1024", "particles": n, "calls": calls,
            "layout": "slab, resident" if resident else "dense",
            "ms_per_step": (t1 - t0) / calls * 1e3,
            "kernel_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in tim.items() if v[1]}}


def run_large_patches(steps: int, warmup: int):
    """The uniform plasma with patches of 64 x 128 cells, whose E/B and J
    tiles exceed the LDS: the library cuts them into x-bins (per-patch
    launch, automatic bin width)."""
    import ctypes

    from paper_2204_12837_amd import inputs as I
    from paper_2204_12837_amd import pic

    wl = I.workload("uniform1024", patch=(64, 128, 1))
    n, secs, tim = run_gpu(wl, steps, warmup)
    ipp = tim["ipp"][0] / tim["ipp"][1]
    bx = int(pic.lib().pic_bin_width(ctypes.byref(pic.make_config(wl))))
    return {"workload": "uniform1024", "patch": [64, 128], "bin_x": bx, "particles": n,
            "steps": steps, "ns_per_particle_step": secs / (n * steps) * 1e9, "ipp_ms": ipp,
            "ipp_hbm_frac": algorithmic_bytes(wl, n) / (ipp * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "kernel_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in tim.items() if v[1]}}


def run_maxwell(steps: int = 50):
    """The field solver (pic_maxwell) on the 2D benchmark grid (1024^2) and
    the 3D one (256x128x128): ms per Yee step and GB/s of its algorithmic
    bytes (96 B per node for Ampere + 72 B for Faraday)."""
    import numpy as np
    import torch

    from paper_2204_12837_amd import inputs as I
    from paper_2204_12837_amd import pic

    out = {}
    for name in ("uniform1024", "expansion3d"):
        wl = I.workload(name)
        rng = np.random.default_rng(7)
        shp = (3, wl.n[2] if wl.dim == 3 else 1, wl.n[1], wl.n[0])
        E, B, J = (torch.from_numpy(rng.standard_normal(shp) * 1e-3).to("cuda:0")
                   for _ in range(3))
        ctx = pic.Context(wl)
        ctx.maxwell(E, B, J, 2)
        torch.cuda.synchronize()
        ctx.timing(True)
        t0 = time.perf_counter()
        ctx.maxwell(E, B, J, steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms, n = ctx.timing_read()["maxwell"]
        ctx.timing(False)
        ctx.check()
        ctx.close()
        cells = wl.n_cells
        kern = ms / n
        gbs = 168.0 * cells / (kern * 1e-3) / 1e9
        out[name] = {"cells": cells, "steps": steps, "ms_per_step": (t1 - t0) / steps * 1e3,
                     "kernel_ms_per_step": kern, "algorithmic_GBs": gbs,
                     "hbm_frac": gbs / HBM_PEAK_GBS}
    return out


def run_cycle(steps: int, warmup: int):
    """The self-consistent loop (pic_cycle: particle step, then field step)
    on the 2D benchmark workload, in one call."""
    import torch

    from paper_2204_12837_amd import inputs as I
    from paper_2204_12837_amd import pic

    wl = I.workload("uniform1024")
    inp = I.generate(wl)
    ctx = pic.Context(wl)
    sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    E, B, J = pic.upload_fields(inp, "cuda:0")
    ctx.bin(sp)
    ctx.cycle(sp, E, B, J, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.cycle(sp, E, B, J, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.check()
    ctx.close()
    n = sum(s.n for s in sp)
    del sp, E, B, J
    torch.cuda.empty_cache()
    return {"workload": "uniform1024", "particles": n, "steps": steps,
            "ms_per_step": (t1 - t0) / steps * 1e3, "particle_steps_per_s": n * steps / (t1 - t0)}


def run_rho(reps: int = 20):
    """The charge density (pic_rho) of the 2D benchmark's 33.5M particles:
    ms per call and GB/s of its algorithmic bytes (x, y, w read: 24 B per
    particle; rho written: 8 B per node)."""
    import torch

    from paper_2204_12837_amd import inputs as I
    from paper_2204_12837_amd import pic

    wl = I.workload("uniform1024")
    inp = I.generate(wl)
    ctx = pic.Context(wl)
    sp = pic.upload(inp, "cuda:0", n_slabs=ctx.n_slabs)
    ctx.bin(sp)
    rho = torch.zeros((1, wl.n[1], wl.n[0]), dtype=torch.float64, device="cuda:0")
    ctx.rho(sp, rho)
    torch.cuda.synchronize()
    ctx.timing(True)
    for _ in range(reps):
        ctx.rho(sp, rho)
    ms, n = ctx.timing_read()["rho"]
    ctx.timing(False)
    ctx.check()
    ctx.close()
    n_p = sp[0].n
    del sp
    torch.cuda.empty_cache()
    kern = ms / n
    gbs = (24.0 * n_p + 8.0 * wl.n_cells) / (kern * 1e-3) / 1e9
    return {"workload": "uniform1024", "particles": n_p, "kernel_ms": kern,
            "particles_per_s": n_p / (kern * 1e-3), "algorithmic_GBs": gbs,
            "hbm_frac": gbs / HBM_PEAK_GBS}


def run_adjoint(every: int = 5):
    """Forward (with checkpoints) and backward of the adjoint workload:
    L = sum W.J after 20 steps of 256^2 cells x 16 ppc, gradients with
    respect to the initial momenta and the fields."""
    import torch

    from paper_2204_12837_amd import adjoint as ADJ
    from paper_2204_12837_amd import inputs as I

    wl = I.workload("adjoint256")
    inp = I.generate(wl)
    s = inp.species[0]
    dev = "cuda:0"
    times = []
    ctx = None  # one context for every repetition: its scratch and graphs stay warm
    for rep in range(3):
        run = ADJ.StepRun(wl, torch.from_numpy(s.x).to(dev), torch.from_numpy(s.wt).to(dev),
                          torch.from_numpy(s.id).to(dev), s.q, s.m, wl.steps, every, ctx=ctx)
        u0 = torch.from_numpy(s.u).to(dev).requires_grad_(True)
        E = torch.from_numpy(inp.E).to(dev).requires_grad_(True)
        B = torch.from_numpy(inp.B).to(dev).requires_grad_(True)
        W = torch.from_numpy(inp.W).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = ADJ.PicSteps.apply(u0, E, B, run)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        (W * J).sum().backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        run.ctx.check()
        ctx = run.ctx
        times.append((t1 - t0, t2 - t1))
    fw, bw = min(times, key=lambda t: t[0] + t[1])
    n = s.x.shape[1]
    out = {"workload": "adjoint256", "particles": n, "steps": wl.steps, "checkpoint_every": every,
           "forward_ms": fw * 1e3, "backward_ms": bw * 1e3,
           "gradient_particle_steps_per_s": n * wl.steps / (fw + bw)}
    # the self-consistent loop (particle step + field step per step), same particles
    crun = ADJ.CycleRun(wl, torch.from_numpy(s.x).to(dev), torch.from_numpy(s.wt).to(dev),
                        torch.from_numpy(s.id).to(dev), s.q, s.m, wl.steps, ctx=ctx)
    ctimes = []
    for rep in range(2):
        u0 = torch.from_numpy(s.u).to(dev).requires_grad_(True)
        E = torch.from_numpy(inp.E).to(dev).requires_grad_(True)
        B = torch.from_numpy(inp.B).to(dev).requires_grad_(True)
        W = torch.from_numpy(inp.W).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J, E1, B1 = ADJ.PicCycle.apply(u0, E, B, crun)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ((W * J).sum() + (E1 * E1).sum()).backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        crun.ctx.check()
        ctimes.append((t1 - t0, t2 - t1))
    cf, cb = min(ctimes, key=lambda t: t[0] + t[1])
    out["self_consistent"] = {"forward_ms": cf * 1e3, "backward_ms": cb * 1e3,
                              "checkpoint_every": 1}
    return out


def cpu_baseline(sample_steps: int):
    """The CPU oracle (serial, one core) on a strip of the uniform workload:
    1024 x 64 cells with the same density, momenta and fields, periodic."""
    import oracle as O
    from paper_2204_12837_amd import inputs as I

    wl = I.workload("uniform1024", n=(1024, 64, 1), seed=2002)
    inp = I.generate(wl)
    sps = O.species_from(inp)
    for s in sps:
        O.bin(wl, s)
    n = sum(s.n for s in sps)
    t0 = time.perf_counter()
    for _ in range(sample_steps):
        O.step(wl, sps, inp.E, inp.B)
    dt = time.perf_counter() - t0
    return {"value": n * sample_steps / dt, "unit": "particle-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"uniform plasma strip 1024x64 cells, 32 ppc ({n} particles), "
                      f"{sample_steps} steps, serial scalar C (one thread) on {cpu_model()}",
            "seconds": round(dt, 3), "host": host_cpu(),
            # the paper's own figure, derived from its one-core timing of the
            # 3D plasma-expansion case on a Xeon Gold 6230 (context only)
            "paper_context": {"value": 2.0e6, "unit": "particle-steps/s per core",
                              "cpu": "Intel Xeon Gold 6230 (one core)"}}


def copy_bandwidth(gib: float = 2.0, reps: int = 5) -> float:
    """Measured HBM bandwidth of a plain float64 device-to-device copy of
    `gib` GiB (bytes read plus bytes written per second, in GB/s), timed
    with events on the current stream after one untimed copy."""
    import torch

    n = int(gib * 2 ** 30 / 8)
    src = torch.rand(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n * 8 / (ms * 1e-3) / 1e9


def copy_calibration(gib: float) -> int:
    """A plain float64 device-to-device copy of known size: reads and writes
    `gib` GiB each per launch."""
    import torch

    n = int(gib * 2 ** 30 / 8)
    src = torch.rand(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 5
    print(json.dumps({"copy_bytes_each_way": n * 8, "ms": dt * 1e3,
                      "GBps_read_plus_write": 2 * n * 8 / dt / 1e9}), flush=True)
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform1024")
    ap.add_argument("--no-imbalanced", action="store_true", help="skip the imbalanced workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D two-species workload")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint workload")
    ap.add_argument("--no-maxwell", action="store_true",
                    help="skip the field solver and the charge density")
    ap.add_argument("--no-large-patches", action="store_true",
                    help="skip the 64x128-cell patches (x-bins) workload")
    ap.add_argument("--cpu-steps", type=int, default=24)
    ap.add_argument("--mode", choices=("per_patch", "persistent"), default="per_patch",
                    help="launch of the main workload's fused kernel")
    ap.add_argument("--chunk", type=int, default=0, help="persistent mode: particles per unit")
    ap.add_argument("--wg", type=int, default=0, help="threads per workgroup (0 = library default)")
    ap.add_argument("--bin-x", type=int, default=0, help="x-bin width (0 = library default)")
    ap.add_argument("--order", choices=("random", "cell_interleaved"), default="random",
                    help="particle order inside each patch of the main workload's inputs")
    ap.add_argument("--main-only", action="store_true",
                    help="time only the main workload (e.g. for counter passes)")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only run a plain device copy of this many GiB (5 times), to scale "
                         "HBM traffic counters")
    args = ap.parse_args(argv)
    if args.copy_calibration > 0:
        return copy_calibration(args.copy_calibration)
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; the step would "
              "shard by patch collections with J-halo and particle exchanges between GPUs",
              file=sys.stderr)
        return 2

    from paper_2204_12837_amd import inputs as I

    wl = I.workload(args.workload)
    inp0 = I.generate(wl, order=args.order)
    # the per-kernel HIP events (roofline) come from one call; the headline
    # throughput from the same call without them (plain eager launches)
    launch = dict(mode=1 if args.mode == "persistent" else 0, chunk=args.chunk, wg=args.wg,
                  bin_x=args.bin_x)
    n, secs_ev, tim = run_gpu(wl, args.steps, args.warmup, inp=inp0, **launch)
    _, secs, _ = run_gpu(wl, args.steps, args.warmup, inp=inp0, timing=False, **launch)
    value = n * args.steps / secs
    ipp_ms, ipp_n = tim["ipp"]
    ipp_avg = ipp_ms / max(ipp_n, 1)
    abytes = algorithmic_bytes(wl, n)
    achieved = abytes / (ipp_avg * 1e-3) / 1e9
    traffic = measured_traffic(args.workload)
    copy_bw = copy_bandwidth()
    lds = measured_lds(args.workload)
    per_kernel = {k: round(v[0] / max(v[1], 1), 4) for k, v in tim.items() if v[1]}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "order": args.order, "dim": wl.dim,
                   "cells": list(wl.n[:wl.dim]),
                   "patch": list(wl.patch[:wl.dim]), "particles": n,
                   "species": len(wl.species), "mode": args.mode, "layout": "slab"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": FUSED_KERNEL, "algorithmic_bytes": abytes, "avg_ms": ipp_avg,
                     # the same achieved rate against a measured plain copy
                     "copy_GBps_measured": copy_bw, "frac_of_copy": achieved / copy_bw,
                     # bytes the counters saw per launch, per second of the kernel
                     "traffic_GBps": (traffic / (ipp_avg * 1e-3) / 1e9) if traffic else None,
                     # the second ceiling: float64 LDS atomic adds per second
                     "lds_atomics_per_particle": lds["lds_atomics_per_particle"] if lds else None,
                     "lds_atomics_per_s": (lds["lds_atomics_per_particle"] * n / (ipp_avg * 1e-3))
                     if lds else None},
        "kernel_ms": per_kernel,
        "with_kernel_events": {"ms_per_step": secs_ev / args.steps * 1e3},
        "interp_push_project_rate": n / (ipp_avg * 1e-3),
    }
    if args.main_only:
        print(json.dumps(out), flush=True)
        return 0
    # the same call replaying captured graphs of eight steps (no per-kernel events)
    _, secs_g, _ = run_gpu(wl, args.steps, args.warmup, inp=inp0, graph=True, **launch)
    del inp0
    out["graph_replay"] = {"ms_per_step": secs_g / args.steps * 1e3,
                           "particle_steps_per_s": n * args.steps / secs_g}
    if not args.no_imbalanced:
        wli = I.workload("imbalanced")
        inpi = I.generate(wli)
        # whole-step times come from plain eager calls, as the headline value
        # does (the library's per-kernel events add about 0.02 ms to each of
        # these short steps); a second, timed call of each leg gives kernel_ms
        ni, si, _ = run_gpu(wli, args.steps, args.warmup, inp=inpi, timing=False)
        _, si_ev, ti = run_gpu(wli, args.steps, args.warmup, inp=inpi)
        tuned = tune_persistent(wli, inpi)
        pers = dict(mode=1, chunk=tuned["chunk"], wg=tuned["wg"], bin_x=tuned.get("bin_x", 0))
        _, sp_, _ = run_gpu(wli, args.steps, args.warmup, inp=inpi, timing=False, **pers)
        _, sp_ev, tp = run_gpu(wli, args.steps, args.warmup, inp=inpi, **pers)
        # the persistent call replaying captured graphs of eight steps
        _, sp_g, _ = run_gpu(wli, args.steps, args.warmup, inp=inpi, graph=True, **pers)
        ns_u = secs / (n * args.steps) * 1e9
        ipp_u = ipp_avg / n * 1e6
        per_k = lambda t: {k: round(v[0] / max(v[1], 1), 4) for k, v in t.items() if v[1]}
        ipp_pp = ti["ipp"][0] / ti["ipp"][1]
        ipp_pe = tp["ipp"][0] / tp["ipp"][1]
        nsps = lambda t: t / (ni * args.steps) * 1e9
        out["imbalanced"] = {
            "workload": "imbalanced", "particles": ni,
            "uniform_ns_per_particle_step": ns_u,
            "per_patch": {"ns_per_particle_step": nsps(si),
                          "ns_per_particle_step_with_kernel_events": nsps(si_ev),
                          "kernel_ms": per_k(ti)},
            "persistent": {"ns_per_particle_step": nsps(sp_),
                           "ns_per_particle_step_with_kernel_events": nsps(sp_ev),
                           "ns_per_particle_step_graph": nsps(sp_g),
                           "chunk": tuned["chunk"], "wg": tuned["wg"], "kernel_ms": per_k(tp),
                           "autotune_trials": tuned["trials"]},
            # fused-kernel time per particle, the quantity the task scheduling balances
            "ipp_ns_per_particle": {"uniform_per_patch": ipp_u,
                                    "imbalanced_per_patch": ipp_pp / ni * 1e6,
                                    "imbalanced_persistent": ipp_pe / ni * 1e6},
            "ipp_ratio_persistent_vs_uniform": (ipp_pe / ni) / (ipp_avg / n),
            "ipp_speedup_persistent_vs_per_patch": ipp_pp / ipp_pe,
            "step_ratio_persistent_vs_uniform": (sp_ / ni) / (secs / n),
            "step_speedup_persistent_vs_per_patch": si / sp_,
        }
        # the same workload with reflecting particle walls along x (the paper's
        # radiation-pressure case: reflective in x, periodic in y), persistent
        wlw = dataclasses.replace(wli, particle_bc=(1, 0, 0))
        _, sw, _ = run_gpu(wlw, args.steps, args.warmup, inp=inpi, timing=False, **pers)
        _, _, tw = run_gpu(wlw, args.steps, args.warmup, inp=inpi, **pers)
        ipp_w = tw["ipp"][0] / tw["ipp"][1]
        out["imbalanced"]["x_walls_persistent"] = {
            "ns_per_particle_step": nsps(sw), "kernel_ms": per_k(tw),
            "ipp_ns_per_particle": ipp_w / ni * 1e6,
            "ipp_ratio_vs_periodic": ipp_w / ipp_pe,
            "step_ratio_vs_periodic": sw / sp_,
        }
        # and with removing walls along x (particles reaching them are deleted)
        wlr = dataclasses.replace(wli, particle_bc=(2, 0, 0))
        _, sr, _ = run_gpu(wlr, args.steps, args.warmup, inp=inpi, timing=False, **pers)
        _, _, tr = run_gpu(wlr, args.steps, args.warmup, inp=inpi, **pers)
        out["imbalanced"]["trace"] = run_trace(inpi, tuned["chunk"], tuned["wg"])
        out["imbalanced"]["x_remove_persistent"] = {
            "ns_per_particle_step": nsps(sr), "kernel_ms": per_k(tr),
            "ipp_ratio_vs_periodic": (tr["ipp"][0] / tr["ipp"][1]) / ipp_pe,
            "step_ratio_vs_periodic": sr / sp_,
        }
    if not args.no_3d:
        out["expansion3d"] = run_expansion3d(min(args.steps, 50), args.warmup)
    if not args.no_large_patches:
        out["large_patches"] = run_large_patches(min(args.steps, 50), args.warmup)
    out["split_entry_points"] = run_split()
    out["one_step_calls"] = run_short_calls()
    out["one_step_calls_resident"] = run_short_calls(resident=True)
    if not args.no_maxwell:
        out["maxwell"] = run_maxwell()
        out["rho"] = run_rho()
        out["cycle"] = run_cycle(min(args.steps, 50), args.warmup)
    if not args.no_adjoint:
        out["adjoint"] = run_adjoint()
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline(args.cpu_steps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
