"""Autotuner for the persistent launch: picks the work-unit size (chunk, in
particles), the workgroup size and (in 3D) the x-bin width for a workload
by timing a step's fused kernel and exchange on the live particles, and
caches the choice in a JSON file keyed by the GPU architecture, the
library build (a digest of libpic.so, so a rebuilt kernel is tuned again),
the dimension, the patch shape, the number of species and a coarse
histogram of the per-patch populations.

The paper tunes its task granularity (the bin width) by hand per physical
set-up; this does the same search automatically.  All timing is done by
the library's own HIP-event timing of the fused kernel class.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import pic

CHUNKS = (512, 1024, 2048, 4096, 8192)
WGS = (128, 256)
WGS_3D = (512, 1024)


def cache_path() -> str:
    p = os.environ.get("PIC_TUNE_CACHE")
    if p:
        return p
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "pic_mi355x", "tune.json")


def population_key(counts: np.ndarray) -> str:
    """Coarse shape of the per-patch population histogram: log2 of the mean
    occupied-patch population, log2 of max/mean (half steps) and the empty
    fraction (tenths)."""
    counts = np.asarray(counts, dtype=np.int64)
    occ = counts[counts > 0]
    if occ.size == 0:
        return "empty"
    mean = occ.mean()
    lm = int(round(math.log2(max(mean, 1))))
    sk = round(2 * math.log2(max(counts.max() / mean, 1.0))) / 2
    ef = int(round(10 * (1 - occ.size / counts.size)))
    return f"m{lm}_s{sk}_e{ef}"


_LIB_DIGEST: Optional[str] = None


def library_digest() -> str:
    """Short digest of the built library (its kernels decide the timings)."""
    global _LIB_DIGEST
    if _LIB_DIGEST is None:
        import hashlib

        h = hashlib.sha256()
        with open(pic.LIB_PATH, "rb") as fh:
            for block in iter(lambda: fh.read(1 << 20), b""):
                h.update(block)
        _LIB_DIGEST = h.hexdigest()[:16]
    return _LIB_DIGEST


def _key(wl, counts) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    patch = "x".join(str(p) for p in wl.patch[:wl.dim])
    return (f"{arch}|lib{library_digest()}|{wl.dim}d|p{patch}|s{len(wl.species)}|"
            f"{population_key(counts)}")


def _load(path: str) -> Dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def bin_candidates(wl) -> Tuple[int, ...]:
    """x-bin widths to try: the library's choice (0), and in 3D half the
    patch when that is at least 4 cells."""
    if wl.dim == 3 and wl.patch[0] % 2 == 0 and wl.patch[0] // 2 >= 4:
        return (0, wl.patch[0] // 2)
    return (0,)


def tune(wl, species: Sequence[pic.Species], E, B, J, steps: int = 3,
         chunks: Sequence[int] = CHUNKS, wgs: Sequence[int] = WGS, use_cache: bool = True,
         path: Optional[str] = None, bins: Optional[Sequence[int]] = None) -> Dict:
    """Best (chunk, wg, bin_x) for the persistent launch on these particles.
    The particles advance by (1 + steps) steps per candidate."""
    path = path or cache_path()
    counts = np.concatenate([np.diff(s.offset.cpu().numpy()) for s in species])
    key = _key(wl, counts)
    cache = _load(path)
    if use_cache and key in cache:
        out = dict(cache[key])
        out["cached"] = True
        return out
    trials: List[Tuple[float, float, int, int, int]] = []
    if wl.dim == 3 and tuple(wgs) == WGS:
        wgs = WGS_3D
    bins = bin_candidates(wl) if bins is None else tuple(bins)
    for bx in bins:
        for wg in wgs:
            for chunk in chunks:
                ctx = pic.Context(wl, mode=pic.MODE_PERSISTENT, chunk=chunk, wg_size=wg, bin_x=bx)
                ctx.bin(species)
                ctx.step(species, E, B, J, nsteps=1)
                ctx.timing(True)
                ctx.step(species, E, B, J, nsteps=steps)
                t = ctx.timing_read()
                ctx.check()
                ctx.close()
                ipp = t["ipp"][0] / max(t["ipp"][1], 1)
                exch = t["exchange"][0] / max(t["exchange"][1], 1) if "exchange" in t else 0.0
                trials.append((ipp + exch, ipp, chunk, wg, bx))
    _, ms, chunk, wg, bx = min(trials)
    out = {"chunk": chunk, "wg": wg, "bin_x": bx, "ipp_ms": ms, "key": key,
           "trials": [{"chunk": c, "wg": w, "bin_x": b, "ipp_ms": round(i, 4),
                       "step_ms": round(t, 4)} for t, i, c, w, b in trials]}
    cache[key] = out
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as fh:
            json.dump(cache, fh, indent=1)
    except OSError:
        pass
    out = dict(out)
    out["cached"] = False
    return out
