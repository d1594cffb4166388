"""Build the HIP library ``libpic.so`` for gfx950 with hipcc (in-tree).

Flags: -ffp-contract=off (the interpolation and push repeat a fixed
operation sequence), -munsafe-fp-atomics (float64 atomic adds lower to the
hardware instructions instead of compare-and-swap loops), packed-fp32 code
generation disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["pic_api.hip", "pic_kernels.hip", "pic_slab.hip", "pic_sort.hip", "pic_adjoint.hip",
           "pic_maxwell.hip", "pic_rho.hip"]
HEADERS = ["pic_common.h", "pic_device.h", "pic_fields.h", os.path.join(ROOT, "include", "pic.h")]
LIB = os.path.join(HERE, "libpic.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _obj(src: str) -> str:
    return os.path.join(CSRC, "_build", os.path.splitext(src)[0] + ".o")


def _stale(out: str, deps) -> bool:
    if not os.path.exists(out):
        return True
    t = os.path.getmtime(out)
    return any(os.path.getmtime(d) > t for d in deps)


def build(force: bool = True, verbose: bool = False) -> str:
    os.makedirs(os.path.join(CSRC, "_build"), exist_ok=True)
    hdrs = [h if os.path.isabs(h) else os.path.join(CSRC, h) for h in HEADERS]
    objs, cmds = [], []
    for src in SOURCES:
        s = os.path.join(CSRC, src)
        o = _obj(src)
        objs.append(o)
        if force or _stale(o, [s, *hdrs]):
            cmds.append([HIPCC, *FLAGS, "-c", s, "-o", o])

    def compile_one(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    # one hipcc per source, at most as many at once as there are CPUs (8 here)
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1) or 1) as ex:
        list(ex.map(compile_one, cmds))
    if force or _stale(LIB, objs):
        tmp = LIB + ".tmp"
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force="--lazy" not in sys.argv, verbose=True)
