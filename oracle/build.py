"""Build the CPU oracle's shared libraries with gcc (test infrastructure).

Three builds of the same source: ``liborc.so`` in double precision (the
parity oracle), ``liborc_ld.so`` in x87 long double and ``liborc_q.so`` in
binary128 (finite-difference references).  Both with -O2 -ffp-contract=off and no fast-math.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pic_oracle.c")
LIBS = {
    "liborc.so": [],
    "liborc_ld.so": ["-DORC_REAL=long double"],
    "liborc_q.so": ["-DORC_QUAD", "-std=gnu11"],
}
CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall"]


def lib_path(name: str = "liborc.so") -> str:
    return os.path.join(HERE, name)


def build(force: bool = True) -> None:
    for name, extra in LIBS.items():
        out = lib_path(name)
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
            continue
        tmp = out + ".tmp"
        cmd = ["gcc", *CFLAGS, *extra, "-o", tmp, SRC, "-lm"]
        if "-std=gnu11" in extra:
            cmd.remove("-std=c11")
        subprocess.run(cmd, check=True, cwd=HERE)
        os.replace(tmp, out)


if __name__ == "__main__":
    build(force="--lazy" not in sys.argv)
