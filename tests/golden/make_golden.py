"""Writes tests/golden/oracle_uniform64_digest.json: a digest of the CPU
oracle's state after 10 steps of the seeded uniform64 workload (per-patch
counts, exact sums of the particle arrays and of J), and
tests/golden/oracle_walls_digest.json: the same for a fast plasma (thermal
spread 0.5) between removing walls along x and reflecting walls along y,
which exercises the mirror and the deletion.  Calls only the oracle
and the input generator; the stored values guard the oracle against
unintended changes (a deliberate change of its arithmetic rewrites this file
and names the passage of the paper that justifies it).

    python tests/golden/make_golden.py
"""
import hashlib
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)


def _walls_workload():
    import dataclasses

    from paper_2204_12837_amd import inputs as I

    wl = I.custom(2, (32, 24), (8, 8), ppc=6, seed=77, sigma=0.5, bz0=0.5, steps=10)
    return dataclasses.replace(wl, particle_bc=(2, 1, 0))


def digest(walls=False):
    import oracle as O
    from paper_2204_12837_amd import inputs as I

    wl = _walls_workload() if walls else I.workload("uniform64")
    inp = I.generate(wl)
    sps = O.species_from(inp)
    for s in sps:
        O.bin(wl, s)
    J = None
    for _ in range(wl.steps):
        J = O.step(wl, sps, inp.E, inp.B)
    s = sps[0]
    h = hashlib.sha256()
    for a in (s.off, s.id, s.x, s.u, s.w, J):
        h.update(np.ascontiguousarray(a).tobytes())
    return {
        "workload": "walls" if walls else "uniform64", "steps": wl.steps, "particles": int(s.n),
        "counts_first16": np.diff(s.off)[:16].tolist(),
        "sum_x": [math.fsum(s.x[a]) for a in range(2)],
        "sum_u": [math.fsum(s.u[a]) for a in range(3)],
        "sum_J": [math.fsum(J[c].ravel()) for c in range(3)],
        "sum_abs_J": [math.fsum(np.abs(J[c]).ravel()) for c in range(3)],
        "sha256": h.hexdigest(),
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "oracle_uniform64_digest.json"), "w") as fh:
        json.dump(digest(), fh, indent=1)
    with open(os.path.join(HERE, "oracle_walls_digest.json"), "w") as fh:
        json.dump(digest(walls=True), fh, indent=1)
