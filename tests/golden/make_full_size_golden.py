"""Write the oracle's expected values for the full-size water workloads.

Runs ONLY the FP64 oracle (oracle/) on the seeded inputs of
paper_2601_18838_amd/systems.py and stores, per workload: R, r0, E_rec and
the potentials and forces of 64 sampled particles (seed 44, without
replacement).  The GPU tests compare the library against these stored values.

Usage (CPU, minutes):  python tests/golden/make_full_size_golden.py [name ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import skp, spme  # noqa: E402
from paper_2601_18838_amd import systems  # noqa: E402

WORKLOADS = {w.name: w for w in (systems.WATER_1M, systems.WATER_200K_NONCUBIC)}


def make(wl):
    t0 = time.time()
    pos, q = wl.particles()
    pl = skp.Plan(wl.box, wl.grid, wl.order, wl.beta, tol=wl.tol)
    Q = spme.spread(pos, q, wl.box, wl.grid, wl.order)
    Phi = pl.apply(Q)
    phi, F = spme.gather(pos, q, wl.box, wl.grid, wl.order, Phi)
    idx = np.sort(np.random.default_rng(44).choice(len(q), 64, replace=False))
    out = {"workload": wl.name, "rank": pl.rank, "r0": pl.r0, "E_rec": 0.5 * float(q @ phi),
           "sum_F": F.sum(axis=0).tolist(), "rms_F": float(np.sqrt((F ** 2).mean())),
           "sample_index": idx.tolist(), "phi": phi[idx].tolist(), "F": F[idx].tolist(),
           "source": "oracle FP64: nested-SVD SKP-PME at the tolerance rule, this script",
           "seconds": time.time() - t0}
    with open(os.path.join(HERE, wl.name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    print(wl.name, "R", pl.rank, "E_rec", out["E_rec"], f"{out['seconds']:.0f}s", flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(WORKLOADS)):
        make(WORKLOADS[name])
