"""Write the oracle's expected values for the full-size water workloads.

Runs ONLY the FP64 oracle (oracle/) on the seeded inputs of
paper_2601_18838_amd/systems.py and stores, per workload: R, r0, E_rec and
the potentials and forces of 64 sampled particles (seed 44, without
replacement); for the 64-system batch, every system's E_rec and 8 sampled
particles.  The GPU tests compare the library against these stored values.

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
BATCH_NAME = "batch64_pm1"
BATCH_SAMPLES = 8   # sampled particles per batch system


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


def make_batch():
    """The 64 independent +-1 systems of the batched evaluation: per system
    R, r0, E_rec and the potentials and forces of BATCH_SAMPLES particles
    (seed 45 + system index, without replacement)."""
    t0 = time.time()
    out = {"workload": BATCH_NAME, "systems": [],
           "source": "oracle FP64: nested-SVD SKP-PME at each system's R, this script"}
    for k, (wl, pos, q) in enumerate(systems.batch_systems(count=64)):
        pl = skp.Plan(wl.box, wl.grid, wl.order, wl.beta, rank=wl.rank)
        Q = spme.spread(pos, q, wl.box, wl.grid, wl.order)
        Phi = pl.apply(Q)
        phi, F = spme.gather(pos, q, wl.box, wl.grid, wl.order, Phi)
        idx = np.sort(np.random.default_rng(45 + k).choice(len(q), BATCH_SAMPLES,
                                                            replace=False))
        out["systems"].append({"rank": pl.rank, "r0": pl.r0, "n": len(q),
                               "E_rec": 0.5 * float(q @ phi), "sample_index": idx.tolist(),
                               "phi": phi[idx].tolist(), "F": F[idx].tolist()})
        print(k, wl.grid, "p", wl.order, "R", pl.rank, "n", len(q), f"{time.time() - t0:.0f}s",
              flush=True)
    out["seconds"] = time.time() - t0
    with open(os.path.join(HERE, BATCH_NAME + ".json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(WORKLOADS) + [BATCH_NAME]):
        if name == BATCH_NAME:
            make_batch()
        else:
            make(WORKLOADS[name])
