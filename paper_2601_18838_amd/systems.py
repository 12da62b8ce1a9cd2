"""Seeded synthetic particle systems (inputs only; no method arithmetic).

The paper's experiments use synthetic, quasi-uniform particle clouds
(Sec. 5); this module builds the workloads the library is measured on, with
NumPy's PCG64 generator so every consumer sees identical arrays:

* ``uniform_pm1``: positions uniform in the box, charges +1 / -1 alternating;
* ``water``: rigid three-site molecules (O -0.834, two H +0.417 at 0.9572 from
  O with a 104.52 degree H-O-H angle), O uniform in the box, orientation
  uniform on SO(3) (unit quaternion from a normalised 4-D Gaussian), atom
  order O, H, H;
* ``batch_systems``: independent neutral +-1 systems of log-uniform size on
  grids drawn from a fixed list, for the batched evaluation.

Positions are wrapped into [0, L) and, like charges, rounded to float32
representable values, so a float32 and a float64 evaluation see the same
inputs.  Nothing here computes any part of the reciprocal sum.
"""
from dataclasses import dataclass, field
import math

import numpy as np


def _f32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def _wrap(pos, box):
    box = np.asarray(box, np.float64)
    return pos - np.floor(pos / box[None, :]) * box[None, :]


def uniform_pm1(n, box, seed):
    """n charges +1/-1 (alternating), positions uniform in the box."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, np.float64)
    pos = rng.uniform(0.0, 1.0, size=(n, 3)) * box[None, :]
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return _f32(_wrap(pos, box)), _f32(q)


def random_rotations(rng, n):
    """n rotation matrices uniform on SO(3) from normalised 4-D Gaussians."""
    g = rng.standard_normal((n, 4))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    w, x, y, z = g.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


WATER_BOND = 0.9572
WATER_ANGLE_DEG = 104.52
WATER_Q = (-0.834, 0.417, 0.417)


def water(nmol, box, seed):
    """nmol rigid water-like triplets; returns (pos[3*nmol, 3], q[3*nmol])."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, np.float64)
    centre = rng.uniform(0.0, 1.0, size=(nmol, 3)) * box[None, :]
    half = math.radians(WATER_ANGLE_DEG) / 2.0
    local = np.array([[0.0, 0.0, 0.0],
                      [WATER_BOND * math.sin(half), WATER_BOND * math.cos(half), 0.0],
                      [-WATER_BOND * math.sin(half), WATER_BOND * math.cos(half), 0.0]])
    R = random_rotations(rng, nmol)
    sites = centre[:, None, :] + np.einsum('nij,kj->nki', R, local)
    pos = sites.reshape(-1, 3)
    q = np.tile(np.array(WATER_Q), nmol)
    return _f32(_wrap(pos, box)), _f32(q)


@dataclass
class Workload:
    """One reciprocal-space workload: particles, box, grid and SKP settings."""
    name: str
    box: tuple
    grid: tuple
    order: int
    beta: float
    rank: int = 0          # > 0: fixed number of Kronecker terms
    tol: float = 0.0       # used when rank <= 0: relative Frobenius tail
    kind: str = "pm1"
    n: int = 0
    seed: int = 0
    extra: dict = field(default_factory=dict)

    def particles(self):
        if self.kind == "pm1":
            return uniform_pm1(self.n, self.box, self.seed)
        if self.kind == "water":
            return water(self.n // 3, self.box, self.seed)
        raise ValueError(self.kind)


# The five workloads: a small fp64 correctness case, a 1e5-atom water box,
# a 1e6-atom precision case, a non-cubic differentiation case and a batch.
SMALL_PM1 = Workload("pm1_n1000_g16_p4", (20.0, 20.0, 20.0), (16, 16, 16), 4, 0.35,
                     rank=8, kind="pm1", n=1000, seed=1)
WATER_100K = Workload("water_n99999_g96_p4", (100.0, 100.0, 100.0), (96, 96, 96), 4,
                      0.34, tol=1e-6, kind="water", n=99999, seed=2)
WATER_1M = Workload("water_n1000002_g128_p6", (215.0, 215.0, 215.0), (128, 128, 128),
                    6, 0.34, tol=1e-6, kind="water", n=1000002, seed=3)
WATER_200K_NONCUBIC = Workload("water_n200001_g80x100x120_p4", (120.0, 150.0, 180.0),
                               (80, 100, 120), 4, 0.34, tol=1e-6, kind="water",
                               n=200001, seed=4)

# The paper's own discretisation (per-cell Lagrange interpolation with the
# mode-truncated kernel): 10 cells of 8 nodes per axis (70 grid points),
# |m_j| <= 10, a 20^3 box at beta = 0.35 (the Gaussian is e^-20 at m = 10).
LAGRANGE_M10 = Workload("lagrange_pm1_n100000_c10_L8_m10", (20.0, 20.0, 20.0), (70, 70, 70), 8,
                        0.35, tol=1e-6, kind="pm1", n=100000, seed=6,
                        extra={"interpolation": "lagrange", "mode_cutoff": 10, "cells": 10})

BATCH_GRIDS = [(32, 32, 32), (48, 48, 48), (64, 64, 64), (64, 64, 96),
               (80, 96, 112), (96, 96, 96), (96, 128, 160)]


def batch_systems(count=64, base_seed=5000):
    """Independent neutral +-1 systems: N log-uniform in [5e3, 3e5] (even),
    grid from BATCH_GRIDS with unit spacing, p in {4, 6}, R in 6..24, beta 0.34."""
    out = []
    for s in range(count):
        rng = np.random.default_rng(base_seed + s)
        n = 2 * int(round(math.exp(rng.uniform(math.log(5e3), math.log(3e5))) / 2))
        grid = BATCH_GRIDS[int(rng.integers(len(BATCH_GRIDS)))]
        p = int(rng.choice([4, 6]))
        rank = int(rng.integers(6, 25))
        box = tuple(float(k) for k in grid)
        pos = rng.uniform(0.0, 1.0, size=(n, 3)) * np.asarray(box)[None, :]
        q = np.concatenate([np.ones(n // 2), -np.ones(n // 2)])
        q = q[rng.permutation(n)]
        wl = Workload(f"batch{s}", box, grid, p, 0.34, rank=rank, kind="given", n=n,
                      seed=base_seed + s)
        out.append((wl, _f32(_wrap(pos, box)), _f32(q)))
    return out
