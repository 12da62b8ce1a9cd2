"""Cardinal B-splines for smooth PME interpolation (oracle; test infrastructure).

The paper interpolates particles onto product grids (Sec. 2.2) and names
B-splines as the alternative to its Lagrange choice; this module follows the
textbook smooth-PME definitions:

* M_2(u) = 1 - |u - 1| on [0, 2], zero elsewhere;
* M_n(u) = [u M_{n-1}(u) + (n - u) M_{n-1}(u - 1)] / (n - 1);
* M_n'(u) = M_{n-1}(u) - M_{n-1}(u - 1);
* |b(m)|^2 = 1 / |sum_{k=0}^{n-2} M_n(k + 1) exp(2 pi i m k / K)|^2.

Pinned by: the closed-form cubic spline, partition of unity, unit integral,
symmetry, central differences for the derivative, and exact interpolation of
exp(2 pi i m u / K) at integer u (which fixes |b(m)|^2's index range and
argument) -- tests/test_oracle_bspline.py.
"""
import numpy as np


def mp(u, p):
    """M_p(u) evaluated elementwise by the two-term recursion, in float64."""
    u = np.asarray(u, dtype=np.float64)
    if p < 2:
        raise ValueError("spline order must be >= 2")
    if p == 2:
        return np.where((u >= 0.0) & (u <= 2.0), 1.0 - np.abs(u - 1.0), 0.0)
    return (u * mp(u, p - 1) + (p - u) * mp(u - 1.0, p - 1)) / (p - 1)


def dmp(u, p):
    """dM_p/du = M_{p-1}(u) - M_{p-1}(u - 1)."""
    u = np.asarray(u, dtype=np.float64)
    return mp(u, p - 1) - mp(u - 1.0, p - 1)


def bmod2(K, p):
    """|b(m)|^2 for m = 0..K-1 on a periodic axis of K points."""
    m = np.arange(K, dtype=np.float64)
    k = np.arange(p - 1, dtype=np.float64)          # k = 0 .. p-2
    terms = mp(k + 1.0, p)[None, :] * np.exp(2j * np.pi * np.outer(m, k) / K)
    s = terms.sum(axis=1)
    return 1.0 / np.abs(s) ** 2


def stencil(u, K, p):
    """Grid indices and weights touched by a particle at scaled coordinate u.

    For u in [0, K): grid point k_t = (floor(u) - t) mod K carries weight
    M_p(u - floor(u) + t), t = 0..p-1 (these are all k with 0 < u - k < p up
    to periodic images).  Returns (idx[..., p], w[..., p], dw[..., p]).
    """
    u = np.asarray(u, dtype=np.float64)
    fl = np.floor(u)
    f = u - fl
    t = np.arange(p, dtype=np.float64)
    idx = np.mod(fl[..., None].astype(np.int64) - np.arange(p), K)
    w = mp(f[..., None] + t, p)
    dw = dmp(f[..., None] + t, p)
    return idx, w, dw
