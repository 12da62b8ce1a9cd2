"""Rank study of the two SKP constructions (test infrastructure, CPU only).

For a workload, the number of Kronecker terms R against the error it leaves,
for the nested SVD (Sec. 2.1.1; terms kept by weight) and the sinc quadrature
(Sec. 2.1.2; R = 2N + 1 nodes, best h): the relative max-norm and Frobenius
errors of the kernel symbol, and the relative error of E_rec against FFT
smooth PME (the exact convolution on the same grid).  The analogue of the
paper's compression-rate figures, computed with the oracle alone.

Usage:  python -m oracle.rank_study [water_100k | pm1_1000]
"""
import sys
import time

import numpy as np

from . import quadrature as qd
from . import skp, spme


def study(box, K, p, beta, pos, q, svd_ranks, quad_N):
    exact = spme.spme(pos, q, box, K, p, beta)
    th = exact["theta_hat"]
    Q = exact["Q"]
    thmax, thnorm = th.max(), np.linalg.norm(th)
    rows = []
    full = skp.Plan(box, K, p, beta)
    for R in svd_ranks:
        terms = full.all_terms[:R]
        rec = skp.reconstruct(terms, th.shape)
        Phi = skp.apply(Q, skp.factors(terms), skp.zero_mode_value(terms))
        rec[0, 0, 0] = 0.0
        e = 0.5 * float((Q * Phi).sum())
        rows.append(("nested_svd", R, np.abs(rec - th).max() / thmax,
                     np.linalg.norm(rec - th) / thnorm, abs(e - exact["E_rec"]) / abs(exact["E_rec"])))
    for N in quad_N:
        h, err = qd.best_h(box, K, p, beta, N)
        terms = qd.terms(box, K, p, beta, N, h)
        rec = skp.reconstruct(terms, th.shape)
        Phi = skp.apply(Q, skp.factors(terms), skp.zero_mode_value(terms))
        rec[0, 0, 0] = 0.0
        e = 0.5 * float((Q * Phi).sum())
        rows.append(("sinc", 2 * N + 1, err, np.linalg.norm(rec - th) / thnorm,
                     abs(e - exact["E_rec"]) / abs(exact["E_rec"])))
    return rows


def main(name):
    from paper_2601_18838_amd import systems
    if name == "water_100k":
        wl = systems.WATER_100K
        pos, q = wl.particles()
        box, K, p, beta = wl.box, wl.grid, wl.order, wl.beta
        svd_ranks = [8, 16, 24, 32, 48, 64, 73, 96, 128]
        quad_N = [4, 8, 12, 16, 20, 24, 32, 40]
    else:
        wl = systems.SMALL_PM1
        pos, q = wl.particles()
        box, K, p, beta = wl.box, wl.grid, wl.order, wl.beta
        svd_ranks = [4, 8, 12, 16, 22, 32, 48]
        quad_N = [2, 4, 6, 8, 11, 16, 24]
    t0 = time.time()
    rows = study(box, K, p, beta, pos, q, svd_ranks, quad_N)
    print(f"# {wl.name}: grid {K}, p={p}, beta={beta}; errors against FFT smooth PME "
          f"({time.time() - t0:.0f} s)")
    print("| construction | R | max-norm symbol err | Frobenius symbol err | E_rec rel err |")
    print("|---|---|---|---|---|")
    for (m, R, ei, ef, ee) in rows:
        print(f"| {m} | {R} | {ei:.2e} | {ef:.2e} | {ee:.2e} |")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "pm1_1000")
