"""Pins of the direct-Ewald oracle: Madelung constant, beta independence,
Newton's third law and finite differences."""
import os

import numpy as np

from oracle import ewald

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "madelung_nacl.txt")


def read_golden(path):
    with open(path) as f:
        return float([l for l in f if not l.startswith("#") and l.strip()][0])


def small_system(n=24, box=(7.0, 8.0, 9.0), seed=11):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 1, (n, 3)) * np.asarray(box)
    q = rng.uniform(-1, 1, n)
    q -= q.mean()
    return pos, q, np.asarray(box)


def test_madelung_nacl():
    """Rock-salt lattice (unit spacing, 6^3 ions in a periodic 6^3 box)."""
    M = read_golden(GOLDEN)
    n = 6
    g = np.arange(n)
    ijk = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1).T
    pos = ijk.astype(np.float64)
    q = np.where(ijk.sum(axis=1) % 2 == 0, 1.0, -1.0)
    box = np.array([6.0, 6.0, 6.0])
    r = ewald.direct_ewald(pos, q, box, beta=1.5, rcut=5.5, kmax=20)
    e_pair = r["E"] / (len(q) / 2)
    assert abs(e_pair + M) < 1e-11, (e_pair, -M)


def test_total_energy_independent_of_beta():
    pos, q, box = small_system()
    energies = []
    for beta in (0.6, 0.75, 0.9):
        r = ewald.direct_ewald(pos, q, box, beta=beta, rcut=9.0, kmax=16)
        energies.append(r["E"])
    # the split moves energy between the terms, the total must not change
    assert max(energies) - min(energies) < 1e-10 * abs(energies[0])


def test_non_neutral_beta_independence_needs_background_term():
    pos, q, box = small_system(seed=3)
    q = q + 0.2                                       # net charge
    e = [ewald.direct_ewald(pos, q, box, b, 9.0, 16)["E"] for b in (0.6, 0.9)]
    assert abs(e[0] - e[1]) < 1e-10 * abs(e[0])
    no_bg = [ewald.direct_ewald(pos, q, box, b, 9.0, 16) for b in (0.6, 0.9)]
    no_bg = [d["E"] - d["E_neutral"] for d in no_bg]
    assert abs(no_bg[0] - no_bg[1]) > 1e-3


def test_newton_third_law():
    pos, q, box = small_system()
    r = ewald.direct_ewald(pos, q, box, beta=0.75, rcut=9.0, kmax=16)
    fscale = np.abs(r["F"]).max()
    assert np.abs(r["F_real"].sum(axis=0)).max() < 1e-12 * fscale
    assert np.abs(r["F_rec"].sum(axis=0)).max() < 1e-12 * fscale


def test_forces_central_differences():
    pos, q, box = small_system(n=12)
    beta, rc, km = 0.75, 9.0, 16
    r = ewald.direct_ewald(pos, q, box, beta, rc, km)
    h = 1e-5
    for i in (0, 5, 11):
        for d in range(3):
            pp = pos.copy()
            pm = pos.copy()
            pp[i, d] += h
            pm[i, d] -= h
            ep = ewald.direct_ewald(pp, q, box, beta, rc, km)["E"]
            em = ewald.direct_ewald(pm, q, box, beta, rc, km)["E"]
            fd = -(ep - em) / (2 * h)
            assert abs(fd - r["F"][i, d]) < 1e-7 * max(1.0, abs(r["F"][i, d]))


def test_reciprocal_potential_gives_energy_and_force():
    pos, q, box = small_system(n=10)
    e, phi, f = ewald.reciprocal(pos, q, box, 0.8, 14)
    assert abs(0.5 * q @ phi - e) < 1e-12 * abs(e)
    h = 1e-5
    for d in range(3):
        pp = pos.copy()
        pm = pos.copy()
        pp[3, d] += h
        pm[3, d] -= h
        fd = -(ewald.reciprocal(pp, q, box, 0.8, 14)[0]
               - ewald.reciprocal(pm, q, box, 0.8, 14)[0]) / (2 * h)
        assert abs(fd - f[3, d]) < 1e-7 * max(1.0, abs(f[3, d]))
