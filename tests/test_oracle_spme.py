"""Pins of the FFT-based smooth-PME oracle against direct Ewald and identities."""
import itertools

import numpy as np
import pytest

from oracle import ewald, spme


def system(n=30, box=(8.0, 9.0, 10.0), seed=5, neutral=True):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 1, (n, 3)) * np.asarray(box)
    q = rng.uniform(-1, 1, n)
    if neutral:
        q -= q.mean()
    return pos, q, np.asarray(box, np.float64)


def test_converges_to_direct_ewald():
    """Energy, potentials and forces approach the exact reciprocal sum as the
    grid and the spline order grow (non-cubic box and grid)."""
    pos, q, box = system()
    beta = 0.9
    e_ref, phi_ref, f_ref = ewald.reciprocal(pos, q, box, beta, kmax=24)
    errs = []
    for K, p in [((16, 18, 20), 4), ((24, 27, 30), 6), ((40, 45, 50), 10)]:
        r = spme.spme(pos, q, box, K, p, beta)
        errs.append((abs(r["E_rec"] - e_ref) / abs(e_ref),
                     np.linalg.norm(r["phi"] - phi_ref) / np.linalg.norm(phi_ref),
                     np.linalg.norm(r["F"] - f_ref) / np.linalg.norm(f_ref)))
    for k in range(3):
        assert errs[0][k] > errs[1][k] > errs[2][k]
    assert errs[2][0] < 1e-9 and errs[2][1] < 1e-8 and errs[2][2] < 1e-7


def test_energy_identities():
    pos, q, box = system(neutral=False)
    K, p, beta = (12, 10, 14), 6, 0.7
    r = spme.spme(pos, q, box, K, p, beta)
    e_grid = 0.5 * float((r["Q"] * r["Phi"]).sum())
    e_modes = 0.5 * float((r["theta_hat"] * np.abs(np.fft.fftn(r["Q"])) ** 2).sum())
    assert abs(e_grid - r["E_rec"]) < 1e-12 * abs(r["E_rec"])
    assert abs(e_modes - r["E_rec"]) < 1e-12 * abs(r["E_rec"])


def test_fft_convolution_against_brute_force():
    """Phi(k) = sum_g theta_rec(k - g) Q(g), theta_rec(d) = sum_m th(m) e^{2 pi i m.d/K},
    evaluated by explicit sums on a tiny grid."""
    K = (4, 5, 6)
    box = np.array([3.0, 4.0, 5.0])
    th = spme.theta_hat(box, K, 4, 0.9)
    rng = np.random.default_rng(0)
    Q = rng.standard_normal(K)
    idx = list(itertools.product(*[range(k) for k in K]))
    Kv = np.array(K, np.float64)
    trec = np.zeros(K)
    for d in idx:
        s = 0.0
        for m in idx:
            s += th[m] * np.cos(2 * np.pi * np.dot(np.array(m) / Kv, d))
        trec[d] = s
    Phi_bf = np.zeros(K)
    for k in idx:
        Phi_bf[k] = sum(trec[tuple(np.mod(np.subtract(k, g), K))] * Q[g] for g in idx)
    np.testing.assert_allclose(spme.convolve_fft(Q, th), Phi_bf, rtol=1e-12,
                               atol=1e-14 * np.abs(Phi_bf).max())


def test_theta_hat_symmetry_and_zero_mode():
    K, box = (8, 10, 12), np.array([5.0, 6.0, 7.0])
    th = spme.theta_hat(box, K, 4, 0.8)
    assert th[0, 0, 0] == 0.0
    assert np.all(th.ravel()[1:] > 0)
    for ax in range(3):
        r = np.take(th, np.mod(-np.arange(K[ax]), K[ax]), axis=ax)
        np.testing.assert_allclose(r, th, rtol=1e-14)


def test_grid_shift_invariance():
    pos, q, box = system()
    K, p, beta = (12, 15, 16), 4, 0.8
    e0 = spme.spme(pos, q, box, K, p, beta)["E_rec"]
    shift = np.array([3 * box[0] / K[0], -box[1] / K[1], 5 * box[2] / K[2]])
    e1 = spme.spme(pos + shift, q, box, K, p, beta)["E_rec"]
    assert abs(e1 - e0) < 1e-11 * abs(e0)
    # an arbitrary shift only moves the energy by the discretisation error
    e2 = spme.spme(pos + np.array([0.123, 0.456, 0.789]), q, box, K, p, beta)["E_rec"]
    e_ref = ewald.reciprocal(pos, q, box, beta, 20)[0]
    assert abs(e2 - e0) < 4 * abs(e0 - e_ref) + 1e-12


def test_partition_of_unity_and_constant_potential():
    pos, q, box = system(neutral=False)
    K, p = (9, 10, 11), 6
    Q = spme.spread(pos, q, box, K, p)
    assert abs(Q.sum() - q.sum()) < 1e-13 * np.abs(q).sum()
    phi, F = spme.gather(pos, q, box, K, p, np.full(K, 2.5))
    np.testing.assert_allclose(phi, 2.5, rtol=1e-14)
    assert np.abs(F).max() < 1e-13


def test_spread_gather_adjoint():
    """sum_k Q(k) X(k) = sum_i q_i (gather of X)_i for any grid X."""
    pos, q, box = system(neutral=False)
    K, p = (9, 10, 11), 4
    X = np.random.default_rng(2).standard_normal(K)
    Q = spme.spread(pos, q, box, K, p)
    phi, _ = spme.gather(pos, q, box, K, p, X)
    assert abs((Q * X).sum() - q @ phi) < 1e-12 * np.abs(q @ phi)


@pytest.mark.parametrize("p", [4, 6])
def test_forces_central_differences(p):
    pos, q, box = system(n=16)
    K, beta = (12, 14, 16), 0.8
    r = spme.spme(pos, q, box, K, p, beta)
    h = 1e-6
    for i in (0, 7):
        for d in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, d] += h
            pm[i, d] -= h
            fd = -(spme.spme(pp, q, box, K, p, beta)["E_rec"]
                   - spme.spme(pm, q, box, K, p, beta)["E_rec"]) / (2 * h)
            assert abs(fd - r["F"][i, d]) < 1e-6 * max(1.0, abs(r["F"][i, d]))
