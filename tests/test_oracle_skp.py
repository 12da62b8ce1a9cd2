"""Pins of the SKP oracle: nested-SVD exactness and truncation identities,
circulant factors, mode-product orientation, equality with FFT-based SPME at
full rank, the constant correction, symmetry and the energy bound."""
import itertools

import numpy as np
import pytest

from oracle import skp, spme

BOX = np.array([9.0, 11.0, 13.0])
K = (8, 10, 12)


def system(n=40, seed=7, neutral=True):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 1, (n, 3)) * BOX
    q = rng.uniform(-1, 1, n)
    if neutral:
        q -= q.mean()
    return pos, q


@pytest.fixture(scope="module")
def full_plan():
    return skp.Plan(BOX, K, 4, 0.7)


def test_full_rank_reconstruction(full_plan):
    th = full_plan.theta
    rec = skp.reconstruct(full_plan.all_terms, th.shape)
    assert np.abs(rec - th).max() < 1e-13 * th.max()


def test_terms_orthonormal_and_sorted(full_plan):
    t = full_plan.all_terms
    w = np.array([x[0] for x in t])
    assert np.all(np.diff(w) <= 0)
    for k in (0, 3, 10):
        for v in t[k][1:4]:
            assert abs(np.linalg.norm(v) - 1.0) < 1e-12
    # rank-1 tensors of distinct terms are orthogonal
    def flat(x):
        return (x[1][:, None, None] * x[2][None, :, None] * x[3][None, None, :]).ravel()
    G = np.array([flat(x) for x in t[:12]])
    np.testing.assert_allclose(G @ G.T, np.eye(12), atol=1e-12)


@pytest.mark.parametrize("R", [1, 3, 8, 20])
def test_truncation_identity_and_svd_bound(full_plan, R):
    th = full_plan.theta
    kept = full_plan.all_terms[:R]
    actual = np.linalg.norm(th - skp.reconstruct(kept, th.shape))
    tail = np.sqrt(sum(x[0] ** 2 for x in full_plan.all_terms[R:]))
    assert abs(actual - tail) <= 1e-10 * np.linalg.norm(th) + 1e-6 * actual
    assert skp.svd_bound(th, full_plan.all_terms, kept) >= actual * (1 - 1e-12)


def test_tolerance_selection_is_minimal():
    pl = skp.Plan(BOX, K, 4, 0.7, tol=1e-5)
    nrm = np.linalg.norm(pl.theta)
    err_R = np.linalg.norm(pl.theta - skp.reconstruct(pl.terms, pl.theta.shape))
    err_Rm1 = np.linalg.norm(pl.theta - skp.reconstruct(pl.terms[:-1], pl.theta.shape))
    assert err_R <= 1e-5 * nrm * (1 + 1e-9) and err_Rm1 > 1e-5 * nrm


def test_circulant_factor_is_symmetric_with_the_mode_vector_as_spectrum(full_plan):
    w, x, y, u, _, _ = full_plan.all_terms[2]
    for a in (x, y, u):
        A, im = skp.circulant(a)
        n = len(a)
        assert im < 1e-12
        np.testing.assert_allclose(A, A.T, atol=1e-14)
        np.testing.assert_allclose(np.roll(np.roll(A, 1, 0), 1, 1), A, atol=1e-14)
        # A e_m = n a(m) e_m for the Fourier vector e_m(h) = exp(2 pi i m h / n)
        for m in (0, 1, n // 2):
            e = np.exp(2j * np.pi * m * np.arange(n) / n)
            np.testing.assert_allclose(A @ e, n * a[m] * e, atol=1e-12)


def test_mode_products_equal_dense_kronecker():
    """One term applied by the oracle equals (A (x) B (x) C) vec(Q) with the
    grid stored row-major (k3 fastest)."""
    rng = np.random.default_rng(1)
    shp = (3, 4, 5)
    A, B, C = (rng.standard_normal((n, n)) for n in shp)
    Q = rng.standard_normal(shp)
    out = skp.apply(Q, [(1.0, A, B, C)], 0.0)
    dense = np.kron(np.kron(A, B), C) @ Q.ravel()
    np.testing.assert_allclose(out.ravel(), dense, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("neutral", [True, False])
@pytest.mark.parametrize("p", [4, 6])
def test_full_rank_equals_fft_spme(neutral, p):
    pos, q = system(neutral=neutral)
    pl = skp.Plan(BOX, K, p, 0.7)
    a = pl.evaluate(pos, q)
    b = spme.spme(pos, q, BOX, K, p, 0.7)
    assert abs(a["E_rec"] - b["E_rec"]) < 1e-12 * abs(b["E_rec"])
    np.testing.assert_allclose(a["phi"], b["phi"], atol=1e-12 * np.abs(b["phi"]).max())
    np.testing.assert_allclose(a["F"], b["F"], atol=1e-12 * np.abs(b["F"]).max())


def test_correction_removes_zero_mode_of_truncated_symbol():
    """Truncated SKP + correction == FFT convolution with the truncated symbol
    whose m = 0 value is zeroed; without the correction they differ by exactly
    theta_R(0) * sum(Q) (the sign of the correction)."""
    pos, q = system(neutral=False)
    pl = skp.Plan(BOX, K, 4, 0.7, rank=6)
    Q = spme.spread(pos, q, BOX, K, 4)
    th_R = skp.reconstruct(pl.terms, pl.theta.shape)
    c0 = th_R[0, 0, 0]
    assert abs(c0 - pl.c0) < 1e-14 * abs(c0) and abs(c0) > 1e-6 * pl.theta.max()
    th_R0 = th_R.copy()
    th_R0[0, 0, 0] = 0.0
    ref = spme.convolve_fft(Q, th_R0)
    out = pl.apply(Q)
    np.testing.assert_allclose(out, ref, atol=1e-12 * np.abs(ref).max())
    uncorrected = skp.apply(Q, pl.facs, 0.0)
    np.testing.assert_allclose(uncorrected - out, c0 * Q.sum(), rtol=1e-10)


def test_operator_symmetry():
    pl = skp.Plan(BOX, K, 4, 0.7, rank=9)
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal(K), rng.standard_normal(K)
    a = float((x * pl.apply(y)).sum())
    b = float((y * pl.apply(x)).sum())
    assert abs(a - b) < 1e-12 * max(abs(a), 1.0)


@pytest.mark.parametrize("R", [2, 5, 12])
def test_energy_error_bound(R):
    """|E_R - E| <= 1/2 ||theta_R - theta||_inf * G * sum_k Q(k)^2 (Parseval)."""
    pos, q = system()
    pl_R = skp.Plan(BOX, K, 4, 0.7, rank=R)
    e_R = pl_R.evaluate(pos, q)["E_rec"]
    ex = spme.spme(pos, q, BOX, K, 4, 0.7)
    th_R = skp.reconstruct(pl_R.terms, pl_R.theta.shape)
    th_R[0, 0, 0] = 0.0
    G = np.prod(K)
    bound = 0.5 * np.abs(th_R - pl_R.theta).max() * G * float((ex["Q"] ** 2).sum())
    assert abs(e_R - ex["E_rec"]) <= bound


def test_neutral_systems_ignore_the_zero_mode_value():
    pos, q = system()
    pl = skp.Plan(BOX, K, 4, 0.7, rank=7)
    Q = spme.spread(pos, q, BOX, K, 4)
    a = skp.apply(Q, pl.facs, pl.c0)
    b = skp.apply(Q, pl.facs, 123.0)
    assert np.abs(a - b).max() < 1e-11 * np.abs(a).max()


def test_axis_order_matters_on_non_cubic_grids():
    """Separating axis 2 first (the paper's order) is a definite choice: the
    first SVD's singular values are those of the axis-2 unfolding."""
    pl = skp.Plan(BOX, K, 4, 0.7)
    th = pl.theta
    s2 = np.linalg.svd(np.transpose(th, (2, 0, 1)).reshape(K[2], -1), compute_uv=False)
    outer = {}
    for t in pl.all_terms:
        outer.setdefault(t[4], 0.0)
        outer[t[4]] += t[0] ** 2
    got = np.sqrt(np.array([outer[i] for i in sorted(outer)]))
    np.testing.assert_allclose(got, s2[:len(got)], rtol=1e-10)
