"""Pins of the rectangular cos/sin factor oracle (Sec. 2.3 Eq. kronw, Sec. 2.4
Eq. VtV): V^T S V against the complex-exponential circulant, the
orthogonality of the real Fourier rows, and the operator applied through two
thin products per mode product against the circulant mode products."""
import numpy as np
import pytest

from oracle import lagrange as lg
from oracle import quadrature as qd
from oracle import rect, skp, spme


@pytest.mark.parametrize("K,M", [(8, 4), (9, 4), (12, 3), (35, 12), (16, 8)])
def test_real_rows_are_orthogonal(K, M):
    F, modes = rect.real_rows(K, M)
    G = F @ F.T
    expect = np.array([K if m == 0 or 2 * m == K else K / 2 for m in modes], float)
    np.testing.assert_allclose(G, np.diag(expect), atol=1e-10)
    assert F.shape == (len(modes), K) and len(modes) == min(2 * M + 1, K)


@pytest.mark.parametrize("K,M", [(8, 4), (9, 4), (12, 3), (35, 12)])
def test_vtsv_equals_the_exponential_circulant(K, M):
    rng = np.random.default_rng(K + M)
    a = np.zeros(K)
    half = rng.standard_normal(M + 1)               # signed, like SVD vectors
    for m in range(M + 1):
        a[m] = half[m]
        a[(-m) % K] = half[m]
    V, S, F, d = rect.rect_factor(a, M)
    assert V.shape[0] == min(2 * M + 1, K)
    np.testing.assert_allclose(V.T @ (S[:, None] * V), rect.circulant_of(a), atol=1e-12)


def test_quadrature_factors_have_nonnegative_weights():
    """The sinc-quadrature mode vectors are positive: A = V^T V exactly as in
    Eq. VtV (S = I)."""
    box, K, p, beta = (20.0, 20.0, 20.0), (16, 16, 16), 4, 0.35
    for (w, x, y, u, _, _) in qd.terms(box, K, p, beta, 5, 0.9):
        for vec in (x, y, u):
            _, S, _, _ = rect.rect_factor(vec)
            assert np.all(S > 0)


@pytest.mark.parametrize("kind", ["bspline", "lagrange"])
def test_operator_through_rectangular_factors_equals_the_circulant_one(kind):
    rng = np.random.default_rng(8)
    if kind == "bspline":
        pl = skp.Plan((9.0, 11.0, 13.0), (8, 10, 12), 4, 0.7, rank=9)
        M = (None, None, None)
    else:
        pl = lg.Plan((10.0, 11.0, 12.0), (2, 3, 3), 5, 3, 0.6, rank=7)
        M = (3, 3, 3)
        for j in range(3):
            for t in pl.terms:
                assert rect.mode_cut(t[1 + j], 1e-14) <= 3
    Q = rng.standard_normal(pl.K)
    np.testing.assert_allclose(rect.apply(Q, pl.terms, pl.c0, M), pl.apply(Q),
                               atol=1e-12 * np.abs(pl.apply(Q)).max())
