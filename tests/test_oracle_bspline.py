"""Pins of the oracle's cardinal B-splines against closed forms and identities."""
import numpy as np
import pytest

from oracle import bspline


def cubic_closed_form(u):
    """M_4 written piecewise (the cubic cardinal B-spline)."""
    u = np.asarray(u, np.float64)
    out = np.zeros_like(u)
    a = (u >= 0) & (u < 1)
    b = (u >= 1) & (u < 2)
    c = (u >= 2) & (u < 3)
    d = (u >= 3) & (u <= 4)
    out[a] = u[a] ** 3 / 6
    out[b] = (-3 * u[b] ** 3 + 12 * u[b] ** 2 - 12 * u[b] + 4) / 6
    out[c] = (3 * u[c] ** 3 - 24 * u[c] ** 2 + 60 * u[c] - 44) / 6
    out[d] = (4 - u[d]) ** 3 / 6
    return out


def test_cubic_matches_closed_form():
    u = np.linspace(-1.0, 5.0, 1201)
    np.testing.assert_allclose(bspline.mp(u, 4), cubic_closed_form(u), atol=1e-15)


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6, 7, 8, 10])
def test_partition_unity_integral_symmetry_support(p):
    f = np.linspace(0.0, 1.0, 101)
    s = sum(bspline.mp(f + t, p) for t in range(p))
    np.testing.assert_allclose(s, 1.0, atol=1e-14)
    u = np.linspace(0.0, p, 20001)
    integral = np.trapezoid(bspline.mp(u, p), u)
    assert abs(integral - 1.0) < 1e-7
    np.testing.assert_allclose(bspline.mp(u, p), bspline.mp(p - u, p), atol=1e-14)
    assert np.all(bspline.mp(np.array([-0.5, -1e-3, p + 1e-3, p + 2.0]), p) == 0.0)


@pytest.mark.parametrize("p", [3, 4, 6, 8])
def test_derivative_central_difference(p):
    u = np.linspace(0.05, p - 0.05, 397)
    h = 1e-6
    fd = (bspline.mp(u + h, p) - bspline.mp(u - h, p)) / (2 * h)
    np.testing.assert_allclose(bspline.dmp(u, p), fd, atol=2e-8)


@pytest.mark.parametrize("K,p", [(16, 4), (17, 4), (24, 6), (32, 8), (10, 2)])
def test_bmod_exact_interpolation_at_grid_points(K, p):
    """|b(m)|^2 |sum_k M_p(u - k) e^{2 pi i m k / K}|^2 = 1 at integer u.

    At integer u the B-spline interpolant of e^{2 pi i m u/K} is exact up to
    the factor b(m); this characterises |b(m)|^2 independently of the form in
    which the oracle writes it (index range and spline argument included).
    """
    b2 = bspline.bmod2(K, p)
    m = np.arange(K)
    for u0 in [0, 3, K - 1]:
        k = np.arange(-3 * K, 3 * K)
        w = bspline.mp(u0 - k, p)                    # all periodic images
        s = (w[None, :] * np.exp(2j * np.pi * np.outer(m, k) / K)).sum(axis=1)
        np.testing.assert_allclose(b2 * np.abs(s) ** 2, 1.0, rtol=1e-12)


def test_bmod_interpolation_converges_off_grid():
    """Off the grid the exponential-spline interpolant converges with p."""
    K, m, u0 = 32, 3, 5.37
    errs = []
    for p in (4, 6, 8):
        k = np.arange(-2 * K, 2 * K)
        s = (bspline.mp(u0 - k, p) * np.exp(2j * np.pi * m * k / K)).sum()
        # |b(m)| * |interpolant| approximates |e^{...}| = 1
        errs.append(abs(np.sqrt(bspline.bmod2(K, p)[m]) * abs(s) - 1.0))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-6


def test_stencil_weights_and_wrap():
    K, p = 8, 4
    u = np.array([0.0, 0.25, 7.999, 8.0, 3.5])
    idx, w, dw = bspline.stencil(u, K, p)
    np.testing.assert_allclose(w.sum(axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(dw.sum(axis=1), 0.0, atol=1e-14)
    assert idx.min() >= 0 and idx.max() < K
    # u = K is the same point as u = 0
    np.testing.assert_array_equal(idx[3], idx[0])
    np.testing.assert_allclose(w[3], w[0])
    # the weight on k is M_p(u - k) taken mod K
    for i, uu in enumerate(u):
        for t in range(p):
            k = idx[i, t]
            d = (uu - k) % K
            assert abs(w[i, t] - bspline.mp(d, p)) < 1e-14
