"""Pins of the per-cell Lagrange KPME oracle (Sec. 2.2, Sec. 4.1): the
Lagrange basis, the interpolation error of the exponentials against the
textbook remainder bound, the direct alpha_M sum against direct Ewald, the
convergence of the interpolated method to the direct alpha_M sum, full-rank
SKP equal to the FFT form, the correction, and finite differences."""
import numpy as np
import pytest

from oracle import ewald
from oracle import lagrange as lg
from oracle import skp, spme


@pytest.mark.parametrize("L", [2, 4, 5, 8])
def test_basis_is_cardinal_partition_of_unity_and_polynomial_exact(L):
    h = lg.nodes(L)
    np.testing.assert_allclose(lg.basis(h, L), np.eye(L), atol=1e-14)
    t = np.linspace(-1, 1, 97)
    S = lg.basis(t, L)
    np.testing.assert_allclose(S.sum(axis=1), 1.0, atol=1e-13)
    for k in range(L):                      # degree < L reproduced exactly
        np.testing.assert_allclose(S @ h ** k, t ** k, atol=1e-12)
    eps = 1e-6
    fd = (lg.basis(t + eps, L) - lg.basis(t - eps, L)) / (2 * eps)
    np.testing.assert_allclose(lg.dbasis(t, L), fd, atol=1e-7 * L ** 3)


@pytest.mark.parametrize("m,L", [(1, 4), (3, 6), (5, 8), (8, 8), (8, 12)])
def test_exponential_interpolation_within_the_lagrange_remainder_bound(m, L):
    """On a cell of width w = 2 (box 20, 10 cells): |e^{2 pi i m x / 20} -
    I[.](x)| <= (2 pi m / 20)^L / L! max |prod_s (x - x_s)| (the remainder
    the convergence rates of Thm. 3 rest on), and the error falls with L."""
    box, Kc = 20.0, 10
    x = np.linspace(0.0, 2.0, 2001)[:-1] + 4.0      # inside cell 2
    idx, W, _ = lg.stencil(x, box, Kc, L)
    K = Kc * (L - 1)
    grid_x = np.arange(K) * box / K
    f = np.exp(2j * np.pi * m * grid_x / box)
    interp = (W * f[idx]).sum(axis=1)
    err = np.abs(interp - np.exp(2j * np.pi * m * x / box)).max()
    xs = 4.0 + np.arange(L) * 2.0 / (L - 1)
    node_poly = np.abs(np.prod(x[:, None] - xs[None, :], axis=1)).max()
    fact = float(np.prod(np.arange(1, L + 1)))
    bound = (2 * np.pi * m / box) ** L / fact * node_poly
    assert err <= bound * (1 + 1e-9)
    if L >= 6:
        idx2, W2, _ = lg.stencil(x, box, Kc, L - 2)
        gx2 = np.arange(Kc * (L - 3)) * box / (Kc * (L - 3))
        err2 = np.abs((W2 * np.exp(2j * np.pi * m * gx2 / box)[idx2]).sum(axis=1)
                      - np.exp(2j * np.pi * m * x / box)).max()
        assert err < err2


def test_direct_alpha_m_equals_direct_ewald_reciprocal_sum():
    """With M = 12 on a 10^3 box at beta = 0.7 the Gaussian has decayed to
    e^{-29} at the cube's face, so the cube sum equals direct Ewald's sphere
    sum |m| <= 12 (module ewald, pinned by the Madelung constant)."""
    rng = np.random.default_rng(3)
    box = np.array([10.0, 10.0, 10.0])
    pos = rng.uniform(0, 1, (30, 3)) * box
    q = rng.uniform(-1, 1, 30)
    q -= q.mean()
    e, phi, F = lg.direct_alpha_m(pos, q, box, 12, 0.7)
    ref = ewald.reciprocal(pos, q, box, 0.7, 12.0)
    assert abs(e - ref[0]) < 1e-11 * abs(ref[0])
    np.testing.assert_allclose(phi, ref[1], atol=1e-11 * np.abs(ref[1]).max())
    np.testing.assert_allclose(F, ref[2], atol=1e-11 * np.abs(ref[2]).max())


def test_kpme_converges_to_the_direct_alpha_m_sum():
    """Finer interpolation (more nodes per cell) drives the interpolated
    method to the direct mode sum at the same M (non-neutral charges)."""
    rng = np.random.default_rng(4)
    box = np.array([10.0, 11.0, 12.0])
    pos = rng.uniform(0, 1, (25, 3)) * box
    q = rng.uniform(-1, 1, 25)
    M, beta = 5, 0.6
    e_ref, phi_ref, F_ref = lg.direct_alpha_m(pos, q, box, M, beta)
    errs = []
    for L in (4, 6, 8, 10, 12):
        r = lg.kpme_fft(pos, q, box, (4, 4, 4), L, M, beta)
        errs.append(np.abs(r["phi"] - phi_ref).max() / np.abs(phi_ref).max())
    assert all(a > 10 * b for a, b in zip(errs, errs[1:]))   # geometric
    assert errs[-1] < 1e-7
    assert abs(r["E_rec"] - e_ref) < 1e-7 * abs(e_ref)
    np.testing.assert_allclose(r["F"], F_ref, atol=1e-5 * np.abs(F_ref).max())


def test_full_rank_skp_equals_the_fft_form():
    rng = np.random.default_rng(5)
    box = np.array([9.0, 11.0, 13.0])
    pos = rng.uniform(0, 1, (30, 3)) * box
    q = rng.uniform(-1, 1, 30)                       # non-neutral
    Kc, L, M, beta = (2, 3, 3), 5, 3, 0.7
    pl = lg.Plan(box, Kc, L, M, beta)
    a = pl.evaluate(pos, q)
    b = lg.kpme_fft(pos, q, box, Kc, L, M, beta)
    assert abs(a["E_rec"] - b["E_rec"]) < 1e-12 * abs(b["E_rec"])
    np.testing.assert_allclose(a["phi"], b["phi"], atol=1e-12 * np.abs(b["phi"]).max())
    np.testing.assert_allclose(a["F"], b["F"], atol=1e-12 * np.abs(b["F"]).max())


def test_correction_removes_the_truncated_zero_mode():
    rng = np.random.default_rng(6)
    box = np.array([9.0, 11.0, 13.0])
    pos = rng.uniform(0, 1, (30, 3)) * box
    q = rng.uniform(-1, 1, 30)
    Kc, L, M, beta = (2, 3, 3), 5, 3, 0.7
    pl = lg.Plan(box, Kc, L, M, beta, rank=5)
    Q = lg.spread(pos, q, box, Kc, L)
    th = skp.reconstruct(pl.terms, pl.K)
    assert abs(th[0, 0, 0] - pl.c0) < 1e-14 * abs(pl.c0) and abs(pl.c0) > 0
    th[0, 0, 0] = 0.0
    ref = spme.convolve_fft(Q, th)
    np.testing.assert_allclose(pl.apply(Q), ref, atol=1e-12 * np.abs(ref).max())


def test_modes_beyond_m_are_zero_and_aliasing_is_refused():
    a = lg.alpha_hat((10.0, 10.0, 10.0), (12, 12, 12), 4, 0.7)
    mp = spme.signed_modes(12)
    assert np.all(a[np.abs(mp) > 4] == 0) and np.all(a[:, np.abs(mp) > 4] == 0)
    assert np.all(a[1:5, 1:5, 1:5] > 0)
    with pytest.raises(ValueError):
        lg.alpha_hat((10.0, 10.0, 10.0), (12, 12, 12), 6, 0.7)


def test_forces_are_minus_the_energy_gradient():
    rng = np.random.default_rng(7)
    box = np.array([10.0, 11.0, 12.0])
    pos = rng.uniform(0, 1, (20, 3)) * box
    q = rng.uniform(-1, 1, 20)
    q -= q.mean()
    Kc, L, M, beta = (3, 3, 3), 6, 5, 0.6
    r = lg.kpme_fft(pos, q, box, Kc, L, M, beta)
    h = 1e-5
    for i, j in ((0, 0), (3, 1), (7, 2)):
        p1, p2 = pos.copy(), pos.copy()
        p1[i, j] += h
        p2[i, j] -= h
        e1 = lg.kpme_fft(p1, q, box, Kc, L, M, beta)["E_rec"]
        e2 = lg.kpme_fft(p2, q, box, Kc, L, M, beta)["E_rec"]
        assert abs(-(e1 - e2) / (2 * h) - r["F"][i, j]) < 1e-6 * np.abs(r["F"]).max()
