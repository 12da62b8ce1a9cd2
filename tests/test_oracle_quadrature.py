"""Pins of the sinc-quadrature SKP oracle (Sec. 2.1.2): the rule against
closed-form integrals, the exponential sum against 1/x, the Kronecker terms
against the FFT smooth-PME symbol, the correction constant, the brute-force
selection of (N, h), and the quadrature SKP-PME against FFT smooth PME."""
import numpy as np
import pytest

from oracle import quadrature as qd
from oracle import skp, spme

BOX = np.array([9.0, 11.0, 13.0])
K = (8, 10, 12)
P, BETA = 4, 0.7


def system(n=40, seed=7, neutral=True):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 1, (n, 3)) * BOX
    q = rng.uniform(-1, 1, n)
    if neutral:
        q -= q.mean()
    return pos, q


@pytest.mark.parametrize("g,exact", [
    (lambda t: np.exp(-t), 1.0),
    (lambda t: np.exp(-3.0 * t), 1.0 / 3.0),
    (lambda t: t * np.exp(-2.0 * t), 0.25),
    (lambda t: t * t * np.exp(-t), 2.0),
    (lambda t: np.exp(-t) * np.cos(t), 0.5),
])
def test_rule_integrates_closed_forms_over_the_half_line(g, exact):
    """The weights and nodes come from t = log(1 + e^s) and the trapezoidal
    rule in s: sum_l omega_l g(lambda_l) -> int_0^inf g(t) dt for any g that
    decays exponentially (a dropped Jacobian or a wrong node fails this)."""
    omega, lam = qd.sinc_rule(120, np.pi / np.sqrt(241.0))
    assert abs(float((omega * g(lam)).sum()) - exact) < 1e-7 * max(1.0, exact)


def test_exponential_sum_converges_to_the_inverse():
    x = np.logspace(0.0, 3.0, 301)
    errs = []
    for N in (10, 30, 120):
        h, _ = min(((h, np.abs(x * qd.exp_sum(x, N, h) - 1).max()) for h in qd.h_candidates(N)),
                   key=lambda t: t[1])
        errs.append(np.abs(x * qd.exp_sum(x, N, h) - 1).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6


def test_terms_reconstruct_the_smooth_pme_symbol():
    """At a converged rule the terms rebuild theta_hat (module spme, the FFT
    smooth-PME kernel) at every m != 0, and their value at m = 0 is the
    correction constant c_Lambda = s sum omega / (pi V)."""
    N, h, err = qd.select(BOX, K, P, BETA, 1e-12)
    th = spme.theta_hat(BOX, K, P, BETA)
    rec = skp.reconstruct(qd.terms(BOX, K, P, BETA, N, h), th.shape)
    c = qd.correction_constant(BOX, N, h)
    assert abs(rec[0, 0, 0] - c) < 1e-13 * c
    rec[0, 0, 0] = 0.0
    assert np.abs(rec - th).max() < 1e-11 * th.max()


@pytest.mark.parametrize("N", [3, 8, 15])
def test_symbol_error_equals_the_reconstructed_error(N):
    """The per-argument error used to choose h equals the error of the
    reconstructed term sum over the whole mode grid."""
    h, err = qd.best_h(BOX, K, P, BETA, N)
    th = spme.theta_hat(BOX, K, P, BETA)
    rec = skp.reconstruct(qd.terms(BOX, K, P, BETA, N, h), th.shape)
    rec[0, 0, 0] = 0.0
    direct = np.abs(rec - th).max() / th.max()
    assert abs(direct - err) <= 1e-12 + 1e-9 * direct


@pytest.mark.parametrize("tol", [1e-3, 1e-6])
def test_selection_meets_tolerance_and_is_minimal(tol):
    N, h, err = qd.select(BOX, K, P, BETA, tol)
    assert err <= tol
    if N > 0:
        _, err_prev = qd.best_h(BOX, K, P, BETA, N - 1)
        assert err_prev > tol
    pl = qd.Plan(BOX, K, P, BETA, tol=tol)
    assert (pl.N, pl.h, pl.rank, pl.r0) == (N, h, 2 * N + 1, 2 * N + 1)


def test_quadrature_skp_pme_matches_fft_spme():
    """With a converged rule the whole oracle path (spread, three mode
    products per quadrature term, correction, gather) equals FFT smooth PME,
    on a non-neutral system so the correction matters."""
    pos, q = system(neutral=False)
    pl = qd.Plan(BOX, K, P, BETA, tol=1e-13)
    a = pl.evaluate(pos, q)
    b = spme.spme(pos, q, BOX, K, P, BETA)
    assert abs(a["E_rec"] - b["E_rec"]) < 1e-10 * abs(b["E_rec"])
    np.testing.assert_allclose(a["phi"], b["phi"], atol=1e-10 * np.abs(b["phi"]).max())
    np.testing.assert_allclose(a["F"], b["F"], atol=1e-10 * np.abs(b["F"]).max())


def test_correction_removes_the_quadrature_zero_mode():
    """Quadrature SKP + correction == FFT convolution with the quadrature
    symbol whose m = 0 value is zeroed (non-neutral charges)."""
    pos, q = system(neutral=False)
    pl = qd.Plan(BOX, K, P, BETA, N=4)
    Q = spme.spread(pos, q, BOX, K, P)
    th_L = skp.reconstruct(pl.terms, K)
    assert abs(th_L[0, 0, 0] - pl.c0) < 1e-13 * abs(pl.c0)
    th_L[0, 0, 0] = 0.0
    ref = spme.convolve_fft(Q, th_L)
    np.testing.assert_allclose(pl.apply(Q), ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("N", [2, 6])
def test_energy_error_bound(N):
    """|E_Lambda - E| <= 1/2 ||theta_Lambda - theta||_inf * G * sum_k Q(k)^2."""
    pos, q = system()
    pl = qd.Plan(BOX, K, P, BETA, N=N)
    e_L = pl.evaluate(pos, q)["E_rec"]
    ex = spme.spme(pos, q, BOX, K, P, BETA)
    bound = 0.5 * pl.sym_err * pl.theta.max() * np.prod(K) * float((ex["Q"] ** 2).sum())
    assert abs(e_L - ex["E_rec"]) <= bound * (1 + 1e-9)
