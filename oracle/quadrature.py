"""Sinc-quadrature Sum of Kronecker Products (oracle; test infrastructure).

The second construction of the kernel's SKP in the paper (Sec. 2.1.2,
Eqs. one_over_r_int and quaddecompalpham): write 1/x as the integral of
exp(-t x) over t > 0 and discretise it with the cardinal-sine (sinc) rule

    omega_l = h / (1 + exp(-l h)),  lambda_l = log(1 + exp(l h)),  l = -N..N,

so that 1/x ~ sum_l omega_l exp(-lambda_l x).  The Gaussian factor of the
kernel and exp(-lambda x) both factor over the axes, so every node is one
Kronecker term and no SVD is needed.

Applied to the smooth-PME symbol (module ``spme``; this plays the paper's
alpha_M with alpha(0) = 0):

    theta_hat(m) = exp(-pi^2 |m_hat|^2 / beta^2) / (pi V |m_hat|^2) prod_j |b_j(m_j)|^2.

Reading (the paper states the rule for integer modes, where |m|^2 >= 1 for
every m != 0): with box lengths, |m_hat|^2 = sum_j (m'_j / L_j)^2 can be
below 1, so the quadrature is applied to x = s |m_hat|^2 with
s = max_j L_j^2, which makes x >= 1 for every m != 0:
1 / |m_hat|^2 = s / x ~ s sum_l omega_l exp(-lambda_l s |m_hat|^2).  Term l then
has weight s omega_l / (pi V) and per-axis mode vectors

    a_{l,j}(m) = |b_j(m)|^2 exp(-(s lambda_l + pi^2 / beta^2) (m'_j / L_j)^2),

and the operator's value at m = 0 is c_Lambda = s sum_l omega_l / (pi V), the
constant the correction removes (Eq. quaddecompalpham: the paper's
c_Lambda = sum_l omega_l, here with the s / (pi V) scaling).

The lifting factor h: the paper tries several values of h for each N by
brute force, measuring the error on every argument |m|^2 that occurs, and
keeps the best.  Here the error of a rule is the largest symbol error over
the mode grid relative to the largest symbol value,
max_{m != 0} |theta_Lambda(m) - theta_hat(m)| / max theta_hat, and the
candidates are h0 2^(k/8), k = -24..16, around the asymptotic choice
h0 = pi / sqrt(2N + 1).  For a tolerance, N is the smallest whose best h
meets it.

Terms are returned in the nested-SVD oracle's format (unit vectors, weight
omega, one group per term), so ``skp.factors`` and ``skp.apply`` evaluate
them unchanged.

Pinned by: the rule integrating other closed-form integrals over (0, inf),
the exponential sum converging to 1/x, the term reconstruction converging to
the FFT smooth-PME symbol, the correction constant against the reconstruction
at m = 0, the selection's error bound and minimality, and the full quadrature
SKP-PME against FFT smooth PME -- tests/test_oracle_quadrature.py.
"""
import numpy as np

from . import bspline, skp, spme


def sinc_rule(N, h):
    """Weights and nodes of the sinc rule for integrals over (0, inf)."""
    l = np.arange(-N, N + 1, dtype=np.float64)
    omega = h / (1.0 + np.exp(-l * h))
    lam = np.log1p(np.exp(l * h))
    return omega, lam


def exp_sum(x, N, h):
    """sum_l omega_l exp(-lambda_l x), the rule's approximation of 1/x."""
    omega, lam = sinc_rule(N, h)
    x = np.asarray(x, np.float64)
    return (omega[None, :] * np.exp(-np.outer(x.ravel(), lam))).sum(axis=1).reshape(x.shape)


def arg_scale(box):
    """s = max_j L_j^2: x = s |m_hat|^2 >= 1 for every non-zero mode."""
    return float(np.max(np.asarray(box, np.float64)) ** 2)


def mode_args(box, K):
    """x(m) = s |m_hat|^2 on the full mode grid (x(0) = 0)."""
    box = np.asarray(box, np.float64)
    mh2 = [(spme.signed_modes(K[j]) / box[j]) ** 2 for j in range(3)]
    m2 = mh2[0][:, None, None] + mh2[1][None, :, None] + mh2[2][None, None, :]
    return arg_scale(box) * m2


def terms(box, K, p, beta, N, h):
    """The 2N+1 Kronecker terms (omega, x, y, u, l, 0), unit vectors."""
    box = np.asarray(box, np.float64)
    V = float(np.prod(box))
    s = arg_scale(box)
    omega, lam = sinc_rule(N, h)
    bm = [bspline.bmod2(K[j], p) for j in range(3)]
    mh2 = [(spme.signed_modes(K[j]) / box[j]) ** 2 for j in range(3)]
    out = []
    for l in range(len(omega)):
        vecs, norm = [], 1.0
        for j in range(3):
            a = bm[j] * np.exp(-(s * lam[l] + np.pi ** 2 / beta ** 2) * mh2[j])
            n = np.linalg.norm(a)
            vecs.append(a / n)
            norm *= n
        out.append((s * omega[l] / (np.pi * V) * norm, vecs[0], vecs[1], vecs[2], l, 0))
    return out


def correction_constant(box, N, h):
    """c_Lambda = s sum_l omega_l / (pi V)."""
    box = np.asarray(box, np.float64)
    omega, _ = sinc_rule(N, h)
    return arg_scale(box) * float(omega.sum()) / (np.pi * float(np.prod(box)))


def _weighted_args(box, K, p, beta):
    """Distinct non-zero arguments x with the largest relative symbol value
    theta_hat / max theta_hat among the modes that share them."""
    th = spme.theta_hat(box, K, p, beta)
    x = mode_args(box, K).ravel()
    w = (th / th.max()).ravel()
    keep = x > 0
    ux, inv = np.unique(x[keep], return_inverse=True)
    wmax = np.zeros(len(ux))
    np.maximum.at(wmax, inv, w[keep])
    return ux, wmax


def symbol_error(box, K, p, beta, N, h, _args=None):
    """max_{m != 0} |theta_Lambda(m) - theta_hat(m)| / max theta_hat.

    For m != 0, theta_Lambda(m) = theta_hat(m) * x * exp_sum(x) with
    x = s |m_hat|^2 (the kernel's factors other than 1/x are kept exactly),
    so the error is theta_hat(m) |x exp_sum(x) - 1|; it is evaluated once per
    distinct argument with the largest theta_hat that has it."""
    ux, wmax = _args if _args is not None else _weighted_args(box, K, p, beta)
    return float((wmax * np.abs(ux * exp_sum(ux, N, h) - 1.0)).max())


def h_candidates(N):
    h0 = np.pi / np.sqrt(2 * N + 1)
    return h0 * 2.0 ** (np.arange(-24, 17) / 8.0)


def best_h(box, K, p, beta, N, _args=None):
    """Brute-force choice of h for a given N: (h, error)."""
    args = _args if _args is not None else _weighted_args(box, K, p, beta)
    errs = [symbol_error(box, K, p, beta, N, h, args) for h in h_candidates(N)]
    k = int(np.argmin(errs))
    return float(h_candidates(N)[k]), float(errs[k])


def select(box, K, p, beta, tol, n_max=400):
    """Smallest N whose best h has symbol_error <= tol: (N, h, error)."""
    args = _weighted_args(box, K, p, beta)
    for N in range(0, n_max + 1):
        h, e = best_h(box, K, p, beta, N, args)
        if e <= tol:
            return N, h, e
    raise ValueError("no sinc rule with N <= n_max meets the tolerance")


class Plan(skp.Plan):
    """Oracle plan with sinc-quadrature terms (N, h given, or N from tol)."""

    def __init__(self, box, K, p, beta, N=None, h=None, tol=None):
        self.box = np.asarray(box, np.float64)
        self.K = tuple(int(k) for k in K)
        self.p = int(p)
        self.beta = float(beta)
        if N is None:
            N, h, _ = select(self.box, self.K, self.p, self.beta, tol)
        elif h is None:
            h, _ = best_h(self.box, self.K, self.p, self.beta, N)
        self.N, self.h = int(N), float(h)
        self.theta = spme.theta_hat(self.box, self.K, self.p, self.beta)
        self.terms = terms(self.box, self.K, self.p, self.beta, self.N, self.h)
        self.all_terms = self.terms
        self.rank = len(self.terms)
        self.r0 = self.rank
        self.facs = skp.factors(self.terms)
        self.c0 = skp.zero_mode_value(self.terms)
        self.sym_err = symbol_error(self.box, self.K, self.p, self.beta, self.N, self.h)
        recon = skp.reconstruct(self.terms, self.K)
        self.trunc_err = float(np.sqrt(((recon - self.theta) ** 2).sum()))
