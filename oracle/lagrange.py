"""Paper-faithful KPME with per-cell Lagrange interpolation (oracle; test
infrastructure).

The paper's own discretisation (Sec. 2.2 and Sec. 4.1): the box is cut into
K_c cells per axis; on each cell an equispaced product grid of L nodes per
axis, end points included (Eq. interp1d with nodes -1 = h_0 < ... <
h_{L-1} = 1 mapped onto the cell), carries the Lagrange interpolation of
every particle of that cell (Eq. interpnd); the kernel is the mode-truncated
alpha_M, every mode with |m_j| <= M (Sec. 1.2, Eq. sumhexpr; Sec. 2.1).

Readings:

* Normalisation as for smooth PME (Cartesian units): the operator applied to
  the charges is phi(x) = (1 / (pi V)) sum_{0 < |m|_inf <= M}
  exp(-pi^2 |m_hat|^2 / beta^2) / |m_hat|^2 Re(S(m) exp(-2 pi i m_hat . x)),
  m_hat = m / L (``direct_alpha_m``): the paper's H_M q with its missing
  1/(pi V) restored (tin-foil boundary, alpha(0) = 0).
* Shared boundary nodes: the last node of cell c and the first of cell c+1
  are the same point, and the operator depends on node positions only, so
  the K_c L nodes per axis collapse to one periodic, equispaced grid of
  K = K_c (L - 1) points; a particle in cell c uses grid points
  c (L - 1) + s, s = 0..L-1 (mod K).  A particle on a cell boundary belongs
  to the cell above it (the paper assigns such particles arbitrarily).
* Kernel on that grid: the per-axis Fourier matrices of the nodes turn the
  interactions between cells (the block matrix of Sec. 4.1) into one
  periodic convolution on the K-point grid with symbol
  alpha_hat(m) = exp(-pi^2 |m_hat|^2 / beta^2) / (pi V |m_hat|^2) for
  0 < |m'_j| <= M on every axis and 0 otherwise (no B-spline moduli: the
  interpolation is of the exponentials themselves); 2M + 1 <= K is
  required so that no two retained modes alias on the grid.
* The SKP of alpha_hat is built exactly as for smooth PME (module ``skp``:
  nested SVD, circulant factors, mode products, correction).

Pinned by: the Lagrange basis (cardinality at the nodes, partition of unity,
exact reproduction of polynomials of degree < L, central differences), the
textbook Lagrange remainder bound for e^{2 pi i m x / L} on a cell (the
convergence the paper's Thm. 3 relies on), the direct alpha_M sum against
direct Ewald's reciprocal sum when M covers the Gaussian, convergence of the
FFT form to the direct alpha_M sum as cells shrink, full-rank SKP equal to
the FFT form, and finite differences of the energy --
tests/test_oracle_lagrange.py.
"""
import itertools

import numpy as np

from . import skp, spme


def nodes(L):
    """Equispaced interpolation nodes on [-1, 1], end points included."""
    return -1.0 + 2.0 * np.arange(L) / (L - 1)


def basis(t, L):
    """S(h_s, t) = prod_{r != s} (t - h_r) / (h_s - h_r) for t in [-1, 1]
    (Eq. interp1d after the affine map phi_I); returns [..., L]."""
    h = nodes(L)
    t = np.asarray(t, np.float64)[..., None]
    out = np.ones(t.shape[:-1] + (L,))
    for s in range(L):
        for r in range(L):
            if r != s:
                out[..., s] *= (t[..., 0] - h[r]) / (h[s] - h[r])
    return out


def dbasis(t, L):
    """d S(h_s, t) / dt by the product rule."""
    h = nodes(L)
    t = np.asarray(t, np.float64)
    out = np.zeros(t.shape + (L,))
    for s in range(L):
        for r in range(L):
            if r == s:
                continue
            term = np.full(t.shape, 1.0 / (h[s] - h[r]))
            for u in range(L):
                if u != s and u != r:
                    term = term * (t - h[u]) / (h[s] - h[u])
            out[..., s] += term
    return out


def stencil(x, box_len, Kc, L):
    """Grid indices, weights and d/dx weights of coordinates x on one axis.

    The cell of x (K_c cells of width w = box_len / K_c) is c = floor(u),
    u = K_c (x / box_len mod 1); its L nodes are grid points c (L - 1) + s
    (mod K = K_c (L - 1)); the weights are the Lagrange basis at
    t = 2 (u - c) - 1 in [-1, 1], and d/dx = (2 K_c / box_len) d/dt."""
    x = np.asarray(x, np.float64)
    s = x / box_len
    s = s - np.floor(s)
    u = s * Kc
    c = np.floor(u)
    c = np.where(c >= Kc, c - Kc, c)             # u rounded up to K_c
    t = 2.0 * (u - c) - 1.0
    K = Kc * (L - 1)
    idx = np.mod(c[..., None].astype(np.int64) * (L - 1) + np.arange(L), K)
    return idx, basis(t, L), dbasis(t, L) * (2.0 * Kc / box_len)


def grid_size(Kc, L):
    return tuple(int(k) * (L - 1) for k in Kc)


def alpha_hat(box, K, M, beta):
    """Mode-truncated kernel on the K1 x K2 x K3 DFT grid (zero beyond |m'_j| > M)."""
    box = np.asarray(box, np.float64)
    V = float(np.prod(box))
    for k in K:
        if 2 * M + 1 > k:
            raise ValueError("2M + 1 must not exceed the grid size (aliasing)")
    mp = [spme.signed_modes(K[j]) for j in range(3)]
    keep = [np.abs(mp[j]) <= M for j in range(3)]
    mh = [mp[j] / box[j] for j in range(3)]
    m2 = (mh[0][:, None, None] ** 2 + mh[1][None, :, None] ** 2
          + mh[2][None, None, :] ** 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        a = np.exp(-np.pi ** 2 * m2 / beta ** 2) / (np.pi * V * m2)
    a[0, 0, 0] = 0.0
    mask = keep[0][:, None, None] & keep[1][None, :, None] & keep[2][None, None, :]
    return np.where(mask, a, 0.0)


def _stencils(pos, box, Kc, L):
    pos = np.asarray(pos, np.float64)
    return [stencil(pos[:, j], box[j], Kc[j], L) for j in range(3)]


def spread(pos, q, box, Kc, L):
    """Q(g) = sum_i q_i W_i(g), W_i the product Lagrange basis of i's cell."""
    q = np.asarray(q, np.float64)
    K = grid_size(Kc, L)
    (i0, w0, _), (i1, w1, _), (i2, w2, _) = _stencils(pos, box, Kc, L)
    Q = np.zeros(K)
    for a in range(L):
        for b in range(L):
            for c in range(L):
                np.add.at(Q, (i0[:, a], i1[:, b], i2[:, c]), q * w0[:, a] * w1[:, b] * w2[:, c])
    return Q


def gather(pos, q, box, Kc, L, Phi):
    """phi_i = sum_g W_i(g) Phi(g); F_i = -q_i grad_x phi_i."""
    q = np.asarray(q, np.float64)
    (i0, w0, d0), (i1, w1, d1), (i2, w2, d2) = _stencils(pos, box, Kc, L)
    n = len(q)
    phi = np.zeros(n)
    g = np.zeros((n, 3))
    for a in range(L):
        for b in range(L):
            for c in range(L):
                v = Phi[i0[:, a], i1[:, b], i2[:, c]]
                phi += w0[:, a] * w1[:, b] * w2[:, c] * v
                g[:, 0] += d0[:, a] * w1[:, b] * w2[:, c] * v
                g[:, 1] += w0[:, a] * d1[:, b] * w2[:, c] * v
                g[:, 2] += w0[:, a] * w1[:, b] * d2[:, c] * v
    return phi, -q[:, None] * g


def kpme_fft(pos, q, box, Kc, L, M, beta):
    """The exact (untruncated-rank) KPME: spread, periodic convolution with
    alpha_hat through FFTs, gather.  Returns a dict like spme.spme."""
    q = np.asarray(q, np.float64)
    box = np.asarray(box, np.float64)
    K = grid_size(Kc, L)
    a = alpha_hat(box, K, M, beta)
    Q = spread(pos, q, box, Kc, L)
    Phi = spme.convolve_fft(Q, a)
    phi, F = gather(pos, q, box, Kc, L, Phi)
    return {"E_rec": 0.5 * float(q @ phi), "phi": phi, "F": F, "Q": Q, "Phi": Phi,
            "alpha_hat": a}


def direct_alpha_m(pos, q, box, M, beta):
    """The paper's H_M q at the particles, summed mode by mode over the cube
    0 < |m|_inf <= M; returns (E_rec, phi, F)."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(q, np.float64)
    box = np.asarray(box, np.float64)
    V = float(np.prod(box))
    r = np.arange(-M, M + 1)
    m = np.array([v for v in itertools.product(r, r, r) if any(v)], np.float64)
    mh = m / box[None, :]
    mh2 = (mh ** 2).sum(axis=1)
    f = np.exp(-np.pi ** 2 * mh2 / beta ** 2) / mh2
    ph = np.exp(2j * np.pi * (pos @ mh.T))           # [N, modes]
    S = q @ ph
    phi = (np.real(np.conj(ph) * S[None, :]) @ f) / (np.pi * V)
    im = np.imag(np.conj(S)[None, :] * ph)
    F = (2.0 / V) * q[:, None] * ((im * f[None, :]) @ mh)
    return 0.5 * float(q @ phi), phi, F


class Plan(skp.Plan):
    """Oracle plan: nested-SVD SKP of alpha_hat on the Lagrange grid."""

    def __init__(self, box, Kc, L, M, beta, rank=None, tol=None):
        self.box = np.asarray(box, np.float64)
        self.Kc = tuple(int(k) for k in Kc)
        self.L = int(L)
        self.M = int(M)
        self.K = grid_size(self.Kc, self.L)
        self.p = self.L
        self.beta = float(beta)
        self.theta = alpha_hat(self.box, self.K, self.M, self.beta)
        self.all_terms = skp.nested_svd_terms(self.theta)
        if rank is None and tol is None:
            rank = len(self.all_terms)
        self.terms = skp.select_terms(self.all_terms, self.theta, rank=rank, tol=tol)
        self.rank = len(self.terms)
        self.facs = skp.factors(self.terms)
        self.c0 = skp.zero_mode_value(self.terms)
        self.r0 = len({t[4] for t in self.terms})
        dropped = self.all_terms[self.rank:]
        self.trunc_err = float(np.sqrt(sum(t[0] ** 2 for t in dropped)))

    def evaluate(self, pos, q):
        q = np.asarray(q, np.float64)
        Q = spread(pos, q, self.box, self.Kc, self.L)
        Phi = self.apply(Q)
        phi, F = gather(pos, q, self.box, self.Kc, self.L, Phi)
        return {"E_rec": 0.5 * float(q @ phi), "phi": phi, "F": F, "Q": Q, "Phi": Phi}
