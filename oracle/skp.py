"""Sum-of-Kronecker-Products reciprocal operator (oracle; test infrastructure).

The method of the paper applied to the smooth-PME grid kernel theta_hat
(module ``spme``), which plays the role of the paper's alpha_M (Sec. 2.1):

1. Nested SVD (Sec. 2.1.1, Eq. last_decomp_kron): unfold theta_hat with
   axis 2 as rows (I_2°, a K3 x K1K2 matrix) and take its SVD
   sum_i s_i u_i v_i^T; reshape each right vector v_i into a K1 x K2 matrix
   (I_1°) and take its SVD sum_j s_ij x_ij y_ij^T.  Every pair (i, j) is a
   term with weight omega = s_i s_ij and per-axis mode vectors
   (axis 0: x_ij, axis 1: y_ij, axis 2: u_i).  Whether the inner matrix has
   axis 0 or axis 1 as rows gives the same terms (an SVD of the transpose).
2. Truncation: sort the terms by |omega| (stable; ties keep (i, j) order) and
   keep the top R, or the smallest R whose dropped tail has Frobenius norm
   <= tol * ||theta_hat||_F.  The terms are orthonormal rank-1 tensors, so the
   dropped tail's Frobenius norm is exactly sqrt(sum of dropped omega^2);
   Eq. estimate_svd bounds it from above.
3. Real per-axis factors (Sec. 2.3-2.4, Eqs. kronw, VtV): each mode vector a
   is even in m, so its circulant A[g, h] = sum_m a(m) exp(2 pi i m (g-h)/K)
   is real and symmetric; the operator is Theta_R = sum_r omega_r A_r (x) B_r (x) C_r
   (Eq. formfinale between the spread S_Y and the gather S_X*).
4. Application (Sec. 3.2-3.3, Alg. 1 / Alg. 2): three mode products per term
   with a library tensordot, summed over terms, no grouping.
5. Correction (Sec. 4.1 Eq. termbonsum, Alg. 4): the truncated symbol is not
   zero at m = 0; its value c = theta_hat_R(0) = sum_r omega_r a_r(0) b_r(0) c_r(0)
   times sum(Q) = sum(q) is subtracted from every grid value of Phi.

Pinned by: exact reconstruction at full rank, the exact Frobenius tail
identity and the Eq. estimate_svd bound, equality with FFT-based SPME at full
rank on non-cubic grids, the correction against an FFT convolution with the
truncated symbol (m = 0 zeroed), operator symmetry and the energy bound --
tests/test_oracle_skp.py.
"""
import numpy as np

from . import spme


def nested_svd_terms(th):
    """All terms (omega, x, y, u, i, j) of the nested SVD of theta_hat.

    Terms whose outer singular value is below the numerical rank threshold
    (K3 * eps * s_1) or whose inner one is below K * eps * s_i1 are omitted:
    their vectors are rounding noise.  Returned sorted by omega descending,
    stable in (i, j).
    """
    K1, K2, K3 = th.shape
    T = np.transpose(th, (2, 0, 1)).reshape(K3, K1 * K2)   # I_2°: rows = axis 2
    U, s, Vt = np.linalg.svd(T, full_matrices=False)
    eps = np.finfo(np.float64).eps
    terms = []
    for i in range(len(s)):
        if s[i] <= K3 * eps * s[0]:
            break
        Vi = Vt[i].reshape(K1, K2)                          # I_1°(v_i)
        X, si, Yt = np.linalg.svd(Vi, full_matrices=False)
        for j in range(len(si)):
            if si[j] <= max(K1, K2) * eps * si[0]:
                break
            terms.append((s[i] * si[j], X[:, j].copy(), Yt[j].copy(),
                          U[:, i].copy(), i, j))
    order = sorted(range(len(terms)), key=lambda k: -terms[k][0])  # stable
    return [terms[k] for k in order]


def select_terms(terms, th, rank=None, tol=None):
    """Top-R terms, or the smallest R with dropped-tail Frobenius <= tol*||th||_F."""
    if rank is not None:
        return terms[:rank]
    norm2 = float((th ** 2).sum())
    w2 = np.array([t[0] ** 2 for t in terms])
    tail = np.concatenate([np.cumsum(w2[::-1])[::-1], [0.0]])  # tail[R] = sum_{r>=R}
    # account for the part of ||th||^2 not represented by any kept-able term
    missing = max(norm2 - float(w2.sum()), 0.0)
    for R in range(len(terms) + 1):
        if np.sqrt(tail[R] + missing) <= tol * np.sqrt(norm2):
            return terms[:R]
    return terms


def svd_bound(th, terms_all, kept):
    """Right-hand side of Eq. estimate_svd for the kept (i, j) set."""
    K1, K2, K3 = th.shape
    T = np.transpose(th, (2, 0, 1)).reshape(K3, K1 * K2)
    _, s, Vt = np.linalg.svd(T, full_matrices=False)
    kept_ij = {(t[4], t[5]) for t in kept}
    kept_i = {i for (i, _) in kept_ij}
    outer = np.sqrt(sum(s[i] ** 2 for i in range(len(s)) if i not in kept_i))
    inner = 0.0
    for i in kept_i:
        si = np.linalg.svd(Vt[i].reshape(K1, K2), compute_uv=False)
        inner += s[i] * np.sqrt(sum(si[j] ** 2 for j in range(len(si))
                                    if (i, j) not in kept_ij))
    return outer + inner


def reconstruct(terms, shape):
    """sum_r omega_r x_r (x) y_r (x) u_r on the mode grid."""
    out = np.zeros(shape)
    for (w, x, y, u, _, _) in terms:
        out += w * x[:, None, None] * y[None, :, None] * u[None, None, :]
    return out


def circulant(a):
    """A[g, h] = sum_m a(m) exp(2 pi i m (g - h) / K).

    Returns (real part, largest |imaginary part|).  The exact mode vectors are
    even, so the imaginary part is rounding noise (checked by ``factors``).
    """
    K = len(a)
    d = np.arange(K)
    F = np.exp(2j * np.pi * np.outer(np.arange(K), d) / K)   # F[m, d]
    col = a @ F                                                # c(d) = sum_m a(m) e^{2 pi i m d/K}
    g = d[:, None] - d[None, :]
    return col.real[np.mod(g, K)], float(np.abs(col.imag).max())


def factors(terms):
    """Real circulant factors (omega, A, B, C) for every term.

    The imaginary parts dropped here must be negligible in the operator:
    omega * |Im| <= 1e-9 * omega_1 (rounding noise of small singular values).
    """
    out = []
    w1 = max((t[0] for t in terms), default=1.0)
    for (w, x, y, u, _, _) in terms:
        mats = [circulant(v) for v in (x, y, u)]
        for (_, im) in mats:
            assert w * im <= 1e-9 * w1, "mode vector is not even: complex circulant"
        out.append((w, mats[0][0], mats[1][0], mats[2][0]))
    return out


def zero_mode_value(terms):
    """theta_hat_R(0) = sum_r omega_r x_r(0) y_r(0) u_r(0)."""
    return float(sum(w * x[0] * y[0] * u[0] for (w, x, y, u, _, _) in terms))


def apply(Q, facs, c0):
    """Phi = sum_r omega_r Q x_1 A_r x_2 B_r x_3 C_r, then Phi -= c0 * sum(Q)."""
    Phi = np.zeros_like(Q, dtype=np.float64)
    for (w, A, B, C) in facs:
        X = np.tensordot(A, Q, axes=(1, 0))                    # contract g1 -> (k1, g2, g3)
        X = np.transpose(np.tensordot(B, X, axes=(1, 1)), (1, 0, 2))  # contract g2
        X = np.tensordot(X, C, axes=(2, 1))                    # contract g3 -> (k1, k2, k3)
        Phi += w * X
    Phi -= c0 * float(Q.sum())
    return Phi


class Plan:
    """Oracle plan: theta_hat, the selected terms and their circulant factors."""

    def __init__(self, box, K, p, beta, rank=None, tol=None):
        self.box = np.asarray(box, np.float64)
        self.K = tuple(int(k) for k in K)
        self.p = int(p)
        self.beta = float(beta)
        self.theta = spme.theta_hat(self.box, self.K, self.p, self.beta)
        self.all_terms = nested_svd_terms(self.theta)
        if rank is None and tol is None:
            rank = len(self.all_terms)
        self.terms = select_terms(self.all_terms, self.theta, rank=rank, tol=tol)
        self.rank = len(self.terms)
        self.facs = factors(self.terms)
        self.c0 = zero_mode_value(self.terms)
        self.r0 = len({t[4] for t in self.terms})
        dropped = self.all_terms[self.rank:]
        self.trunc_err = float(np.sqrt(sum(t[0] ** 2 for t in dropped)))

    def apply(self, Q):
        return apply(Q, self.facs, self.c0)

    def evaluate(self, pos, q):
        q = np.asarray(q, np.float64)
        Q = spme.spread(pos, q, self.box, self.K, self.p)
        Phi = self.apply(Q)
        phi, F = spme.gather(pos, q, self.box, self.K, self.p, Phi)
        return {"E_rec": 0.5 * float(q @ phi), "phi": phi, "F": F, "Q": Q,
                "Phi": Phi}


def backward(plan, pos, q, g_energy, g_pot):
    """Gradients of L = g_energy * (E_rec + E_self + E_neutral) + sum_i g_pot_i phi_i.

    phi = S* Theta S q with Theta the corrected (symmetric) operator; with
    Phi = Theta S q and Psi = Theta S g_pot:
      dL/dr_i = grad W_i . [(g_energy q_i + g_pot_i) Phi + q_i Psi]
      dL/dq_i = g_energy (phi_i - 2 beta q_i / sqrt(pi) - pi sum(q) / (V beta^2)) + W_i . Psi
    Written from the chain rule of the definitions above; pinned by central
    finite differences of `Plan.evaluate` (tests/test_oracle_backward.py).
    """
    q = np.asarray(q, np.float64)
    n = len(q)
    g_pot = np.zeros(n) if g_pot is None else np.asarray(g_pot, np.float64)
    ones = np.ones(n)
    Phi = plan.apply(spme.spread(pos, q, plan.box, plan.K, plan.p))
    Psi = plan.apply(spme.spread(pos, g_pot, plan.box, plan.K, plan.p))
    phi, f_phi = spme.gather(pos, ones, plan.box, plan.K, plan.p, Phi)
    psi, f_psi = spme.gather(pos, ones, plan.box, plan.K, plan.p, Psi)
    grad_w_phi, grad_w_psi = -f_phi, -f_psi        # gradient of W_i . grid
    V = float(np.prod(plan.box))
    grad_pos = (g_energy * q + g_pot)[:, None] * grad_w_phi + q[:, None] * grad_w_psi
    grad_q = g_energy * (phi - 2.0 * plan.beta * q / np.sqrt(np.pi)
                         - np.pi * q.sum() / (V * plan.beta ** 2)) + psi
    return grad_pos, grad_q
