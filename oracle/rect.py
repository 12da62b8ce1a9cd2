"""Rectangular real cos/sin factors of the Kronecker terms (oracle; test
infrastructure).

The paper's compressed real format (Sec. 2.3, Eq. kronw; Sec. 2.4, Eq. VtV):
a per-axis factor whose mode vector a(m) is even and vanishes for |m'| > M is

    A[g, h] = sum_m a(m) e^{2 pi i m (g - h) / K}
            = a(0) + sum_{m=1}^{M} 2 a(m) [cos(t_m g) cos(t_m h) + sin(t_m g) sin(t_m h)],

t_m = 2 pi m / K, i.e. A = F^T diag(d) F with the real, rectangular
(2M + 1) x K matrix F of rows 1, cos(t_m g), sin(t_m g) (m = 1..M) and the
weights d = (a(0), 2 a(m), 2 a(m), ...); at the Nyquist mode m = K / 2 of an
even K the sine row vanishes and is dropped, and its weight is a(K/2).
Written as in Eq. VtV, A = V^T S V with V = diag(sqrt|d|) F and S the signs
of d (S = I for the non-negative vectors of the quadrature; nested-SVD
vectors can change sign).  A mode product by A is then two thin products,
V X and V^T (S V X) (Sec. 3.2-3.3).

Pinned by: V^T S V against the circulant built from complex exponentials
(module skp), the orthogonality F F^T = diag(K, K/2, ..., K/2[, K]) of the
real Fourier rows, and the operator through rectangular factors against the
circulant one -- tests/test_oracle_rect.py.
"""
import numpy as np

from . import skp


def mode_cut(a, tol=0.0):
    """Largest |m'| with a non-zero entry of the even mode vector a."""
    K = len(a)
    m = np.arange(K)
    ms = np.where(m <= K // 2, m, K - m)
    nz = np.abs(a) > tol * max(np.abs(a).max(), 1e-300)
    return int(ms[nz].max()) if nz.any() else 0


def real_rows(K, M):
    """F (rows x K) and the mode m of each row: 1, then cos and sin rows for
    m = 1..M (no sine row at m = K / 2)."""
    g = np.arange(K, dtype=np.float64)
    rows, modes = [np.ones(K)], [0]
    for m in range(1, M + 1):
        t = 2.0 * np.pi * m / K
        rows.append(np.cos(t * g))
        modes.append(m)
        if 2 * m != K:
            rows.append(np.sin(t * g))
            modes.append(m)
    return np.array(rows), np.array(modes)


def rect_factor(a, M=None):
    """(V, S, F, d) of the even mode vector a (length K, zero beyond |m'| > M)."""
    a = np.asarray(a, np.float64)
    K = len(a)
    if M is None:
        M = K // 2
    F, modes = real_rows(K, M)
    d = np.array([a[m] if m == 0 or 2 * m == K else 2.0 * a[m] for m in modes])
    V = np.sqrt(np.abs(d))[:, None] * F
    S = np.sign(d)
    return V, S, F, d


def mode_product(X, V, S, axis):
    """X x_axis (V^T S V): two thin products along one axis."""
    Z = np.tensordot(V, X, axes=(1, axis))            # (rows, ...) -- V X
    Z = S.reshape((-1,) + (1,) * (X.ndim - 1)) * Z
    Y = np.tensordot(V.T, Z, axes=(1, 0))            # (K, ...) -- V^T (S V X)
    return np.moveaxis(Y, 0, axis)


def apply(Q, terms, c0, M=(None, None, None)):
    """Phi = sum_r omega_r Q x_1 A_r x_2 B_r x_3 C_r with every factor in
    rectangular form, then Phi -= c0 sum(Q)."""
    Phi = np.zeros_like(Q, dtype=np.float64)
    for (w, x, y, u, _, _) in terms:
        X = Q
        for axis, (vec, m) in enumerate(zip((x, y, u), M)):
            V, S, _, _ = rect_factor(vec, m)
            X = mode_product(X, V, S, axis)
        Phi += w * X
    Phi -= c0 * float(Q.sum())
    return Phi


def circulant_of(a):
    """The circulant of module skp (complex-exponential definition), real part."""
    return skp.circulant(a)[0]
