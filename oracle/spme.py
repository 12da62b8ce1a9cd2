"""Classical smooth PME with FFTs (oracle; test infrastructure).

The FFT-based particle-mesh method the paper sets out to replace (Sec. 1.2):
interpolate charges on a periodic K1 x K2 x K3 grid with order-p cardinal
B-splines, convolve with the reciprocal kernel through FFTs, interpolate back.

Definitions (textbook smooth PME, Cartesian units, orthorhombic box):

* u_ij = K_j * (x_ij / L_j mod 1); particle i touches k = (floor(u) - t) mod K
  with weight M_p(u - floor(u) + t), t = 0..p-1 (module ``bspline``);
* Q(k) = sum_i q_i W_i(k),  W_i(k) = prod_j M_p(...);
* theta_hat(m) = exp(-pi^2 |m_hat|^2 / beta^2) / (pi V |m_hat|^2)
                 * prod_j |b_j(m_j)|^2,  theta_hat(0) = 0,
  m_hat_j = m'_j / L_j with m'_j = m_j if m_j <= K_j/2 else m_j - K_j
  (the paper's alpha_M with alpha(0) = 0, Sec. 2.1, carrying 1/(pi V) and the
  B-spline moduli);
* Phi = G * ifftn(theta_hat * fftn(Q)), G = K1 K2 K3: the periodic convolution
  with theta_rec(k) = sum_m theta_hat(m) exp(2 pi i m.k / K);
* phi_i = sum_k W_i(k) Phi(k);  E_rec = 1/2 sum_i q_i phi_i = 1/2 sum_k Q Phi;
* F_i = -q_i sum_k grad W_i(k) Phi(k), d/dx_j = (K_j / L_j) d/du_j.

Pinned by: convergence to direct Ewald as K and p grow, the three energy
identities, a single-mode eigenvector test, grid-shift invariance, partition
of unity and central finite differences -- tests/test_oracle_spme.py.
"""
import numpy as np

from . import bspline


def scaled_coords(pos, box, K):
    """u_ij = K_j (x_ij / L_j mod 1), in float64."""
    pos = np.asarray(pos, np.float64)
    box = np.asarray(box, np.float64)
    s = pos / box[None, :]
    s = s - np.floor(s)
    return s * np.asarray(K, np.float64)[None, :]


def signed_modes(K):
    """m' = m if m <= K/2 else m - K, for m = 0..K-1."""
    m = np.arange(K)
    return np.where(m <= K // 2, m, m - K).astype(np.float64)


def theta_hat(box, K, p, beta):
    """Reciprocal kernel on the K1 x K2 x K3 mode grid, theta_hat(0) = 0."""
    box = np.asarray(box, np.float64)
    V = float(np.prod(box))
    mh = [signed_modes(K[j]) / box[j] for j in range(3)]
    m2 = (mh[0][:, None, None] ** 2 + mh[1][None, :, None] ** 2
          + mh[2][None, None, :] ** 2)
    b = [bspline.bmod2(K[j], p) for j in range(3)]
    bb = b[0][:, None, None] * b[1][None, :, None] * b[2][None, None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        th = np.exp(-np.pi ** 2 * m2 / beta ** 2) / (np.pi * V * m2) * bb
    th[0, 0, 0] = 0.0
    return th


def _stencils(pos, box, K, p):
    u = scaled_coords(pos, box, K)
    return [bspline.stencil(u[:, j], K[j], p) for j in range(3)]


def spread(pos, q, box, K, p):
    """Q(k) = sum_i q_i W_i(k) by scattering every stencil point (np.add.at)."""
    q = np.asarray(q, np.float64)
    st = _stencils(pos, box, K, p)
    (i0, w0, _), (i1, w1, _), (i2, w2, _) = st
    Q = np.zeros(tuple(K), np.float64)
    for a in range(p):
        for b in range(p):
            for c in range(p):
                np.add.at(Q, (i0[:, a], i1[:, b], i2[:, c]),
                          q * w0[:, a] * w1[:, b] * w2[:, c])
    return Q


def convolve_fft(Q, th):
    """Phi = G * ifftn(theta_hat * fftn(Q)); the result is real."""
    G = Q.size
    Phi = G * np.fft.ifftn(th * np.fft.fftn(Q))
    assert np.abs(Phi.imag).max() <= 1e-9 * max(1.0, np.abs(Phi.real).max())
    return Phi.real


def gather(pos, q, box, K, p, Phi):
    """phi_i = sum_k W_i(k) Phi(k) and F_i = -q_i sum_k grad W_i(k) Phi(k)."""
    q = np.asarray(q, np.float64)
    box = np.asarray(box, np.float64)
    st = _stencils(pos, box, K, p)
    (i0, w0, d0), (i1, w1, d1), (i2, w2, d2) = st
    n = len(q)
    phi = np.zeros(n)
    g = np.zeros((n, 3))
    for a in range(p):
        for b in range(p):
            for c in range(p):
                v = Phi[i0[:, a], i1[:, b], i2[:, c]]
                phi += w0[:, a] * w1[:, b] * w2[:, c] * v
                g[:, 0] += d0[:, a] * w1[:, b] * w2[:, c] * v
                g[:, 1] += w0[:, a] * d1[:, b] * w2[:, c] * v
                g[:, 2] += w0[:, a] * w1[:, b] * d2[:, c] * v
    scale = np.asarray(K, np.float64) / box
    force = -q[:, None] * g * scale[None, :]
    return phi, force


def spme(pos, q, box, K, p, beta):
    """Full SPME reciprocal evaluation; returns a dict (E_rec, phi, F, Q, Phi)."""
    q = np.asarray(q, np.float64)
    th = theta_hat(box, K, p, beta)
    Q = spread(pos, q, box, K, p)
    Phi = convolve_fft(Q, th)
    phi, F = gather(pos, q, box, K, p, Phi)
    return {"E_rec": 0.5 * float(q @ phi), "phi": phi, "F": F, "Q": Q,
            "Phi": Phi, "theta_hat": th}
