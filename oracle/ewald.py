"""Direct Ewald summation in an orthorhombic periodic box (oracle; test infrastructure).

Ground truth for the periodic Coulomb problem of Sec. 1.1 (Eq.
qmutheta_coulomb), split as in Sec. 1.2 (Eq. tau with tau = erf(beta r)) into

* a short-range real-space sum  E_real = 1/2 sum_{i,j} sum'_n q_i q_j erfc(beta r)/r,
  r = |r_i - r_j + n L| <= r_cut, the prime excluding i = j at n = 0;
* the reciprocal sum (Eqs. hexpr, sumhexpr written in Cartesian units,
  m_hat = (m1/L1, m2/L2, m3/L3), V = L1 L2 L3, tin-foil boundary, alpha(0) = 0):
  E_rec = 1/(2 pi V) sum_{m != 0} exp(-pi^2 |m_hat|^2 / beta^2) / |m_hat|^2 |S(m)|^2,
  S(m) = sum_j q_j exp(2 pi i m_hat . r_j);
* the self term E_self = -(beta / sqrt(pi)) sum q_i^2;
* the neutralising-background term E_neutral = -pi (sum q)^2 / (2 V beta^2).

Potentials phi_i split the same way, with E = 1/2 sum q_i phi_i term by term;
forces are F_i = -dE/dr_i.  Coulomb constant 1 (Gaussian units).

Pinned by: the NaCl Madelung constant (tests/golden/madelung_nacl.txt),
independence of the total energy from beta, Newton's third law and central
finite differences -- tests/test_oracle_ewald.py.
"""
import itertools
import math

import numpy as np
from scipy.special import erfc


def _mode_list(box, kmax):
    """Integer mode vectors m != 0 with Euclidean |m| <= kmax."""
    r = int(math.floor(kmax))
    rng = np.arange(-r, r + 1)
    m = np.array(list(itertools.product(rng, rng, rng)), dtype=np.float64)
    n2 = (m ** 2).sum(axis=1)
    keep = (n2 > 0) & (n2 <= kmax * kmax + 1e-9)
    return m[keep]


def reciprocal(pos, q, box, beta, kmax):
    """Reciprocal-space energy, potentials and forces by explicit mode sums."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(q, np.float64)
    box = np.asarray(box, np.float64)
    V = float(np.prod(box))
    m = _mode_list(box, kmax)
    mh = m / box[None, :]                        # m_hat
    mh2 = (mh ** 2).sum(axis=1)
    f = np.exp(-np.pi ** 2 * mh2 / beta ** 2) / mh2
    energy = 0.0
    phi = np.zeros(len(q))
    force = np.zeros((len(q), 3))
    chunk = 512
    for s in range(0, len(m), chunk):
        mhc = mh[s:s + chunk]
        fc = f[s:s + chunk]
        ph = np.exp(2j * np.pi * (pos @ mhc.T))  # [N, M]  e^{2 pi i m_hat . r_j}
        S = q @ ph                               # structure factor per mode
        energy += float((fc * np.abs(S) ** 2).sum()) / (2.0 * np.pi * V)
        phi += (np.real(np.conj(ph) * S[None, :]) @ fc) / (np.pi * V)
        im = np.imag(np.conj(S)[None, :] * ph)   # Im(S*(m) e^{2 pi i m_hat . r_i})
        force += (2.0 / V) * q[:, None] * ((im * fc[None, :]) @ mhc)
    return energy, phi, force


def real_space(pos, q, box, beta, rcut):
    """Short-range real-space energy, potentials and forces with an image loop."""
    pos = np.asarray(pos, np.float64)
    q = np.asarray(q, np.float64)
    box = np.asarray(box, np.float64)
    n = len(q)
    nimg = [int(math.ceil(rcut / L)) for L in box]
    phi = np.zeros(n)
    force = np.zeros((n, 3))
    d0 = pos[:, None, :] - pos[None, :, :]
    for s in itertools.product(*[range(-k, k + 1) for k in nimg]):
        shift = np.array(s, np.float64) * box
        d = d0 + shift[None, None, :]
        r = np.sqrt((d ** 2).sum(axis=2))
        mask = r <= rcut
        if s == (0, 0, 0):
            np.fill_diagonal(mask, False)
        rs = np.where(mask, r, 1.0)
        pot = np.where(mask, erfc(beta * rs) / rs, 0.0)
        phi += pot @ q
        dpot = np.where(mask, erfc(beta * rs) / rs ** 2
                        + 2.0 * beta / math.sqrt(math.pi)
                        * np.exp(-(beta * rs) ** 2) / rs, 0.0)
        # F_i = sum_j q_i q_j dpot * (r_i - r_j + nL) / r
        force += q[:, None] * np.einsum('ij,ijk->ik', dpot * q[None, :] / rs, d)
    energy = 0.5 * float(q @ phi)
    return energy, phi, force


def direct_ewald(pos, q, box, beta, rcut, kmax):
    """All four Ewald terms; returns a dict of energies, potentials and forces."""
    q = np.asarray(q, np.float64)
    box = np.asarray(box, np.float64)
    V = float(np.prod(box))
    e_real, phi_real, f_real = real_space(pos, q, box, beta, rcut)
    e_rec, phi_rec, f_rec = reciprocal(pos, q, box, beta, kmax)
    qs = float(q.sum())
    e_self = -beta / math.sqrt(math.pi) * float((q ** 2).sum())
    e_neutral = -math.pi * qs ** 2 / (2.0 * V * beta ** 2)
    phi_self = -2.0 * beta * q / math.sqrt(math.pi)
    phi_neutral = np.full(len(q), -math.pi * qs / (V * beta ** 2))
    return {
        "E_real": e_real, "E_rec": e_rec, "E_self": e_self,
        "E_neutral": e_neutral,
        "E": e_real + e_rec + e_self + e_neutral,
        "phi_real": phi_real, "phi_rec": phi_rec,
        "phi": phi_real + phi_rec + phi_self + phi_neutral,
        "F_real": f_real, "F_rec": f_rec, "F": f_real + f_rec,
    }


def self_and_neutral(q, box, beta):
    """(E_self, E_neutral) for charges q in box -- textbook Ewald constants."""
    q = np.asarray(q, np.float64)
    V = float(np.prod(box))
    qs = float(q.sum())
    return (-beta / math.sqrt(math.pi) * float((q ** 2).sum()),
            -math.pi * qs ** 2 / (2.0 * V * beta ** 2))
