// Host FP64 factor construction for the Kronecker-product reciprocal operator.
//
// The kernel is the smooth-PME symbol
//   theta_hat(m) = exp(-pi^2 |m_hat|^2 / beta^2) / (pi V |m_hat|^2) prod_j |b_j(m_j)|^2,
// theta_hat(0) = 0 (the paper's alpha_M with alpha(0) = 0, Sec. 2.1), and its
// Sum of Kronecker Products comes from the nested SVD of Sec. 2.1.1
// (Eq. last_decomp_kron): axis 2 is separated first, then each right singular
// vector, reshaped to K1 x K2, is decomposed again.
//
// theta_hat is even in every m_j, so every singular vector with a non-zero
// singular value is even (the reflection m_j -> -m_j maps each unfolding onto
// itself).  The SVDs are therefore taken on the folded half domain
// h = |m'| in [0, floor(K/2)] with weights w(h) = sqrt(multiplicity of h),
// which preserves inner products: the singular values are those of the full
// unfoldings, and a folded vector a'(h) unfolds to a(m) = a'(|m'|) / w(|m'|).
// The SVDs are one-sided (Hestenes) Jacobi iterations in FP64, which keep
// high relative accuracy in the small singular values that decide truncation.
#include "factors.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace kpme {

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

// M_n evaluated at u by the two-term recursion of the cardinal B-splines.
double bspline_eval(double u, int n) {
  if (n == 2) return (u >= 0.0 && u <= 2.0) ? 1.0 - std::fabs(u - 1.0) : 0.0;
  return (u * bspline_eval(u, n - 1) + (n - u) * bspline_eval(u - 1.0, n - 1)) / (n - 1);
}

// Thin SVD of a (rows x cols) matrix stored column-major, by one-sided Jacobi
// on its columns (requires cols <= rows).  On return: s[k] descending,
// left[k*rows + r] (unit columns for s > 0), right[k*cols + c] (orthonormal).
bool jacobi_svd_cols(int rows, int cols, std::vector<double> W,
                     std::vector<double>* s, std::vector<double>* left,
                     std::vector<double>* right) {
  std::vector<double> V(static_cast<size_t>(cols) * cols, 0.0);
  for (int c = 0; c < cols; ++c) V[static_cast<size_t>(c) * cols + c] = 1.0;
  const double tol = 1e-15;
  bool converged = false;
  for (int sweep = 0; sweep < 80 && !converged; ++sweep) {
    converged = true;
    for (int p = 0; p < cols - 1; ++p) {
      double* wp = &W[static_cast<size_t>(p) * rows];
      for (int q = p + 1; q < cols; ++q) {
        double* wq = &W[static_cast<size_t>(q) * rows];
        double a = 0.0, b = 0.0, g = 0.0;
        for (int r = 0; r < rows; ++r) {
          a += wp[r] * wp[r];
          b += wq[r] * wq[r];
          g += wp[r] * wq[r];
        }
        if (a == 0.0 || b == 0.0) continue;
        if (std::fabs(g) <= tol * std::sqrt(a * b)) continue;
        converged = false;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) /
                         (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t);
        const double sn = c * t;
        for (int r = 0; r < rows; ++r) {
          const double x = wp[r], y = wq[r];
          wp[r] = c * x - sn * y;
          wq[r] = sn * x + c * y;
        }
        double* vp = &V[static_cast<size_t>(p) * cols];
        double* vq = &V[static_cast<size_t>(q) * cols];
        for (int r = 0; r < cols; ++r) {
          const double x = vp[r], y = vq[r];
          vp[r] = c * x - sn * y;
          vq[r] = sn * x + c * y;
        }
      }
    }
  }
  if (!converged) return false;
  std::vector<double> norms(cols);
  for (int c = 0; c < cols; ++c) {
    double a = 0.0;
    const double* w = &W[static_cast<size_t>(c) * rows];
    for (int r = 0; r < rows; ++r) a += w[r] * w[r];
    norms[c] = std::sqrt(a);
  }
  std::vector<int> order(cols);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return norms[x] > norms[y]; });
  s->assign(cols, 0.0);
  left->assign(static_cast<size_t>(cols) * rows, 0.0);
  right->assign(static_cast<size_t>(cols) * cols, 0.0);
  for (int k = 0; k < cols; ++k) {
    const int c = order[k];
    (*s)[k] = norms[c];
    const double inv = norms[c] > 0 ? 1.0 / norms[c] : 0.0;
    for (int r = 0; r < rows; ++r)
      (*left)[static_cast<size_t>(k) * rows + r] = W[static_cast<size_t>(c) * rows + r] * inv;
    for (int r = 0; r < cols; ++r)
      (*right)[static_cast<size_t>(k) * cols + r] = V[static_cast<size_t>(c) * cols + r];
  }
  return true;
}

// Thin SVD of a row-major (m x n) matrix: A = sum_k s_k u_k v_k^T with
// u[k*m + i], v[k*n + j].
bool svd_rowmajor(int m, int n, const std::vector<double>& A, std::vector<double>* s,
                  std::vector<double>* u, std::vector<double>* v) {
  if (n <= m) {
    // columns of A (length m), column-major copy
    std::vector<double> W(static_cast<size_t>(n) * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) W[static_cast<size_t>(j) * m + i] = A[static_cast<size_t>(i) * n + j];
    return jacobi_svd_cols(m, n, std::move(W), s, u, v);
  }
  // columns of A^T are the rows of A (length n)
  std::vector<double> W(A.begin(), A.end());
  return jacobi_svd_cols(n, m, std::move(W), s, v, u);
}

}  // namespace

std::vector<double> bspline_at_integers(int p) {
  std::vector<double> out(p + 1, 0.0);
  for (int k = 0; k <= p; ++k) out[k] = bspline_eval(static_cast<double>(k), p);
  return out;
}

std::vector<double> bspline_moduli(int K, int p) {
  const std::vector<double> Mk = bspline_at_integers(p);
  std::vector<double> out(K);
  for (int m = 0; m < K; ++m) {
    double re = 0.0, im = 0.0;
    for (int k = 0; k <= p - 2; ++k) {
      const long r = (static_cast<long>(m) * k) % K;
      const double ang = 2.0 * kPi * static_cast<double>(r) / K;
      re += Mk[k + 1] * std::cos(ang);
      im += Mk[k + 1] * std::sin(ang);
    }
    out[m] = 1.0 / (re * re + im * im);
  }
  return out;
}

std::vector<double> circulant_column(const std::vector<double>& a) {
  const int K = static_cast<int>(a.size());
  std::vector<double> ct(K);
  for (int r = 0; r < K; ++r) ct[r] = std::cos(2.0 * kPi * r / K);
  std::vector<double> col(K, 0.0);
  for (int d = 0; d < K; ++d) {
    double acc = 0.0;
    for (int m = 0; m < K; ++m) acc += a[m] * ct[(static_cast<long>(m) * d) % K];
    col[d] = acc;
  }
  return col;
}

bool build_factors(const double box[3], const int K[3], int p, double beta, int rank,
                   double tol, const KernelSpec& ks, FactorSet* out, std::string* err) {
  const double V = box[0] * box[1] * box[2];
  int H[3];
  std::vector<double> w[3], bm[3], mh2[3];
  for (int j = 0; j < 3; ++j) {
    H[j] = K[j] / 2 + 1;
    w[j].resize(H[j]);
    const std::vector<double> bfull = ks.lagrange ? std::vector<double>() : bspline_moduli(K[j], p);
    bm[j].resize(H[j]);
    for (int h = 0; h < H[j]; ++h) bm[j][h] = ks.axis_factor(bfull, h);
    mh2[j].resize(H[j]);
    for (int h = 0; h < H[j]; ++h) {
      const bool single = (h == 0) || (K[j] % 2 == 0 && h == K[j] / 2);
      w[j][h] = single ? 1.0 : std::sqrt(2.0);
      const double mh = h / box[j];
      mh2[j][h] = mh * mh;
    }
  }
  // Folded unfolding T'[h3][h1*H2 + h2] = w1 w2 w3 theta_hat.
  const int H12 = H[0] * H[1];
  std::vector<double> T(static_cast<size_t>(H[2]) * H12);
  double norm2 = 0.0;
  for (int h3 = 0; h3 < H[2]; ++h3)
    for (int h1 = 0; h1 < H[0]; ++h1)
      for (int h2 = 0; h2 < H[1]; ++h2) {
        double th = 0.0;
        if (h1 || h2 || h3) {
          const double m2 = mh2[0][h1] + mh2[1][h2] + mh2[2][h3];
          th = std::exp(-kPi * kPi * m2 / (beta * beta)) / (kPi * V * m2) *
               bm[0][h1] * bm[1][h2] * bm[2][h3];
        }
        const double v = w[0][h1] * w[1][h2] * w[2][h3] * th;
        T[static_cast<size_t>(h3) * H12 + h1 * H[1] + h2] = v;
        norm2 += v * v;
      }
  out->theta_norm = std::sqrt(norm2);

  std::vector<double> s, U, Vt;
  if (!svd_rowmajor(H[2], H12, T, &s, &U, &Vt)) {
    *err = "outer Jacobi SVD did not converge";
    return false;
  }
  const double eps = 2.220446049250313e-16;
  struct Raw { double omega; int i, j; };
  std::vector<Raw> raw;
  std::vector<std::vector<double>> inner_x, inner_y;
  std::vector<std::vector<double>> inner_s;
  const int nouter = static_cast<int>(s.size());
  inner_x.resize(nouter);
  inner_y.resize(nouter);
  inner_s.resize(nouter);
  for (int i = 0; i < nouter; ++i) {
    if (!(s[i] > K[2] * eps * s[0])) break;
    std::vector<double> Vi(Vt.begin() + static_cast<size_t>(i) * H12,
                           Vt.begin() + static_cast<size_t>(i + 1) * H12);
    std::vector<double> si, X, Y;
    if (!svd_rowmajor(H[0], H[1], Vi, &si, &X, &Y)) {
      *err = "inner Jacobi SVD did not converge";
      return false;
    }
    inner_x[i] = X;
    inner_y[i] = Y;
    inner_s[i] = si;
    for (int j = 0; j < static_cast<int>(si.size()); ++j) {
      if (!(si[j] > std::max(K[0], K[1]) * eps * si[0])) break;
      raw.push_back({s[i] * si[j], i, j});
    }
  }
  std::stable_sort(raw.begin(), raw.end(),
                   [](const Raw& a, const Raw& b) { return a.omega > b.omega; });
  out->total_terms = static_cast<int>(raw.size());

  int R;
  if (rank > 0) {
    R = std::min<int>(rank, static_cast<int>(raw.size()));
  } else {
    double all = 0.0;
    for (const Raw& r : raw) all += r.omega * r.omega;
    const double missing = std::max(norm2 - all, 0.0);
    std::vector<double> tail(raw.size() + 1, 0.0);
    for (int r = static_cast<int>(raw.size()) - 1; r >= 0; --r)
      tail[r] = tail[r + 1] + raw[r].omega * raw[r].omega;
    R = static_cast<int>(raw.size());
    for (int r = 0; r <= static_cast<int>(raw.size()); ++r)
      if (std::sqrt(tail[r] + missing) <= tol * std::sqrt(norm2)) { R = r; break; }
  }
  double dropped = 0.0;
  for (size_t r = R; r < raw.size(); ++r) dropped += raw[r].omega * raw[r].omega;
  out->trunc_err = std::sqrt(dropped);

  auto unfold = [&](const double* folded, int axis) {
    std::vector<double> full(K[axis]);
    for (int m = 0; m < K[axis]; ++m) {
      const int ms = (m <= K[axis] / 2) ? m : m - K[axis];
      const int h = ms < 0 ? -ms : ms;
      full[m] = folded[h] / w[axis][h];
    }
    return full;
  };
  out->K[0] = K[0]; out->K[1] = K[1]; out->K[2] = K[2];
  out->terms.clear();
  double c0 = 0.0;
  for (int r = 0; r < R; ++r) {
    const Raw& rw = raw[r];
    Term t;
    t.omega = rw.omega;
    t.group = rw.i;
    t.inner = rw.j;
    t.v[0] = unfold(&inner_x[rw.i][static_cast<size_t>(rw.j) * H[0]], 0);
    t.v[1] = unfold(&inner_y[rw.i][static_cast<size_t>(rw.j) * H[1]], 1);
    t.v[2] = unfold(&U[static_cast<size_t>(rw.i) * H[2]], 2);
    c0 += t.omega * t.v[0][0] * t.v[1][0] * t.v[2][0];
    out->terms.push_back(std::move(t));
  }
  out->zero_mode = c0;
  return true;
}

}  // namespace kpme
