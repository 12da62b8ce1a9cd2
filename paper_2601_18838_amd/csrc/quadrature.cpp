// Host FP64 sinc-quadrature factors of the smooth-PME reciprocal kernel.
//
// 1/x is the integral of exp(-t x) over t > 0 (Sec. 2.1.2, Eq.
// one_over_r_int); the cardinal-sine rule with nodes lambda_l = log(1 + e^{lh})
// and weights omega_l = h / (1 + e^{-lh}), l = -N..N, turns it into a sum of
// exponentials.  The smooth-PME symbol
//   theta_hat(m) = exp(-pi^2 |m_hat|^2 / beta^2) / (pi V |m_hat|^2) prod_j |b_j(m_j)|^2
// keeps its Gaussian and B-spline factors exactly, and 1 / |m_hat|^2 is
// written as s / x with x = s |m_hat|^2, s = max_j L_j^2, so that x >= 1 for
// every m != 0 (the range the paper's rule is stated for).  Each node is then
// one Kronecker term (Eq. quaddecompalpham) with weight s omega_l / (pi V)
// and per-axis mode vectors
//   a_{l,j}(m) = |b_j(m)|^2 exp(-(s lambda_l + pi^2 / beta^2) (m'_j / L_j)^2),
// and the operator's value at m = 0, c = s sum_l omega_l / (pi V), is what
// the constant correction removes.
//
// The lifting factor h is chosen as the paper does, by trying values of h
// for the given N and measuring the error on every argument that occurs:
// for m != 0 the quadrature symbol is theta_hat(m) x q(x) with
// q(x) = sum_l omega_l e^{-lambda_l x}, so the max-norm error relative to
// max theta_hat is max over the distinct x of W(x) |x q(x) - 1|, W(x) the
// largest theta_hat / max theta_hat among the modes with that x (computed on
// the folded, even half domain).  Plan-time only.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <utility>

#include "factors.hpp"

namespace kpme {

namespace {

constexpr double kPiQ = 3.141592653589793238462643383279502884;

struct WeightedArgs {
  std::vector<double> x;  // distinct non-zero arguments s |m_hat|^2, ascending
  std::vector<double> w;  // largest relative symbol value at each
};

// max over the arguments of W(x) |x q(x) - 1| for the rule (N, h)
double rule_error(const WeightedArgs& wa, int N, double h) {
  std::vector<double> om(2 * N + 1), la(2 * N + 1);
  for (int l = -N; l <= N; ++l) {
    om[l + N] = h / (1.0 + std::exp(-l * h));
    la[l + N] = std::log1p(std::exp(l * h));
  }
  double worst = 0.0;
  for (size_t i = 0; i < wa.x.size(); ++i) {
    const double x = wa.x[i];
    double q = 0.0;
    for (int k = 0; k < 2 * N + 1; ++k) q += om[k] * std::exp(-la[k] * x);
    worst = std::max(worst, wa.w[i] * std::fabs(x * q - 1.0));
  }
  return worst;
}

// Best h on the geometric scan h0 2^(k/16), k = -48..32, h0 = pi / sqrt(2N + 1):
// every fourth point first, then the points within 3/16 of an octave of the
// best of those.
std::pair<double, double> best_rule_h(const WeightedArgs& wa, int N) {
  const double h0 = kPiQ / std::sqrt(2.0 * N + 1.0);
  int best_k = 0;
  double best_e = -1.0;
  auto visit = [&](int k) {
    const double e = rule_error(wa, N, h0 * std::exp2(k / 16.0));
    if (best_e < 0.0 || e < best_e) { best_e = e; best_k = k; }
  };
  for (int k = -48; k <= 32; k += 4) visit(k);
  const int kc = best_k;
  for (int k = std::max(-48, kc - 3); k <= std::min(32, kc + 3); ++k)
    if (k != kc) visit(k);
  return {h0 * std::exp2(best_k / 16.0), best_e};
}

}  // namespace

bool build_factors_quadrature(const double box[3], const int K[3], int p, double beta,
                              int rank, double tol, double h, const KernelSpec& ks,
                              FactorSet* out, std::string* err) {
  const double V = box[0] * box[1] * box[2];
  const double s = std::pow(std::max(box[0], std::max(box[1], box[2])), 2);
  // folded half domain: h_j = |m'_j| in [0, K_j / 2], multiplicity 1 or 2
  int H[3];
  std::vector<double> bm[3], mh2[3], mult[3];
  for (int j = 0; j < 3; ++j) {
    H[j] = K[j] / 2 + 1;
    const std::vector<double> full = ks.lagrange ? std::vector<double>() : bspline_moduli(K[j], p);
    bm[j].resize(H[j]);
    mh2[j].resize(H[j]);
    mult[j].resize(H[j]);
    for (int i = 0; i < H[j]; ++i) {
      bm[j][i] = ks.axis_factor(full, i);
      const double mh = i / box[j];
      mh2[j][i] = mh * mh;
      mult[j][i] = (i == 0 || (K[j] % 2 == 0 && i == K[j] / 2)) ? 1.0 : 2.0;
    }
  }
  // symbol on the folded domain, its maximum and Frobenius norm
  const size_t nf = static_cast<size_t>(H[0]) * H[1] * H[2];
  std::vector<double> xs(nf), th(nf);
  double thmax = 0.0, norm2 = 0.0;
  for (int a = 0; a < H[0]; ++a)
    for (int b = 0; b < H[1]; ++b)
      for (int c = 0; c < H[2]; ++c) {
        const size_t i = (static_cast<size_t>(a) * H[1] + b) * H[2] + c;
        const double m2 = mh2[0][a] + mh2[1][b] + mh2[2][c];
        xs[i] = s * m2;
        th[i] = (i == 0) ? 0.0
                         : std::exp(-kPiQ * kPiQ * m2 / (beta * beta)) / (kPiQ * V * m2) *
                               bm[0][a] * bm[1][b] * bm[2][c];
        thmax = std::max(thmax, th[i]);
        norm2 += mult[0][a] * mult[1][b] * mult[2][c] * th[i] * th[i];
      }
  if (!(thmax > 0.0)) {
    *err = "the kernel symbol vanishes on this grid";
    return false;
  }
  // distinct arguments with their largest relative symbol value
  WeightedArgs wa;
  {
    std::vector<size_t> idx(nf - 1);
    std::iota(idx.begin(), idx.end(), size_t(1));
    std::sort(idx.begin(), idx.end(), [&](size_t u, size_t v) { return xs[u] < xs[v]; });
    for (size_t i : idx) {
      const double w = th[i] / thmax;
      if (!wa.x.empty() && xs[i] == wa.x.back()) {
        wa.w.back() = std::max(wa.w.back(), w);
      } else {
        wa.x.push_back(xs[i]);
        wa.w.push_back(w);
      }
    }
  }
  // the rule: N fixed by the rank, or the smallest N whose best h meets tol
  int N;
  double err_inf;
  if (rank > 0) {
    if (rank % 2 == 0) {
      *err = "the sinc rule has 2N + 1 nodes: the rank must be odd";
      return false;
    }
    N = (rank - 1) / 2;
    if (h > 0.0) {
      err_inf = rule_error(wa, N, h);
    } else {
      const auto b = best_rule_h(wa, N);
      h = b.first;
      err_inf = b.second;
    }
  } else {
    // the best error falls with N: bracket by doubling, then bisect
    auto best_at = [&](int n) { return h > 0.0 ? std::make_pair(h, rule_error(wa, n, h))
                                               : best_rule_h(wa, n); };
    constexpr int kMaxN = 512;
    int lo = -1, hi = 0;
    std::pair<double, double> at_hi = best_at(0);
    while (at_hi.second > tol) {
      lo = hi;
      hi = hi == 0 ? 1 : 2 * hi;
      if (hi > kMaxN) {
        *err = "no sinc rule with N <= 512 meets the tolerance";
        return false;
      }
      at_hi = best_at(hi);
    }
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      const auto at_mid = best_at(mid);
      if (at_mid.second <= tol) { hi = mid; at_hi = at_mid; } else { lo = mid; }
    }
    N = hi;
    h = at_hi.first;
    err_inf = at_hi.second;
  }

  // terms: unit mode vectors on the full axes, weights carrying the norms
  out->K[0] = K[0]; out->K[1] = K[1]; out->K[2] = K[2];
  out->terms.clear();
  out->theta_norm = std::sqrt(norm2);
  out->quad_N = N;
  out->quad_h = h;
  out->sym_err = err_inf;
  std::vector<std::vector<double>> folded[3];
  std::vector<double> weight(2 * N + 1);
  double c0 = 0.0;
  for (int l = -N; l <= N; ++l) {
    const double om = h / (1.0 + std::exp(-l * h));
    const double la = std::log1p(std::exp(l * h));
    Term t;
    t.group = l + N;
    t.inner = 0;
    double w = s * om / (kPiQ * V);
    for (int j = 0; j < 3; ++j) {
      std::vector<double> f(H[j]);
      for (int i = 0; i < H[j]; ++i)
        f[i] = bm[j][i] * std::exp(-(s * la + kPiQ * kPiQ / (beta * beta)) * mh2[j][i]);
      double n2 = 0.0;
      for (int i = 0; i < H[j]; ++i) n2 += mult[j][i] * f[i] * f[i];
      const double nrm = std::sqrt(n2);
      w *= nrm;
      t.v[j].resize(K[j]);
      for (int m = 0; m < K[j]; ++m) {
        const int ms = (m <= K[j] / 2) ? m : m - K[j];
        t.v[j][m] = f[ms < 0 ? -ms : ms] / nrm;
      }
      for (double& v : f) v /= nrm;
      folded[j].push_back(std::move(f));
    }
    t.omega = w;
    weight[l + N] = w;
    c0 += w * t.v[0][0] * t.v[1][0] * t.v[2][0];
    out->terms.push_back(std::move(t));
  }
  out->zero_mode = c0;
  out->total_terms = 2 * N + 1;
  // ||theta_hat - theta_Lambda||_F over the full mode grid (m = 0 included,
  // where theta_hat is 0 and the quadrature symbol is c)
  double d2 = 0.0;
  for (int a = 0; a < H[0]; ++a)
    for (int b = 0; b < H[1]; ++b)
      for (int c = 0; c < H[2]; ++c) {
        double v = 0.0;
        for (int r = 0; r < 2 * N + 1; ++r)
          v += weight[r] * folded[0][r][a] * folded[1][r][b] * folded[2][r][c];
        const size_t i = (static_cast<size_t>(a) * H[1] + b) * H[2] + c;
        const double d = v - th[i];
        d2 += mult[0][a] * mult[1][b] * mult[2][c] * d * d;
      }
  out->trunc_err = std::sqrt(d2);
  return true;
}

}  // namespace kpme
