// Host-only driver for the plan-time factor construction (nested SVD by
// one-sided Jacobi, sinc quadrature, circulant columns, B-spline moduli),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py.  Each case checks a few invariants that
// hold for any correct run; a sanitizer report or a failed check exits
// non-zero.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "factors.hpp"

namespace {

int failures = 0;

void check(bool ok, const char* what, const char* name) {
  if (!ok) {
    std::fprintf(stderr, "FAIL %s: %s\n", name, what);
    ++failures;
  }
}

void check_set(const kpme::FactorSet& fs, const int K[3], const char* name) {
  check(!fs.terms.empty(), "no terms", name);
  check(std::isfinite(fs.theta_norm) && fs.theta_norm > 0, "theta norm", name);
  check(std::isfinite(fs.trunc_err) && fs.trunc_err >= 0, "tail", name);
  for (const kpme::Term& t : fs.terms) {
    check(std::isfinite(t.omega), "omega", name);
    for (int j = 0; j < 3; ++j) {
      check(static_cast<int>(t.v[j].size()) == K[j], "vector length", name);
      for (double x : t.v[j]) check(std::isfinite(x), "vector entry", name);
    }
  }
}

void nested(const double box[3], const int K[3], int p, double beta, int rank, double tol,
            kpme::KernelSpec ks, const char* name) {
  kpme::FactorSet fs;
  std::string err;
  const bool ok = kpme::build_factors(box, K, p, beta, rank, tol, ks, &fs, &err);
  check(ok, err.c_str(), name);
  if (!ok) return;
  check_set(fs, K, name);
  // the nested-SVD tail is part of the symbol's norm (the quadrature's error
  // also counts m = 0, where its symbol is the constant c)
  check(fs.trunc_err <= fs.theta_norm, "tail below the norm", name);
  if (rank > 0) check(static_cast<int>(fs.terms.size()) <= rank, "rank", name);
  if (rank <= 0) check(fs.trunc_err <= tol * fs.theta_norm * (1 + 1e-12), "tolerance", name);
  for (const kpme::Term& t : fs.terms) {
    const std::vector<double> col = kpme::circulant_column(t.v[0]);
    check(static_cast<int>(col.size()) == K[0], "circulant length", name);
  }
  std::printf("%s: R = %zu, tail %.3e\n", name, fs.terms.size(), fs.trunc_err / fs.theta_norm);
}

void quadrature(const double box[3], const int K[3], int p, double beta, int rank, double tol,
                const char* name) {
  kpme::FactorSet fs;
  std::string err;
  const bool ok = kpme::build_factors_quadrature(box, K, p, beta, rank, tol, 0.0,
                                                 kpme::KernelSpec{}, &fs, &err);
  check(ok, err.c_str(), name);
  if (!ok) return;
  check_set(fs, K, name);
  check(static_cast<int>(fs.terms.size()) == 2 * fs.quad_N + 1, "2N + 1 terms", name);
  check(fs.zero_mode > 0, "c = sum of the weights", name);
  if (rank <= 0) check(fs.sym_err <= tol, "symbol error", name);
  std::printf("%s: N = %d, h = %.4f, symbol error %.3e\n", name, fs.quad_N, fs.quad_h,
              fs.sym_err);
}

}  // namespace

int main() {
  for (int p = 2; p <= 12; p += 2) {
    const std::vector<double> m = kpme::bspline_moduli(20, p);
    check(static_cast<int>(m.size()) == 20, "moduli length", "moduli");
    for (double x : m) check(std::isfinite(x) && x > 0, "moduli positive", "moduli");
  }
  const double cube[3] = {20.0, 20.0, 20.0}, rect[3] = {12.0, 15.0, 18.0};
  const int g16[3] = {16, 16, 16}, g_nc[3] = {20, 25, 30}, g_odd[3] = {9, 11, 13};
  nested(cube, g16, 4, 0.35, 8, 0.0, kpme::KernelSpec{}, "nested 16^3 p4 R8");
  nested(cube, g16, 6, 0.35, 0, 1e-6, kpme::KernelSpec{}, "nested 16^3 p6 tol");
  nested(rect, g_nc, 6, 0.5, 0, 1e-8, kpme::KernelSpec{}, "nested 20x25x30 p6 tol");
  nested(rect, g_odd, 4, 0.6, 1000000, 0.0, kpme::KernelSpec{}, "nested odd grid full rank");
  kpme::KernelSpec lag;
  lag.lagrange = true;
  lag.cutoff = 5;
  const int g_lag[3] = {20, 20, 20};
  nested(cube, g_lag, 6, 0.6, 0, 1e-6, lag, "nested Lagrange M5");
  quadrature(cube, g16, 4, 0.35, 0, 1e-6, "sinc 16^3 tol");
  quadrature(rect, g_nc, 6, 0.5, 21, 0.0, "sinc 20x25x30 R21");
  if (failures) {
    std::fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
