// The Kronecker operator through rectangular real cos/sin factors (Sec. 2.3,
// Eq. kronw; Sec. 2.4, Eq. VtV).
//
// A per-axis factor with an even mode vector a(m) that vanishes beyond
// |m'| <= M is A = F^T diag(d) F: F the n x K matrix of the real Fourier rows
// 1, cos(2 pi m g / K), sin(2 pi m g / K) (m = 1..M; no sine row at the
// Nyquist mode of an even K; n = min(2M + 1, K)) and d = (a(0), 2 a(m),
// 2 a(m), ...) (a(K/2) at the Nyquist row).  F does not depend on the term,
// only d does, so the whole operator is
//   sum_r omega_r A_r (x) B_r (x) C_r
//     = (F1 (x) F2 (x) F3)^T  D  (F1 (x) F2 (x) F3),
//   D = sum_r omega_r d_r1 (x) d_r2 (x) d_r3   (an n1 x n2 x n3 diagonal):
// every term's two thin products per mode product (V X, then V^T (S V X))
// share their outer factors, so they are taken once for all terms -- three
// thin products into the real mode basis, one scaling by D, three back.
// Each thin product contracts the last axis of a row-major 3-D array and
// puts the new axis first, Y[n][a][b] = sum_c X[a][b][c] W[n][c]: three of
// them cycle the axes back to [k1][k2][k3].  They are plain GEMMs and run on
// rocBLAS; the scaling, the constant correction and the energy partials are
// kernels here.  FP64 and FP32.
#include <rocblas/rocblas.h>

#include <cmath>
#include <vector>

#include "batch_launch.hpp"
#include "device_common.hpp"
#include "kernels.hpp"
#include "rect.hpp"

namespace kpme {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void rect_scale(T* __restrict__ Y, const T* __restrict__ D,
                                                  long n) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += 256L * gridDim.x) Y[i] *= D[i];
}

// Phi -= c0 sum(Q) in place, and (epart != NULL) per-workgroup FP64 sums of
// Q Phi over the values written, with the workgroup grid of the circulant
// path's finalize (finalize_blocks() partials, one per 32 x 32 (k2, k3) tile
// of a k1 plane).
template <typename T>
__global__ __launch_bounds__(256) void rect_finalize(T* __restrict__ Phi, int K1, int K2, int K3,
                                                     const double* __restrict__ sumQ, double c0,
                                                     const T* __restrict__ Q,
                                                     double* __restrict__ epart) {
  __shared__ double red[16];
  const int k1 = blockIdx.z, k2b = blockIdx.x * 32, k3b = blockIdx.y * 32, t = threadIdx.x;
  const T corr = static_cast<T>(c0 * sumQ[0]);
  double e = 0.0;
  for (int j = t >> 5; j < 32; j += 8) {
    const int k2 = k2b + j, k3 = k3b + (t & 31);
    if (k2 < K2 && k3 < K3) {
      const long at = (static_cast<long>(k1) * K2 + k2) * K3 + k3;
      const T v = Phi[at] - corr;
      Phi[at] = v;
      if (epart) e += static_cast<double>(Q[at]) * static_cast<double>(v);
    }
  }
  if (epart) {
    double v[1] = {e};
    block_reduce<1, 1>(v, red);
    if (t == 0)
      epart[(static_cast<long>(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = v[0];
  }
}

// Y[n][ab] = sum_c X[ab][c] W[n][c] (row-major): in column-major terms
// Y^T = X^T-view times W-view, one GEMM.
rocblas_status rotate(rocblas_handle h, bool fp64, long ab, int n, int c, const void* X,
                      const void* W, void* Y) {
  if (fp64) {
    const double one = 1.0, zero = 0.0;
    return rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none,
                         static_cast<rocblas_int>(ab), n, c, &one,
                         static_cast<const double*>(X), c, static_cast<const double*>(W), c,
                         &zero, static_cast<double*>(Y), static_cast<rocblas_int>(ab));
  }
  const float one = 1.f, zero = 0.f;
  return rocblas_sgemm(h, rocblas_operation_transpose, rocblas_operation_none,
                       static_cast<rocblas_int>(ab), n, c, &one, static_cast<const float*>(X), c,
                       static_cast<const float*>(W), c, &zero, static_cast<float*>(Y),
                       static_cast<rocblas_int>(ab));
}

hipError_t from_rocblas(rocblas_status s) {
  if (s == rocblas_status_success) return hipSuccess;
  if (s == rocblas_status_memory_error) return hipErrorOutOfMemory;
  return hipErrorLaunchFailure;
}

}  // namespace

std::vector<double> rect_rows(int K, int M, std::vector<int>* modes) {
  std::vector<double> F;
  modes->clear();
  const double pi = 3.141592653589793238462643383279502884;
  auto row = [&](int m, bool sine) {
    for (int g = 0; g < K; ++g) {
      // exact angle reduction: m g mod K before the trigonometric call
      const double t = 2.0 * pi * static_cast<double>((static_cast<long>(m) * g) % K) / K;
      F.push_back(m == 0 ? 1.0 : (sine ? std::sin(t) : std::cos(t)));
    }
    modes->push_back(m);
  };
  row(0, false);
  for (int m = 1; m <= M; ++m) {
    row(m, false);
    if (2 * m != K) row(m, true);
  }
  return F;
}

std::vector<double> rect_weights(const std::vector<double>& a, const std::vector<int>& modes) {
  const int K = static_cast<int>(a.size());
  std::vector<double> d(modes.size());
  for (size_t i = 0; i < modes.size(); ++i) {
    const int m = modes[i];
    d[i] = (m == 0 || 2 * m == K) ? a[m] : 2.0 * a[m];
  }
  return d;
}

hipError_t rect_create_handle(void** handle) {
  rocblas_handle h = nullptr;
  const rocblas_status s = rocblas_create_handle(&h);
  *handle = h;
  return from_rocblas(s);
}

void rect_destroy_handle(void* handle) {
  if (handle) (void)rocblas_destroy_handle(static_cast<rocblas_handle>(handle));
}

hipError_t launch_rect_apply(const RectArgs& a, hipStream_t st) {
  if (record_unsupported()) return hipSuccess;
  rocblas_handle h = static_cast<rocblas_handle>(a.handle);
  rocblas_status s = rocblas_set_stream(h, st);
  const bool f64 = a.fp64;
  const int K1 = a.K[0], K2 = a.K[1], K3 = a.K[2];
  const int n1 = a.n[0], n2 = a.n[1], n3 = a.n[2];
  // forward: Q[K1][K2][K3] -> [n3][K1][K2] -> [n2][n3][K1] -> [n1][n2][n3]
  if (s == rocblas_status_success) s = rotate(h, f64, static_cast<long>(K1) * K2, n3, K3, a.Q, a.F[2], a.wa);
  if (s == rocblas_status_success) s = rotate(h, f64, static_cast<long>(n3) * K1, n2, K2, a.wa, a.F[1], a.wb);
  if (s == rocblas_status_success) s = rotate(h, f64, static_cast<long>(n2) * n3, n1, K1, a.wb, a.F[0], a.wa);
  if (s != rocblas_status_success) return from_rocblas(s);
  const long nd = static_cast<long>(n1) * n2 * n3;
  const unsigned blocks = static_cast<unsigned>(std::min<long>((nd + 255) / 256, 8192));
  if (f64)
    hipLaunchKernelGGL((rect_scale<double>), dim3(blocks), dim3(256), 0, st,
                       static_cast<double*>(a.wa), static_cast<const double*>(a.D), nd);
  else
    hipLaunchKernelGGL((rect_scale<float>), dim3(blocks), dim3(256), 0, st,
                       static_cast<float*>(a.wa), static_cast<const float*>(a.D), nd);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // back: [n1][n2][n3] -> [K3][n1][n2] -> [K2][K3][n1] -> [K1][K2][K3]
  s = rotate(h, f64, static_cast<long>(n1) * n2, K3, n3, a.wa, a.Ft[2], a.wb);
  if (s == rocblas_status_success) s = rotate(h, f64, static_cast<long>(K3) * n1, K2, n2, a.wb, a.Ft[1], a.wa);
  if (s == rocblas_status_success) s = rotate(h, f64, static_cast<long>(K2) * K3, K1, n1, a.wa, a.Ft[0], a.Phi);
  return from_rocblas(s);
}

hipError_t launch_rect_finalize(const RectArgs& a, hipStream_t st) {
  if (record_unsupported()) return hipSuccess;
  dim3 gf((a.K[1] + 31) / 32, (a.K[2] + 31) / 32, a.K[0]);
  if (a.fp64)
    hipLaunchKernelGGL((rect_finalize<double>), gf, dim3(256), 0, st, static_cast<double*>(a.Phi),
                       a.K[0], a.K[1], a.K[2], a.sumQ, a.c0, static_cast<const double*>(a.Q),
                       a.epart);
  else
    hipLaunchKernelGGL((rect_finalize<float>), gf, dim3(256), 0, st, static_cast<float*>(a.Phi),
                       a.K[0], a.K[1], a.K[2], a.sumQ, a.c0, static_cast<const float*>(a.Q),
                       a.epart);
  return hipGetLastError();
}

}  // namespace kpme
