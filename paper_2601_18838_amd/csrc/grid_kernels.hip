// Particle <-> grid kernels: order-p cardinal B-spline spread and gather
// (the interpolation S_Y and its transpose S_X* of Eq. formfinale, in the
// B-spline form named in Sec. 2.2), and the FP64 energy reduction.
#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"

namespace kpme {

namespace {

// w[t] = M_P(f + t), dw[t] = M_P'(f + t) for t = 0..P-1 and f in [0, 1):
// the order-n values follow from order n-1 by
//   M_n(f+t) = [(f+t) M_{n-1}(f+t) + (n-f-t) M_{n-1}(f+t-1)] / (n-1),
// and M_P'(u) = M_{P-1}(u) - M_{P-1}(u-1).
template <typename T, int P>
__device__ __forceinline__ void bspline(T f, T* w, T* dw) {
  w[0] = T(1);
#pragma unroll
  for (int t = 1; t < P; ++t) w[t] = T(0);
#pragma unroll
  for (int n = 2; n <= P; ++n) {
    if (n == P) {
#pragma unroll
      for (int t = 0; t < P; ++t) dw[t] = w[t] - (t > 0 ? w[t - 1] : T(0));
    }
    const T inv = T(1) / T(n - 1);
#pragma unroll
    for (int t = n - 1; t >= 0; --t) {
      const T left = (f + T(t)) * w[t];
      const T right = (t > 0) ? (T(n) - f - T(t)) * w[t - 1] : T(0);
      w[t] = (left + right) * inv;
    }
  }
}

// Scaled coordinate of one axis, computed in double: u = K (x / L mod 1);
// returns the fractional part and sets the base grid index floor(u) mod K.
template <typename T>
__device__ __forceinline__ T scaled(T x, double L, int K, int& base) {
  double s = static_cast<double>(x) / L;
  s -= floor(s);
  const double u = s * K;
  const double fl = floor(u);
  int b = static_cast<int>(fl);
  if (b >= K) b -= K;
  // a non-finite coordinate must not index outside the grid (its NaN weights
  // still propagate into the results)
  if (!(b >= 0 && b < K)) b = 0;
  base = b;
  return static_cast<T>(u - fl);
}

template <typename T>
__global__ void zero_kernel(T* p, long n) {
  for (long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<long>(gridDim.x) * blockDim.x)
    p[i] = T(0);
}

template <typename T, int P>
__global__ __launch_bounds__(256) void spread_atomic(long n, const T* __restrict__ pos,
                                                     const T* __restrict__ q,
                                                     T* __restrict__ grid, GridGeom g) {
  const long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  T w[3][P], dw[P];
  int base[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const T f = scaled(pos[3 * i + j], g.L[j], g.K[j], base[j]);
    bspline<T, P>(f, w[j], dw);
  }
  const T qi = q[i];
  const int K1 = g.K[0], K2 = g.K[1], K3 = g.K[2];
  for (int a = 0; a < P; ++a) {
    int ka = base[0] - a;
    if (ka < 0) ka += K1;
    const T wa = qi * w[0][a];
    for (int b = 0; b < P; ++b) {
      int kb = base[1] - b;
      if (kb < 0) kb += K2;
      const T wab = wa * w[1][b];
      T* row = grid + (static_cast<long>(ka) * K2 + kb) * K3;
#pragma unroll
      for (int c = 0; c < P; ++c) {
        int kc = base[2] - c;
        if (kc < 0) kc += K3;
        atomicAdd(&row[kc], wab * w[2][c]);
      }
    }
  }
}

template <typename T, int P>
__global__ __launch_bounds__(256) void gather_direct(long n, const T* __restrict__ pos,
                                                     const T* __restrict__ q,
                                                     const T* __restrict__ grid,
                                                     T* __restrict__ pot,
                                                     T* __restrict__ force, GridGeom g) {
  const long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  T w[3][P], dw[3][P];
  int base[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const T f = scaled(pos[3 * i + j], g.L[j], g.K[j], base[j]);
    bspline<T, P>(f, w[j], dw[j]);
  }
  const int K1 = g.K[0], K2 = g.K[1], K3 = g.K[2];
  int kc[P];
#pragma unroll
  for (int c = 0; c < P; ++c) {
    kc[c] = base[2] - c;
    if (kc[c] < 0) kc[c] += K3;
  }
  T phi = 0, g0 = 0, g1 = 0, g2 = 0;
  for (int a = 0; a < P; ++a) {
    int ka = base[0] - a;
    if (ka < 0) ka += K1;
    T sa = 0, sa1 = 0, sa2 = 0;  // sums over b of (w1 s, dw1 s, w1 s')
    for (int b = 0; b < P; ++b) {
      int kb = base[1] - b;
      if (kb < 0) kb += K2;
      const T* row = grid + (static_cast<long>(ka) * K2 + kb) * K3;
      T s = 0, s2 = 0;
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const T v = row[kc[c]];
        s += w[2][c] * v;
        s2 += dw[2][c] * v;
      }
      sa += w[1][b] * s;
      sa1 += dw[1][b] * s;
      sa2 += w[1][b] * s2;
    }
    phi += w[0][a] * sa;
    g0 += dw[0][a] * sa;
    g1 += w[0][a] * sa1;
    g2 += w[0][a] * sa2;
  }
  if (pot) pot[i] = phi;
  if (force) {
    const T qi = q[i];
    force[3 * i + 0] = -qi * g0 * static_cast<T>(K1 / g.L[0]);
    force[3 * i + 1] = -qi * g1 * static_cast<T>(K2 / g.L[1]);
    force[3 * i + 2] = -qi * g2 * static_cast<T>(K3 / g.L[2]);
  }
}

// Per-block FP64 partial sums of (q pot, q, q^2), then one block combines
// them in a fixed order: the result does not depend on scheduling.
template <typename T>
__global__ __launch_bounds__(256) void energy_partial(long n, const T* __restrict__ q,
                                                      const T* __restrict__ pot,
                                                      double* __restrict__ part) {
  __shared__ double red[3][256];
  const long per = (n + gridDim.x - 1) / gridDim.x;
  const long b = per * blockIdx.x, e = (b + per < n) ? b + per : n;
  double s0 = 0, s1 = 0, s2 = 0;
  for (long i = b + threadIdx.x; i < e; i += blockDim.x) {
    const double qi = static_cast<double>(q[i]);
    s0 += qi * static_cast<double>(pot[i]);
    s1 += qi;
    s2 += qi * qi;
  }
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = s1;
  red[2][threadIdx.x] = s2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) part[3 * blockIdx.x + k] = red[k][0];
}

__global__ __launch_bounds__(256) void energy_final(const double* __restrict__ part, int nb,
                                                    double beta, double volume,
                                                    double* __restrict__ e4) {
  __shared__ double red[3][256];
  double s[3] = {0, 0, 0};
  for (int i = threadIdx.x; i < nb; i += 256)
    for (int k = 0; k < 3; ++k) s[k] += part[3 * i + k];
  for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double pi = 3.141592653589793238462643383279502884;
    const double e_rec = 0.5 * red[0][0];
    const double e_self = -beta / sqrt(pi) * red[2][0];
    const double e_neu = -pi * red[1][0] * red[1][0] / (2.0 * volume * beta * beta);
    e4[0] = e_rec;
    e4[1] = e_self;
    e4[2] = e_neu;
    e4[3] = e_rec + e_self + e_neu;
  }
}

template <typename T, int P>
hipError_t spread_p(const GridGeom& g, int64_t n, const void* pos, const void* q, void* grid,
                    hipStream_t st) {
  const unsigned blocks = static_cast<unsigned>((n + 255) / 256);
  hipLaunchKernelGGL((spread_atomic<T, P>), dim3(blocks), dim3(256), 0, st,
                     static_cast<long>(n), static_cast<const T*>(pos),
                     static_cast<const T*>(q), static_cast<T*>(grid), g);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t gather_p(const GridGeom& g, int64_t n, const void* pos, const void* q,
                    const void* grid, void* pot, void* force, hipStream_t st) {
  const unsigned blocks = static_cast<unsigned>((n + 255) / 256);
  hipLaunchKernelGGL((gather_direct<T, P>), dim3(blocks), dim3(256), 0, st,
                     static_cast<long>(n), static_cast<const T*>(pos),
                     static_cast<const T*>(q), static_cast<const T*>(grid),
                     static_cast<T*>(pot), static_cast<T*>(force), g);
  return hipGetLastError();
}

#define KPME_ORDER_SWITCH(P, CALL) \
  switch (P) {                     \
    case 4: return CALL(4);        \
    case 6: return CALL(6);        \
    case 8: return CALL(8);        \
    case 10: return CALL(10);      \
    case 12: return CALL(12);      \
    default: return hipErrorInvalidValue; \
  }

}  // namespace

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  const long n = static_cast<long>(bytes / 4);
  const unsigned blocks = static_cast<unsigned>(std::min<long>((n + 255) / 256, 4096));
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((zero_kernel<float>), dim3(blocks), dim3(256), 0, st,
                     static_cast<float*>(p), n);
  return hipGetLastError();
}

hipError_t launch_spread_atomic(int prec, const GridGeom& g, int64_t n, const void* pos,
                                const void* q, void* grid, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (prec == PREC_FP64) {
#define CALL(P) spread_p<double, P>(g, n, pos, q, grid, st)
    KPME_ORDER_SWITCH(g.p, CALL)
#undef CALL
  }
#define CALL(P) spread_p<float, P>(g, n, pos, q, grid, st)
  KPME_ORDER_SWITCH(g.p, CALL)
#undef CALL
}

hipError_t launch_gather_direct(int prec, const GridGeom& g, int64_t n, const void* pos,
                                const void* q, const void* grid, void* pot, void* force,
                                hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (prec == PREC_FP64) {
#define CALL(P) gather_p<double, P>(g, n, pos, q, grid, pot, force, st)
    KPME_ORDER_SWITCH(g.p, CALL)
#undef CALL
  }
#define CALL(P) gather_p<float, P>(g, n, pos, q, grid, pot, force, st)
  KPME_ORDER_SWITCH(g.p, CALL)
#undef CALL
}

hipError_t launch_energy(int prec, int64_t n, const void* q, const void* pot, double beta,
                         double volume, double* scratch, double* energy4, hipStream_t st) {
  const int nb = kSumBlocks;
  if (prec == PREC_FP64)
    hipLaunchKernelGGL((energy_partial<double>), dim3(nb), dim3(256), 0, st,
                       static_cast<long>(n), static_cast<const double*>(q),
                       static_cast<const double*>(pot), scratch);
  else
    hipLaunchKernelGGL((energy_partial<float>), dim3(nb), dim3(256), 0, st,
                       static_cast<long>(n), static_cast<const float*>(q),
                       static_cast<const float*>(pot), scratch);
  hipLaunchKernelGGL(energy_final, dim3(1), dim3(256), 0, st, scratch, nb, beta, volume,
                     energy4);
  return hipGetLastError();
}

}  // namespace kpme
