// Particle <-> grid kernels: order-p cardinal B-spline spread and gather
// (the interpolation S_Y and its transpose S_X* of Eq. formfinale, in the
// B-spline form named in Sec. 2.2), and the FP64 energy reduction.
#include <algorithm>

#include "batch_launch.hpp"
#include "device_common.hpp"
#include "kernels.hpp"

namespace kpme {

namespace {

// w[t] = M_P(f + t), dw[t] = M_P'(f + t) for t = 0..P-1 and f in [0, 1).
// With W_n = (n-1)! M_n the order-n values follow from order n-1 by
//   W_n(f+t) = (f+t) W_{n-1}(f+t) + (n-f-t) W_{n-1}(f+t-1),
// of which only the n entries t = 0..n-1 are non-zero (W_{n-1}(f+n-1) and
// W_{n-1}(f-1) vanish), and M_P'(u) = M_{P-1}(u) - M_{P-1}(u-1); the
// factorials are divided out at the end.
template <typename T, int P>
__device__ __forceinline__ void bspline(T f, T* w, T* dw) {
  w[0] = T(1);
#pragma unroll
  for (int n = 2; n <= P; ++n) {
    if (n == P) {
      dw[0] = w[0];
#pragma unroll
      for (int t = 1; t < P - 1; ++t) dw[t] = w[t] - w[t - 1];
      dw[P - 1] = -w[P - 2];
    }
    w[n - 1] = (T(1) - f) * w[n - 2];
#pragma unroll
    for (int t = n - 2; t >= 1; --t) w[t] = (f + T(t)) * w[t] + (T(n - t) - f) * w[t - 1];
    w[0] = f * w[0];
  }
  double fw = 1.0, fd = 1.0;
#pragma unroll
  for (int k = 2; k < P; ++k) {
    fw *= k;
    if (k < P - 1) fd *= k;
  }
  const T sw = static_cast<T>(1.0 / fw), sd = static_cast<T>(1.0 / fd);
#pragma unroll
  for (int t = 0; t < P; ++t) {
    w[t] *= sw;
    dw[t] *= sd;
  }
}

// Scaled coordinate of one axis, computed in double: u = K (x / L mod 1),
// with x / L taken as x times the host-computed 1 / L; returns the fractional
// part and sets the base grid index floor(u) mod K.
//
// The compiler may fuse x * invL with the subtraction of its floor into one
// FMA, which subtracts from the exact product: for x on the box face
// (x = L) the exact product can lie just below the rounded 1.0, so s comes
// out as a tiny negative number, u slightly below 0, floor(u) = -1 and the
// fraction ~1.  That is the same stencil as base 0 with fraction 0, and is
// kept as such by wrapping the base into [0, K) from either side.
template <typename T>
__device__ __forceinline__ T scaled(T x, double invL, int K, int& base) {
  double s = static_cast<double>(x) * invL;
  s -= floor(s);
  const double u = s * K;
  const double fl = floor(u);
  int b = static_cast<int>(fl);
  if (b >= K) b -= K;
  if (b < 0) b += K;
  // a non-finite coordinate must not index outside the grid (its NaN weights
  // still propagate into the results)
  if (!(b >= 0 && b < K)) b = 0;
  base = b;
  return static_cast<T>(u - fl);
}

// Scaled coordinate and stencil base of one axis for either interpolation
// rule (GridGeom::cell), computed in double:
//   B-spline (cell == 0): u = K (x / L mod 1), base = floor(u) mod K, and the
//     returned fractional part f in [0, 1) gives the weights M_p(f + t);
//   Lagrange (cell = p - 1): the particle's cell c = floor(u / cell) has the
//     nodes c cell + s, s = 0..p-1 (end points shared with the neighbouring
//     cells); base = (c + 1) cell mod K, its last node, and the returned
//     xi = u - c cell in [0, cell] is the position inside the cell.
// Either way grid point (base - t) mod K carries stencil weight w[t].  Binning
// and every spread and gather call this same function, so a particle's base
// (and with it its brick) is the same everywhere.
template <typename T>
__device__ __forceinline__ T stencil_coord(T x, double invL, int K, int cell, int& base) {
  if (cell == 0) return scaled(x, invL, K, base);
  double s = static_cast<double>(x) * invL;
  s -= floor(s);
  double u = s * K;
  const int Kc = K / cell;
  int c = static_cast<int>(floor(u / cell));
  if (c >= Kc) {  // u rounded up to K: the first cell
    c -= Kc;
    u -= K;
  }
  if (c < 0) {    // u slightly below 0 (see scaled): the last cell
    c += Kc;
    u += K;
  }
  // a non-finite coordinate must not index outside the grid (its NaN weights
  // still propagate into the results)
  if (!(c >= 0 && c < Kc)) {
    c = 0;
    u = 0.0;
  }
  int b = (c + 1) * cell;
  if (b >= K) b -= K;
  base = b;
  return static_cast<T>(u - static_cast<double>(c) * cell);
}

// prod_{r != s} (s - r) over the nodes 0..P-1.
__host__ __device__ constexpr double lagrange_denom(int s, int P) {
  double d = 1.0;
  for (int r = 0; r < P; ++r)
    if (r != s) d *= static_cast<double>(s - r);
  return d;
}

// Lagrange basis of the P integer nodes 0..P-1 of one cell (Eq. interp1d with
// the cell mapped onto them) at xi: w[t] = l_{P-1-t}(xi) with
// l_s(xi) = prod_{r != s} (xi - r) / (s - r), and dw[t] its derivative in xi,
// from prefix and suffix products of (xi - r) and their derivatives.
template <typename T, int P>
__device__ __forceinline__ void lagrange(T xi, T* w, T* dw) {
  T pre[P + 1], dpre[P + 1], suf[P + 1], dsuf[P + 1];
  pre[0] = T(1);
  dpre[0] = T(0);
#pragma unroll
  for (int r = 0; r < P; ++r) {
    pre[r + 1] = pre[r] * (xi - T(r));
    dpre[r + 1] = dpre[r] * (xi - T(r)) + pre[r];
  }
  suf[P] = T(1);
  dsuf[P] = T(0);
#pragma unroll
  for (int r = P - 1; r >= 0; --r) {
    suf[r] = suf[r + 1] * (xi - T(r));
    dsuf[r] = dsuf[r + 1] * (xi - T(r)) + suf[r + 1];
  }
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const T inv = static_cast<T>(1.0 / lagrange_denom(s, P));
    w[P - 1 - s] = pre[s] * suf[s + 1] * inv;
    dw[P - 1 - s] = (dpre[s] * suf[s + 1] + pre[s] * dsuf[s + 1]) * inv;
  }
}

// Stencil weights and their derivatives in u for either rule.
template <typename T, int P>
__device__ __forceinline__ void stencil_weights(T f, int cell, T* w, T* dw) {
  if (cell == 0)
    bspline<T, P>(f, w, dw);
  else
    lagrange<T, P>(f, w, dw);
}

template <typename T>
__global__ void zero_kernel(T* p, long n) {
  for (long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<long>(gridDim.x) * blockDim.x)
    p[i] = T(0);
}

// The energy job of an evaluation (see EnergyJob), in a fixed order; one
// workgroup, every thread calls it.
__device__ void run_energy_job(const EnergyJob& ej) {
  __shared__ double red[48];
  double v[3] = {0.0, 0.0, 0.0};  // sum Q Phi, sum q, sum q^2
  const int nt = blockDim.x;
  for (int i0 = threadIdx.x; i0 < ej.nfin; i0 += 4 * nt) {  // four loads in flight
    double x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = i0 + u * nt < ej.nfin ? ej.epart[i0 + u * nt] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) v[0] += x[u];
  }
  for (int i0 = threadIdx.x; i0 < ej.nq; i0 += 4 * nt) {
    double2 x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      x[u] = i0 + u * nt < ej.nq ? *reinterpret_cast<const double2*>(&ej.qpart[2 * (i0 + u * nt)])
                                 : double2{0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      v[1] += x[u].x;
      v[2] += x[u].y;
    }
  }
  block_reduce<3, 3>(v, red);
  if (threadIdx.x == 0) {
    const double pi = 3.141592653589793238462643383279502884;
    const double e_rec = 0.5 * v[0];
    const double e_self = -ej.beta / sqrt(pi) * v[2];
    const double e_neu = -pi * v[1] * v[1] / (2.0 * ej.volume * ej.beta * ej.beta);
    ej.e4[0] = e_rec;
    ej.e4[1] = e_self;
    ej.e4[2] = e_neu;
    ej.e4[3] = e_rec + e_self + e_neu;
  }
}

__device__ __forceinline__ void energy_job_body(EnergyJob ej, const Wg) { run_energy_job(ej); }
__global__ __launch_bounds__(256) void energy_job_kernel(EnergyJob ej) { run_energy_job(ej); }

// Per-workgroup FP64 (sum q, sum q^2) of the scatter.  Every thread calls it.
__device__ void charge_partials(double s1, double s2, double* qpart, int blk) {
  __shared__ double red[32];
  double v[2] = {s1, s2};
  block_reduce<2, 2>(v, red);
  if (threadIdx.x == 0) {
    qpart[2 * blk] = v[0];
    qpart[2 * blk + 1] = v[1];
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
    const T f = stencil_coord(pos[3 * i + j], g.invL[j], g.K[j], g.cell, base[j]);
    stencil_weights<T, P>(f, g.cell, w[j], dw[j]);
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
    force[3 * i + 0] = -qi * g0 * static_cast<T>(K1 * g.invL[0]);
    force[3 * i + 1] = -qi * g1 * static_cast<T>(K2 * g.invL[1]);
    force[3 * i + 2] = -qi * g2 * static_cast<T>(K3 * g.invL[2]);
  }
}

// ---------------------------------------------------------------------------
// Binning: particles are counting-sorted by the grid brick that holds their
// base index floor(u) (brick edge E_j, NB_j = ceil(K_j / E_j) bricks per axis).

template <typename T>
__device__ __forceinline__ int brick_of_particle(const T* __restrict__ pos, long i,
                                                 const GridGeom& g, const BinGeom& bg) {
  int bid = 0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    int base;
    (void)stencil_coord(pos[3 * i + j], g.invL[j], g.K[j], g.cell, base);
    // edges are 8 unless the axis is shorter (a uniform branch)
    bid = bid * bg.nb[j] + (bg.edge[j] == 8 ? base >> 3 : base / bg.edge[j]);
  }
  return bid;
}

// Histogram with a per-workgroup LDS copy (up to kLdsHist bricks): each
// workgroup ranks its particles inside the bricks in LDS, then reserves one
// range per brick with a single global atomic.  count[] must be zero on entry.
// The global atomics on one counter are serialised, so on large systems
// their number per counter (about the number of workgroups) sets the time:
// workgroups of 1024 threads from kCountBig particles on (1M atoms, 4,096
// bricks: 24.8 -> 14.3 us), 256 below (more workgroups in flight; equal or
// slightly faster up to ~1e5 particles).
constexpr int kBinPer = 4;         // particles per thread of the scatter
constexpr int kCountPer = 8;       // particles per thread of the LDS-histogram count
constexpr long kCountBig = 32L * 1024 * kCountPer;
constexpr int kLdsHist = 8192;     // bricks handled with an LDS histogram

template <typename T, int NT>
__device__ __forceinline__ void bin_count_lds_body(long n, const T* __restrict__ pos,
                                                     GridGeom g, BinGeom bg,
                                                     int* __restrict__ brick_of,
                                                     int* __restrict__ slot,
                                                     int* __restrict__ count,
    const Wg wg) {
  __shared__ int hist[kLdsHist];
  const int nb = bg.nbricks;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  const long base = static_cast<long>(wg.x) * blockDim.x * kCountPer;
  int bid[kCountPer], loc[kCountPer];
#pragma unroll
  for (int k = 0; k < kCountPer; ++k) {
    const long i = base + static_cast<long>(k) * blockDim.x + threadIdx.x;
    bid[k] = -1;
    if (i < n) {
      bid[k] = brick_of_particle(pos, i, g, bg);
      loc[k] = atomicAdd(&hist[bid[k]], 1);
    }
  }
  __syncthreads();
  // one global atomic per non-empty brick (hist then holds this block's
  // base), issued kFlush at a time so that their round trips overlap
  static_assert(kLdsHist % NT == 0, "the flush covers the histogram in one pass");
  constexpr int kFlush = kLdsHist / NT;
  for (int b0 = threadIdx.x; b0 < nb; b0 += kFlush * blockDim.x) {
    int c[kFlush];
#pragma unroll
    for (int k = 0; k < kFlush; ++k) {
      const int b = b0 + k * static_cast<int>(blockDim.x);
      c[k] = b < nb ? hist[b] : 0;
    }
#pragma unroll
    for (int k = 0; k < kFlush; ++k)
      if (c[k]) c[k] = atomicAdd(&count[b0 + k * static_cast<int>(blockDim.x)], c[k]);
#pragma unroll
    for (int k = 0; k < kFlush; ++k) {
      const int b = b0 + k * static_cast<int>(blockDim.x);
      if (b < nb) hist[b] = c[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kCountPer; ++k) {
    const long i = base + static_cast<long>(k) * blockDim.x + threadIdx.x;
    if (bid[k] >= 0) {
      brick_of[i] = bid[k];
      slot[i] = hist[bid[k]] + loc[k];
    }
  }
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void bin_count_lds(long n, const T* __restrict__ pos,
                                                               GridGeom g, BinGeom bg,
                                                               int* __restrict__ brick_of,
                                                               int* __restrict__ slot,
                                                               int* __restrict__ count) {
  bin_count_lds_body<T, NT>(n, pos, g, bg, brick_of, slot, count, Wg::plain());
}

template <typename T>
__global__ __launch_bounds__(256) void bin_count(long n, const T* __restrict__ pos,
                                                 GridGeom g, BinGeom bg,
                                                 int* __restrict__ brick_of,
                                                 int* __restrict__ slot,
                                                 int* __restrict__ count) {
  const long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const int bid = brick_of_particle(pos, i, g, bg);
  brick_of[i] = bid;
  slot[i] = atomicAdd(&count[bid], 1);
}

// Exclusive scan of the brick counts in one workgroup of 1024 threads:
// offset[b] = sum_{c < b} count[c], offset[nbricks] = n; count[] is reset to
// zero for the next binning.
__global__ __launch_bounds__(1024) void bin_scan(int* __restrict__ count, int nbricks,
                                                 int* __restrict__ offset) {
  __shared__ int wsum[16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int per = (nbricks + 1023) / 1024;
  const int b0 = t * per, b1 = min(b0 + per, nbricks);
  int s = 0;
  for (int b = b0; b < b1; ++b) s += count[b];
  // inclusive scan: within each wave by shuffles, then over the 16 wave totals
  int inc = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int v = __shfl_up(inc, d, 64);
    if (lane >= d) inc += v;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  if (w == 0) {
    int x = lane < 16 ? wsum[lane] : 0;
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
      const int v = __shfl_up(x, d, 64);
      if (lane >= d) x += v;
    }
    if (lane < 16) wsum[lane] = x;
  }
  __syncthreads();
  int run = inc - s + (w > 0 ? wsum[w - 1] : 0);
  for (int b = b0; b < b1; ++b) {
    offset[b] = run;
    run += count[b];
    count[b] = 0;
  }
  if (t == 1023) offset[nbricks] = wsum[15];
}

// Scatter with the scan folded in (nbricks <= kLdsHist, and few workgroups
// times bricks): every workgroup takes the exclusive prefix of the brick
// counts into LDS (workgroup 0 also stores it to offset[0..nbricks]) and
// scatters kBinPer particles per thread; the counts are cleared later, by
// the spread (one workgroup per brick), for the next binning.
template <typename T>
__device__ __forceinline__ void bin_scan_scatter_body(long n, const T* __restrict__ pos,
                                                        const T* __restrict__ q,
                                                        const int* __restrict__ brick_of,
                                                        const int* __restrict__ slot,
                                                        const int* __restrict__ count,
                                                        int nbricks, int* __restrict__ offset,
                                                        T* __restrict__ sorted,
                                                        int* __restrict__ perm,
                                                        double* __restrict__ qpart,
    const Wg wg) {
  __shared__ int off[kLdsHist + 1];
  __shared__ int wsum[4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int per = (nbricks + 255) / 256;
  const int b0 = min(t * per, nbricks), b1 = min(b0 + per, nbricks);
  int s = 0;
  for (int c0 = b0; c0 < b1; c0 += 8) {  // eight loads in flight at a time
    int c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] = c0 + u < b1 ? count[c0 + u] : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (c0 + u < b1) {
        off[c0 + u] = s;
        s += c[u];
      }
  }
  int inc = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int v = __shfl_up(inc, d, 64);
    if (lane >= d) inc += v;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int base = inc - s;
  for (int k = 0; k < w; ++k) base += wsum[k];
  for (int b = b0; b < b1; ++b) off[b] += base;
  if (t == 255) off[nbricks] = base + s;  // thread 255's range ends at nbricks
  __syncthreads();
  if (wg.x == 0)
    for (int b = t; b <= nbricks; b += 256) offset[b] = off[b];
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int k = 0; k < kBinPer; ++k) {
    const long i = (wg.x * static_cast<long>(kBinPer) + k) * 256 + t;
    if (i >= n) break;
    const long d = off[brick_of[i]] + slot[i];
    const T qi = q[i];
    sorted[4 * d + 0] = pos[3 * i + 0];
    sorted[4 * d + 1] = pos[3 * i + 1];
    sorted[4 * d + 2] = pos[3 * i + 2];
    sorted[4 * d + 3] = qi;
    perm[d] = static_cast<int>(i);
    s1 += static_cast<double>(qi);
    s2 += static_cast<double>(qi) * static_cast<double>(qi);
  }
  if (qpart) charge_partials(s1, s2, qpart, wg.x);
}

template <typename T>
__global__ __launch_bounds__(256) void bin_scan_scatter(long n, const T* __restrict__ pos,
                                                        const T* __restrict__ q,
                                                        const int* __restrict__ brick_of,
                                                        const int* __restrict__ slot,
                                                        const int* __restrict__ count,
                                                        int nbricks, int* __restrict__ offset,
                                                        T* __restrict__ sorted,
                                                        int* __restrict__ perm,
                                                        double* __restrict__ qpart) {
  bin_scan_scatter_body<T>(n, pos, q, brick_of, slot, count, nbricks, offset, sorted, perm, qpart, Wg::plain());
}

template <typename T>
__global__ __launch_bounds__(256) void bin_scatter(long n, const T* __restrict__ pos,
                                                   const T* __restrict__ q,
                                                   const int* __restrict__ brick_of,
                                                   const int* __restrict__ slot,
                                                   const int* __restrict__ offset,
                                                   T* __restrict__ sorted,
                                                   int* __restrict__ perm,
                                                   double* __restrict__ qpart) {
  const long i = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  double s1 = 0.0, s2 = 0.0;
  if (i < n) {
    const long d = offset[brick_of[i]] + slot[i];
    const T qi = q[i];
    sorted[4 * d + 0] = pos[3 * i + 0];
    sorted[4 * d + 1] = pos[3 * i + 1];
    sorted[4 * d + 2] = pos[3 * i + 2];
    sorted[4 * d + 3] = qi;
    perm[d] = static_cast<int>(i);
    s1 = static_cast<double>(qi);
    s2 = s1 * s1;
  }
  if (qpart) charge_partials(s1, s2, qpart, blockIdx.x);
}

// Owner-computes spread: one workgroup per grid brick.  It visits the
// particles binned in the home bricks whose stencils reach it (per-axis
// lists nbr[axis][brick] = {count, b0, b1, ...}, at most 4^3 combinations,
// flattened into one candidate range), adds the stencil points that fall
// inside its brick into an LDS tile with LDS atomics, and stores the tile:
// every grid value is written exactly once, with no global atomics.  It also
// writes the tile's FP64 sum and largest magnitude (part2[brick] = {sum, max})
// for the correction and the FP16X3 grid scale.  The tile accumulates in FP64
// for every precision (the LDS FP64 add is also the faster one on gfx950).
//
// Most candidates from neighbouring home bricks do not reach the brick (for
// 8-point bricks and P = 4, about a third of them do), and a wave pays for
// the stencil loop of its busiest lane, so a first pass compacts the
// candidates that reach the brick into an LDS list: wave w examines the
// 64-candidate runs w, w + 4, ... of the pass and appends the hits in order to
// its own segment (ballot prefix, deterministic).  The stencil pass then runs
// over the concatenated segments.  E8: every brick edge is 8 (compile-time tile
// strides).
constexpr int kHomeThreads = 256;  // threads per brick of the home-computes spread
static_assert(kHomeThreads % 64 == 0 && kHomeThreads <= 256, "spread_home's launch bound");
constexpr int kSpreadCand = 1024;  // candidates examined per pass, 256 per wave

template <typename T, int P, bool E8>
__device__ __forceinline__ void spread_brick_body(const T* __restrict__ sorted,
                                                    const int* __restrict__ offset,
                                                    const int* __restrict__ nbr,
                                                    T* __restrict__ grid,
                                                    double* __restrict__ part2,
                                                    int* __restrict__ count, GridGeom g,
                                                    BinGeom bg,
    const Wg wg) {
  static_assert(P <= 9, "at most four home bricks per axis (8-point bricks)");
  extern __shared__ __attribute__((aligned(16))) char smem[];
  double* tile = reinterpret_cast<double*>(smem);
  __shared__ int hstart[64], hpre[65];
  __shared__ int list[kSpreadCand], wcnt[4];
  __shared__ double red[32];
  const int E0 = E8 ? 8 : bg.edge[0], E1 = E8 ? 8 : bg.edge[1], E2 = E8 ? 8 : bg.edge[2];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // neighbouring bricks (which read overlapping particle lists) share an XCD
  const int brick = wg_order(wg, wg.x, wg.nx);
  if (threadIdx.x == 0) count[brick] = 0;  // the scatter has read it: ready for the next binning
  int own[3], rest = brick;
  own[2] = rest % bg.nb[2]; rest /= bg.nb[2];
  own[1] = rest % bg.nb[1];
  own[0] = rest / bg.nb[1];
  int lo[3], ext[3];
  lo[0] = own[0] * E0;
  lo[1] = own[1] * E1;
  lo[2] = own[2] * E2;
#pragma unroll
  for (int j = 0; j < 3; ++j) ext[j] = min(j == 0 ? E0 : j == 1 ? E1 : E2, g.K[j] - lo[j]);
  const int ntile = E0 * E1 * E2;
  for (int e = threadIdx.x; e < ntile; e += blockDim.x) tile[e] = 0.0;
  const int* n0 = nbr + kNbrRec * (0 * bg.nbmax + own[0]);
  const int* n1 = nbr + kNbrRec * (1 * bg.nbmax + own[1]);
  const int* n2 = nbr + kNbrRec * (2 * bg.nbmax + own[2]);
  const int nh = n0[0] * n1[0] * n2[0];  // <= 64 home bricks
  if (threadIdx.x < 64) {
    // lane c loads home brick c's particle range; exclusive prefix of the
    // range lengths by shuffles (lanes >= nh add nothing)
    const int c = threadIdx.x;
    int start = 0, cnt = 0;
    if (c < nh) {
      const int a2 = c % n2[0], a1 = (c / n2[0]) % n1[0], a0 = c / (n1[0] * n2[0]);
      const int hb = (n0[1 + a0] * bg.nb[1] + n1[1 + a1]) * bg.nb[2] + n2[1 + a2];
      start = offset[hb];
      cnt = offset[hb + 1] - start;
    }
    int inc = cnt;
#pragma unroll
    for (int dl = 1; dl < 64; dl <<= 1) {
      const int v = __shfl_up(inc, dl, 64);
      if (c >= dl) inc += v;
    }
    if (c < nh) {
      hstart[c] = start;
      hpre[c] = inc - cnt;
    }
    if (c == 63) hpre[nh] = inc;
  }
  __syncthreads();
  const int total = hpre[nh];
  for (int c0 = 0; c0 < total; c0 += kSpreadCand) {
    // pass 1: compact the candidates whose stencil reaches this brick
    int nw = 0;
#pragma unroll
    for (int k = 0; k < kSpreadCand / 256; ++k) {
      const int v = c0 + 64 * (4 * k + wave) + lane;
      bool hit = false;
      int i = 0;
      if (v < total) {
        int c = 0;
        while (hpre[c + 1] <= v) ++c;
        i = hstart[c] + (v - hpre[c]);
        hit = true;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          int base;
          (void)stencil_coord(sorted[4L * i + j], g.invL[j], g.K[j], g.cell, base);
          bool any = false;
#pragma unroll
          for (int t = 0; t < P; ++t) {
            int kk = base - t;
            if (kk < 0) kk += g.K[j];
            const int dd = kk - lo[j];
            any = any || (dd >= 0 && dd < ext[j]);
          }
          hit = hit && any;
        }
      }
      const unsigned long long m = __ballot(hit);
      const int below = __builtin_amdgcn_mbcnt_hi(static_cast<unsigned>(m >> 32),
                                                  __builtin_amdgcn_mbcnt_lo(static_cast<unsigned>(m), 0));
      if (hit) list[(kSpreadCand / 4) * wave + nw + below] = i;
      nw += __popcll(m);
    }
    if (lane == 0) wcnt[wave] = nw;
    __syncthreads();
    // pass 2: the stencils of the listed particles, segments in wave order
    const int s1 = wcnt[0], s2 = s1 + wcnt[1], s3 = s2 + wcnt[2], nl = s3 + wcnt[3];
    for (int u = threadIdx.x; u < nl; u += blockDim.x) {
      const int w = (u >= s1) + (u >= s2) + (u >= s3);
      const int segbase = w == 0 ? 0 : w == 1 ? s1 : w == 2 ? s2 : s3;
      const long i = list[(kSpreadCand / 4) * w + u - segbase];
      T w3[3][P], dw[P];
      int d[3][P];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        int base;
        const T f = stencil_coord(sorted[4 * i + j], g.invL[j], g.K[j], g.cell, base);
        stencil_weights<T, P>(f, g.cell, w3[j], dw);
#pragma unroll
        for (int t = 0; t < P; ++t) {
          int k = base - t;
          if (k < 0) k += g.K[j];
          const int dd = k - lo[j];
          d[j][t] = (dd >= 0 && dd < ext[j]) ? dd : -1;
        }
      }
      const double qi = static_cast<double>(sorted[4 * i + 3]);
      double wz[P];
#pragma unroll
      for (int cc = 0; cc < P; ++cc) wz[cc] = static_cast<double>(w3[2][cc]);
      for (int a = 0; a < P; ++a) {
        if (d[0][a] < 0) continue;
        const double wa = qi * static_cast<double>(w3[0][a]);
        for (int b = 0; b < P; ++b) {
          if (d[1][b] < 0) continue;
          const double wab = wa * static_cast<double>(w3[1][b]);
          double* row = tile + (d[0][a] * E1 + d[1][b]) * E2;
#pragma unroll
          for (int cc = 0; cc < P; ++cc)
            if (d[2][cc] >= 0) atomicAdd(&row[d[2][cc]], wab * wz[cc]);
        }
      }
    }
    __syncthreads();  // the list is rewritten by the next pass; the tile is read below
  }
  double s = 0.0, m = 0.0;
  for (int e = threadIdx.x; e < ntile; e += blockDim.x) {
    const int c = e % E2, b = (e / E2) % E1, a = e / (E1 * E2);
    if (a < ext[0] && b < ext[1] && c < ext[2]) {
      const T v = static_cast<T>(tile[e]);
      grid[(static_cast<long>(lo[0] + a) * g.K[1] + lo[1] + b) * g.K[2] + lo[2] + c] = v;
      s += static_cast<double>(v);
      m = fmax(m, fabs(static_cast<double>(v)));
    }
  }
  double v[2] = {s, m};
  block_reduce<1, 2>(v, red);
  if (threadIdx.x == 0) {
    part2[2 * brick] = v[0];
    part2[2 * brick + 1] = v[1];
  }
}

template <typename T, int P, bool E8>
__global__ __launch_bounds__(256) void spread_brick(const T* __restrict__ sorted,
                                                    const int* __restrict__ offset,
                                                    const int* __restrict__ nbr,
                                                    T* __restrict__ grid,
                                                    double* __restrict__ part2,
                                                    int* __restrict__ count, GridGeom g,
                                                    BinGeom bg) {
  spread_brick_body<T, P, E8>(sorted, offset, nbr, grid, part2, count, g, bg, Wg::plain());
}

// Home-computes spread, pass 1: one workgroup (kHomeThreads threads, one
// particle per thread at a time) per grid brick adds the stencils of
// the particles binned in that brick into an LDS tile covering the brick and
// the P - 1 planes below it on each axis, H_j = edge_j + P - 1 points, where
// every stencil point of those particles falls (no masking, each particle
// visited once), then stores the tile, rounded from the FP64 LDS sums to T,
// to tiles[brick].  Local tile coordinate of grid point k_j:
// k_j - lo_j + P - 1 (unwrapped).
template <typename T, int P>
__global__ __launch_bounds__(256) void spread_home(const T* __restrict__ sorted,
                                                  const int* __restrict__ offset,
                                                  T* __restrict__ tiles,
                                                  int* __restrict__ count, GridGeom g, BinGeom bg) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  double* tile = reinterpret_cast<double*>(smem);
  const int brick = xcd_order(blockIdx.x, gridDim.x);
  if (threadIdx.x == 0) count[brick] = 0;  // the scatter has read it: ready for the next binning
  int own[3], rest = brick;
  own[2] = rest % bg.nb[2]; rest /= bg.nb[2];
  own[1] = rest % bg.nb[1];
  own[0] = rest / bg.nb[1];
  int lo[3], H[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    lo[j] = own[j] * bg.edge[j];
    H[j] = bg.edge[j] + P - 1;
  }
  const int ntile = H[0] * H[1] * H[2];
  for (int e = threadIdx.x; e < ntile; e += blockDim.x) tile[e] = 0.0;
  __syncthreads();
  const int i0 = offset[brick], i1 = offset[brick + 1];
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    T w[3][P], dw[P];
    int l[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      int base;
      const T f = stencil_coord(sorted[4L * i + j], g.invL[j], g.K[j], g.cell, base);
      stencil_weights<T, P>(f, g.cell, w[j], dw);
      // the particle was binned by the same floor, so base lies in this
      // brick; the clamp only keeps a corrupted input inside the tile
      l[j] = min(max(base - lo[j] + P - 1, P - 1), H[j] - 1);
    }
    const T qi = sorted[4L * i + 3];
#pragma unroll
    for (int a = 0; a < P; ++a) {
      const T wa = qi * w[0][a];
#pragma unroll
      for (int b = 0; b < P; ++b) {
        const T wab = wa * w[1][b];
        double* row = tile + ((l[0] - a) * H[1] + l[1] - b) * H[2] + l[2];
#pragma unroll
        for (int c = 0; c < P; ++c) atomicAdd(row - c, static_cast<double>(wab * w[2][c]));
      }
    }
  }
  __syncthreads();
  T* out = tiles + static_cast<long>(brick) * ntile;
  for (int e = threadIdx.x; e < ntile; e += blockDim.x) out[e] = static_cast<T>(tile[e]);
}

// Home-computes spread, pass 1, on the matrix cores (float grids): the tile of
// a brick is T[a][b][c] = sum_i s_i(a) wy_i(b) wz_i(c), with s_i(a) =
// q_i wx_i(a) the charge-weighted x weight of particle i at tile plane a (zero
// off its stencil) and wy_i, wz_i its y and z weights placed at their tile
// positions.  Plane a is therefore one 16 x 16 rank-n update,
// T_a = sum_k (s_k(a) wy_k) wz_k^T, taken four particles at a time by
// v_mfma_f32_16x16x4f32 (A = s(a) wy, B = wz; FP32 accumulation).  The
// particles of a chunk are ordered by their x base in the brick with a
// stable, ballot-based counting sort, so that the particles reaching plane a
// (bases a - P + 1 .. a) form one contiguous range and each plane's k-steps
// cover only that range.  Eight waves: the first four stage the chunk's
// particles, and wave w accumulates planes w and w + 8 in its MFMA
// accumulators over every chunk and stores them at the end; the
// tile values are exact products rounded to FP32 and summed in FP32 in a
// fixed order.  Needs every tile extent <= 16 (edge + P - 1).
constexpr int kMfmaChunk = 256;   // particles staged per chunk (one per thread of waves 0-3)
constexpr int kMfmaWaves = 8;     // waves per workgroup; wave w owns planes w, w + 8
// three workgroups per CU fit in LDS (3 x 51 KB): six waves per SIMD, which
// caps the kernel at 80 VGPRs
constexpr int kMfmaWavesPerEu = 6;

__device__ __forceinline__ unsigned long long lanemask_lt() {
  const unsigned lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

template <int P>
__device__ __forceinline__ void spread_home_mfma_body(const float* __restrict__ sorted,
                                                       const int* __restrict__ offset,
                                                       float* __restrict__ tiles,
                                                       int* __restrict__ count, GridGeom g,
                                                       BinGeom bg,
    const Wg wg) {
  static_assert(P <= 9, "tile extents must stay within 16 (brick edge 8)");
  static_assert(2 * kMfmaWaves >= 16, "two planes per wave cover a 16-plane tile");
  // padded per-particle rows, in sorted slot order: q wx at its x planes,
  // wy at its y positions, wz at its z positions (zero elsewhere)
  // (eight rows past the chunk: the k-loops read up to seven slots past a
  // plane's range, and the rows past the chunk's particles are zero)
  __shared__ __attribute__((aligned(16))) float sx[kMfmaChunk + 8][16];
  __shared__ __attribute__((aligned(16))) float sy[kMfmaChunk + 8][16];
  __shared__ __attribute__((aligned(16))) float sz[kMfmaChunk + 8][16];
  __shared__ int wcount[4][16];   // per wave, particles per x base
  __shared__ int boff[4][17];     // per wave, first slot of each x base
  __shared__ int bstart[17];      // first slot of each x base in the chunk
  const int brick = wg_order(wg, wg.x, wg.nx);
  if (threadIdx.x == 0) count[brick] = 0;  // the scatter has read it: ready for the next binning
  int own[3], rest = brick;
  own[2] = rest % bg.nb[2]; rest /= bg.nb[2];
  own[1] = rest % bg.nb[1];
  own[0] = rest / bg.nb[1];
  int lo[3], H[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    lo[j] = own[j] * bg.edge[j];
    H[j] = bg.edge[j] + P - 1;
  }
  const int E0 = bg.edge[0];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);
  const int col = lane & 15, kq = lane >> 4;
  floatx4 acc[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) acc[u] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int i0 = offset[brick], i1 = offset[brick + 1];
  for (int c0 = i0; c0 < i1; c0 += kMfmaChunk) {
    const int n = min(kMfmaChunk, i1 - c0);
    // this thread's particle: tile bases and weights
    const int t = threadIdx.x;
    float w[3][P], dw[P];
    int l[3] = {0, 0, 0};
    int bin = -1;
    float qi = 0.f;
    if (t < n) {
      // (x, y, z, q) of one particle in one 16-byte load
      const float4 pq = reinterpret_cast<const float4*>(sorted)[c0 + t];
      const float xyz[3] = {pq.x, pq.y, pq.z};
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        int base;
        const float f = stencil_coord(xyz[j], g.invL[j], g.K[j], g.cell, base);
        stencil_weights<float, P>(f, g.cell, w[j], dw);
        l[j] = min(max(base - lo[j] + P - 1, P - 1), H[j] - 1);
      }
      qi = pq.w;
      bin = l[0] - (P - 1);
    }
    // stable counting sort by x base: ballots give the rank inside the wave
    int rank = 0;
    if (wave_u < 4) {
      for (int v = 0; v < E0; ++v) {
        const unsigned long long m = __ballot(bin == v);
        if (bin == v) rank = __popcll(m & lanemask_lt());
        if (lane == 0) wcount[wave][v] = __popcll(m);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int acc_s = 0;
      for (int v = 0; v < E0; ++v) {
        bstart[v] = acc_s;
        for (int ww = 0; ww < 4; ++ww) {
          boff[ww][v] = acc_s;
          acc_s += wcount[ww][v];
        }
      }
      bstart[E0] = acc_s;
    }
    __syncthreads();
    if (t < n) {
      const int slot = boff[wave][bin] + rank;
      // the rows are cleared, then the P weights of each axis are written
      // at their tile positions (one thread's LDS writes land in order):
      // tile index l_j - s carries weight w_j[s]
      const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int e = 0; e < 16; e += 4) {
        *reinterpret_cast<float4*>(&sx[slot][e]) = z4;
        *reinterpret_cast<float4*>(&sy[slot][e]) = z4;
        *reinterpret_cast<float4*>(&sz[slot][e]) = z4;
      }
#pragma unroll
      for (int s = 0; s < P; ++s) {
        sx[slot][l[0] - s] = qi * w[0][s];
        sy[slot][l[1] - s] = w[1][s];
        sz[slot][l[2] - s] = w[2][s];
      }
    } else if (t < n + 8) {
      const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int e = 0; e < 16; e += 4) {
        *reinterpret_cast<float4*>(&sx[t][e]) = z4;
        *reinterpret_cast<float4*>(&sy[t][e]) = z4;
        *reinterpret_cast<float4*>(&sz[t][e]) = z4;
      }
    }
    __syncthreads();
    // planes a = wave + 8u; the particles reaching plane a have x base in
    // [a - P + 1, a]: slots [bstart[max(0, a - P + 1)], bstart[min(a, E0 - 1) + 1]).
    // The bounds are wave-uniform (read into scalar registers), so each
    // plane is one straight loop of unconditional products over its range;
    // the lanes of a step past the range contribute zeros.
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int a = wave_u + kMfmaWaves * u;
      if (a >= H[0]) break;
      const int ps = __builtin_amdgcn_readfirstlane(bstart[max(0, a - P + 1)]);
      const int pe = __builtin_amdgcn_readfirstlane(bstart[min(a, E0 - 1) + 1]);
      // operands of particle k for this lane: A[b][k] = s_k(a) wy_k(b) with
      // b = col, B[k][c] = wz_k(c) with c = col; the next step's operands
      // are read while this step's product runs
      // (no masks: a slot in [pe, n) holds a particle whose x planes lie
      // above a, so its s(a) is zero, and the rows from n on are zero)
      float yb = sx[ps + kq][a] * sy[ps + kq][col], zc = sz[ps + kq][col];
      for (int k0 = ps; k0 < pe; k0 += 4) {
        const int kn = k0 + 4 + kq;   // <= pe + 6 <= n + 6
        const float xn = sx[kn][a], yn = sy[kn][col], zn = sz[kn][col];
        acc[u] = mfma_k4(yb, zc, acc[u]);
        yb = xn * yn;
        zc = zn;
      }
    }
    __syncthreads();   // the rows are rewritten by the next chunk
  }
  // D[b][c] with b = 4 kq + r, c = col in register r
  const int ntile = H[0] * H[1] * H[2];
  float* out = tiles + static_cast<long>(brick) * ntile;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int a = wave + kMfmaWaves * u;
    if (a >= H[0] || col >= H[2]) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int b = 4 * kq + r;
      if (b < H[1]) out[(a * H[1] + b) * H[2] + col] = acc[u][r];
    }
  }
}

template <int P>
__global__ __launch_bounds__(64 * kMfmaWaves) __attribute__((amdgpu_waves_per_eu(kMfmaWavesPerEu)))
void spread_home_mfma(const float* __restrict__ sorted,
                                                       const int* __restrict__ offset,
                                                       float* __restrict__ tiles,
                                                       int* __restrict__ count, GridGeom g,
                                                       BinGeom bg) {
  spread_home_mfma_body<P>(sorted, offset, tiles, count, g, bg, Wg::plain());
}

// Pass 2, persistent form for grids where every owner brick is reached by
// exactly two home bricks per axis (itself and the next one, periodically)
// and every tile extent is at most the axis length (BinGeom::two_homes):
// workgroup w takes a contiguous range of owner bricks, derives the home
// bricks and tile offsets of each from its brick coordinates, and loads the
// eight tile values of its point in the next brick while it adds and stores
// those of the current one.  Per point the eight values are added in FP64
// in the order of spread_combine (home lists ascending per axis), so the
// grid is the same; the workgroup's FP64 (sum, max) over all its points goes
// to part2[w].
constexpr int kCombineThreads = 512;
constexpr int kCombineMaxBricks = 64;

int combine_workgroups(int nbricks) {
  const int target = 4 * 256;
  const int per = std::max(1, (nbricks + target - 1) / target);
  return (nbricks + per - 1) / per;
}

template <typename T, int P>
__device__ __forceinline__ void spread_combine_pf_body(
    const T* __restrict__ tiles, T* __restrict__ grid, double* __restrict__ part2, GridGeom g,
    BinGeom bg,
    const Wg wg) {
  __shared__ double red[32];
  const int wl = wg_order(wg, wg.x, wg.nx);
  const int nb = bg.nbricks;
  const int b_begin = static_cast<int>(static_cast<long>(wl) * nb / wg.nx);
  const int b_end = static_cast<int>(static_cast<long>(wl + 1) * nb / wg.nx);
  int H[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) H[j] = bg.edge[j] + P - 1;
  const int ntile = H[0] * H[1] * H[2];
  // this thread's point of a brick (edges are the full 8 or the axis)
  const int e = threadIdx.x;
  const int npts = bg.edge[0] * bg.edge[1] * bg.edge[2];
  const bool has = e < npts;
  const int x2 = e % bg.edge[2], x1 = (e / bg.edge[2]) % bg.edge[1],
            x0 = e / (bg.edge[1] * bg.edge[2]);
  const int x[3] = {x0, x1, x2};
  // the eight (tile, offset) pairs of point x in owner brick `brick`, in the
  // order of the general kernel, and whether each lies in its tile
  // brick coordinates, advanced one brick at a time along the range (one
  // division for the first brick only)
  int own[3];
  {
    int rest = b_begin;
    own[2] = rest % bg.nb[2];
    rest /= bg.nb[2];
    own[1] = rest % bg.nb[1];
    own[0] = rest / bg.nb[1];
  }
  auto advance = [&]() {
    if (++own[2] == bg.nb[2]) {
      own[2] = 0;
      if (++own[1] == bg.nb[1]) {
        own[1] = 0;
        ++own[0];
      }
    }
  };
  auto locate = [&](long* at, bool* in, long* gat) {
    int hid[3][2], l[3][2];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int nxt = own[j] + 1 == bg.nb[j] ? 0 : own[j] + 1;
      hid[j][0] = min(own[j], nxt);   // ascending, as the neighbour lists
      hid[j][1] = max(own[j], nxt);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        int d = (own[j] - hid[j][h]) * bg.edge[j] + P - 1;
        if (d < 0) d += g.K[j];
        if (d >= g.K[j]) d -= g.K[j];
        int v = x[j] + d;
        if (v >= g.K[j]) v -= g.K[j];
        l[j][h] = v;
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int a = q >> 2, b = (q >> 1) & 1, c = q & 1;
      in[q] = has && l[0][a] < H[0] && l[1][b] < H[1] && l[2][c] < H[2];
      // clamped into the tile: every lane loads (no divergent branch), and
      // the values outside it are dropped by the select below
      at[q] = static_cast<long>((hid[0][a] * bg.nb[1] + hid[1][b]) * bg.nb[2] + hid[2][c]) * ntile +
              (min(l[0][a], H[0] - 1) * H[1] + min(l[1][b], H[1] - 1)) * H[2] +
              min(l[2][c], H[2] - 1);
    }
    *gat = (static_cast<long>(own[0] * bg.edge[0] + x0) * g.K[1] + own[1] * bg.edge[1] + x1) *
               g.K[2] + own[2] * bg.edge[2] + x2;
  };
  T v[8];
  bool in[8];
  long gat = 0;
  if (b_begin < b_end) {
    long at[8];
    locate(at, in, &gat);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const T t = tiles[at[q]];
      v[q] = in[q] ? t : T(0);
    }
  }
  double s = 0.0, m = 0.0;
  for (int brick = b_begin; brick < b_end; ++brick) {
    T cur[8];
    bool cin[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      cur[q] = v[q];
      cin[q] = in[q];
    }
    const long cgat = gat;
    if (brick + 1 < b_end) {   // the next brick's values in flight
      long at[8];
      advance();
      locate(at, in, &gat);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
      const T t = tiles[at[q]];
      v[q] = in[q] ? t : T(0);
    }
    }
    if (has) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (cin[q]) acc += static_cast<double>(cur[q]);
      const T val = static_cast<T>(acc);
      grid[cgat] = val;
      s += static_cast<double>(val);
      m = fmax(m, fabs(static_cast<double>(val)));
    }
  }
  double r[2] = {s, m};
  block_reduce<1, 2>(r, red);
  if (threadIdx.x == 0) {
    part2[2 * wg.x] = r[0];
    part2[2 * wg.x + 1] = r[1];
  }
}

template <typename T, int P>
__global__ __launch_bounds__(kCombineThreads) void spread_combine_pf(
    const T* __restrict__ tiles, T* __restrict__ grid, double* __restrict__ part2, GridGeom g,
    BinGeom bg) {
  spread_combine_pf_body<T, P>(tiles, grid, part2, g, bg, Wg::plain());
}

// Pass 2: one workgroup per grid brick sums, for each of its points and in a
// fixed order, the tiles of the home bricks whose stencils reach it (the
// per-axis lists nbr[axis][brick] = {count, b0, b1, ...}).  Point x_j of the
// owner brick sits in tile h at local coordinate x_j + d_j(h) with
// d_j(h) = (lo_owner - lo_h + P - 1) reduced so that the image lies in the
// tile (when a stencil is wider than the grid, further images at + m K_j are
// summed too).  Writes every grid value once and the brick's FP64 (sum, max)
// to part2[brick].
template <typename T, int P>
__global__ __launch_bounds__(512) void spread_combine(const T* __restrict__ tiles,
                                                      const int* __restrict__ nbr,
                                                      T* __restrict__ grid,
                                                      double* __restrict__ part2, GridGeom g,
                                                      BinGeom bg) {
  __shared__ double red[32];
  __shared__ int dlt[3][kNbrRec], hid[3][kNbrRec];
  const int brick = xcd_order(blockIdx.x, gridDim.x);
  int own[3], rest = brick;
  own[2] = rest % bg.nb[2]; rest /= bg.nb[2];
  own[1] = rest % bg.nb[1];
  own[0] = rest / bg.nb[1];
  int lo[3], ext[3], H[3], cnt[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    lo[j] = own[j] * bg.edge[j];
    ext[j] = min(bg.edge[j], g.K[j] - lo[j]);
    H[j] = bg.edge[j] + P - 1;
    cnt[j] = nbr[kNbrRec * (j * bg.nbmax + own[j])];
  }
  if (threadIdx.x < 3 * (kNbrRec - 1)) {
    const int j = threadIdx.x / (kNbrRec - 1), x = threadIdx.x % (kNbrRec - 1);
    const int* list = nbr + kNbrRec * (j * bg.nbmax + own[j]);
    if (x < list[0]) {
      // smallest non-negative image of lo_owner - lo_h + P - 1 modulo K_j
      int d = lo[j] - list[1 + x] * bg.edge[j] + P - 1;
      while (d < 0) d += g.K[j];
      while (d >= g.K[j]) d -= g.K[j];
      dlt[j][x] = d;
      hid[j][x] = list[1 + x];
    }
  }
  __syncthreads();
  const int ntile = H[0] * H[1] * H[2];
  double s = 0.0, m = 0.0;
  const int npts = ext[0] * ext[1] * ext[2];
  // two home bricks per axis and tiles no longer than the axis (every tile
  // holds at most one image of a point): the eight tile values of a point
  // are loaded together, then added in the order of the general loop below
  const bool two = cnt[0] == 2 && cnt[1] == 2 && cnt[2] == 2 && g.K[0] >= H[0] &&
                   g.K[1] >= H[1] && g.K[2] >= H[2];
  for (int e = threadIdx.x; e < npts; e += blockDim.x) {
    const int x2 = e % ext[2], x1 = (e / ext[2]) % ext[1], x0 = e / (ext[1] * ext[2]);
    double acc = 0.0;
    if (two) {
      int l[3][2];
      const int x[3] = {x0, x1, x2};
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          int v = x[j] + dlt[j][h];
          if (v >= g.K[j]) v -= g.K[j];
          l[j][h] = v;   // in this tile when < H[j]
        }
      T v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int a = q >> 2, b = (q >> 1) & 1, c = q & 1;
        const bool in = l[0][a] < H[0] && l[1][b] < H[1] && l[2][c] < H[2];
        const long at = static_cast<long>((hid[0][a] * bg.nb[1] + hid[1][b]) * bg.nb[2] + hid[2][c]) *
                            ntile + (l[0][a] * H[1] + l[1][b]) * H[2] + l[2][c];
        v[q] = in ? tiles[at] : T(0);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int a = q >> 2, b = (q >> 1) & 1, c = q & 1;
        if (l[0][a] < H[0] && l[1][b] < H[1] && l[2][c] < H[2]) acc += static_cast<double>(v[q]);
      }
    } else {
      for (int a = 0; a < cnt[0]; ++a) {
        int l0 = x0 + dlt[0][a];
        if (l0 >= g.K[0]) l0 -= g.K[0];
        for (; l0 < H[0]; l0 += g.K[0])
          for (int b = 0; b < cnt[1]; ++b) {
            int l1 = x1 + dlt[1][b];
            if (l1 >= g.K[1]) l1 -= g.K[1];
            for (; l1 < H[1]; l1 += g.K[1])
              for (int c = 0; c < cnt[2]; ++c) {
                int l2 = x2 + dlt[2][c];
                if (l2 >= g.K[2]) l2 -= g.K[2];
                const T* t = tiles + static_cast<long>((hid[0][a] * bg.nb[1] + hid[1][b]) * bg.nb[2] +
                                                       hid[2][c]) * ntile +
                             (l0 * H[1] + l1) * H[2];
                for (; l2 < H[2]; l2 += g.K[2]) acc += static_cast<double>(t[l2]);
              }
          }
      }
    }
    const T v = static_cast<T>(acc);
    grid[(static_cast<long>(lo[0] + x0) * g.K[1] + lo[1] + x1) * g.K[2] + lo[2] + x2] = v;
    s += static_cast<double>(v);
    m = fmax(m, fabs(static_cast<double>(v)));
  }
  double v[2] = {s, m};
  block_reduce<1, 2>(v, red);
  if (threadIdx.x == 0) {
    part2[2 * brick] = v[0];
    part2[2 * brick + 1] = v[1];
  }
}

// Gather in binned order (neighbouring threads read neighbouring grid
// values); results are written back to the caller's order through perm.
// With an energy job, one extra last workgroup runs it.
template <typename T, int P>
__device__ __forceinline__ void gather_sorted_body(long n, const T* __restrict__ sorted,
                                                     const int* __restrict__ perm,
                                                     const T* __restrict__ grid,
                                                     T* __restrict__ pot,
                                                     T* __restrict__ force,
                                                     EnergyJob ej, GridGeom g,
    const Wg wg) {
  // with an energy job, one extra last workgroup runs it beside the gather
  const int nwork = wg.nx - (ej.e4 ? 1 : 0);
  if (static_cast<int>(wg.x) == nwork) {
    run_energy_job(ej);
    return;
  }
  // neighbouring particle blocks (neighbouring bricks) share an XCD's L2
  const int blk = wg_order(wg, wg.x, nwork);
  const long s = blk * static_cast<long>(blockDim.x) + threadIdx.x;
  if (s < n) {
    T w[3][P], dw[3][P];
    int base[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const T f = stencil_coord(sorted[4 * s + j], g.invL[j], g.K[j], g.cell, base[j]);
      stencil_weights<T, P>(f, g.cell, w[j], dw[j]);
    }
    const int K1 = g.K[0], K2 = g.K[1], K3 = g.K[2];
    int kc[P];
#pragma unroll
    for (int c = 0; c < P; ++c) {
      kc[c] = base[2] - c;
      if (kc[c] < 0) kc[c] += K3;
    }
    T phi = 0, g0 = 0, g1 = 0, g2 = 0;
    // unrolled so that a whole plane (small P: the whole stencil) of loads is
    // in flight at once
    constexpr int UA = P <= 4 ? P : 1, UB = P <= 8 ? P : 1;
#pragma unroll UA
    for (int a = 0; a < P; ++a) {
      int ka = base[0] - a;
      if (ka < 0) ka += K1;
      // plane a's weights by selection (no dynamic register indexing)
      T wa = w[0][0], dwa = dw[0][0];
#pragma unroll
      for (int t = 1; t < P; ++t)
        if (a == t) {
          wa = w[0][t];
          dwa = dw[0][t];
        }
      T sa = 0, sa1 = 0, sa2 = 0;
#pragma unroll UB
      for (int b = 0; b < P; ++b) {
        int kb = base[1] - b;
        if (kb < 0) kb += K2;
        const T* row = grid + (static_cast<long>(ka) * K2 + kb) * K3;
        T sv = 0, s2 = 0;
#pragma unroll
        for (int c = 0; c < P; ++c) {
          const T v = row[kc[c]];
          sv += w[2][c] * v;
          s2 += dw[2][c] * v;
        }
        sa += w[1][b] * sv;
        sa1 += dw[1][b] * sv;
        sa2 += w[1][b] * s2;
      }
      phi += wa * sa;
      g0 += dwa * sa;
      g1 += wa * sa1;
      g2 += wa * sa2;
    }
    const long i = perm[s];
    const T qi = sorted[4 * s + 3];
    if (pot) pot[i] = phi;
    if (force) {
      force[3 * i + 0] = -qi * g0 * static_cast<T>(K1 * g.invL[0]);
      force[3 * i + 1] = -qi * g1 * static_cast<T>(K2 * g.invL[1]);
      force[3 * i + 2] = -qi * g2 * static_cast<T>(K3 * g.invL[2]);
    }
  }
}

template <typename T, int P>
__global__ __launch_bounds__(256) void gather_sorted(long n, const T* __restrict__ sorted,
                                                     const int* __restrict__ perm,
                                                     const T* __restrict__ grid,
                                                     T* __restrict__ pot,
                                                     T* __restrict__ force,
                                                     EnergyJob ej, GridGeom g) {
  gather_sorted_body<T, P>(n, sorted, perm, grid, pot, force, ej, g, Wg::plain());
}

// Gather in binned order with P lanes per particle (spline orders up to 4):
// lane a of a particle's group takes the stencil plane k1 = base0 - a (P^2
// loads), and the group's plane sums are added by shuffles.  Four times the
// threads of gather_sorted keep more loads in flight.  Partial sums per
// workgroup as in gather_sorted.
template <typename T, int P>
__device__ __forceinline__ void gather_sorted_planes_body(long n, const T* __restrict__ sorted,
                                                            const int* __restrict__ perm,
                                                            const T* __restrict__ grid,
                                                            T* __restrict__ pot,
                                                            T* __restrict__ force,
                                                            EnergyJob ej, GridGeom g,
    const Wg wg) {
  static_assert(P == 4, "one lane per plane, four lanes per particle");
  // with an energy job, one extra last workgroup runs it beside the gather
  const int nwork = wg.nx - (ej.e4 ? 1 : 0);
  if (static_cast<int>(wg.x) == nwork) {
    run_energy_job(ej);
    return;
  }
  const int blk = wg_order(wg, wg.x, nwork);
  const long s = (blk * static_cast<long>(blockDim.x) + threadIdx.x) / P;
  const int a = threadIdx.x % P;
  T phi = 0, g0 = 0, g1 = 0, g2 = 0;
  const bool live = s < n;
  T qi = 0;
  // the destination index is loaded first; its latency hides behind the stencil
  const long dst = live && a == 0 ? perm[s] : 0;
  if (live) {
    T w[3][P], dw[3][P];
    int base[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const T f = stencil_coord(sorted[4 * s + j], g.invL[j], g.K[j], g.cell, base[j]);
      stencil_weights<T, P>(f, g.cell, w[j], dw[j]);
    }
    qi = sorted[4 * s + 3];
    const int K1 = g.K[0], K2 = g.K[1], K3 = g.K[2];
    int kc[P];
#pragma unroll
    for (int c = 0; c < P; ++c) {
      kc[c] = base[2] - c;
      if (kc[c] < 0) kc[c] += K3;
    }
    int ka = base[0] - a;
    if (ka < 0) ka += K1;
    // this lane's weights of axis 0 (a runtime index into the unrolled array)
    T wa = w[0][0], dwa = dw[0][0];
#pragma unroll
    for (int t = 1; t < P; ++t)
      if (a == t) {
        wa = w[0][t];
        dwa = dw[0][t];
      }
    T sa = 0, sa1 = 0, sa2 = 0;
#pragma unroll
    for (int b = 0; b < P; ++b) {
      int kb = base[1] - b;
      if (kb < 0) kb += K2;
      const T* row = grid + (static_cast<long>(ka) * K2 + kb) * K3;
      T sv = 0, s2 = 0;
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const T v = row[kc[c]];
        sv += w[2][c] * v;
        s2 += dw[2][c] * v;
      }
      sa += w[1][b] * sv;
      sa1 += dw[1][b] * sv;
      sa2 += w[1][b] * s2;
    }
    phi = wa * sa;
    g0 = dwa * sa;
    g1 = wa * sa1;
    g2 = wa * sa2;
  }
  // sums over the particle's P lanes (aligned groups of the wave)
#pragma unroll
  for (int o = 1; o < P; o <<= 1) {
    phi += __shfl_xor(phi, o, 64);
    g0 += __shfl_xor(g0, o, 64);
    g1 += __shfl_xor(g1, o, 64);
    g2 += __shfl_xor(g2, o, 64);
  }
  if (live && a == 0) {
    const long i = dst;
    if (pot) pot[i] = phi;
    if (force) {
      force[3 * i + 0] = -qi * g0 * static_cast<T>(g.K[0] * g.invL[0]);
      force[3 * i + 1] = -qi * g1 * static_cast<T>(g.K[1] * g.invL[1]);
      force[3 * i + 2] = -qi * g2 * static_cast<T>(g.K[2] * g.invL[2]);
    }
  }
}

template <typename T, int P>
__global__ __launch_bounds__(256) void gather_sorted_planes(long n, const T* __restrict__ sorted,
                                                            const int* __restrict__ perm,
                                                            const T* __restrict__ grid,
                                                            T* __restrict__ pot,
                                                            T* __restrict__ force,
                                                            EnergyJob ej, GridGeom g) {
  gather_sorted_planes_body<T, P>(n, sorted, perm, grid, pot, force, ej, g, Wg::plain());
}

// The binned record (x, y, z, q) of slot s in one 16-byte load (float) or two
// (double).
__device__ __forceinline__ void load_record(const float* sorted, long s, float* r) {
  const float4 v = reinterpret_cast<const float4*>(sorted)[s];
  r[0] = v.x;
  r[1] = v.y;
  r[2] = v.z;
  r[3] = v.w;
}
__device__ __forceinline__ void load_record(const double* sorted, long s, double* r) {
  const double2 a = reinterpret_cast<const double2*>(sorted)[2 * s];
  const double2 b = reinterpret_cast<const double2*>(sorted)[2 * s + 1];
  r[0] = a.x;
  r[1] = a.y;
  r[2] = b.x;
  r[3] = b.y;
}

// Gather by brick: one workgroup per grid brick stages in LDS the potential
// values that the stencils of the particles binned in it read -- the brick
// and the P - 1 planes below it on each axis, H_j = edge_j + P - 1 points,
// wrapped periodically -- then interpolates those particles from LDS, one
// particle per thread (every stencil point is inside the tile: no masking).
// Results go back to the caller's order through perm.  With an energy job,
// one extra last workgroup runs it.
constexpr int kGatherThreads = 256;
constexpr int kGatherMaxBricks = 64;   // bricks per workgroup of the persistent gather

// Workgroups of the persistent gather: one per brick up to `target` (the
// plan's BinGeom::gather_wgs), then the same number of bricks per workgroup
// up to one (at most kGatherMaxBricks, since the grid has at most 32^3
// bricks).  A plan alone on the device takes sixteen per CU: on the 1M-atom
// box (4,096 bricks) one brick per workgroup measured 55.5 us against 57.2
// with four (about five workgroups per CU) and 67.4 with six.  In a batch,
// whose systems fill the device together, five per CU keeps the per-workgroup
// cost down (64-system batch gather 375 -> 329 us).
int gather_pf_workgroups(int nbricks, int target) {
  const int per = std::max(1, (nbricks + target - 1) / target);
  return (nbricks + per - 1) / per;
}

template <typename T, int P>
__global__ __launch_bounds__(kGatherThreads) void gather_brick(const T* __restrict__ sorted,
                                                              const int* __restrict__ offset,
                                                              const int* __restrict__ perm,
                                                              const T* __restrict__ grid,
                                                              T* __restrict__ pot,
                                                              T* __restrict__ force, EnergyJob ej,
                                                              GridGeom g, BinGeom bg) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  T* tile = reinterpret_cast<T*>(smem);
  // with an energy job, one extra last workgroup runs it beside the gather
  const int nwork = gridDim.x - (ej.e4 ? 1 : 0);
  if (static_cast<int>(blockIdx.x) == nwork) {
    run_energy_job(ej);
    return;
  }
  const int brick = xcd_order(blockIdx.x, nwork);
  int own[3], rest = brick;
  own[2] = rest % bg.nb[2]; rest /= bg.nb[2];
  own[1] = rest % bg.nb[1];
  own[0] = rest / bg.nb[1];
  int lo[3], H[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    lo[j] = own[j] * bg.edge[j];
    H[j] = bg.edge[j] + P - 1;
  }
  const int K1 = g.K[0], K2 = g.K[1], K3 = g.K[2];
  // the tile, one (t0, t1) row of H2 consecutive k3 values per 16 lanes
  // (a row start is wrapped once per row; within a row k3 wraps at most
  // once, every tile extent being below 2 K_j)
  {
    const int nrows = H[0] * H[1];
    const int c16 = threadIdx.x & 15;
    for (int r = threadIdx.x >> 4; r < nrows; r += kGatherThreads / 16) {
      const int t0 = r / H[1], t1 = r - t0 * H[1];
      int k0 = lo[0] - (P - 1) + t0, k1 = lo[1] - (P - 1) + t1;
      while (k0 < 0) k0 += K1;
      while (k0 >= K1) k0 -= K1;
      while (k1 < 0) k1 += K2;
      while (k1 >= K2) k1 -= K2;
      const T* src = grid + (static_cast<long>(k0) * K2 + k1) * K3;
      for (int c = c16; c < H[2]; c += 16) {
        int k2 = lo[2] - (P - 1) + c;
        while (k2 < 0) k2 += K3;
        while (k2 >= K3) k2 -= K3;
        tile[r * H[2] + c] = src[k2];
      }
    }
  }
  __syncthreads();
  const int i0 = offset[brick], i1 = offset[brick + 1];
  for (int s = i0 + threadIdx.x; s < i1; s += blockDim.x) {
    T rec[4];
    load_record(sorted, s, rec);
    T w[3][P], dw[3][P];
    int l[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      int base;
      const T f = stencil_coord(rec[j], g.invL[j], g.K[j], g.cell, base);
      stencil_weights<T, P>(f, g.cell, w[j], dw[j]);
      // binned by the same floor: base lies in this brick (the clamp only
      // keeps a corrupted input inside the tile)
      l[j] = min(max(base - lo[j] + P - 1, P - 1), H[j] - 1);
    }
    T phi = 0, g0 = 0, g1 = 0, g2 = 0;
    constexpr int UB = P <= 8 ? P : 1;
    // one plane at a time (P^2 values in flight): a fully unrolled stencil
    // holds every value in registers and leaves one wave per SIMD
#pragma unroll 1
    for (int a = 0; a < P; ++a) {
      T wa = w[0][0], dwa = dw[0][0];
#pragma unroll
      for (int t = 1; t < P; ++t)
        if (a == t) {
          wa = w[0][t];
          dwa = dw[0][t];
        }
      T sa = 0, sa1 = 0, sa2 = 0;
#pragma unroll UB
      for (int b = 0; b < P; ++b) {
        const T* row = tile + ((l[0] - a) * H[1] + l[1] - b) * H[2] + l[2];
        T sv = 0, s2 = 0;
#pragma unroll
        for (int c = 0; c < P; ++c) {
          const T v = row[-c];
          sv += w[2][c] * v;
          s2 += dw[2][c] * v;
        }
        sa += w[1][b] * sv;
        sa1 += dw[1][b] * sv;
        sa2 += w[1][b] * s2;
      }
      phi += wa * sa;
      g0 += dwa * sa;
      g1 += wa * sa1;
      g2 += wa * sa2;
    }
    const long i = perm[s];
    const T qi = rec[3];
    if (pot) pot[i] = phi;
    if (force) {
      force[3 * i + 0] = -qi * g0 * static_cast<T>(K1 * g.invL[0]);
      force[3 * i + 1] = -qi * g1 * static_cast<T>(K2 * g.invL[1]);
      force[3 * i + 2] = -qi * g2 * static_cast<T>(K3 * g.invL[2]);
    }
  }
}

// The same gather, persistent and software-pipelined (tile extents <= 16,
// i.e. P <= 9): workgroup w takes a contiguous range of bricks and, while it
// interpolates the particles of one brick from LDS, already holds in
// registers the next brick's tile values (rows (t0, t1) of H2 consecutive
// values, 16 lanes per row, kPfRows rows per thread) and the records and
// perm entries of its first kGatherThreads particles.  The brick offsets of
// the range are staged in LDS once.  Results and summation order per
// particle are those of gather_brick.
template <typename T, int P, bool E8>
__device__ __forceinline__ void gather_brick_pf_body(
    const T* __restrict__ sorted, const int* __restrict__ offset, const int* __restrict__ perm,
    const T* __restrict__ grid, T* __restrict__ pot, T* __restrict__ force, EnergyJob ej,
    GridGeom g, BinGeom bg,
    const Wg wg) {
  static_assert(P <= 9, "rows of at most 16 values");
  constexpr int HM = 8 + P - 1;                       // largest tile extent (edge <= 8)
  constexpr int kPfRows = (HM * HM + kGatherThreads / 16 - 1) / (kGatherThreads / 16);
  extern __shared__ __attribute__((aligned(16))) char smem[];
  T* tile = reinterpret_cast<T*>(smem);
  __shared__ int offs[kGatherMaxBricks + 1];
  const int nwork = wg.nx - (ej.e4 ? 1 : 0);
  if (static_cast<int>(wg.x) == nwork) {
    run_energy_job(ej);
    return;
  }
  const int wl = wg_order(wg, wg.x, nwork);
  const int nb = bg.nbricks;
  const int b_begin = static_cast<int>(static_cast<long>(wl) * nb / nwork);
  const int b_end = static_cast<int>(static_cast<long>(wl + 1) * nb / nwork);
  const int tid = threadIdx.x;
  for (int k = tid; k <= b_end - b_begin; k += kGatherThreads) offs[k] = offset[b_begin + k];
  // E8: every brick edge is 8, so the tile strides are compile-time
  // constants (LDS offsets of the stencil rows become immediates)
  int H[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) H[j] = E8 ? 8 + P - 1 : bg.edge[j] + P - 1;
  const int K1 = g.K[0], K2 = g.K[1], K3 = g.K[2];
  const int nrows = H[0] * H[1];
  const int c16 = tid & 15;
  auto lo_of = [&](int brick, int* lo) {
    int rest = brick;
    const int o2 = rest % bg.nb[2];
    rest /= bg.nb[2];
    lo[2] = o2 * bg.edge[2];
    lo[1] = (rest % bg.nb[1]) * bg.edge[1];
    lo[0] = (rest / bg.nb[1]) * bg.edge[0];
  };
  // the tile values of a brick this thread stages: row r = tid / 16 + 16 k
  // k mod K for the tile's grid indices; with 8-point bricks an index is at
  // most one period off (k in [-(P - 1), K + 7), K >= 8)
  auto wrap = [](int k, int K) {
    if (E8) {
      k = k < 0 ? k + K : k;
      return k >= K ? k - K : k;
    }
    while (k < 0) k += K;
    while (k >= K) k -= K;
    return k;
  };
  auto load_tile = [&](int brick, T* reg) {
    int lo[3];
    lo_of(brick, lo);
    int r = tid >> 4;
    int t0 = r / H[1], t1 = r - t0 * H[1];
    const int k2 = wrap(lo[2] - (P - 1) + min(c16, H[2] - 1), K3);
#pragma unroll
    for (int k = 0; k < kPfRows; ++k) {
      // every lane loads (rows past the tile and lanes past H2 read a
      // clamped in-tile point, and their values are not stored)
      const int tt0 = min(t0, H[0] - 1);
      const int k0 = wrap(lo[0] - (P - 1) + tt0, K1), k1 = wrap(lo[1] - (P - 1) + t1, K2);
      reg[k] = grid[(static_cast<long>(k0) * K2 + k1) * K3 + k2];
      r += kGatherThreads / 16;
      t1 += kGatherThreads / 16;
      while (t1 >= H[1]) {
        t1 -= H[1];
        ++t0;
      }
    }
  };
  auto store_tile = [&](const T* reg) {
    int r = tid >> 4;
#pragma unroll
    for (int k = 0; k < kPfRows; ++k) {
      if (r < nrows && c16 < H[2]) tile[r * H[2] + c16] = reg[k];
      r += kGatherThreads / 16;
    }
  };
  T treg[kPfRows];
  T rec[4] = {T(0), T(0), T(0), T(0)};
  int pm = 0;
  __syncthreads();   // offs
  // a brick without particles needs no tile (its offsets are uniform)
  if (b_begin < b_end && offs[1] > offs[0]) {
    load_tile(b_begin, treg);
    const int s = offs[0] + tid;
    if (s < offs[1]) {
      load_record(sorted, s, rec);
      pm = perm[s];
    }
  }
  for (int b = b_begin; b < b_end; ++b) {
    const int i0 = offs[b - b_begin], i1 = offs[b - b_begin + 1];
    if (i1 > i0) {
      store_tile(treg);
      __syncthreads();
    }
    T rc[4] = {rec[0], rec[1], rec[2], rec[3]};
    int pc = pm;
    if (b + 1 < b_end && offs[b - b_begin + 2] > i1) {   // next brick's values in flight
      load_tile(b + 1, treg);
      const int s = i1 + tid;
      if (s < offs[b - b_begin + 2]) {
        load_record(sorted, s, rec);
        pm = perm[s];
      }
    }
    if (i1 == i0) continue;
    int lo[3];
    lo_of(b, lo);
    for (int s = i0 + tid; s < i1; s += kGatherThreads) {
      if (s != i0 + tid) {
        load_record(sorted, s, rc);
        pc = perm[s];
      }
      T w[3][P], dw[3][P];
      int l[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        int base;
        const T f = stencil_coord(rc[j], g.invL[j], g.K[j], g.cell, base);
        stencil_weights<T, P>(f, g.cell, w[j], dw[j]);
        l[j] = min(max(base - lo[j] + P - 1, P - 1), H[j] - 1);
      }
      T phi = 0, g0 = 0, g1 = 0, g2 = 0;
      constexpr int UB = P <= 8 ? P : 1;
      // the stencil's lowest tile point: every read below is at a
      // non-negative, compile-time offset (E8) from a plane's start
      const T* st0 = tile + ((l[0] - (P - 1)) * H[1] + l[1] - (P - 1)) * H[2] + l[2] - (P - 1);
      // the x weights rotate down one place per plane (no indexed select)
      T wr[P], dwr[P];
#pragma unroll
      for (int t = 0; t < P; ++t) {
        wr[t] = w[0][t];
        dwr[t] = dw[0][t];
      }
#pragma unroll 1
      for (int a = 0; a < P; ++a) {
        const T wa = wr[0], dwa = dwr[0];
#pragma unroll
        for (int t = 0; t + 1 < P; ++t) {
          wr[t] = wr[t + 1];
          dwr[t] = dwr[t + 1];
        }
        const T* plane = st0 + (P - 1 - a) * (H[1] * H[2]);
        T sa = 0, sa1 = 0, sa2 = 0;
#pragma unroll UB
        for (int bb = 0; bb < P; ++bb) {
          const T* row = plane + (P - 1 - bb) * H[2];
          T sv = 0, s2 = 0;
#pragma unroll
          for (int c = 0; c < P; ++c) {
            const T v = row[P - 1 - c];
            sv += w[2][c] * v;
            s2 += dw[2][c] * v;
          }
          sa += w[1][bb] * sv;
          sa1 += dw[1][bb] * sv;
          sa2 += w[1][bb] * s2;
        }
        phi += wa * sa;
        g0 += dwa * sa;
        g1 += wa * sa1;
        g2 += wa * sa2;
      }
      const long i = pc;
      const T qi = rc[3];
      if (pot) pot[i] = phi;
      if (force) {
        force[3 * i + 0] = -qi * g0 * static_cast<T>(K1 * g.invL[0]);
        force[3 * i + 1] = -qi * g1 * static_cast<T>(K2 * g.invL[1]);
        force[3 * i + 2] = -qi * g2 * static_cast<T>(K3 * g.invL[2]);
      }
    }
    __syncthreads();   // every tile read done before the next store
  }
}

template <typename T, int P, bool E8>
__global__ __launch_bounds__(kGatherThreads) void gather_brick_pf(
    const T* __restrict__ sorted, const int* __restrict__ offset, const int* __restrict__ perm,
    const T* __restrict__ grid, T* __restrict__ pot, T* __restrict__ force, EnergyJob ej,
    GridGeom g, BinGeom bg) {
  gather_brick_pf_body<T, P, E8>(sorted, offset, perm, grid, pot, force, ej, g, bg, Wg::plain());
}

// sorted2[d] = (x, y, z, g[perm[d]]): the binned positions with a second
// per-particle value (the adjoint's upstream potential gradient) as charge.
template <typename T>
__global__ __launch_bounds__(256) void resort_charges(long n, const T* __restrict__ sorted,
                                                      const int* __restrict__ perm,
                                                      const T* __restrict__ gval,
                                                      T* __restrict__ sorted2) {
  const long d = blockIdx.x * static_cast<long>(blockDim.x) + threadIdx.x;
  if (d >= n) return;
  sorted2[4 * d + 0] = sorted[4 * d + 0];
  sorted2[4 * d + 1] = sorted[4 * d + 1];
  sorted2[4 * d + 2] = sorted[4 * d + 2];
  sorted2[4 * d + 3] = gval ? gval[perm[d]] : T(0);
}

// Adjoint gather (binned order): with Phi = Theta S q and Psi = Theta S g,
//   grad_pos_i = grad W_i . [(gE q_i + g_i) Phi + q_i Psi]
//   grad_q_i   = gE (W_i . Phi + self_i + neutral) + W_i . Psi
// self_i = -2 beta q_i / sqrt(pi), neutral = -pi sum(q) / (V beta^2).
template <typename T, int P>
__global__ __launch_bounds__(256) void gather_backward(
    long n, const T* __restrict__ sorted, const int* __restrict__ perm,
    const T* __restrict__ Phi, const T* __restrict__ Psi, const double* __restrict__ g_energy,
    const T* __restrict__ g_pot, const double* __restrict__ sumq, double beta, double volume,
    T* __restrict__ grad_pos, T* __restrict__ grad_q, GridGeom g) {
  const long s = xcd_order(blockIdx.x, gridDim.x) * static_cast<long>(blockDim.x) + threadIdx.x;
  if (s >= n) return;
  T w[3][P], dw[3][P];
  int base[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const T f = stencil_coord(sorted[4 * s + j], g.invL[j], g.K[j], g.cell, base[j]);
    stencil_weights<T, P>(f, g.cell, w[j], dw[j]);
  }
  const int K1 = g.K[0], K2 = g.K[1], K3 = g.K[2];
  int kc[P];
#pragma unroll
  for (int c = 0; c < P; ++c) {
    kc[c] = base[2] - c;
    if (kc[c] < 0) kc[c] += K3;
  }
  // v[0]: W.grid, v[1..3]: derivatives along the three axes (in u units)
  T vf[4] = {0, 0, 0, 0}, vs[4] = {0, 0, 0, 0};
  // one plane of Phi and Psi loads in flight (a whole unrolled stencil of
  // both holds too many registers)
  constexpr int UB = P <= 8 ? P : 1;
#pragma unroll 1
  for (int a = 0; a < P; ++a) {
    int ka = base[0] - a;
    if (ka < 0) ka += K1;
    T wa = w[0][0], dwa = dw[0][0];
#pragma unroll
    for (int t = 1; t < P; ++t)
      if (a == t) {
        wa = w[0][t];
        dwa = dw[0][t];
      }
#pragma unroll UB
    for (int b = 0; b < P; ++b) {
      int kb = base[1] - b;
      if (kb < 0) kb += K2;
      const long row = (static_cast<long>(ka) * K2 + kb) * K3;
      T sf = 0, sf2 = 0, ss = 0, ss2 = 0;
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const T x = Phi[row + kc[c]];
        sf += w[2][c] * x;
        sf2 += dw[2][c] * x;
        if (Psi) {
          const T y = Psi[row + kc[c]];
          ss += w[2][c] * y;
          ss2 += dw[2][c] * y;
        }
      }
      const T wab = wa * w[1][b];
      vf[0] += wab * sf;
      vf[1] += dwa * w[1][b] * sf;
      vf[2] += wa * dw[1][b] * sf;
      vf[3] += wab * sf2;
      vs[0] += wab * ss;
      vs[1] += dwa * w[1][b] * ss;
      vs[2] += wa * dw[1][b] * ss;
      vs[3] += wab * ss2;
    }
  }
  const long i = perm[s];
  const T qi = sorted[4 * s + 3];
  const T ge = g_energy ? static_cast<T>(*g_energy) : T(0);
  const T gp = g_pot ? g_pot[i] : T(0);
  if (grad_pos) {
    const T cf = ge * qi + gp;
#pragma unroll
    for (int j = 0; j < 3; ++j)
      grad_pos[3 * i + j] = (cf * vf[1 + j] + qi * vs[1 + j]) * static_cast<T>(g.K[j] * g.invL[j]);
  }
  if (grad_q) {
    const double pi = 3.141592653589793238462643383279502884;
    const double self_i = -2.0 * beta * static_cast<double>(qi) / sqrt(pi);
    const double neutral = -pi * sumq[0] / (volume * beta * beta);
    grad_q[i] = ge * (vf[0] + static_cast<T>(self_i + neutral)) + vs[0];
  }
}

// Per-block FP64 partial sums of (q pot, q, q^2), then one block combines
// them in a fixed order: the result does not depend on scheduling.
template <typename T>
__global__ __launch_bounds__(256) void energy_partial(long n, const T* __restrict__ q,
                                                      const T* __restrict__ pot,
                                                      double* __restrict__ part) {
  __shared__ double red[48];
  const long per = (n + gridDim.x - 1) / gridDim.x;
  const long b = per * blockIdx.x, e = (b + per < n) ? b + per : n;
  double s0 = 0, s1 = 0, s2 = 0;
  for (long i = b + threadIdx.x; i < e; i += blockDim.x) {
    const double qi = static_cast<double>(q[i]);
    s0 += qi * static_cast<double>(pot[i]);
    s1 += qi;
    s2 += qi * qi;
  }
  double v[3] = {s0, s1, s2};
  block_reduce<3, 3>(v, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) part[3 * blockIdx.x + k] = v[k];
}

__global__ __launch_bounds__(256) void energy_final(const double* __restrict__ part, int nb,
                                                    double beta, double volume,
                                                    double* __restrict__ e4) {
  __shared__ double red[48];
  double s[3] = {0, 0, 0};
  for (int i0 = threadIdx.x; i0 < nb; i0 += 4 * 256) {  // four triples in flight
    double x[4][3];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < 3; ++k) x[u][k] = i0 + 256 * u < nb ? part[3 * (i0 + 256 * u) + k] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < 3; ++k) s[k] += x[u][k];
  }
  block_reduce<3, 3>(s, red);
  if (threadIdx.x == 0) {
    const double pi = 3.141592653589793238462643383279502884;
    const double e_rec = 0.5 * s[0];
    const double e_self = -beta / sqrt(pi) * s[2];
    const double e_neu = -pi * s[1] * s[1] / (2.0 * volume * beta * beta);
    e4[0] = e_rec;
    e4[1] = e_self;
    e4[2] = e_neu;
    e4[3] = e_rec + e_self + e_neu;
  }
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

namespace {

// Workgroups of the folded scan-and-scatter kernel (at least one).
int64_t scatter_blocks(int64_t n) {
  const int64_t per = 256 * kBinPer;
  return std::max<int64_t>(1, (n + per - 1) / per);
}

// The scan goes into the scatter when the LDS histogram is used and the
// workgroups' copies of the scan read at most 2^21 counts in all; otherwise
// one workgroup scans.
bool scan_in_scatter(const Bins& b, int64_t n) {
  return b.geom.nbricks <= kLdsHist && scatter_blocks(n) * b.geom.nbricks <= (int64_t(1) << 21);
}

template <typename T, int NT>
hipError_t count_lds_t(const GridGeom& g, const Bins& b, int64_t n, const void* pos,
                       hipStream_t st) {
  const long per = static_cast<long>(NT) * kCountPer;
  const unsigned blocks = static_cast<unsigned>((n + per - 1) / per);
  return launch_or_record<NT, bin_count_lds_body<T, NT>>(
      LS_BIN_COUNT, bin_count_lds<T, NT>, dim3(blocks), 0, st, static_cast<long>(n),
      static_cast<const T*>(pos), g, b.geom, b.brick_of, b.slot, b.count);
}

template <typename T>
hipError_t bin_t(const GridGeom& g, const Bins& b, int64_t n, const void* pos, hipStream_t st) {
  if (n > 0) {
    if (b.geom.nbricks <= kLdsHist) {
      hipError_t e = n >= kCountBig ? count_lds_t<T, 1024>(g, b, n, pos, st)
                                    : count_lds_t<T, 256>(g, b, n, pos, st);
      if (e != hipSuccess) return e;
    } else {
      if (record_unsupported()) return hipSuccess;
      const unsigned blocks = static_cast<unsigned>((n + 255) / 256);
      hipLaunchKernelGGL((bin_count<T>), dim3(blocks), dim3(256), 0, st, static_cast<long>(n),
                         static_cast<const T*>(pos), g, b.geom, b.brick_of, b.slot, b.count);
    }
  }
  if (!scan_in_scatter(b, n)) {
    if (record_unsupported()) return hipSuccess;
    hipLaunchKernelGGL(bin_scan, dim3(1), dim3(1024), 0, st, b.count, b.geom.nbricks, b.offset);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t scatter_t(const Bins& b, int64_t n, const void* pos, const void* q, double* qpart,
                     hipStream_t st) {
  if (scan_in_scatter(b, n)) {
    // at least one workgroup: it stores the offsets also for n = 0
    const unsigned blocks = static_cast<unsigned>(scatter_blocks(n));
    return launch_or_record<256, bin_scan_scatter_body<T>>(
        LS_BIN_SCATTER, bin_scan_scatter<T>, dim3(blocks), 0, st, static_cast<long>(n),
        static_cast<const T*>(pos), static_cast<const T*>(q),
        static_cast<const int*>(b.brick_of), static_cast<const int*>(b.slot),
        static_cast<const int*>(b.count), b.geom.nbricks, b.offset, static_cast<T*>(b.sorted),
        b.perm, qpart);
  }
  if (n == 0) return hipSuccess;
  if (record_unsupported()) return hipSuccess;
  const unsigned blocks = static_cast<unsigned>((n + 255) / 256);
  hipLaunchKernelGGL((bin_scatter<T>), dim3(blocks), dim3(256), 0, st, static_cast<long>(n),
                     static_cast<const T*>(pos), static_cast<const T*>(q), b.brick_of, b.slot,
                     b.offset, static_cast<T*>(b.sorted), b.perm, qpart);
  return hipGetLastError();
}

// Spread dispatch by spline order: for P <= 4 the owner-computes kernel (one
// pass, each particle seen by ~(1 + (P-1)/8)^3 owner bricks); for larger P
// the two-pass home-computes scheme, which sees each particle once.
template <typename T, int P>
hipError_t spread_brick_p(const GridGeom& g, const Bins& b, const void* src, void* grid,
                          double* part2, hipStream_t st) {
  const T* srt = static_cast<const T*>(src ? src : b.sorted);
  // the owner spread for low orders, FP64 at order 4, and sparse plans
  bool owner = P < 4 || (P == 4 && sizeof(T) == 8);
  if constexpr (P <= 9) owner = owner || b.geom.sparse;
  if (owner) {
    const size_t lds = sizeof(double) * b.geom.edge[0] * b.geom.edge[1] * b.geom.edge[2];
    const bool e8 = b.geom.edge[0] == 8 && b.geom.edge[1] == 8 && b.geom.edge[2] == 8;
    const int* off = b.offset;
    const int* nbr = b.nbr;
    if constexpr (P <= 9) {
      if (e8)
        return launch_or_record<256, spread_brick_body<T, P, true>>(
            LS_SPREAD, spread_brick<T, P, true>, dim3(b.geom.nbricks), lds, st, srt, off, nbr,
            static_cast<T*>(grid), part2, b.count, g, b.geom);
      return launch_or_record<256, spread_brick_body<T, P, false>>(
          LS_SPREAD, spread_brick<T, P, false>, dim3(b.geom.nbricks), lds, st, srt, off, nbr,
          static_cast<T*>(grid), part2, b.count, g, b.geom);
    }
    return hipErrorInvalidValue;
  }
  const int ntile = (b.geom.edge[0] + P - 1) * (b.geom.edge[1] + P - 1) * (b.geom.edge[2] + P - 1);
  if constexpr (sizeof(T) == 4 && P <= 9) {
    // float grids: the matrix-core tile spread (every brick edge <= 8)
    const int* off = b.offset;
    hipError_t e = launch_or_record_w<64 * kMfmaWaves, kMfmaWavesPerEu, spread_home_mfma_body<P>>(
        LS_SPREAD, spread_home_mfma<P>, dim3(b.geom.nbricks), 0, st, srt, off,
        static_cast<float*>(b.tiles), b.count, g, b.geom);
    if (e != hipSuccess) return e;
  } else {
    if (record_unsupported()) return hipSuccess;
    hipLaunchKernelGGL((spread_home<T, P>), dim3(b.geom.nbricks), dim3(kHomeThreads),
                       sizeof(double) * ntile, st, srt, b.offset, static_cast<T*>(b.tiles),
                       b.count, g, b.geom);
  }
  if (b.geom.two_homes) {
    const int nw = combine_workgroups(b.geom.nbricks);
    if ((b.geom.nbricks + nw - 1) / nw > kCombineMaxBricks ||
        b.geom.edge[0] * b.geom.edge[1] * b.geom.edge[2] > kCombineThreads)
      return hipErrorInvalidValue;
    return launch_or_record<kCombineThreads, spread_combine_pf_body<T, P>>(
        LS_COMBINE, spread_combine_pf<T, P>, dim3(nw), 0, st, static_cast<const T*>(b.tiles),
        static_cast<T*>(grid), part2, g, b.geom);
  }
  if (record_unsupported()) return hipSuccess;
  hipLaunchKernelGGL((spread_combine<T, P>), dim3(b.geom.nbricks), dim3(512), 0, st,
                     static_cast<const T*>(b.tiles), b.nbr, static_cast<T*>(grid), part2, g,
                     b.geom);
  return hipGetLastError();
}

// Gather dispatch: for FP32 and spline orders above 4 the brick-tiled kernel
// (each potential value staged once in LDS and read by every stencil that
// needs it); otherwise particles read the grid directly (fewer particles per
// brick and smaller stencils do not amortise the staging).
template <typename T, int P>
hipError_t gather_brick_p(const GridGeom& g, const Bins& b, int64_t n, const void* grid,
                          void* pot, void* force, const EnergyJob& ej, hipStream_t st) {
  if (P < 4 || (P > 4 && sizeof(T) == 8)) {
    // direct stencil reads per particle (low orders, FP64)
    const unsigned blocks = static_cast<unsigned>((n + 255) / 256) + (ej.e4 ? 1 : 0);
    return launch_or_record<256, gather_sorted_body<T, P>>(
        LS_GATHER, gather_sorted<T, P>, dim3(blocks), 0, st, static_cast<long>(n),
        static_cast<const T*>(b.sorted), static_cast<const int*>(b.perm),
        static_cast<const T*>(grid), static_cast<T*>(pot), static_cast<T*>(force), ej, g);
  }
  if constexpr (sizeof(T) == 4 && P > 4 && P <= 9) {
    const int ntile = (b.geom.edge[0] + P - 1) * (b.geom.edge[1] + P - 1) * (b.geom.edge[2] + P - 1);
    const int nw = gather_pf_workgroups(b.geom.nbricks, b.geom.gather_wgs);
    if ((b.geom.nbricks + nw - 1) / nw > kGatherMaxBricks) return hipErrorInvalidValue;
    const bool e8 = b.geom.edge[0] == 8 && b.geom.edge[1] == 8 && b.geom.edge[2] == 8;
    if (e8)
      return launch_or_record<kGatherThreads, gather_brick_pf_body<T, P, true>>(
          LS_GATHER, gather_brick_pf<T, P, true>, dim3(nw + (ej.e4 ? 1 : 0)), sizeof(T) * ntile,
          st, static_cast<const T*>(b.sorted), static_cast<const int*>(b.offset),
          static_cast<const int*>(b.perm), static_cast<const T*>(grid), static_cast<T*>(pot),
          static_cast<T*>(force), ej, g, b.geom);
    return launch_or_record<kGatherThreads, gather_brick_pf_body<T, P, false>>(
        LS_GATHER, gather_brick_pf<T, P, false>, dim3(nw + (ej.e4 ? 1 : 0)), sizeof(T) * ntile,
        st, static_cast<const T*>(b.sorted), static_cast<const int*>(b.offset),
        static_cast<const int*>(b.perm), static_cast<const T*>(grid), static_cast<T*>(pot),
        static_cast<T*>(force), ej, g, b.geom);
  }
  if (P == 4) {
    const unsigned blocks = static_cast<unsigned>((n + 63) / 64) + (ej.e4 ? 1 : 0);
    return launch_or_record<256, gather_sorted_planes_body<T, 4>>(
        LS_GATHER, gather_sorted_planes<T, 4>, dim3(blocks), 0, st, static_cast<long>(n),
        static_cast<const T*>(b.sorted), static_cast<const int*>(b.perm),
        static_cast<const T*>(grid), static_cast<T*>(pot), static_cast<T*>(force), ej, g);
  }
  // FP32, P > 9: the brick tile without prefetch
  if (record_unsupported()) return hipSuccess;
  const int ntile = (b.geom.edge[0] + P - 1) * (b.geom.edge[1] + P - 1) * (b.geom.edge[2] + P - 1);
  hipLaunchKernelGGL((gather_brick<T, P>), dim3(b.geom.nbricks + (ej.e4 ? 1 : 0)),
                     dim3(kGatherThreads), sizeof(T) * ntile, st,
                     static_cast<const T*>(b.sorted), b.offset, b.perm,
                     static_cast<const T*>(grid), static_cast<T*>(pot), static_cast<T*>(force),
                     ej, g, b.geom);
  return hipGetLastError();
}


}  // namespace

// Number of (sum, max) pairs the binned spread writes: one per workgroup of
// the persistent combine, else one per brick.
int spread_partials(const BinGeom& bg, int p, bool fp64) {
  const bool home = p > 4 || (p == 4 && !fp64);
  return (home && !bg.sparse && bg.two_homes) ? combine_workgroups(bg.nbricks) : bg.nbricks;
}

// Number of (sum q, sum q^2) pairs the scatter writes.
int scatter_partials(const Bins& b, int64_t n) {
  if (scan_in_scatter(b, n)) return static_cast<int>(scatter_blocks(n));
  return static_cast<int>((n + 255) / 256);
}

hipError_t launch_bin(int prec, const GridGeom& g, const Bins& b, int64_t n, const void* pos,
                      const void* q, double* qpart, hipStream_t st) {
  hipError_t e = prec == PREC_FP64 ? bin_t<double>(g, b, n, pos, st) : bin_t<float>(g, b, n, pos, st);
  if (e != hipSuccess) return e;
  return prec == PREC_FP64 ? scatter_t<double>(b, n, pos, q, qpart, st)
                           : scatter_t<float>(b, n, pos, q, qpart, st);
}

hipError_t launch_spread_binned(int prec, const GridGeom& g, const Bins& b, void* grid,
                                double* part2, hipStream_t st, const void* src) {
  if (prec == PREC_FP64) {
#define CALL(P) spread_brick_p<double, P>(g, b, src, grid, part2, st)
    KPME_ORDER_SWITCH(g.p, CALL)
#undef CALL
  }
#define CALL(P) spread_brick_p<float, P>(g, b, src, grid, part2, st)
  KPME_ORDER_SWITCH(g.p, CALL)
#undef CALL
}

hipError_t launch_gather_binned(int prec, const GridGeom& g, const Bins& b, int64_t n,
                                const void* grid, void* pot, void* force, const EnergyJob& ej,
                                hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (prec == PREC_FP64) {
#define CALL(P) gather_brick_p<double, P>(g, b, n, grid, pot, force, ej, st)
    KPME_ORDER_SWITCH(g.p, CALL)
#undef CALL
  }
#define CALL(P) gather_brick_p<float, P>(g, b, n, grid, pot, force, ej, st)
  KPME_ORDER_SWITCH(g.p, CALL)
#undef CALL
}

template <typename T, int P>
hipError_t gather_backward_p(const GridGeom& g, const Bins& b, int64_t n, const void* Phi,
                             const void* Psi, const double* g_energy, const void* g_pot,
                             const double* sumq, double beta, double volume, void* grad_pos,
                             void* grad_q, hipStream_t st) {
  const unsigned blocks = static_cast<unsigned>((n + 255) / 256);
  hipLaunchKernelGGL((gather_backward<T, P>), dim3(blocks), dim3(256), 0, st,
                     static_cast<long>(n), static_cast<const T*>(b.sorted), b.perm,
                     static_cast<const T*>(Phi), static_cast<const T*>(Psi), g_energy,
                     static_cast<const T*>(g_pot), sumq, beta, volume,
                     static_cast<T*>(grad_pos), static_cast<T*>(grad_q), g);
  return hipGetLastError();
}

hipError_t launch_resort_charges(int prec, const Bins& b, int64_t n, const void* gval,
                                 void* sorted2, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = static_cast<unsigned>((n + 255) / 256);
  if (prec == PREC_FP64)
    hipLaunchKernelGGL((resort_charges<double>), dim3(blocks), dim3(256), 0, st,
                       static_cast<long>(n), static_cast<const double*>(b.sorted), b.perm,
                       static_cast<const double*>(gval), static_cast<double*>(sorted2));
  else
    hipLaunchKernelGGL((resort_charges<float>), dim3(blocks), dim3(256), 0, st,
                       static_cast<long>(n), static_cast<const float*>(b.sorted), b.perm,
                       static_cast<const float*>(gval), static_cast<float*>(sorted2));
  return hipGetLastError();
}

hipError_t launch_gather_backward(int prec, const GridGeom& g, const Bins& b, int64_t n,
                                  const void* Phi, const void* Psi, const double* g_energy,
                                  const void* g_pot, const double* sumq, double beta,
                                  double volume, void* grad_pos, void* grad_q,
                                  hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (prec == PREC_FP64) {
#define CALL(P) gather_backward_p<double, P>(g, b, n, Phi, Psi, g_energy, g_pot, sumq, beta, \
                                             volume, grad_pos, grad_q, st)
    KPME_ORDER_SWITCH(g.p, CALL)
#undef CALL
  }
#define CALL(P) gather_backward_p<float, P>(g, b, n, Phi, Psi, g_energy, g_pot, sumq, beta, \
                                            volume, grad_pos, grad_q, st)
  KPME_ORDER_SWITCH(g.p, CALL)
#undef CALL
}

hipError_t launch_energy_job(const EnergyJob& ej, hipStream_t st) {
  if (!ej.e4) return hipSuccess;
  return launch_or_record<256, energy_job_body>(LS_GATHER, energy_job_kernel, dim3(1), 0, st, ej);
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
