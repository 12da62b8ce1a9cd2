// Sum-of-Kronecker-Products reciprocal operator on the matrix cores (gfx950).
//
// Phi = sum_r omega_r (A_r (x) B_r (x) C_r) Q - c sum(Q) (Eq. formfinale with
// the correction of Eq. termbonsum), evaluated as the mode products of
// Alg. 2, grouped by the nested-SVD structure (Sec. 2.1.1): all terms of
// outer index i share their axis-2 factor C_i.
//
//  stage 1  Y_i = Q x_3 C_i for the r0 distinct C_i: one GEMM with rows
//           (i, k3), columns the K1 x K2 slab position and inner index g3;
//           written slab-major [i][k3][g1][g2] (zero-padded to K1P x K2P).
//  stage 2  per slab k3 and range of terms:
//           Phi_k3 += sum_t A_t . Y_{g(t),k3} . B_t^T   (omega folded into A_t)
//           Each wave owns NC output columns; T = Y . B_t^T stays in the MFMA
//           accumulators and is fed straight back as the B operand of
//           A_t . T (the K index of an MFMA may be permuted consistently in
//           both operands, so the accumulator layout is used as is).
//  final    sums the stage-2 partial slabs in a fixed order, transposes to
//           [k1][k2][k3] and subtracts c * sum(Q).
//
// Precisions: FP64 and FP32 use the 16x16x4 MFMAs; BF16X3 splits every
// operand into bf16 hi + lo and issues hi*hi + hi*lo + lo*hi on the
// 16x16x32 bf16 MFMA with FP32 accumulation.
#include "batch_launch.hpp"
#include "device_common.hpp"
#include "kernels.hpp"

namespace kpme {

namespace {

constexpr int S1 = 64;  // stage-1 output tile (rows and columns)

// ----------------------------------------------------------------------------
// Stage 1, split precision (BF16X3 / FP16X3), one wave per block: a tile of
// 64 slab positions p = g1 K2P + g2 (rows of Q, the MFMA A operand) against
// kS1Tiles 16-row tiles of C (rows n = (i, k3), the B operand), looping over
// the K3P / 32 chunks of g3 with the next chunk's Q values in flight.
// The 64 positions are dealt to the four 16-row MFMA tiles so that tile u,
// accumulator row 4a + r, holds position 16a + 4u + r: a lane then owns 16
// consecutive positions of one output row and stores them as 32 bytes per
// plane.  Q is multiplied by the grid scale (a power of two, FP16X3) before
// its split, the FP32 result by sy (a power of two) before Y's split.
// C hi/lo: [nrows][K3P] (pre-scaled, zero-padded); Y hi/lo: [nrows][slab].
constexpr int kS1Tiles = 4;

// Grid sum and FP16X3 grid scale from np partial (sum, max|.|) pairs, which
// the split stage-1 kernels reduce themselves when there are few of them (no
// separate launch): the scale 2^(13 - floor(log2 max)) brings the largest
// grid value into [2^13, 2^14) (1 for an all-zero or non-finite grid).  With
// `store` the workgroup writes (sum, scale) to sums[0..1] for the later
// stages.  part == nullptr: sums[0..1] were computed before; nothing is
// reduced.  Returns the scale when `want_scale`, else 1.  Every thread of the
// workgroup calls it, with the same arguments.
__device__ float grid_scalars(const double* __restrict__ part, int np, double* __restrict__ sums,
                              bool want_scale, bool store) {
  __shared__ double red[32];
  __shared__ double scale;
  if (!part) return want_scale ? static_cast<float>(sums[1]) : 1.0f;
  if (!want_scale && !store) return 1.0f;
  double v[2] = {0.0, 0.0};
  // eight pairs per thread in flight at a time (the partials come from
  // another kernel, most of them from other XCDs' caches)
  for (int i0 = threadIdx.x; i0 < np; i0 += 8 * blockDim.x) {
    double2 x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * blockDim.x;
      x[u] = i < np ? *reinterpret_cast<const double2*>(&part[2 * i]) : double2{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      v[0] += x[u].x;
      v[1] = fmax(v[1], x[u].y);
    }
  }
  block_reduce<1, 2>(v, red);
  if (threadIdx.x == 0) {
    const double m = v[1];
    scale = (m > 0.0 && m < 1e300) ? ldexp(1.0, 13 - ilogb(m)) : 1.0;
    if (store) {
      sums[0] = v[0];
      sums[1] = scale;
    }
  }
  __syncthreads();
  return want_scale ? static_cast<float>(scale) : 1.0f;
}

template <typename H>
__device__ __forceinline__ void stage1_x3_body(
    const float* __restrict__ Q, const H* __restrict__ Chi, const H* __restrict__ Clo,
    H* __restrict__ Yhi, H* __restrict__ Ylo, int K1, int K2, int K3, int K3P, int K2P,
    long slab, int nrows, const double* __restrict__ part, int np, double* __restrict__ sums,
    int scale_q, float sy,
    const Wg wg) {
  typedef typename HVec<H>::v8 v8;
  const int lane = threadIdx.x, q = lane >> 4, m = lane & 15;
  // logical order: the n splits of one position tile are consecutive (and so
  // share an XCD and its L2 copy of the Q tile)
  const int L = wg_order(wg, wg.linear(), wg.count());
  const long p0 = static_cast<long>(L / wg.nx) * 64;
  const int nt0 = (L % wg.nx) * kS1Tiles;
  const float sq = grid_scalars(part, np, sums, scale_q != 0, wg.linear() == 0);
  const bool vec4 = (K3 & 3) == 0;  // rows 16-byte aligned, 4-float groups all in or out
  // Q rows of this lane's A-operand rows: tile u holds p = p0 + 16 (m / 4) + 4 u + m % 4
  const float* row[4];
  bool valid[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const long p = p0 + 16 * (m >> 2) + 4 * u + (m & 3);
    const int g1 = static_cast<int>(p / K2P), g2 = static_cast<int>(p % K2P);
    valid[u] = g1 < K1 && g2 < K2;
    row[u] = Q + (static_cast<long>(valid[u] ? g1 : 0) * K2 + (valid[u] ? g2 : 0)) * K3;
  }
  auto load = [&](int kc, float (&x)[4][8]) {
    const int k0 = 32 * kc + 8 * q;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (vec4) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = k0 + 4 * h;
          float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
          if (valid[u] && k < K3) v = *reinterpret_cast<const float4*>(&row[u][k]);
          x[u][4 * h] = v.x; x[u][4 * h + 1] = v.y; x[u][4 * h + 2] = v.z; x[u][4 * h + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[u][e] = (valid[u] && k0 + e < K3) ? row[u][k0 + e] : 0.f;
      }
    }
  };
  // C fragments (B operand) of the wave's n tiles for one K chunk
  auto loadc = [&](int kc, v8 (&bh)[kS1Tiles], v8 (&bl)[kS1Tiles]) {
#pragma unroll
    for (int t = 0; t < kS1Tiles; ++t) {
      const int n = (nt0 + t) * 16 + m;
      bh[t] = v8{};
      bl[t] = v8{};
      if (n < nrows) {
        bh[t] = *reinterpret_cast<const v8*>(&Chi[static_cast<long>(n) * K3P + 32 * kc + 8 * q]);
        bl[t] = *reinterpret_cast<const v8*>(&Clo[static_cast<long>(n) * K3P + 32 * kc + 8 * q]);
      }
    }
  };
  floatx4 acc[kS1Tiles][4];
#pragma unroll
  for (int t = 0; t < kS1Tiles; ++t)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[t][u] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int nkc = K3P / 32;
  float x[4][8];
  v8 bh[kS1Tiles], bl[kS1Tiles];
  load(0, x);
  loadc(0, bh, bl);
  for (int kc = 0; kc < nkc; ++kc) {
    v8 ah[4], al[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        H h, l;
        split_h<H>(sq * x[u][e], h, l);
        ah[u][e] = h;
        al[u][e] = l;
      }
    v8 ch[kS1Tiles], cl[kS1Tiles];
#pragma unroll
    for (int t = 0; t < kS1Tiles; ++t) {
      ch[t] = bh[t];
      cl[t] = bl[t];
    }
    // the next chunk's operands load while this chunk's MFMAs run
    if (kc + 1 < nkc) {
      load(kc + 1, x);
      loadc(kc + 1, bh, bl);
    }
#pragma unroll
    for (int t = 0; t < kS1Tiles; ++t) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[t][u] = mfma_h(ah[u], ch[t], acc[t][u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[t][u] = mfma_h(ah[u], cl[t], acc[t][u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[t][u] = mfma_h(al[u], ch[t], acc[t][u]);
    }
  }
#pragma unroll
  for (int t = 0; t < kS1Tiles; ++t) {
    const int n = (nt0 + t) * 16 + m;
    if (n >= nrows) continue;
    v8 yh[2], yl[2];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        H h, l;
        split_h<H>(sy * acc[t][u][r], h, l);
        yh[u >> 1][4 * (u & 1) + r] = h;
        yl[u >> 1][4 * (u & 1) + r] = l;
      }
    const long o = static_cast<long>(n) * slab + p0 + 16 * q;
    *reinterpret_cast<v8*>(&Yhi[o]) = yh[0];
    *reinterpret_cast<v8*>(&Yhi[o + 8]) = yh[1];
    *reinterpret_cast<v8*>(&Ylo[o]) = yl[0];
    *reinterpret_cast<v8*>(&Ylo[o + 8]) = yl[1];
  }
}

template <typename H>
__global__ __launch_bounds__(64) void stage1_x3(
    const float* __restrict__ Q, const H* __restrict__ Chi, const H* __restrict__ Clo,
    H* __restrict__ Yhi, H* __restrict__ Ylo, int K1, int K2, int K3, int K3P, int K2P,
    long slab, int nrows, const double* __restrict__ part, int np, double* __restrict__ sums,
    int scale_q, float sy) {
  stage1_x3_body<H>(Q, Chi, Clo, Yhi, Ylo, K1, K2, K3, K3P, K2P, slab, nrows, part, np, sums, scale_q, sy, Wg::plain());
}

// Stage 1, split precision, K3P <= 160 (NK = K3P / 32 chunks): a workgroup
// of four waves takes one tile of 64 positions; its Q rows are split into
// hi/lo once, into LDS, and every wave keeps the A fragments of the whole K
// range in registers while it streams its share of the 16-row C tiles
// (gridDim.x workgroups per position tile; the plan picks that split, since
// the C tiles of one workgroup should spread evenly over its four waves),
// the next tile's C fragments in flight.  Position dealing and output layout
// as in stage1_x3.

template <typename H, int NK>
__device__ __forceinline__ void stage1_x3_lds_body(
    const float* __restrict__ Q, const H* __restrict__ Chi, const H* __restrict__ Clo,
    H* __restrict__ Yhi, H* __restrict__ Ylo, int K1, int K2, int K3, int K2P, long slab,
    int nrows, const double* __restrict__ part, int np, double* __restrict__ sums, int scale_q,
    float sy,
    const Wg wg) {
  typedef typename HVec<H>::v8 v8;
  constexpr int K3P = 32 * NK, QSTR = K3P + 8;
  __shared__ __attribute__((aligned(16))) H Qh[64 * QSTR], Ql[64 * QSTR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4, m = lane & 15;
  // logical order: the splits of one position tile are consecutive (one XCD)
  const int L = wg_order(wg, wg.linear(), wg.count());
  const int nsplit = wg.nx;
  const long p0 = static_cast<long>(L / nsplit) * 64;
  const int split = L % nsplit;
  // Q tile (row r = p - p0, zero outside the grid and for k >= K3) into
  // registers; the loads are in flight while the grid scalars are reduced
  constexpr int c4n = K3P / 4, QIT = 64 * c4n / 256;
  float x[QIT][4];
#pragma unroll
  for (int it = 0; it < QIT; ++it) {
    const int e = tid + 256 * it;
    const int r = e / c4n, k = 4 * (e % c4n);
    const long p = p0 + r;
    const int g1 = static_cast<int>(p / K2P), g2 = static_cast<int>(p % K2P);
    const bool valid = g1 < K1 && g2 < K2;
    const float* row = Q + (static_cast<long>(valid ? g1 : 0) * K2 + (valid ? g2 : 0)) * K3;
#pragma unroll
    for (int h = 0; h < 4; ++h) x[it][h] = 0.f;
    if ((K3 & 3) == 0) {
      if (valid && k < K3) {
        const float4 v = *reinterpret_cast<const float4*>(&row[k]);
        x[it][0] = v.x; x[it][1] = v.y; x[it][2] = v.z; x[it][3] = v.w;
      }
    } else {
#pragma unroll
      for (int h = 0; h < 4; ++h) x[it][h] = (valid && k + h < K3) ? row[k + h] : 0.f;
    }
  }
  const float sq = grid_scalars(part, np, sums, scale_q != 0, wg.linear() == 0);
  // scaled and split into LDS hi/lo
#pragma unroll
  for (int it = 0; it < QIT; ++it) {
    const int e = tid + 256 * it;
    const int r = e / c4n, k = 4 * (e % c4n);
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      H hi, lo;
      split_h<H>(sq * x[it][h], hi, lo);
      Qh[r * QSTR + k + h] = hi;
      Ql[r * QSTR + k + h] = lo;
    }
  }
  __syncthreads();
  // A fragments of the whole K range: tile u, lane (q, m) holds position
  // row 8 (m / 4) + 4 u + m % 4 (u < 2), 32 + 8 (m / 4) + 4 (u - 2) + m % 4
  // (u >= 2), columns 32 kc + 8 q .. + 7, so that output lane (q, m) holds
  // positions 8 q .. 8 q + 7 and 32 + 8 q .. + 7 of column m: each Y store
  // instruction then writes 64 contiguous bytes per column
  v8 ah[NK][4], al[NK][4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = u < 2 ? 8 * (m >> 2) + 4 * u + (m & 3) : 32 + 8 * (m >> 2) + 4 * (u - 2) + (m & 3);
#pragma unroll
    for (int kc = 0; kc < NK; ++kc) {
      ah[kc][u] = *reinterpret_cast<const v8*>(&Qh[r * QSTR + 32 * kc + 8 * q]);
      al[kc][u] = *reinterpret_cast<const v8*>(&Ql[r * QSTR + 32 * kc + 8 * q]);
    }
  }
  const int ntiles = (nrows + 15) / 16;
  const int per = (ntiles + nsplit - 1) / nsplit;
  const int t0 = split * per, t1 = min(ntiles, t0 + per);
  auto loadc = [&](int t, v8 (&bh)[NK], v8 (&bl)[NK]) {
    const int n = 16 * t + m;
#pragma unroll
    for (int kc = 0; kc < NK; ++kc) {
      bh[kc] = v8{};
      bl[kc] = v8{};
      if (t < t1 && n < nrows) {
        bh[kc] = *reinterpret_cast<const v8*>(&Chi[static_cast<long>(n) * K3P + 32 * kc + 8 * q]);
        bl[kc] = *reinterpret_cast<const v8*>(&Clo[static_cast<long>(n) * K3P + 32 * kc + 8 * q]);
      }
    }
  };
  v8 bh[NK], bl[NK];
  loadc(t0 + wave, bh, bl);
  for (int t = t0 + wave; t < t1; t += 4) {
    v8 ch[NK], cl[NK];
#pragma unroll
    for (int kc = 0; kc < NK; ++kc) {
      ch[kc] = bh[kc];
      cl[kc] = bl[kc];
    }
    loadc(t + 4, bh, bl);  // the wave's next tile
    floatx4 acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < NK; ++kc) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = mfma_h(ah[kc][u], ch[kc], acc[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = mfma_h(ah[kc][u], cl[kc], acc[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = mfma_h(al[kc][u], ch[kc], acc[u]);
    }
    const int n = 16 * t + m;
    if (n < nrows) {
      v8 yh[2], yl[2];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          H h, l;
          split_h<H>(sy * acc[u][r], h, l);
          yh[u >> 1][4 * (u & 1) + r] = h;
          yl[u >> 1][4 * (u & 1) + r] = l;
        }
      const long o = static_cast<long>(n) * slab + p0 + 8 * q;
      *reinterpret_cast<v8*>(&Yhi[o]) = yh[0];
      *reinterpret_cast<v8*>(&Yhi[o + 32]) = yh[1];
      *reinterpret_cast<v8*>(&Ylo[o]) = yl[0];
      *reinterpret_cast<v8*>(&Ylo[o + 32]) = yl[1];
    }
  }
}

template <typename H, int NK>
__global__ __launch_bounds__(256) void stage1_x3_lds(
    const float* __restrict__ Q, const H* __restrict__ Chi, const H* __restrict__ Clo,
    H* __restrict__ Yhi, H* __restrict__ Ylo, int K1, int K2, int K3, int K2P, long slab,
    int nrows, const double* __restrict__ part, int np, double* __restrict__ sums, int scale_q,
    float sy) {
  stage1_x3_lds_body<H, NK>(Q, Chi, Clo, Yhi, Ylo, K1, K2, K3, K2P, slab, nrows, part, np, sums, scale_q, sy, Wg::plain());
}

// Stage 1, FP32 / FP64 (16x16x4 MFMA).  C: [nrows][K3P]; Y: [nrows][slab].
template <typename T>
__global__ __launch_bounds__(256) void stage1_k4(const T* __restrict__ Q,
                                                 const T* __restrict__ C,
                                                 T* __restrict__ Y, int K1, int K2,
                                                 int K3, int K3P, int K2P, long slab,
                                                 int nrows) {
  typedef typename Vec4<T>::type acc_t;
  constexpr int KC = 16, STR = KC + 1;
  __shared__ T As[S1 * STR], Bs[S1 * STR];
  const long m0 = static_cast<long>(blockIdx.x) * S1;
  const int n0 = blockIdx.y * S1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1, q = lane >> 4, m = lane & 15;
  acc_t acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  for (int k0 = 0; k0 < K3P; k0 += KC) {
    __syncthreads();
    for (int e = tid; e < S1 * KC; e += 256) {
      const int r = e / KC, c = e % KC;
      const int n = n0 + r;
      As[r * STR + c] = (n < nrows) ? C[static_cast<long>(n) * K3P + k0 + c] : T(0);
      const long mp = m0 + r;
      const int g1 = static_cast<int>(mp / K2P), g2 = static_cast<int>(mp % K2P);
      const int k = k0 + c;
      Bs[r * STR + c] = (g1 < K1 && g2 < K2 && k < K3)
                            ? Q[(static_cast<long>(g1) * K2 + g2) * K3 + k] : T(0);
    }
    __syncthreads();
    for (int kk = 0; kk < KC / 4; ++kk)
      for (int i = 0; i < 2; ++i) {
        const T a = As[(wr * 32 + 16 * i + m) * STR + 4 * kk + q];
        for (int j = 0; j < 2; ++j) {
          const T b = Bs[(wc * 32 + 16 * j + m) * STR + 4 * kk + q];
          acc[i][j] = mfma_k4(a, b, acc[i][j]);
        }
      }
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int row = n0 + wr * 32 + 16 * i + acc_row<T>(q, r);
        const long col = m0 + wc * 32 + 16 * j + m;
        if (row < nrows && col < slab) Y[row * slab + col] = acc[i][j][r];
      }
}

// ----------------------------------------------------------------------------
// Stage 2, split precision.  One workgroup = (slab s, range of steps); it has
// NS streams of WPS = K2P / (16 CT) waves, and wave w of a stream owns output
// columns [16 CT w, 16 CT (w + 1)).
//
// A_t and B_t are circulant: A_t[k1][g1] = a_t((k1 - g1) mod K1).  Each term
// is stored as shifted copies of its reversed generating vectors,
//   Bv[s][x] = b((-(x + s)) mod K2), s < 8,  Av[s][x] = a((-(x + s)) mod K1), s < 4,
// so that the 8 (resp. 4) consecutive factor entries an MFMA fragment needs
// start at an aligned position of one copy: a term costs a few KB of LDS
// instead of two K x K tiles.  The next term's vectors are fetched into
// registers while the current term computes (double-buffered LDS).  The Y
// slab of the current outer-SVD group stays in LDS.  T is multiplied by st
// (a power of two, FP16X3) before its split.
//
// A step holds NS terms of one outer-SVD group (-1: the stream idles for that
// step); stream k computes the k-th term of every step on the shared Y slab
// with its own vector buffers, and the streams' sums are added through LDS
// at the end, in stream order.  Every wave reads the whole Y slab and its
// columns' B fragments, and the A fragments of all rows, per term: wider
// column tiles (CT) cut that LDS traffic per term, at the cost of
// accumulator registers.  K1P = 128 runs with one wave per SIMD, which may
// then use the full register file.
template <typename H, int RT, int NKC, int CT, int NS>
__device__ __forceinline__ void stage2_x3_body(
    const H* __restrict__ Yhi, const H* __restrict__ Ylo, const H* __restrict__ vec,
    const int* __restrict__ step_term, const int* __restrict__ step_group,
    const int* __restrict__ step_begin, float* __restrict__ Phi_part, int K1, int K2, int K3,
    float st,
    const Wg wg) {
  typedef typename HVec<H>::v8 v8;
  typedef typename HVec<H>::v4 v4;
  static_assert((2 * NKC) % CT == 0, "column tiles must divide K2P / 16");
  constexpr int K1P = RT * 16, K2P = NKC * 32;
  constexpr int WPS = 2 * NKC / CT;             // waves per stream
  constexpr int blen = 2 * K2P + 8 + (K2P % 64 == 0 ? 64 : 0), alen = 2 * K1P + 16;  // x3_blen, x3_alen
  constexpr int plane = 8 * blen + 8 + 4 * alen + 8;  // x3_plane: halves per plane
  constexpr int tsz = 2 * plane;                // halves per term (hi plane, lo plane)
  constexpr int STHR = 64 * WPS;                // threads per stream
  constexpr int PF = (tsz / 8 + STHR - 1) / STHR;  // 16-byte chunks per stream thread
  constexpr int YSTR = K2P;                     // rows swizzled by x3_yswz
  extern __shared__ __attribute__((aligned(16))) char smem[];
  H* Ysh = reinterpret_cast<H*>(smem);
  H* Ysl = Ysh + K1P * YSTR;
  H* vbase = Ysl + K1P * YSTR;                  // [NS][2][tsz]
  // logical order: the term ranges of one slab are consecutive (one XCD and
  // L2 for the slab's Y planes)
  const int L = wg_order(wg, wg.linear(), wg.count());
  const int s = L / wg.ny, part = L % wg.ny;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, q = lane >> 4, m = lane & 15;
  const int strm = wave / WPS, cw = wave - strm * WPS, stid = tid - strm * STHR;
  const int col0 = cw * 16 * CT;
  H* vbuf = vbase + strm * 2 * tsz;
  constexpr long slab = static_cast<long>(K1P) * K2P;
  constexpr int nchunk = tsz / 8;
  floatx4 acc2[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc2[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int s0 = step_begin[part], s1 = step_begin[part + 1];
  // Fragment bases (halves) into one plane of a term's vectors.  Copy s of
  // the B vector holds at x the entry for (k2 - g2) = x + s - K2P, so the B
  // fragment (kc, j) -- g2 = 32 kc + 8 q + e, k2 = col0 + 16 j + m -- starts
  // at u = uB + 32 kc - 16 j in copy (u & 7) at (u & ~7) with
  // uB = 8 q - col0 - m + K2P; the kc, j part is a multiple of 8, hence a
  // constant offset from offB.  Likewise the A half-fragment at K offset 16 d
  // (d = 2 c - i, then 2 c - i + 1) starts at uA + 16 d, uA = 4 q - m + K1P,
  // in copy (uA & 3).  Copy s starts x3_shift_b(s) (B) or kX3ShiftA (A, s >= 1)
  // halves late.  The Y fragment of row m + 16 i and K chunk (kc, q) is chunk
  // (4 kc + q) ^ x3_yswz(NKC, m) of its row (the swizzle of rows m + 16 i is
  // that of row m).
  const int uB = 8 * q - col0 - m + K2P, uA = 4 * q - m + K1P;
  const int sB = uB & 7, sA = uA & 3;
  const int offB = sB * blen + x3_shift_b(sB) + (uB & ~7) - 16;
  const int ysw = x3_yswz(NKC, m);
  auto ycol = [&](int kc) { return 8 * ((4 * kc + q) ^ ysw); };
  const int offA = 8 * blen + 8 + sA * alen + (sA ? kX3ShiftA : 0) + (uA & ~3) - 16 * (RT - 1);
  // prologue: this stream's first term's vectors into its buffer 0
  if (s0 < s1) {
    const int tf = step_term[s0 * NS + strm];
    if (tf >= 0)
      for (int c = stid; c < nchunk; c += STHR)
        *reinterpret_cast<v8*>(&vbuf[8 * c]) =
            *reinterpret_cast<const v8*>(&vec[static_cast<long>(tf) * tsz + 8 * c]);
  }
  int cur = -1;
  for (int sp = s0; sp < s1; ++sp) {
    const int g = step_group[sp];
    const int t = step_term[sp * NS + strm];
    const int tn = (sp + 1 < s1) ? step_term[(sp + 1) * NS + strm] : -1;
    const int buf = (sp - s0) & 1;
    __syncthreads();
    if (g != cur) {
      const H* yh = Yhi + (static_cast<long>(g) * K3 + s) * slab;
      const H* yl = Ylo + (static_cast<long>(g) * K3 + s) * slab;
      constexpr int cpr = K2P / 8;
      for (int e = tid; e < K1P * cpr; e += nthr) {
        const int r = e / cpr, c8 = e % cpr;
        *reinterpret_cast<v8*>(&Ysh[r * YSTR + 8 * (c8 ^ x3_yswz(NKC, r))]) =
            *reinterpret_cast<const v8*>(&yh[static_cast<long>(r) * K2P + 8 * c8]);
        *reinterpret_cast<v8*>(&Ysl[r * YSTR + 8 * (c8 ^ x3_yswz(NKC, r))]) =
            *reinterpret_cast<const v8*>(&yl[static_cast<long>(r) * K2P + 8 * c8]);
      }
      cur = g;
      __syncthreads();
    }
    // prefetch this stream's next term's vectors into registers
    v8 pre[PF];
    if (tn >= 0) {
      const H* src = vec + static_cast<long>(tn) * tsz;
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const int c = stid + k * STHR;
        if (c < nchunk) pre[k] = *reinterpret_cast<const v8*>(&src[8 * c]);
      }
    }
    if (t >= 0) {
    const H* Bvh = vbuf + buf * tsz + offB;
    const H* Bvl = Bvh + plane;
    const H* Avh = vbuf + buf * tsz + offA;
    const H* Avl = Avh + plane;
    // GEMM1: T[g1][k2] = sum_g2 Y[g1][g2] B_t[k2][g2]
    floatx4 acc1[RT][CT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < CT; ++j) acc1[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // (kc, i) steps s = RT kc + i; each loads the Y fragment of step s + 2,
    // and the next-to-last i of a kc also the next kc's B fragments
    constexpr int NSTEP = NKC * RT;
    auto yfrag = [&](int st1, v8& h, v8& l) {
      const int yo = (m + 16 * (st1 % RT)) * YSTR + ycol(st1 / RT);
      h = *reinterpret_cast<const v8*>(&Ysh[yo]);
      l = *reinterpret_cast<const v8*>(&Ysl[yo]);
    };
    v8 bh[CT], bl[CT], nbh[CT], nbl[CT];
#pragma unroll
    for (int j = 0; j < CT; ++j) {
      bh[j] = *reinterpret_cast<const v8*>(&Bvh[16 * (1 - j)]);
      bl[j] = *reinterpret_cast<const v8*>(&Bvl[16 * (1 - j)]);
    }
    // T rows 2c, 2c + 1 of column tile j, multiplied by st and split into
    // 16-bit hi/lo: the B operand of GEMM2's K chunk c (see below).  With
    // 128 rows (kEarlySplit) chunk c is split once its rows are final, one
    // column tile per step, while the remaining MFMAs run: in the last K step
    // of GEMM1 for all but the last chunk, in the first two d steps of GEMM2
    // for the last.  Other tile counts split every chunk before GEMM2 (the
    // early form measured slower there: it spills at 96 x 96).
    constexpr bool kEarlySplit = RT == 8;
    v8 tbh[RT / 2][CT], tbl[RT / 2][CT];
    auto split_tile = [&](int c, int j) {
      v4 h0, l0, h1, l1;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        H h, l;
        split_h<H>(st * acc1[2 * c][j][r], h, l);
        h0[r] = h;
        l0[r] = l;
        split_h<H>(st * acc1[2 * c + 1][j][r], h, l);
        h1[r] = h;
        l1[r] = l;
      }
      tbh[c][j] = cat44<v4, v8>(h0, h1);
      tbl[c][j] = cat44<v4, v8>(l0, l1);
    };
    // the split of chunk c, tile j, happens at GEMM1 step i = 2c + 2 + (j * 2 / CT)
    // of the last kc (rows 2c, 2c + 1 were final at step 2c + 1), or for the
    // last chunk at GEMM2 step dd = j * 2 / CT
    auto split_at = [&](int i) {
      if (!kEarlySplit) return;
#pragma unroll
      for (int c = 0; c < RT / 2 - 1; ++c)
#pragma unroll
        for (int j = 0; j < CT; ++j)
          if (2 * c + 2 + (j * 2) / CT == i) split_tile(c, j);
    };
    v8 ah, al, a1h, a1l;
    yfrag(0, ah, al);
    a1h = ah;
    a1l = al;
    if (NSTEP > 1) yfrag(1, a1h, a1l);
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        const int st1 = kc * RT + i;
        v8 a2h = a1h, a2l = a1l;
        if (st1 + 2 < NSTEP) yfrag(st1 + 2, a2h, a2l);
        if (i + 2 == RT && kc + 1 < NKC) {
#pragma unroll
          for (int j = 0; j < CT; ++j) {
            nbh[j] = *reinterpret_cast<const v8*>(&Bvh[32 * (kc + 1) + 16 * (1 - j)]);
            nbl[j] = *reinterpret_cast<const v8*>(&Bvl[32 * (kc + 1) + 16 * (1 - j)]);
          }
        }
#pragma unroll
        for (int j = 0; j < CT; ++j) acc1[i][j] = mfma_h(ah, bh[j], acc1[i][j]);
#pragma unroll
        for (int j = 0; j < CT; ++j) acc1[i][j] = mfma_h(ah, bl[j], acc1[i][j]);
#pragma unroll
        for (int j = 0; j < CT; ++j) acc1[i][j] = mfma_h(al, bh[j], acc1[i][j]);
        if (kc + 1 == NKC) split_at(i);
        ah = a1h;
        al = a1l;
        a1h = a2h;
        a1l = a2l;
        if (i + 1 == RT && kc + 1 < NKC) {
#pragma unroll
          for (int j = 0; j < CT; ++j) {
            bh[j] = nbh[j];
            bl[j] = nbl[j];
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // GEMM2: Phi[k1][k2] += sum_g1 A_t[k1][g1] T[g1][k2], K chunks of 32 rows
    // of T taken as {32c + 4q + r} u {32c + 16 + 4q + r}, so that the chunk's
    // two accumulator tiles are the B operand; T is multiplied by st and split
    // into 16-bit hi/lo in place.  Because A_t is circulant, the A fragment of
    // output row tile i and chunk c depends on d = 2c - i only: the d loop
    // reads each distinct fragment once and applies it to every (c, i) pair.
    if (!kEarlySplit) {
#pragma unroll
      for (int c = 0; c < RT / 2; ++c)
#pragma unroll
        for (int j = 0; j < CT; ++j) split_tile(c, j);
    }
    auto afrag = [&](const H* base, int dd) {  // dd = d + RT - 1
      return cat44<v4, v8>(*reinterpret_cast<const v4*>(&base[16 * dd]),
                           *reinterpret_cast<const v4*>(&base[16 * dd + 16]));
    };
    ah = afrag(Avh, 0);
    al = afrag(Avl, 0);
#pragma unroll
    for (int dd = 0; dd < 2 * RT - 2; ++dd) {
      v8 nh = ah, nl = al;
      if (dd + 1 < 2 * RT - 2) {
        nh = afrag(Avh, dd + 1);
        nl = afrag(Avl, dd + 1);
      }
      const int d = dd - (RT - 1);
      // the last chunk (first used at dd = RT - 2 = 6)
      if (kEarlySplit) {
#pragma unroll
        for (int j = 0; j < CT; ++j)
          if ((j * 2) / CT == dd) split_tile(RT / 2 - 1, j);
      }
#pragma unroll
      for (int pass = 0; pass < 3; ++pass)
#pragma unroll
        for (int c = 0; c < RT / 2; ++c) {
          const int i = 2 * c - d;
          if (i < 0 || i >= RT) continue;
#pragma unroll
          for (int j = 0; j < CT; ++j) {
            if (pass == 0) acc2[i][j] = mfma_h(ah, tbh[c][j], acc2[i][j]);
            if (pass == 1) acc2[i][j] = mfma_h(ah, tbl[c][j], acc2[i][j]);
            if (pass == 2) acc2[i][j] = mfma_h(al, tbh[c][j], acc2[i][j]);
          }
        }
      ah = nh;
      al = nl;
      __builtin_amdgcn_sched_barrier(0);
    }
    }  // t >= 0
    // publish the prefetched vectors into the other buffer (read after the
    // barrier at the top of the next step)
    if (tn >= 0) {
      H* dst = vbuf + (buf ^ 1) * tsz;
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const int c = stid + k * STHR;
        if (c < nchunk) *reinterpret_cast<v8*>(&dst[8 * c]) = pre[k];
      }
    }
  }
  if (NS > 1) {
    // streams 1.. hand their sums to stream 0 through the (now free) Y area in
    // a lane-private layout; stream 0 adds them in stream order
    float* red = reinterpret_cast<float*>(smem);
    for (int k = 1; k < NS; ++k) {
      __syncthreads();
      if (strm == k) {
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
          for (int j = 0; j < CT; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              red[(((cw * RT + i) * CT + j) * 4 + r) * 64 + lane] = acc2[i][j][r];
      }
      __syncthreads();
      if (strm == 0) {
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
          for (int j = 0; j < CT; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              acc2[i][j][r] += red[(((cw * RT + i) * CT + j) * 4 + r) * 64 + lane];
      }
    }
    if (strm != 0) return;
  }
  float* out = Phi_part + (static_cast<long>(part) * K3 + s) * K1 * K2;
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) {
      const int k2 = col0 + 16 * j + m;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k1 = 16 * i + 4 * q + r;
        if (k1 < K1 && k2 < K2) out[static_cast<long>(k1) * K2 + k2] = acc2[i][j][r];
      }
    }
}

template <typename H, int RT, int NKC, int CT, int NS>
__global__ __launch_bounds__(64 * (2 * NKC / CT) * NS)
__attribute__((amdgpu_waves_per_eu(RT >= 8 ? 1 : 2))) void stage2_x3(
    const H* __restrict__ Yhi, const H* __restrict__ Ylo, const H* __restrict__ vec,
    const int* __restrict__ step_term, const int* __restrict__ step_group,
    const int* __restrict__ step_begin, float* __restrict__ Phi_part, int K1, int K2, int K3,
    float st) {
  stage2_x3_body<H, RT, NKC, CT, NS>(Yhi, Ylo, vec, step_term, step_group, step_begin, Phi_part, K1, K2, K3, st, Wg::plain());
}

// Stage 2, FP32 / FP64 with the 16x16x4 MFMAs.  The factors are symmetric,

// Stage 2, FP32 / FP64 with the 16x16x4 MFMAs.  The factors are symmetric,
// which lets the global-memory operand reads run along rows (coalesced).
template <typename T, int RT, int CT, bool A_LDS>
__global__ __launch_bounds__(512) void stage2_k4(
    const T* __restrict__ Y, const T* __restrict__ A, const T* __restrict__ B,
    const int* __restrict__ term_group, const int* __restrict__ part_begin,
    T* __restrict__ Phi_part, int K1, int K2, int K3, int K2P) {
  typedef typename Vec4<T>::type acc_t;
  constexpr int K1P = RT * 16, ASTR = K1P + 1;
  const int YSTR = K2P + 1;
  extern __shared__ __attribute__((aligned(16))) char smem[];
  T* Ys = reinterpret_cast<T*>(smem);
  T* As = Ys + K1P * YSTR;
  const int s = blockIdx.x, part = blockIdx.y;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, q = lane >> 4, m = lane & 15;
  const int col0 = wave * 16 * CT;
  const long slab = static_cast<long>(K1P) * K2P;
  acc_t acc2[RT][CT];
  for (int i = 0; i < RT; ++i)
    for (int j = 0; j < CT; ++j) acc2[i][j] = acc_t{0, 0, 0, 0};
  const int t0 = part_begin[part], t1 = part_begin[part + 1];
  int cur = -1;
  for (int t = t0; t < t1; ++t) {
    const int g = term_group[t];
    __syncthreads();
    if (g != cur) {
      const T* y = Y + (static_cast<long>(g) * K3 + s) * slab;
      for (int e = tid; e < K1P * K2P; e += nthr) {
        const int r = e / K2P, c = e % K2P;
        Ys[r * YSTR + c] = y[e];
      }
      cur = g;
    }
    const T* a_g = A + static_cast<long>(t) * K1P * K1P;
    if (A_LDS) {
      for (int e = tid; e < K1P * K1P; e += nthr) {
        const int r = e / K1P, c = e % K1P;
        As[r * ASTR + c] = a_g[e];
      }
    }
    __syncthreads();
    if (col0 >= K2P) continue;
    acc_t acc1[RT][CT];
    for (int i = 0; i < RT; ++i)
      for (int j = 0; j < CT; ++j) acc1[i][j] = acc_t{0, 0, 0, 0};
    const T* b_g = B + static_cast<long>(t) * K2P * K2P;
    for (int kc = 0; kc < K2P / 4; ++kc) {
      T b[CT];
      for (int j = 0; j < CT; ++j)  // B_t[k2][g2] = B_t[g2][k2]
        b[j] = b_g[static_cast<long>(4 * kc + q) * K2P + col0 + 16 * j + m];
      for (int i = 0; i < RT; ++i) {
        const T a = Ys[(16 * i + m) * YSTR + 4 * kc + q];
        for (int j = 0; j < CT; ++j) acc1[i][j] = mfma_k4(a, b[j], acc1[i][j]);
      }
    }
    for (int ik = 0; ik < RT; ++ik)
      for (int r = 0; r < 4; ++r) {
        T bb[CT];
        for (int j = 0; j < CT; ++j) bb[j] = acc1[ik][j][r];
        const int g1 = 16 * ik + acc_row<T>(q, r);  // row of T held in register r
        for (int i = 0; i < RT; ++i) {
          // A_t[k1][g1] with k1 = 16 i + m
          const T a = A_LDS ? As[(16 * i + m) * ASTR + g1] : a_g[g1 * K1P + 16 * i + m];
          for (int j = 0; j < CT; ++j) acc2[i][j] = mfma_k4(a, bb[j], acc2[i][j]);
        }
      }
  }
  if (col0 >= K2P) return;
  T* out = Phi_part + (static_cast<long>(part) * K3 + s) * K1 * K2;
  for (int i = 0; i < RT; ++i)
    for (int j = 0; j < CT; ++j) {
      const int k2 = col0 + 16 * j + m;
      for (int r = 0; r < 4; ++r) {
        const int k1 = 16 * i + acc_row<T>(q, r);
        if (k1 < K1 && k2 < K2) out[static_cast<long>(k1) * K2 + k2] = acc2[i][j][r];
      }
    }
}

// Sum the partial slabs [part][k3][k1][k2] in order, transpose to
// [k1][k2][k3] and subtract c * sum(Q).  One workgroup per (k1, 32 x 32 tile
// of k2 x k3); interior tiles of 4-aligned extents move float4 vectors.
// With epart, the workgroup also writes the FP64 sum of Q * Phi over the
// values it stores (the reciprocal energy is half the total).
template <typename A, typename O>
__device__ __forceinline__ void finalize_body(const A* __restrict__ part, int nparts,
                                                O* __restrict__ Phi, int K1, int K2,
                                                int K3, const double* __restrict__ sumQ,
                                                double c0, const double* __restrict__ qscale,
                                                double const_scale, const O* __restrict__ Q,
                                                double* __restrict__ epart,
    const Wg wg) {
  __shared__ A tile[32][33];
  __shared__ double red[16];
  double e = 0.0;
  const int k1 = wg.z, k2b = wg.x * 32, k3b = wg.y * 32;
  const int t = threadIdx.x;
  const long pstride = static_cast<long>(K3) * K1 * K2;
  const bool vec = sizeof(A) == 4 && (K2 & 3) == 0 && (K3 & 3) == 0 && k2b + 32 <= K2 &&
                   k3b + 32 <= K3;
  if (vec) {
    const int r = t >> 3, c4 = (t & 7) * 4;  // k3 row, k2 column group
    const long base = (static_cast<long>(k3b + r) * K1 + k1) * K2 + k2b + c4;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int p = 0; p < nparts; ++p) {
      const float4 w = *reinterpret_cast<const float4*>(&part[p * pstride + base]);
      v.x += w.x; v.y += w.y; v.z += w.z; v.w += w.w;
    }
    tile[r][c4] = v.x;
    tile[r][c4 + 1] = v.y;
    tile[r][c4 + 2] = v.z;
    tile[r][c4 + 3] = v.w;
  } else {
    for (int j = t >> 5; j < 32; j += 8) {
      const int k3 = k3b + j, k2 = k2b + (t & 31);
      A v = 0;
      if (k3 < K3 && k2 < K2) {
        const long base = (static_cast<long>(k3) * K1 + k1) * K2 + k2;
        for (int p = 0; p < nparts; ++p) v += part[p * pstride + base];
      }
      tile[j][t & 31] = v;
    }
  }
  const A corr = static_cast<A>(c0 * sumQ[0]);
  // the partial slabs carry the product of the split-precision scales
  const A unscale = qscale ? static_cast<A>(1.0 / (qscale[0] * const_scale)) : A(1);
  __syncthreads();
  if (vec) {
    const int r = t >> 3, c4 = (t & 7) * 4;  // k2 row, k3 column group
    float4 o;
    o.x = unscale * tile[c4][r] - corr;
    o.y = unscale * tile[c4 + 1][r] - corr;
    o.z = unscale * tile[c4 + 2][r] - corr;
    o.w = unscale * tile[c4 + 3][r] - corr;
    const long at = (static_cast<long>(k1) * K2 + k2b + r) * K3 + k3b + c4;
    *reinterpret_cast<float4*>(&Phi[at]) = o;
    if (epart) {
      const float4 qv = *reinterpret_cast<const float4*>(&Q[at]);
      e = static_cast<double>(qv.x) * o.x + static_cast<double>(qv.y) * o.y +
          static_cast<double>(qv.z) * o.z + static_cast<double>(qv.w) * o.w;
    }
  } else {
    for (int j = t >> 5; j < 32; j += 8) {
      const int k2 = k2b + j, k3 = k3b + (t & 31);
      if (k2 < K2 && k3 < K3) {
        const long at = (static_cast<long>(k1) * K2 + k2) * K3 + k3;
        const O v = static_cast<O>(unscale * tile[t & 31][j] - corr);
        Phi[at] = v;
        if (epart) e += static_cast<double>(Q[at]) * static_cast<double>(v);
      }
    }
  }
  if (epart) {
    double v[1] = {e};
    block_reduce<1, 1>(v, red);
    if (t == 0) epart[(static_cast<long>(wg.z) * wg.ny + wg.y) * wg.nx + wg.x] = v[0];
  }
}

template <typename A, typename O>
__global__ __launch_bounds__(256) void finalize(const A* __restrict__ part, int nparts,
                                                O* __restrict__ Phi, int K1, int K2,
                                                int K3, const double* __restrict__ sumQ,
                                                double c0, const double* __restrict__ qscale,
                                                double const_scale, const O* __restrict__ Q,
                                                double* __restrict__ epart) {
  finalize_body<A, O>(part, nparts, Phi, K1, K2, K3, sumQ, c0, qscale, const_scale, Q, epart, Wg::plain());
}

}  // namespace

int finalize_blocks(int K1, int K2, int K3) { return ((K2 + 31) / 32) * ((K3 + 31) / 32) * K1; }

namespace {

// Fixed-order FP64 sum and max |x| of a grid: per-block partials, then one
// block combines them.
template <typename T>
__global__ __launch_bounds__(256) void sum_partial(const T* __restrict__ x, long n,
                                                   double* __restrict__ part) {
  __shared__ double red[32];
  const long per = (n + gridDim.x - 1) / gridDim.x;
  const long b = per * blockIdx.x, e = (b + per < n) ? b + per : n;
  double acc = 0.0, amax = 0.0;
  for (long i = b + threadIdx.x; i < e; i += blockDim.x) {
    const double v = static_cast<double>(x[i]);
    acc += v;
    amax = fmax(amax, fabs(v));
  }
  double v[2] = {acc, amax};
  block_reduce<1, 2>(v, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = v[0];
    part[2 * blockIdx.x + 1] = v[1];
  }
}

// out[0] = sum; out[1] = 2^(13 - floor(log2 max|x|)), the power of two that
// brings the largest grid value into [2^13, 2^14) for the FP16X3 split
// (1 for an all-zero or non-finite grid).
__device__ __forceinline__ void sum_final_body(const double* __restrict__ part, int np,
                                                 double* __restrict__ out,
    const Wg wg) {
  __shared__ double red[32];
  double v[2] = {0.0, 0.0};
  for (int i0 = threadIdx.x; i0 < np; i0 += 8 * 256) {  // eight pairs in flight
    double2 x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + 256 * u;
      x[u] = i < np ? *reinterpret_cast<const double2*>(&part[2 * i]) : double2{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      v[0] += x[u].x;
      v[1] = fmax(v[1], x[u].y);
    }
  }
  block_reduce<1, 2>(v, red);
  if (threadIdx.x == 0) {
    out[0] = v[0];
    const double m = v[1];
    out[1] = (m > 0.0 && m < 1e300) ? ldexp(1.0, 13 - ilogb(m)) : 1.0;
  }
}

__global__ __launch_bounds__(256) void sum_final(const double* __restrict__ part, int np,
                                                 double* __restrict__ out) {
  sum_final_body(part, np, out, Wg::plain());
}

template <typename K>
hipError_t set_lds(K kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(bytes));
}

// prep: only raise the kernel instance's dynamic-LDS limit (plan creation,
// outside any stream capture); otherwise launch.  NS term streams per
// workgroup (the plan's step schedule is built for that many).
template <typename H, int RT, int NKC, int NS>
hipError_t launch_s2_x3_ns(const SkpArgs& a, hipStream_t st, bool prep) {
  constexpr int K1P = RT * 16, K2P = NKC * 32;
  constexpr int CT = x3_ct(K1P, K2P);
  const size_t tsz = 2 * static_cast<size_t>(x3_plane(K1P, K2P));
  const size_t lds = sizeof(H) * (2 * static_cast<size_t>(K1P) * K2P + 2 * NS * tsz);
  constexpr int NT = 64 * (2 * NKC / CT) * NS, W = RT >= 8 ? 1 : 2;
  const H* yh = static_cast<const H*>(a.Y[0]);
  const H* yl = static_cast<const H*>(a.Y[1]);
  const H* vec = static_cast<const H*>(a.vec);
  const int* sterm = a.step_term;
  const int* sgroup = a.step_group;
  const int* sbegin = a.step_begin;
  float* ppart = static_cast<float*>(a.Phi_part);
  if (prep) {
    // the plain instance and the batched ones (grid and persistent forms)
    hipError_t e = set_lds(stage2_x3<H, RT, NKC, CT, NS>, lds);
    if (e != hipSuccess) return e;
    e = batched_set_lds(
        batched_kernel_w_of<NT, W, stage2_x3_body<H, RT, NKC, CT, NS>>(
            yh, yl, vec, sterm, sgroup, sbegin, ppart, a.K[0], a.K[1], a.K[2], a.st),
        lds);
    if (e != hipSuccess) return e;
    return batched_set_lds(
        batched_kernel_wq_of<NT, W, stage2_x3_body<H, RT, NKC, CT, NS>>(
            yh, yl, vec, sterm, sgroup, sbegin, ppart, a.K[0], a.K[1], a.K[2], a.st),
        lds);
  }
  if (a.K2P != K2P || a.x3_streams != NS || a.blen != x3_blen(K2P) || a.alen != x3_alen(K1P))
    return hipErrorInvalidValue;
  return launch_or_record_w<NT, W, stage2_x3_body<H, RT, NKC, CT, NS>>(
      LS_STAGE2, stage2_x3<H, RT, NKC, CT, NS>, dim3(a.K[2], a.nparts), lds, st, yh, yl, vec,
      sterm, sgroup, sbegin, ppart, a.K[0], a.K[1], a.K[2], a.st);
}

// One or two term streams; at plan creation (prep) both instances get their
// LDS limit, since the autotuner may switch the plan between them.
template <typename H, int RT, int NKC>
hipError_t launch_s2_x3(const SkpArgs& a, hipStream_t st, bool prep) {
  if (prep) {
    hipError_t e = launch_s2_x3_ns<H, RT, NKC, 1>(a, st, true);
    if (e == hipSuccess) e = launch_s2_x3_ns<H, RT, NKC, 2>(a, st, true);
    return e;
  }
  if (a.x3_streams == 2) return launch_s2_x3_ns<H, RT, NKC, 2>(a, st, false);
  return launch_s2_x3_ns<H, RT, NKC, 1>(a, st, false);
}

template <typename H, int RT>
hipError_t launch_s2_x3(const SkpArgs& a, hipStream_t st, bool prep) {
  switch (a.K2P) {
    case 32: return launch_s2_x3<H, RT, 1>(a, st, prep);
    case 64: return launch_s2_x3<H, RT, 2>(a, st, prep);
    case 96: return launch_s2_x3<H, RT, 3>(a, st, prep);
    case 128: return launch_s2_x3<H, RT, 4>(a, st, prep);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int RT, int CT, bool AL>
hipError_t launch_s2_k4(const SkpArgs& a, hipStream_t st, bool prep) {
  const int K1P = RT * 16;
  size_t lds = sizeof(T) * static_cast<size_t>(K1P) * (a.K2P + 1);
  if (AL) lds += sizeof(T) * static_cast<size_t>(K1P) * (K1P + 1);
  if (prep) return set_lds(stage2_k4<T, RT, CT, AL>, lds);
  if (record_unsupported()) return hipSuccess;
  const int threads = 64 * ((a.K2P + 16 * CT - 1) / (16 * CT));
  if (threads > 512) return hipErrorInvalidValue;  // the kernel's launch bound
  hipLaunchKernelGGL((stage2_k4<T, RT, CT, AL>), dim3(a.K[2], a.nparts), dim3(threads), lds, st,
                     static_cast<const T*>(a.Y[0]), static_cast<const T*>(a.A[0]),
                     static_cast<const T*>(a.B[0]), a.term_group, a.part_begin,
                     static_cast<T*>(a.Phi_part), a.K[0], a.K[1], a.K[2], a.K2P);
  return hipGetLastError();
}

template <int RT>
hipError_t dispatch_s2(const SkpArgs& a, hipStream_t st, bool prep) {
  const int K1P = RT * 16;
  if (a.prec == PREC_BF16X3) return launch_s2_x3<bf16, RT>(a, st, prep);
  if (a.prec == PREC_FP16X3) return launch_s2_x3<f16, RT>(a, st, prep);
  if (a.prec == PREC_FP32) {
    const size_t full = sizeof(float) * static_cast<size_t>(K1P) * (a.K2P + 1 + K1P + 1);
    return full <= kMaxLds ? launch_s2_k4<float, RT, 2, true>(a, st, prep)
                           : launch_s2_k4<float, RT, 2, false>(a, st, prep);
  }
  // FP64: one 16-column tile per wave up to K2P = 128 (eight waves), two
  // beyond (at most eight waves for K2P = 256)
  const size_t full = sizeof(double) * static_cast<size_t>(K1P) * (a.K2P + 1 + K1P + 1);
  if (a.K2P > 128)
    return full <= kMaxLds ? launch_s2_k4<double, RT, 2, true>(a, st, prep)
                           : launch_s2_k4<double, RT, 2, false>(a, st, prep);
  return full <= kMaxLds ? launch_s2_k4<double, RT, 1, true>(a, st, prep)
                         : launch_s2_k4<double, RT, 1, false>(a, st, prep);
}

hipError_t stage2_dispatch(const SkpArgs& a, hipStream_t st, bool prep) {
  switch (a.K1P) {
    case 32: return dispatch_s2<2>(a, st, prep);
    case 64: return dispatch_s2<4>(a, st, prep);
    case 96: return dispatch_s2<6>(a, st, prep);
    case 128: return dispatch_s2<8>(a, st, prep);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

size_t stage2_lds_bytes(int prec, int K1P, int K2P, int streams) {
  if (prec == PREC_BF16X3 || prec == PREC_FP16X3) {
    // Y slab (two planes) + two buffers of circulant vectors per stream
    const size_t tsz = 2 * static_cast<size_t>(x3_plane(K1P, K2P));
    return 2 * (2 * static_cast<size_t>(K1P) * K2P + 2 * static_cast<size_t>(streams) * tsz);
  }
  if (prec == PREC_FP32) return sizeof(float) * static_cast<size_t>(K1P) * (K2P + 1);
  return sizeof(double) * static_cast<size_t>(K1P) * (K2P + 1);
}

hipError_t launch_skp_sum(const SkpArgs& a, hipStream_t st) {
  if (record_unsupported()) return hipSuccess;
  const long G = static_cast<long>(a.K[0]) * a.K[1] * a.K[2];
  // sum(Q) in FP64, fixed reduction order
  if (a.prec == PREC_FP64)
    hipLaunchKernelGGL((sum_partial<double>), dim3(kSumBlocks), dim3(256), 0, st,
                       static_cast<const double*>(a.Q), G, a.scratch);
  else
    hipLaunchKernelGGL((sum_partial<float>), dim3(kSumBlocks), dim3(256), 0, st,
                       static_cast<const float*>(a.Q), G, a.scratch);
  hipLaunchKernelGGL(sum_final, dim3(1), dim3(256), 0, st, a.scratch, kSumBlocks, a.sumQ);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const SkpArgs& a, hipStream_t st) {
  if (record_unsupported()) return hipSuccess;
  const long G = static_cast<long>(a.K[0]) * a.K[1] * a.K[2];
  if (a.prec == PREC_FP64)
    hipLaunchKernelGGL((sum_partial<double>), dim3(kSumBlocks), dim3(256), 0, st,
                       static_cast<const double*>(a.Q), G, a.scratch);
  else
    hipLaunchKernelGGL((sum_partial<float>), dim3(kSumBlocks), dim3(256), 0, st,
                       static_cast<const float*>(a.Q), G, a.scratch);
  return hipGetLastError();
}

hipError_t launch_sum_final(const double* part2, int np, double* out, hipStream_t st) {
  return launch_or_record<256, sum_final_body>(LS_GRID_SUM, sum_final, dim3(1), 0, st, part2, np,
                                               out);
}

template <typename H>
hipError_t launch_s1_x3(const SkpArgs& a, int scale_q, float sy, hipStream_t st) {
  const long slab = static_cast<long>(a.K1P) * a.K2P;
  const int nrows = a.r0 * a.K[2];
  const int ntiles = (nrows + 15) / 16;
  const unsigned ptiles = static_cast<unsigned>(slab / 64);
  const unsigned s1split = static_cast<unsigned>(std::max(1, std::min(a.s1_split, ntiles)));
  const float* Q = static_cast<const float*>(a.Q);
  const H* ch = static_cast<const H*>(a.C[0]);
  const H* cl = static_cast<const H*>(a.C[1]);
  H* yh = static_cast<H*>(a.Y[0]);
  H* yl = static_cast<H*>(a.Y[1]);
  const double* spart = a.sum_part;
#define KPME_S1(NK)                                                                          \
  return launch_or_record<256, stage1_x3_lds_body<H, NK>>(                                   \
      LS_STAGE1, stage1_x3_lds<H, NK>, dim3(s1split, ptiles), 0, st, Q, ch, cl, yh, yl,       \
      a.K[0], a.K[1], a.K[2], a.K2P, slab, nrows, spart, a.sum_np, a.sumQ, scale_q, sy)
  switch (a.K3P) {
    case 32: KPME_S1(1);
    case 64: KPME_S1(2);
    case 96: KPME_S1(3);
    case 128: KPME_S1(4);
    case 160: KPME_S1(5);
    default: break;
  }
#undef KPME_S1
  dim3 grid((ntiles + kS1Tiles - 1) / kS1Tiles, ptiles);
  return launch_or_record<64, stage1_x3_body<H>>(LS_STAGE1, stage1_x3<H>, grid, 0, st, Q, ch, cl,
                                                 yh, yl, a.K[0], a.K[1], a.K[2], a.K3P, a.K2P,
                                                 slab, nrows, spart, a.sum_np, a.sumQ, scale_q,
                                                 sy);
}

hipError_t launch_skp_stage1(const SkpArgs& a, hipStream_t st) {
  const long slab = static_cast<long>(a.K1P) * a.K2P;
  const int nrows = a.r0 * a.K[2];
  dim3 g1(static_cast<unsigned>(slab / S1), (nrows + S1 - 1) / S1);
  if (a.prec == PREC_BF16X3) return launch_s1_x3<bf16>(a, 0, 1.0f, st);
  if (a.prec == PREC_FP16X3) return launch_s1_x3<f16>(a, 1, a.sy, st);
  if (record_unsupported()) return hipSuccess;
  if (a.prec == PREC_FP32)
    hipLaunchKernelGGL((stage1_k4<float>), g1, dim3(256), 0, st, static_cast<const float*>(a.Q),
                       static_cast<const float*>(a.C[0]), static_cast<float*>(a.Y[0]), a.K[0],
                       a.K[1], a.K[2], a.K3P, a.K2P, slab, nrows);
  else
    hipLaunchKernelGGL((stage1_k4<double>), g1, dim3(256), 0, st,
                       static_cast<const double*>(a.Q), static_cast<const double*>(a.C[0]),
                       static_cast<double*>(a.Y[0]), a.K[0], a.K[1], a.K[2], a.K3P, a.K2P,
                       slab, nrows);
  return hipGetLastError();
}

hipError_t launch_skp_stage2(const SkpArgs& a, hipStream_t st) {
  return stage2_dispatch(a, st, false);
}

hipError_t prepare_skp_stage2(const SkpArgs& a) { return stage2_dispatch(a, nullptr, true); }

hipError_t launch_skp_finalize(const SkpArgs& a, hipStream_t st) {
  dim3 gf((a.K[1] + 31) / 32, (a.K[2] + 31) / 32, a.K[0]);
  if (a.prec == PREC_FP64 && record_unsupported()) return hipSuccess;
  if (a.prec == PREC_FP64)
    hipLaunchKernelGGL((finalize<double, double>), gf, dim3(256), 0, st,
                       static_cast<const double*>(a.Phi_part), a.nparts,
                       static_cast<double*>(a.Phi), a.K[0], a.K[1], a.K[2], a.sumQ, a.c0,
                       nullptr, 1.0, static_cast<const double*>(a.eQ), a.epart);
  else
    return launch_or_record<256, finalize_body<float, float>>(
        LS_FINALIZE, finalize<float, float>, gf, 0, st, static_cast<const float*>(a.Phi_part),
        a.nparts, static_cast<float*>(a.Phi), a.K[0], a.K[1], a.K[2],
        static_cast<const double*>(a.sumQ), a.c0,
        static_cast<const double*>(a.prec == PREC_FP16X3 ? a.sumQ + 1 : nullptr),
        a.const_scale, static_cast<const float*>(a.eQ), a.epart);
  return hipGetLastError();
}

}  // namespace kpme
