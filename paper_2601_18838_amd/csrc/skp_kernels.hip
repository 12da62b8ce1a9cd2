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
#include "device_common.hpp"
#include "kernels.hpp"

namespace kpme {

namespace {

constexpr int S1 = 64;  // stage-1 output tile (rows and columns)

// ----------------------------------------------------------------------------
// Stage 1, split precision (BF16X3 / FP16X3).  C hi/lo: [nrows][K3P]
// (pre-scaled); Q: fp32 [K1][K2][K3], multiplied by *qscale (a power of two,
// FP16X3 only) before the split; the FP32 accumulator is multiplied by sy
// (a power of two) before Y is split and stored.  Y hi/lo: [nrows][K1P*K2P].
template <typename H>
__global__ __launch_bounds__(256) void stage1_x3(
    const float* __restrict__ Q, const H* __restrict__ Chi, const H* __restrict__ Clo,
    H* __restrict__ Yhi, H* __restrict__ Ylo, int K1, int K2, int K3, int K3P, int K2P,
    long slab, int nrows, const double* __restrict__ qscale, float sy) {
  typedef typename HVec<H>::v8 v8;
  constexpr int KC = 32, STR = KC + 8;
  __shared__ __attribute__((aligned(16))) H Ah[S1 * STR], Al[S1 * STR], Bh[S1 * STR], Bl[S1 * STR];
  const long m0 = static_cast<long>(blockIdx.x) * S1;
  const int n0 = blockIdx.y * S1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1, q = lane >> 4, m = lane & 15;
  const float sq = qscale ? static_cast<float>(*qscale) : 1.0f;
  floatx4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K3P; k0 += KC) {
    __syncthreads();
    for (int e = tid; e < S1 * (KC / 8); e += 256) {
      const int r = e / (KC / 8), c8 = e % (KC / 8);
      const int n = n0 + r;
      v8 vh = {}, vl = {};
      if (n < nrows) {
        vh = *reinterpret_cast<const v8*>(&Chi[static_cast<long>(n) * K3P + k0 + 8 * c8]);
        vl = *reinterpret_cast<const v8*>(&Clo[static_cast<long>(n) * K3P + k0 + 8 * c8]);
      }
      *reinterpret_cast<v8*>(&Ah[r * STR + 8 * c8]) = vh;
      *reinterpret_cast<v8*>(&Al[r * STR + 8 * c8]) = vl;
    }
    for (int e = tid; e < S1 * KC; e += 256) {
      const int r = e / KC, c = e % KC;
      const long mp = m0 + r;
      const int g1 = static_cast<int>(mp / K2P), g2 = static_cast<int>(mp % K2P);
      const int k = k0 + c;
      float x = 0.f;
      if (g1 < K1 && g2 < K2 && k < K3) x = sq * Q[(static_cast<long>(g1) * K2 + g2) * K3 + k];
      H h, l;
      split_h<H>(x, h, l);
      Bh[r * STR + c] = h;
      Bl[r * STR + c] = l;
    }
    __syncthreads();
    v8 ah[2], al[2], bh[2], bl[2];
    for (int i = 0; i < 2; ++i) {
      ah[i] = *reinterpret_cast<const v8*>(&Ah[(wr * 32 + 16 * i + m) * STR + 8 * q]);
      al[i] = *reinterpret_cast<const v8*>(&Al[(wr * 32 + 16 * i + m) * STR + 8 * q]);
      bh[i] = *reinterpret_cast<const v8*>(&Bh[(wc * 32 + 16 * i + m) * STR + 8 * q]);
      bl[i] = *reinterpret_cast<const v8*>(&Bl[(wc * 32 + 16 * i + m) * STR + 8 * q]);
    }
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = mfma_h(ah[i], bh[j], acc[i][j]);
        acc[i][j] = mfma_h(ah[i], bl[j], acc[i][j]);
        acc[i][j] = mfma_h(al[i], bh[j], acc[i][j]);
      }
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int row = n0 + wr * 32 + 16 * i + 4 * q + r;
        const long col = m0 + wc * 32 + 16 * j + m;
        if (row < nrows && col < slab) {
          H h, l;
          split_h<H>(sy * acc[i][j][r], h, l);
          Yhi[row * slab + col] = h;
          Ylo[row * slab + col] = l;
        }
      }
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
// Stage 2, split precision.  One workgroup = (slab s, term part); wave w owns
// output columns [32 w, 32 w + 32).
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
// K1P = 128 runs with at most 256 threads (K2P <= 128) so that one wave per
// SIMD may use the full register file without spilling.
template <typename H, int RT>
__global__ __launch_bounds__(RT >= 8 ? 256 : 512) void stage2_x3(
    const H* __restrict__ Yhi, const H* __restrict__ Ylo, const H* __restrict__ vec,
    const int* __restrict__ term_group, const int* __restrict__ part_begin,
    float* __restrict__ Phi_part, int K1, int K2, int K3, int K2P, int blen, int alen,
    float st) {
  typedef typename HVec<H>::v8 v8;
  typedef typename HVec<H>::v4 v4;
  constexpr int K1P = RT * 16, CT = 2, PF = 4;  // PF: 16-byte prefetch chunks per thread
  const int YSTR = K2P + 8;
  const int plane = 8 * blen + 4 * alen;        // halves per plane of one term
  const int tsz = 2 * plane;                    // halves per term (hi plane, lo plane)
  extern __shared__ __attribute__((aligned(16))) char smem[];
  H* Ysh = reinterpret_cast<H*>(smem);
  H* Ysl = Ysh + K1P * YSTR;
  H* vbuf = Ysl + K1P * YSTR;                   // [2][tsz]
  const int s = blockIdx.x, part = blockIdx.y;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, q = lane >> 4, m = lane & 15;
  const int col0 = wave * 16 * CT;
  const long slab = static_cast<long>(K1P) * K2P;
  const int nchunk = tsz / 8;
  floatx4 acc2[RT][CT];
  for (int i = 0; i < RT; ++i)
    for (int j = 0; j < CT; ++j) acc2[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int t0 = part_begin[part], t1 = part_begin[part + 1];
  // fragment start offsets that do not depend on the term
  //   B: y = (32 kc + 8 q - col0 - 16 j - m) mod K2;  A: y = (32 c + 4 q - 16 i - m) mod K1
  auto md = [](int x, int k) { x %= k; return x < 0 ? x + k : x; };
  const int yb0 = md(8 * q - col0 - m, K2);
  const int ya0 = md(4 * q - m, K1);
  // prologue: term t0's vectors into buffer 0
  for (int c = tid; c < nchunk; c += nthr)
    if (t0 < t1)
      *reinterpret_cast<v8*>(&vbuf[8 * c]) =
          *reinterpret_cast<const v8*>(&vec[static_cast<long>(t0) * tsz + 8 * c]);
  int cur = -1;
  for (int t = t0; t < t1; ++t) {
    const int g = term_group[t];
    const int buf = (t - t0) & 1;
    __syncthreads();
    if (g != cur) {
      const H* yh = Yhi + (static_cast<long>(g) * K3 + s) * slab;
      const H* yl = Ylo + (static_cast<long>(g) * K3 + s) * slab;
      const int cpr = K2P / 8;
      for (int e = tid; e < K1P * cpr; e += nthr) {
        const int r = e / cpr, c8 = e % cpr;
        *reinterpret_cast<v8*>(&Ysh[r * YSTR + 8 * c8]) =
            *reinterpret_cast<const v8*>(&yh[static_cast<long>(r) * K2P + 8 * c8]);
        *reinterpret_cast<v8*>(&Ysl[r * YSTR + 8 * c8]) =
            *reinterpret_cast<const v8*>(&yl[static_cast<long>(r) * K2P + 8 * c8]);
      }
      cur = g;
      __syncthreads();
    }
    // prefetch the next term's vectors into registers
    v8 pre[PF];
    if (t + 1 < t1) {
      const H* src = vec + static_cast<long>(t + 1) * tsz;
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const int c = tid + k * nthr;
        if (c < nchunk) pre[k] = *reinterpret_cast<const v8*>(&src[8 * c]);
      }
    }
    const H* Bvh = vbuf + buf * tsz;
    const H* Avh = Bvh + 8 * blen;
    const H* Bvl = Bvh + plane;
    const H* Avl = Bvl + 8 * blen;
    // GEMM1: T[g1][k2] = sum_g2 Y[g1][g2] B_t[k2][g2]
    floatx4 acc1[RT][CT];
    for (int i = 0; i < RT; ++i)
      for (int j = 0; j < CT; ++j) acc1[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < K2P / 32; ++kc) {
      v8 bh[CT], bl[CT];
      for (int j = 0; j < CT; ++j) {
        const int y = md(yb0 + 32 * kc - 16 * j, K2);
        const int off = (y & 7) * blen + (y & ~7);
        bh[j] = *reinterpret_cast<const v8*>(&Bvh[off]);
        bl[j] = *reinterpret_cast<const v8*>(&Bvl[off]);
      }
      for (int i = 0; i < RT; ++i) {
        const int off = (16 * i + m) * YSTR + 32 * kc + 8 * q;
        const v8 ah = *reinterpret_cast<const v8*>(&Ysh[off]);
        const v8 al = *reinterpret_cast<const v8*>(&Ysl[off]);
        for (int j = 0; j < CT; ++j) {
          acc1[i][j] = mfma_h(ah, bh[j], acc1[i][j]);
          acc1[i][j] = mfma_h(ah, bl[j], acc1[i][j]);
          acc1[i][j] = mfma_h(al, bh[j], acc1[i][j]);
        }
      }
    }
    // split T into 16-bit hi/lo, in the accumulator layout
    typename HVec<H>::v4 th[RT][CT], tl[RT][CT];
    for (int i = 0; i < RT; ++i)
      for (int j = 0; j < CT; ++j)
        for (int r = 0; r < 4; ++r) {
          H h, l;
          split_h<H>(st * acc1[i][j][r], h, l);
          th[i][j][r] = h;
          tl[i][j][r] = l;
        }
    // GEMM2: Phi[k1][k2] += sum_g1 A_t[k1][g1] T[g1][k2], K chunks of 32 rows
    // of T taken as {32c + 4q + r} u {32c + 16 + 4q + r}.
    for (int c = 0; c < RT / 2; ++c) {
      v8 tbh[CT], tbl[CT];
      for (int j = 0; j < CT; ++j) {
        tbh[j] = cat44<v4, v8>(th[2 * c][j], th[2 * c + 1][j]);
        tbl[j] = cat44<v4, v8>(tl[2 * c][j], tl[2 * c + 1][j]);
      }
      for (int i = 0; i < RT; ++i) {
        const int y0 = md(ya0 + 32 * c - 16 * i, K1);
        const int y1 = md(y0 + 16, K1);
        const int o0 = (y0 & 3) * alen + (y0 & ~3), o1 = (y1 & 3) * alen + (y1 & ~3);
        const v8 ah = cat44<v4, v8>(*reinterpret_cast<const v4*>(&Avh[o0]),
                                    *reinterpret_cast<const v4*>(&Avh[o1]));
        const v8 al = cat44<v4, v8>(*reinterpret_cast<const v4*>(&Avl[o0]),
                                    *reinterpret_cast<const v4*>(&Avl[o1]));
        for (int j = 0; j < CT; ++j) {
          acc2[i][j] = mfma_h(ah, tbh[j], acc2[i][j]);
          acc2[i][j] = mfma_h(ah, tbl[j], acc2[i][j]);
          acc2[i][j] = mfma_h(al, tbh[j], acc2[i][j]);
        }
      }
    }
    // publish the prefetched vectors into the other buffer (read after the
    // barrier at the top of the next iteration)
    if (t + 1 < t1) {
      H* dst = vbuf + (buf ^ 1) * tsz;
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const int c = tid + k * nthr;
        if (c < nchunk) *reinterpret_cast<v8*>(&dst[8 * c]) = pre[k];
      }
    }
  }
  float* out = Phi_part + (static_cast<long>(part) * K3 + s) * K1 * K2;
  for (int i = 0; i < RT; ++i)
    for (int j = 0; j < CT; ++j) {
      const int k2 = col0 + 16 * j + m;
      for (int r = 0; r < 4; ++r) {
        const int k1 = 16 * i + 4 * q + r;
        if (k1 < K1 && k2 < K2) out[static_cast<long>(k1) * K2 + k2] = acc2[i][j][r];
      }
    }
}

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
// [k1][k2][k3] and subtract c * sum(Q).
template <typename A, typename O>
__global__ __launch_bounds__(256) void finalize(const A* __restrict__ part, int nparts,
                                                O* __restrict__ Phi, int K1, int K2,
                                                int K3, const double* __restrict__ sumQ,
                                                double c0, const double* __restrict__ qscale,
                                                double const_scale) {
  __shared__ A tile[32][33];
  const int k1 = blockIdx.z, k2b = blockIdx.x * 32, k3b = blockIdx.y * 32;
  const A corr = static_cast<A>(c0 * sumQ[0]);
  // the partial slabs carry the product of the split-precision scales
  const A unscale = qscale ? static_cast<A>(1.0 / (qscale[0] * const_scale)) : A(1);
  const long pstride = static_cast<long>(K3) * K1 * K2;
  for (int j = threadIdx.y; j < 32; j += 8) {
    const int k3 = k3b + j, k2 = k2b + threadIdx.x;
    A v = 0;
    if (k3 < K3 && k2 < K2) {
      const long base = (static_cast<long>(k3) * K1 + k1) * K2 + k2;
      for (int p = 0; p < nparts; ++p) v += part[p * pstride + base];
    }
    tile[j][threadIdx.x] = v;
  }
  __syncthreads();
  for (int j = threadIdx.y; j < 32; j += 8) {
    const int k2 = k2b + j, k3 = k3b + threadIdx.x;
    if (k2 < K2 && k3 < K3)
      Phi[(static_cast<long>(k1) * K2 + k2) * K3 + k3] =
          static_cast<O>(unscale * tile[threadIdx.x][j] - corr);
  }
}

// Fixed-order FP64 sum and max |x| of a grid: per-block partials, then one
// block combines them.
template <typename T>
__global__ __launch_bounds__(256) void sum_partial(const T* __restrict__ x, long n,
                                                   double* __restrict__ part) {
  __shared__ double red[256], mx[256];
  const long per = (n + gridDim.x - 1) / gridDim.x;
  const long b = per * blockIdx.x, e = (b + per < n) ? b + per : n;
  double acc = 0.0, amax = 0.0;
  for (long i = b + threadIdx.x; i < e; i += blockDim.x) {
    const double v = static_cast<double>(x[i]);
    acc += v;
    amax = fmax(amax, fabs(v));
  }
  red[threadIdx.x] = acc;
  mx[threadIdx.x] = amax;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0];
    part[2 * blockIdx.x + 1] = mx[0];
  }
}

// out[0] = sum; out[1] = 2^(13 - floor(log2 max|x|)), the power of two that
// brings the largest grid value into [2^13, 2^14) for the FP16X3 split
// (1 for an all-zero or non-finite grid).
__global__ __launch_bounds__(256) void sum_final(const double* __restrict__ part, int np,
                                                 double* __restrict__ out) {
  __shared__ double red[256], mx[256];
  double acc = 0.0, amax = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) {
    acc += part[2 * i];
    amax = fmax(amax, part[2 * i + 1]);
  }
  red[threadIdx.x] = acc;
  mx[threadIdx.x] = amax;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0];
    const double m = mx[0];
    out[1] = (m > 0.0 && m < 1e300) ? ldexp(1.0, 13 - ilogb(m)) : 1.0;
  }
}

template <typename K>
hipError_t set_lds(K kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(bytes));
}

template <typename H, int RT>
hipError_t launch_s2_x3(const SkpArgs& a, hipStream_t st) {
  const int K1P = RT * 16;
  const size_t tsz = 2 * (8 * static_cast<size_t>(a.blen) + 4 * a.alen);
  const size_t lds = sizeof(H) * (2 * static_cast<size_t>(K1P) * (a.K2P + 8) + 2 * tsz);
  hipError_t e = set_lds(stage2_x3<H, RT>, lds);
  if (e != hipSuccess) return e;
  const int threads = 64 * (a.K2P / 32);
  if (threads > (RT >= 8 ? 256 : 512)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((stage2_x3<H, RT>), dim3(a.K[2], a.nparts), dim3(threads), lds, st,
                     static_cast<const H*>(a.Y[0]), static_cast<const H*>(a.Y[1]),
                     static_cast<const H*>(a.vec), a.term_group, a.part_begin,
                     static_cast<float*>(a.Phi_part), a.K[0], a.K[1], a.K[2], a.K2P, a.blen,
                     a.alen, a.st);
  return hipGetLastError();
}

template <typename T, int RT, int CT, bool AL>
hipError_t launch_s2_k4(const SkpArgs& a, hipStream_t st) {
  const int K1P = RT * 16;
  size_t lds = sizeof(T) * static_cast<size_t>(K1P) * (a.K2P + 1);
  if (AL) lds += sizeof(T) * static_cast<size_t>(K1P) * (K1P + 1);
  hipError_t e = set_lds(stage2_k4<T, RT, CT, AL>, lds);
  if (e != hipSuccess) return e;
  const int threads = 64 * (a.K2P / (16 * CT));
  hipLaunchKernelGGL((stage2_k4<T, RT, CT, AL>), dim3(a.K[2], a.nparts), dim3(threads), lds, st,
                     static_cast<const T*>(a.Y[0]), static_cast<const T*>(a.A[0]),
                     static_cast<const T*>(a.B[0]), a.term_group, a.part_begin,
                     static_cast<T*>(a.Phi_part), a.K[0], a.K[1], a.K[2], a.K2P);
  return hipGetLastError();
}

template <int RT>
hipError_t dispatch_s2(const SkpArgs& a, hipStream_t st) {
  const int K1P = RT * 16;
  if (a.prec == PREC_BF16X3) return launch_s2_x3<bf16, RT>(a, st);
  if (a.prec == PREC_FP16X3) return launch_s2_x3<f16, RT>(a, st);
  if (a.prec == PREC_FP32) {
    const size_t full = sizeof(float) * static_cast<size_t>(K1P) * (a.K2P + 1 + K1P + 1);
    return full <= kMaxLds ? launch_s2_k4<float, RT, 2, true>(a, st)
                           : launch_s2_k4<float, RT, 2, false>(a, st);
  }
  const size_t full = sizeof(double) * static_cast<size_t>(K1P) * (a.K2P + 1 + K1P + 1);
  return full <= kMaxLds ? launch_s2_k4<double, RT, 1, true>(a, st)
                         : launch_s2_k4<double, RT, 1, false>(a, st);
}

}  // namespace

size_t stage2_lds_bytes(int prec, int K1P, int K2P) {
  if (prec == PREC_BF16X3 || prec == PREC_FP16X3) {
    // Y slab (two planes) + two buffers of circulant vectors
    const size_t tsz = 2 * (8 * static_cast<size_t>(x3_blen(K2P)) + 4 * x3_alen(K1P));
    return 2 * (2 * static_cast<size_t>(K1P) * (K2P + 8) + 2 * tsz);
  }
  if (prec == PREC_FP32) return sizeof(float) * static_cast<size_t>(K1P) * (K2P + 1);
  return sizeof(double) * static_cast<size_t>(K1P) * (K2P + 1);
}

hipError_t launch_skp_sum(const SkpArgs& a, hipStream_t st) {
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

hipError_t launch_sum_final(const double* part2, int np, double* out, hipStream_t st) {
  hipLaunchKernelGGL(sum_final, dim3(1), dim3(256), 0, st, part2, np, out);
  return hipGetLastError();
}

hipError_t launch_skp_stage1(const SkpArgs& a, hipStream_t st) {
  const long slab = static_cast<long>(a.K1P) * a.K2P;
  const int nrows = a.r0 * a.K[2];
  dim3 g1(static_cast<unsigned>(slab / S1), (nrows + S1 - 1) / S1);
  if (a.prec == PREC_BF16X3)
    hipLaunchKernelGGL((stage1_x3<bf16>), g1, dim3(256), 0, st, static_cast<const float*>(a.Q),
                       static_cast<const bf16*>(a.C[0]), static_cast<const bf16*>(a.C[1]),
                       static_cast<bf16*>(a.Y[0]), static_cast<bf16*>(a.Y[1]), a.K[0], a.K[1],
                       a.K[2], a.K3P, a.K2P, slab, nrows, nullptr, 1.0f);
  else if (a.prec == PREC_FP16X3)
    hipLaunchKernelGGL((stage1_x3<f16>), g1, dim3(256), 0, st, static_cast<const float*>(a.Q),
                       static_cast<const f16*>(a.C[0]), static_cast<const f16*>(a.C[1]),
                       static_cast<f16*>(a.Y[0]), static_cast<f16*>(a.Y[1]), a.K[0], a.K[1],
                       a.K[2], a.K3P, a.K2P, slab, nrows, a.sumQ + 1, a.sy);
  else if (a.prec == PREC_FP32)
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
  switch (a.K1P) {
    case 32: return dispatch_s2<2>(a, st);
    case 64: return dispatch_s2<4>(a, st);
    case 96: return dispatch_s2<6>(a, st);
    case 128: return dispatch_s2<8>(a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_skp_finalize(const SkpArgs& a, hipStream_t st) {
  dim3 gf((a.K[1] + 31) / 32, (a.K[2] + 31) / 32, a.K[0]);
  if (a.prec == PREC_FP64)
    hipLaunchKernelGGL((finalize<double, double>), gf, dim3(32, 8), 0, st,
                       static_cast<const double*>(a.Phi_part), a.nparts,
                       static_cast<double*>(a.Phi), a.K[0], a.K[1], a.K[2], a.sumQ, a.c0,
                       nullptr, 1.0);
  else
    hipLaunchKernelGGL((finalize<float, float>), gf, dim3(32, 8), 0, st,
                       static_cast<const float*>(a.Phi_part), a.nparts,
                       static_cast<float*>(a.Phi), a.K[0], a.K[1], a.K[2], a.sumQ, a.c0,
                       a.prec == PREC_FP16X3 ? a.sumQ + 1 : nullptr, a.const_scale);
  return hipGetLastError();
}

}  // namespace kpme
