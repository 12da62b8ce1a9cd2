// Device-side types and helpers shared by the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kpme {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef _Float16 f16;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(4 * sizeof(_Float16)))) _Float16 f16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double doublex4;

// Split x = hi + lo into two round-to-nearest-even 16-bit values (bfloat16
// or IEEE half).
template <typename H>
__device__ __forceinline__ void split_h(float x, H& hi, H& lo) {
  hi = static_cast<H>(x);
  lo = static_cast<H>(x - static_cast<float>(hi));
}
__device__ __forceinline__ void split_bf16(float x, bf16& hi, bf16& lo) { split_h<bf16>(x, hi, lo); }

// 8- and 4-wide vectors of a 16-bit element type.
template <typename H> struct HVec;
template <> struct HVec<bf16> { typedef bf16x8 v8; typedef bf16x4 v4; };
template <> struct HVec<f16> { typedef f16x8 v8; typedef f16x4 v4; };

template <typename V4, typename V8>
__device__ __forceinline__ V8 cat44(V4 a, V4 b) {
  return V8{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
}
__device__ __forceinline__ bf16x8 cat44(bf16x4 a, bf16x4 b) { return cat44<bf16x4, bf16x8>(a, b); }
__device__ __forceinline__ f16x8 cat44(f16x4 a, f16x4 b) { return cat44<f16x4, f16x8>(a, b); }

// 16x16x32 bf16 product, FP32 accumulation.  Lane l holds A[l%16][8(l/16)..+7],
// B[8(l/16)..+7][l%16]; D[4(l/16)+r][l%16] in register r.
__device__ __forceinline__ floatx4 mfma_bf16(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// Same shape and lane layout for IEEE half inputs.
__device__ __forceinline__ floatx4 mfma_h(bf16x8 a, bf16x8 b, floatx4 c) { return mfma_bf16(a, b, c); }
__device__ __forceinline__ floatx4 mfma_h(f16x8 a, f16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
// 16x16x4 products: lane l holds A[l%16][l/16], B[l/16][l%16].  The FP32
// form returns D[4(l/16)+r][l%16] in register r, the FP64 form returns
// D[4r+(l/16)][l%16] (measured on gfx950); acc_row gives the row.
__device__ __forceinline__ floatx4 mfma_k4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma_k4(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T> __device__ __forceinline__ int acc_row(int q, int r);
template <> __device__ __forceinline__ int acc_row<float>(int q, int r) { return 4 * q + r; }
template <> __device__ __forceinline__ int acc_row<double>(int q, int r) { return 4 * r + q; }

template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef floatx4 type; };
template <> struct Vec4<double> { typedef doublex4 type; };

}  // namespace kpme

namespace kpme {

// Workgroups are handed to the 8 XCDs (each with its own L2) in turn: linear
// workgroup b runs on XCD b % 8.  xcd_order(b, n) renumbers them so that
// every XCD gets one contiguous range of the logical order; kernels whose
// neighbouring logical workgroups share inputs then reuse them in one L2.
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_order(int b, int n) {
  const int x = b % kNumXcd, i = b / kNumXcd;
  const int per = n / kNumXcd, rem = n % kNumXcd;
  return x * per + min(x, rem) + i;
}
__device__ __forceinline__ int linear_block() {
  return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}
__device__ __forceinline__ int num_blocks() { return gridDim.x * gridDim.y * gridDim.z; }

// Workgroup reduction in a fixed order: sums of v[0..NS) and maxima of
// v[NS..NV), by a butterfly within each wave and then over the waves in wave
// order; the result is in thread 0's v.  The workgroup is whole waves, at
// most 16; red holds 16 * NV doubles of LDS.  Every thread must call it.
template <int NS, int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const double x = __shfl_xor(v[k], o, 64);
      v[k] = k < NS ? v[k] + x : fmax(v[k], x);
    }
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[16 * k + wv] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double a = red[16 * k];
      for (int w = 1; w < nw; ++w) a = k < NS ? a + red[16 * k + w] : fmax(a, red[16 * k + w]);
      v[k] = a;
    }
}

}  // namespace kpme
