// Device-side types and helpers shared by the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kpme {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double doublex4;

// Split x = hi + lo into two round-to-nearest-even bfloat16 values.
__device__ __forceinline__ void split_bf16(float x, bf16& hi, bf16& lo) {
  hi = static_cast<bf16>(x);
  lo = static_cast<bf16>(x - static_cast<float>(hi));
}

__device__ __forceinline__ bf16x8 cat44(bf16x4 a, bf16x4 b) {
  return bf16x8{a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
}

// 16x16x32 bf16 product, FP32 accumulation.  Lane l holds A[l%16][8(l/16)..+7],
// B[8(l/16)..+7][l%16]; D[4(l/16)+r][l%16] in register r.
__device__ __forceinline__ floatx4 mfma_bf16(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
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
