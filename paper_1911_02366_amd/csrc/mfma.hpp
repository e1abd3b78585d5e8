// CDNA4 matrix-core helpers: the 16x16x4 MFMA in FP64 and FP32.
//
// Operand layout within a 64-lane wave (A is 16x4, B is 4x16, D is 16x16),
// measured on gfx950:
//   A: lane l holds A[l % 16][l / 16]
//   B: lane l holds B[l / 16][l % 16]
//   D, FP32: lane l, element r holds D[4 * (l / 16) + r][l % 16]
//   D, FP64: lane l, element r holds D[l / 16 + 4 * r][l % 16]
// Mfma<T>::row(lane, r) returns the D row of (lane, r); the column is lane % 16.
#pragma once

#include <hip/hip_runtime.h>

namespace scdg {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  using acc_t = f64x4;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <>
struct Mfma<float> {
  using acc_t = f32x4;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

}  // namespace scdg
