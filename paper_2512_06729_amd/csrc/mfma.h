// 16x16x4 matrix-core helpers shared by the Schur-update and block-product
// kernels (device code only).
#pragma once

#include <hip/hip_runtime.h>

namespace xod {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32: lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; it receives D[l/16 + 4i][l%16] (f64) or
// D[4(l/16) + i][l%16] (f32), i = 0..3 (layouts checked on gfx950).
__device__ __forceinline__ int mfma_row(double, int lane, int i) { return (lane >> 4) + 4 * i; }
__device__ __forceinline__ int mfma_row(float, int lane, int i) { return 4 * (lane >> 4) + i; }
__device__ __forceinline__ double4_t mfma16(double a, double b, double4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ float4_t mfma16(float a, float b, float4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <class T> struct Vec4;
template <> struct Vec4<double> { typedef double4_t type; };
template <> struct Vec4<float> { typedef float4_t type; };

}  // namespace xod
