// 16x16x4 matrix-core helpers shared by the Schur-update and block-product
// kernels, and global-memory views of device pointers (device code only).
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
// Global-address-space views of device pointers.  Accesses through them
// compile to global_* instructions, counted by vmcnt alone; generic (flat_*)
// accesses also count in lgkmcnt, so waiting for an LDS read would wait for
// every global load in flight as well, and a prefetch could not overlap
// the MFMAs fed from LDS.
template <class T> using GlobalPtr = __attribute__((address_space(1))) T *;
template <class T> __device__ __forceinline__ GlobalPtr<const T> gmem(const T *p) {
  return (GlobalPtr<const T>)p;
}
template <class T> __device__ __forceinline__ GlobalPtr<T> gmem(T *p) { return (GlobalPtr<T>)p; }

template <class T> struct Vec4;
template <> struct Vec4<double> { typedef double4_t type; };
template <> struct Vec4<float> { typedef float4_t type; };

}  // namespace xod
