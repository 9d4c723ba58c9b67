// MFMA operand traits shared by the matrix-core kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace gvt {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Output layout of the 16x16 MFMA blocks (checked with a one-hot lane probe on
// gfx950): lane l holds column l % 16; item v holds row 4*(l/16) + v for the
// FP32 and bf16 instructions but row (l/16) + 4*v for v_mfma_f64_16x16x4f64.
template <class T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

}  // namespace gvt
