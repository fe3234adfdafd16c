// 16x16x4 matrix-core (MFMA) wrappers for gfx950 shared by the factorization and solve kernels.
//
// Operand layout of one 16x16x4 MFMA D = A B + C in a wave of 64 lanes: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; register q of lane l receives D[drow(l, q)][l % 16].
#pragma once
#include <hip/hip_runtime.h>

namespace lobpcg {

template <typename T> struct Mfma;
// Output row of D held by (lane, register q) of a 16x16x4 MFMA (column is lane % 16);
// the FP32 and FP64 forms interleave the rows differently (checked on gfx950).
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 op(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int drow(int lane, int q) { return 4 * (lane / 16) + q; }
};
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int drow(int lane, int q) { return 4 * q + lane / 16; }
};

}  // namespace lobpcg
