// Matrix-core (MFMA) wrappers for gfx950 shared by the kernel files.
#pragma once

#include <hip/hip_runtime.h>

namespace hdsw {

template <class T>
struct MF;
template <>
struct MF<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 mfma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator register i of lane l holds row 4 (l / 16) + i, column l % 16
  static __device__ inline int row(int l, int i) { return 4 * (l >> 4) + i; }
};
template <>
struct MF<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 mfma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator register i of lane l holds row l / 16 + 4 i, column l % 16
  static __device__ inline int row(int l, int i) { return (l >> 4) + 4 * i; }
};

}  // namespace hdsw
