// Matrix-core (MFMA) and cross-lane wrappers for gfx950 shared by the
// kernel files.
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

// Largest value over the 64 lanes of the wave, returned in every lane:
// quad permutations and row mirrors reduce each row of 16 lanes, row
// broadcasts combine the rows into lane 63.
__device__ __forceinline__ unsigned dpp_max(unsigned v, unsigned t) { return v > t ? v : t; }
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  const int iv = (int)v;
  v = dpp_max(v, (unsigned)__builtin_amdgcn_update_dpp(iv, iv, 0xB1, 0xF, 0xF, false));
  int w = (int)v;
  v = dpp_max(v, (unsigned)__builtin_amdgcn_update_dpp(w, w, 0x4E, 0xF, 0xF, false));
  w = (int)v;
  v = dpp_max(v, (unsigned)__builtin_amdgcn_update_dpp(w, w, 0x141, 0xF, 0xF, false));
  w = (int)v;
  v = dpp_max(v, (unsigned)__builtin_amdgcn_update_dpp(w, w, 0x140, 0xF, 0xF, false));
  w = (int)v;
  v = dpp_max(v, (unsigned)__builtin_amdgcn_update_dpp(w, w, 0x142, 0xA, 0xF, false));
  w = (int)v;
  v = dpp_max(v, (unsigned)__builtin_amdgcn_update_dpp(w, w, 0x143, 0xC, 0xF, false));
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

}  // namespace hdsw
