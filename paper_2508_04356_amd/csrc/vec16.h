// 16-byte vector loads of factor storage (FP64, FP32, BF16) widened to the
// accumulation type (FP64 for FP64 storage, FP32 otherwise).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gdsw {

template <typename T>
struct VecW;
template <>
struct VecW<double> {
  static constexpr int W = 2;
  using acc = double;
};
template <>
struct VecW<float> {
  static constexpr int W = 4;
  using acc = float;
};
template <>
struct VecW<uint16_t> {
  static constexpr int W = 8;
  using acc = float;
};

__device__ inline void load16(const double* p, double (&o)[2]) {
  const double2 v = *reinterpret_cast<const double2*>(p);
  o[0] = v.x;
  o[1] = v.y;
}
__device__ inline void load16(const float* p, float (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x;
  o[1] = v.y;
  o[2] = v.z;
  o[3] = v.w;
}
__device__ inline void load16(const uint16_t* p, float (&o)[8]) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    o[2 * i] = __uint_as_float(w[i] << 16);
    o[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
  }
}

}  // namespace gdsw
