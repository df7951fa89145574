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

// Streaming variants: the loads carry the non-temporal hint, so data read
// once does not displace reusable lines from the caches.
typedef double gdsw_d2 __attribute__((ext_vector_type(2)));
typedef float gdsw_f4 __attribute__((ext_vector_type(4)));
typedef uint32_t gdsw_u4 __attribute__((ext_vector_type(4)));

// Factor storage is always device (global) memory.  Its pointers often come
// out of descriptors in memory, where the compiler cannot tell their address
// space and would emit flat loads; a flat load also counts as an LDS access,
// so the wait before the next LDS barrier would wait for every tile load in
// flight.  The cast makes them global loads, counted as vector memory only.
template <typename V>
__device__ inline const __attribute__((address_space(1))) V* as_global(const void* p) {
  return (const __attribute__((address_space(1))) V*)p;
}

__device__ inline void load16_nt(const double* p, double (&o)[2]) {
  const gdsw_d2 v = __builtin_nontemporal_load(as_global<gdsw_d2>(p));
  o[0] = v.x;
  o[1] = v.y;
}
__device__ inline void load16_nt(const float* p, float (&o)[4]) {
  const gdsw_f4 v = __builtin_nontemporal_load(as_global<gdsw_f4>(p));
  o[0] = v.x;
  o[1] = v.y;
  o[2] = v.z;
  o[3] = v.w;
}
__device__ inline void load16_nt(const uint16_t* p, float (&o)[8]) {
  const gdsw_u4 v = __builtin_nontemporal_load(as_global<gdsw_u4>(p));
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    o[2 * i] = __uint_as_float(w[i] << 16);
    o[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
  }
}

__device__ inline void load16(const double* p, double (&o)[2]) {
  const gdsw_d2 v = *as_global<gdsw_d2>(p);
  o[0] = v.x;
  o[1] = v.y;
}
__device__ inline void load16(const float* p, float (&o)[4]) {
  const gdsw_f4 v = *as_global<gdsw_f4>(p);
  o[0] = v.x;
  o[1] = v.y;
  o[2] = v.z;
  o[3] = v.w;
}
__device__ inline void load16(const uint16_t* p, float (&o)[8]) {
  const gdsw_u4 v = *as_global<gdsw_u4>(p);
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    o[2 * i] = __uint_as_float(w[i] << 16);
    o[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
  }
}

// 16-byte loads through a buffer resource (raw buffer, byte offsets): an
// offset past the resource's size reads as zero without a memory access, so
// a piece that is not needed costs no traffic while the load instruction
// stays unconditional (no branch around it, so the compiler's wait counts
// stay exact and later loads stay in flight).  NT: the non-temporal hint.
constexpr uint32_t BUF_SKIP = 0x80000000u;  // past every resource made here

__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  // word 3 = 0x00020000: the raw 32-bit data format of the gfx9 family
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}

template <bool NT>
__device__ inline gdsw_u4 buf_load16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(gdsw_u4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, NT ? 2 : 0));
}
template <bool NT>
__device__ inline void buf_load16(__amdgpu_buffer_rsrc_t r, uint32_t off, double (&o)[2]) {
  const gdsw_d2 v = __builtin_bit_cast(gdsw_d2, buf_load16<NT>(r, off));
  o[0] = v.x;
  o[1] = v.y;
}
template <bool NT>
__device__ inline void buf_load16(__amdgpu_buffer_rsrc_t r, uint32_t off, float (&o)[4]) {
  const gdsw_f4 v = __builtin_bit_cast(gdsw_f4, buf_load16<NT>(r, off));
  o[0] = v.x;
  o[1] = v.y;
  o[2] = v.z;
  o[3] = v.w;
}
template <bool NT>
__device__ inline void buf_load16_bf16(__amdgpu_buffer_rsrc_t r, uint32_t off, float (&o)[8]) {
  const gdsw_u4 v = buf_load16<NT>(r, off);
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    o[2 * i] = __uint_as_float(w[i] << 16);
    o[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
  }
}

// FP32 -> BF16 bits, round to nearest even (NaN stays NaN).
__device__ inline uint16_t to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}

}  // namespace gdsw
