// X_i <- A_i^-1 X_i for several right-hand sides (up to 32 per launch) on
// the matrix cores: v_mfma_f64_16x16x4 (FP64 storage), v_mfma_f32_16x16x4f32
// (FP32) and v_mfma_f32_16x16x32_bf16 (BF16, right-hand sides rounded to
// BF16, FP32 accumulation).  Still HBM bound at 32 right-hand sides
// (8 / 16 / 32 flop per byte of FP64 / FP32 / BF16 storage).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "kernels.h"
#include "vec16.h"

namespace gdsw {
namespace {

// ---- several right-hand sides: MFMA products with the stored inverses ------
//
// Item (f, r0, c0, p) of a multi-RHS plan: output rows [r0, r0 + RB) and
// summation columns [c0, c0 + GEMV_CW) of matrix f for up to 32 right-hand
// sides (two groups of 16).  The work vectors are interleaved: entry
// (row, j) at w[row * ldk + j].  The right-hand sides of the chunk are staged
// in LDS SC columns at a time; each wave owns RB / 4 output rows.  partial
// layout: partial[(p * RB + row) * 32 + j].  Columns beyond the chunk (or n)
// are staged as zero, so padded or foreign matrix entries never contribute.
typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef __bf16 mf_bf8 __attribute__((ext_vector_type(8)));

#ifndef GDSW_GEMM_H
#define GDSW_GEMM_H 1     // FP64/FP32: row groups of 16 E rows per wave
#endif
#ifndef GDSW_GEMM_HB
#define GDSW_GEMM_HB 4    // BF16: 16-row output tiles per wave
#endif
#ifndef GDSW_GEMM_SC
#define GDSW_GEMM_SC 64   // FP64/FP32: columns staged per step
#endif
#ifndef GDSW_GEMM_SCB
#define GDSW_GEMM_SCB 128 // BF16: columns staged per step
#endif

template <typename T>
struct MultiShape;
template <>
struct MultiShape<double> {  // v_mfma_f64_16x16x4: a lane's 16-byte load = 2 rows of one column
  static constexpr int H = GDSW_GEMM_H, RB = 4 * H * 32, SC = GDSW_GEMM_SC;
  using P = double;
};
template <>
struct MultiShape<float> {  // v_mfma_f32_16x16x4f32: 4 rows of one column
  static constexpr int H = GDSW_GEMM_H, RB = 4 * H * 64, SC = GDSW_GEMM_SC;
  using P = float;
};
template <>
struct MultiShape<uint16_t> {  // v_mfma_f32_16x16x32_bf16: 8 entries along the summation index
  static constexpr int H = GDSW_GEMM_HB, RB = 4 * H * 16, SC = GDSW_GEMM_SCB;
  using P = float;
};

__device__ inline uint16_t bf16_bits(double x) { return to_bf16((float)x); }

// Stage rows [c, c + SC) x 32 right-hand sides of the work vectors into LDS
// as the MFMA B operand type.
template <typename T, typename XT, int SC, bool RHS_MAJOR>
__device__ inline void stage_x(XT* xs, const double* __restrict__ x, int64_t ldk, int nrhs, int ccount) {
  for (int idx = threadIdx.x; idx < SC * 32; idx += 256) {
    const int j = idx % 32, col = idx / 32;  // consecutive threads: consecutive right-hand sides of one row
    const double v = (col < ccount && j < nrhs) ? x[(int64_t)col * ldk + j] : 0.0;
    XT o;
    if constexpr (sizeof(XT) == 2)
      o = bf16_bits(v);
    else
      o = (XT)v;
    if constexpr (RHS_MAJOR)
      xs[j * SC + col] = o;
    else
      xs[col * 32 + j] = o;
  }
}

// FP64 and FP32 storage: for each of H row groups h, lane l loads
// E = 16 / sizeof(T) consecutive rows (Rw + 16 E h + E (l % 16) + v) of
// column c + l / 16; MFMA (h, v) uses A[i][k] = M[Rw + 16 E h + E i + v][c + k]
// and B[k][j] = x[c + k][j].
template <typename T, int G>
__global__ __launch_bounds__(256) void gemm_part_kernel(const T* __restrict__ store, const int64_t* __restrict__ OFF,
                                                        const int32_t* __restrict__ N, const int32_t* __restrict__ NP,
                                                        const int64_t* __restrict__ XOFF,
                                                        const int4* __restrict__ items, const double* __restrict__ w,
                                                        int64_t ldk, int nrhs,
                                                        typename MultiShape<T>::P* __restrict__ partial) {
  using S = MultiShape<T>;
  using P = typename S::P;
  using ACC = typename std::conditional<sizeof(T) == 8, mf_d4, mf_f4>::type;
  constexpr int E = 16 / sizeof(T);
  constexpr int H = S::H, RB = S::RB, SC = S::SC;
  __shared__ T xs[SC * 32];
  const int4 item = items[blockIdx.x];
  const int f = item.x, r0 = item.y, c0 = item.z, p = item.w;
  const int n = N[f];
  const int64_t np = NP[f];
  const int cend = min(c0 + GEMV_CW, n);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const int Rw = r0 + wave * (RB / 4);
  bool rok[H];
#pragma unroll
  for (int h = 0; h < H; ++h) rok[h] = Rw + 16 * E * h + E * i < n;
  const T* base = store + OFF[f] + Rw + E * i;
  const double* x = w + XOFF[f] * ldk;
  ACC acc[H][E][G];
#pragma unroll
  for (int h = 0; h < H; ++h)
#pragma unroll
    for (int v = 0; v < E; ++v)
#pragma unroll
      for (int g = 0; g < G; ++g) acc[h][v][g] = ACC{0, 0, 0, 0};
  for (int c = c0; c < cend; c += SC) {
    // every matrix load of the step is issued first (they do not depend on
    // the staged right-hand sides), then the staging, then the products
    constexpr int Q = SC / 4;
    T a[Q][H][E];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int col = c + 4 * q + kq;
#pragma unroll
      for (int h = 0; h < H; ++h) {
        if (rok[h] && col < cend) {
          load16_nt(base + 16 * E * h + (int64_t)col * np, a[q][h]);
        } else {
#pragma unroll
          for (int v = 0; v < E; ++v) a[q][h][v] = 0;
        }
      }
    }
    __syncthreads();
    stage_x<T, T, SC, false>(xs, x + (int64_t)c * ldk, ldk, nrhs, min(SC, cend - c));
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const T b = xs[(4 * q + kq) * 32 + g * 16 + i];
#pragma unroll
        for (int h = 0; h < H; ++h)
#pragma unroll
          for (int v = 0; v < E; ++v) {
            if constexpr (sizeof(T) == 8)
              acc[h][v][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q][h][v], b, acc[h][v][g], 0, 0, 0);
            else
              acc[h][v][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[q][h][v], b, acc[h][v][g], 0, 0, 0);
          }
      }
    }
  }
  // D_(h,v)[i'][j] = y[Rw + 16 E h + E i' + v][16 g + j], j = i.  Accumulator
  // register t of a lane holds output row i' = 4 kq + t for the f32 shape and
  // i' = kq + 4 t for the f64 shape (groups of one row strided by 4).
  P* out = partial + (int64_t)p * RB * 32;
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int v = 0; v < E; ++v)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int ip = sizeof(T) == 8 ? kq + 4 * t : 4 * kq + t;
          out[(int64_t)(wave * (RB / 4) + 16 * E * h + E * ip + v) * 32 + g * 16 + i] = (P)acc[h][v][g][t];
        }
}

// BF16 storage (the stored inverse is symmetric): lane l loads 2 x 8
// entries of column Rw + 16 h + (l % 16), rows c + 16 (l / 16) + 0..15, i.e.
// 16 consecutive summation entries of output row Rw + 16 h + (l % 16).
template <int G>
__global__ __launch_bounds__(256) void gemm_part_bf16_kernel(const uint16_t* __restrict__ store,
                                                             const int64_t* __restrict__ OFF,
                                                             const int32_t* __restrict__ N,
                                                             const int32_t* __restrict__ NP,
                                                             const int64_t* __restrict__ XOFF,
                                                             const int4* __restrict__ items,
                                                             const double* __restrict__ w, int64_t ldk, int nrhs,
                                                             float* __restrict__ partial) {
  using S = MultiShape<uint16_t>;
  constexpr int H = S::H, RB = S::RB, SC = S::SC;
  __shared__ uint16_t xs[32 * SC];  // [rhs][col]
  const int4 item = items[blockIdx.x];
  const int f = item.x, r0 = item.y, c0 = item.z, p = item.w;
  const int n = N[f];
  const int64_t np = NP[f];
  const int cend = min(c0 + GEMV_CW, n);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const int Rw = r0 + wave * (RB / 4);
  const double* x = w + XOFF[f] * ldk;
  mf_f4 acc[H][G];
#pragma unroll
  for (int h = 0; h < H; ++h)
#pragma unroll
    for (int g = 0; g < G; ++g) acc[h][g] = mf_f4{0, 0, 0, 0};
  for (int c = c0; c < cend; c += SC) {
    // matrix loads of the step first, then the staging, then the products
    constexpr int Q = SC / 64;
    gdsw_u4 a[Q][H][2];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int r = c + 64 * q + 16 * kq;  // first summation index of this lane
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int ocol = Rw + 16 * h + i;  // output row = storage column (symmetry)
        a[q][h][0] = gdsw_u4{0, 0, 0, 0};
        a[q][h][1] = gdsw_u4{0, 0, 0, 0};
        if (ocol < n && r < cend) {
          const uint16_t* src = store + OFF[f] + (int64_t)ocol * np + r;
          a[q][h][0] = __builtin_nontemporal_load(reinterpret_cast<const gdsw_u4*>(src));
          a[q][h][1] = __builtin_nontemporal_load(reinterpret_cast<const gdsw_u4*>(src + 8));
        }
      }
    }
    __syncthreads();
    stage_x<uint16_t, uint16_t, SC, true>(xs, x + (int64_t)c * ldk, ldk, nrhs, min(SC, cend - c));
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      mf_bf8 bx[G][2];
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2)
          bx[g][s2] = *reinterpret_cast<const mf_bf8*>(&xs[(g * 16 + i) * SC + 64 * q + 16 * kq + 8 * s2]);
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const mf_bf8 A0 = __builtin_bit_cast(mf_bf8, a[q][h][0]);
        const mf_bf8 A1 = __builtin_bit_cast(mf_bf8, a[q][h][1]);
#pragma unroll
        for (int g = 0; g < G; ++g) {
          acc[h][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, bx[g][0], acc[h][g], 0, 0, 0);
          acc[h][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, bx[g][1], acc[h][g], 0, 0, 0);
        }
      }
    }
  }
  float* out = partial + (int64_t)p * RB * 32;
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        out[(int64_t)(wave * (RB / 4) + 16 * h + 4 * kq + t) * 32 + g * 16 + i] = acc[h][g][t];
}

// Item (f, r0, p0, cnt): w[(XOFF + r0 + t) * ldk + j] = sum_q partial[((p0 + q) * RB + t) * 32 + j].
template <typename P, int RB>
__global__ __launch_bounds__(256) void gemm_sum_kernel(const int32_t* __restrict__ N, const int64_t* __restrict__ XOFF,
                                                       const int4* __restrict__ items, const P* __restrict__ partial,
                                                       double* __restrict__ w, int64_t ldk, int nrhs) {
  const int4 item = items[blockIdx.x];
  const int f = item.x, r0 = item.y, p0 = item.z, cnt = item.w;
  const int n = N[f];
  const int rows = min(RB, n - r0);
  for (int e = threadIdx.x; e < rows * nrhs; e += 256) {
    const int t = e / nrhs, j = e % nrhs;
    double s = 0.0;
    for (int q = 0; q < cnt; ++q) s += (double)partial[((int64_t)(p0 + q) * RB + t) * 32 + j];
    w[(XOFF[f] + r0 + t) * ldk + j] = s;
  }
}

template <typename T>
void gemm_launch(const FactorSet& fs, double* w, int64_t ldk, int nrhs, hipStream_t st) {
  using S = MultiShape<T>;
  using P = typename S::P;
  const FactorSet::GemvPlan& G = fs.gemm;
  if (G.n1 == 0) return;
  P* part = static_cast<P*>(fs.d_partial_m);
  for (int j0 = 0; j0 < nrhs; j0 += 32) {
    const int nr = std::min(32, nrhs - j0);
    double* wj = w + j0;
    KernelTimer* tm = (fs.timer && fs.timer->on && fs.timer->used < KernelTimer::CAP) ? fs.timer : nullptr;
    if (tm) GDSW_HIP(hipEventRecord(tm->ev[2 * tm->used], st));
    if constexpr (sizeof(T) == 2) {
      if (nr > 16)
        gemm_part_bf16_kernel<2><<<G.n1, 256, 0, st>>>(static_cast<const uint16_t*>(fs.store), fs.d_off, fs.d_n,
                                                      fs.d_npad, fs.d_xoff, G.d_items1, wj, ldk, nr, part);
      else
        gemm_part_bf16_kernel<1><<<G.n1, 256, 0, st>>>(static_cast<const uint16_t*>(fs.store), fs.d_off, fs.d_n,
                                                      fs.d_npad, fs.d_xoff, G.d_items1, wj, ldk, nr, part);
    } else {
      if (nr > 16)
        gemm_part_kernel<T, 2><<<G.n1, 256, 0, st>>>(static_cast<const T*>(fs.store), fs.d_off, fs.d_n, fs.d_npad,
                                                     fs.d_xoff, G.d_items1, wj, ldk, nr, part);
      else
        gemm_part_kernel<T, 1><<<G.n1, 256, 0, st>>>(static_cast<const T*>(fs.store), fs.d_off, fs.d_n, fs.d_npad,
                                                     fs.d_xoff, G.d_items1, wj, ldk, nr, part);
    }
    if (tm) {
      GDSW_HIP(hipEventRecord(tm->ev[2 * tm->used++ + 1], st));
      tm->bytes += (double)fs.alg_bytes;
    }
    gemm_sum_kernel<P, S::RB><<<G.n2, 256, 0, st>>>(fs.d_n, fs.d_xoff, G.d_items2, part, wj, ldk, nr);
  }
}

}  // namespace

int gemm_rows(int prec) {
  return prec == P_FP64 ? MultiShape<double>::RB : prec == P_FP32 ? MultiShape<float>::RB : MultiShape<uint16_t>::RB;
}

void gemm_set(const FactorSet& fs, double* w, int64_t ldk, int nrhs, hipStream_t st) {
  if (fs.count == 0 || nrhs == 0) return;
  if (fs.prec == P_FP64)
    gemm_launch<double>(fs, w, ldk, nrhs, st);
  else if (fs.prec == P_FP32)
    gemm_launch<float>(fs, w, ldk, nrhs, st);
  else
    gemm_launch<uint16_t>(fs, w, ldk, nrhs, st);
  GDSW_HIP(hipGetLastError());
}

}  // namespace gdsw
