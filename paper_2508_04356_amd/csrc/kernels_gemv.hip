// y = A_i^-1 x for every stored inverse of a factor set: the single
// right-hand-side apply of the local (and coarse) solves, HBM bound.
//
// Kernel 1: one work-group per (matrix, row block of 64 * E rows, chunk of
// GEMV_CW columns), each lane owning E = 16 / sizeof(T) consecutive rows of
// a column (one 16-byte non-temporal load per column), the waves splitting
// the columns; it writes one partial vector per item.  Kernel 2 sums the
// partials of a row block in chunk order (a fixed order: results are bitwise
// reproducible) and writes the result over x in the work vector.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "vec16.h"

namespace gdsw {
namespace {

#ifndef GDSW_GEMV_NW
#define GDSW_GEMV_NW 4  // waves per matrix-vector work-group
#endif
#ifndef GDSW_GEMV_U
#define GDSW_GEMV_U 8   // columns loaded per wave before the FMAs
#endif
#ifndef GDSW_GEMV_NT
#define GDSW_GEMV_NT 1  // 1: non-temporal loads of the inverses (read once per apply)
#endif

template <typename T, typename V>
__device__ inline void gemv_load(const T* p, V& o) {
  if constexpr (GDSW_GEMV_NT)
    load16_nt(p, o);
  else
    load16(p, o);
}

// ---- batched dense matrix-vector product ----------------------------------

// Item (f, r0, c0, p): rows [r0, r0 + 64 E) and columns [c0, c0 + GEMV_CW)
// of matrix f; partial[p * 64 E + row] = sum over those columns of M x.
template <typename T, int NW>
__global__ __launch_bounds__(64 * NW) void gemv_part_kernel(const T* __restrict__ store,
                                                           const int64_t* __restrict__ OFF,
                                                           const int32_t* __restrict__ N,
                                                           const int32_t* __restrict__ NP,
                                                           const int64_t* __restrict__ XOFF,
                                                           const int4* __restrict__ items,
                                                           const double* __restrict__ w,
                                                           double* __restrict__ partial,
                                                           const int32_t* __restrict__ want) {
  using AT = typename VecW<T>::acc;
  constexpr int E = VecW<T>::W;
  constexpr int RB = 64 * E;
  __shared__ AT xs[GEMV_CW];
  __shared__ AT red[NW][RB];
  const int4 item = items[blockIdx.x];
  const int f = item.x, r0 = item.y, c0 = item.z, p = item.w;
  if (want && !want[f]) return;  // uniform per work-group
  const int n = N[f];
  const int64_t np = NP[f];
  const int ncols = min(GEMV_CW, n - c0);
  const int tid = threadIdx.x;
  const double* x = w + XOFF[f] + c0;
  for (int i = tid; i < GEMV_CW; i += 64 * NW) xs[i] = i < ncols ? (AT)x[i] : (AT)0;
  const int lane = tid & 63, wave = tid >> 6;
  const int rr = r0 + lane * E;
  const bool active = rr < n;
  const T* col = store + OFF[f] + (int64_t)c0 * np + rr;
  AT acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = 0;
  __syncthreads();
  if (active) {
    constexpr int U = GDSW_GEMV_U;
    int c = wave;
    for (; c + (U - 1) * NW < ncols; c += U * NW) {
      AT v[U][E];
#pragma unroll
      for (int u = 0; u < U; ++u) gemv_load(col + (int64_t)(c + u * NW) * np, v[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const AT xv = xs[c + u * NW];
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = fma(v[u][e], xv, acc[e]);
      }
    }
    for (; c < ncols; c += NW) {
      AT v[E];
      gemv_load(col + (int64_t)c * np, v);
      const AT xv = xs[c];
#pragma unroll
      for (int e = 0; e < E; ++e) acc[e] = fma(v[e], xv, acc[e]);
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) red[wave][lane * E + e] = acc[e];
  __syncthreads();
  for (int r = tid; r < RB; r += 64 * NW) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) s += (double)red[q][r];
    partial[(int64_t)p * RB + r] = s;
  }
}

// Item (f, r0, p0, cnt): x[r0 + t] = sum_{q < cnt} partial[(p0 + q) * RB + t].
template <int RB>
__global__ __launch_bounds__(256) void gemv_sum_kernel(const int32_t* __restrict__ N,
                                                       const int64_t* __restrict__ XOFF,
                                                       const int4* __restrict__ items,
                                                       const double* __restrict__ partial, double* __restrict__ w,
                                                       const int32_t* __restrict__ want) {
  const int4 item = items[blockIdx.x];
  const int f = item.x, r0 = item.y, p0 = item.z, cnt = item.w;
  if (want && !want[f]) return;
  const int n = N[f];
  for (int t = threadIdx.x; t < RB; t += 256) {
    if (r0 + t >= n) break;
    double s = 0.0;
    for (int q = 0; q < cnt; ++q) s += partial[(int64_t)(p0 + q) * RB + t];
    w[XOFF[f] + r0 + t] = s;
  }
}

template <typename T>
void gemv_launch(const FactorSet& fs, double* w, hipStream_t st, int slot, const int32_t* want) {
  const FactorSet::GemvPlan& G = fs.gemv[slot];
  if (G.n1 == 0) return;
  constexpr int RB = 64 * VecW<T>::W;
  KernelTimer* tm = (slot == 0 && fs.timer && fs.timer->on && fs.timer->used < KernelTimer::CAP) ? fs.timer : nullptr;
  if (tm) GDSW_HIP(hipEventRecord(tm->ev[2 * tm->used], st));
  gemv_part_kernel<T, GDSW_GEMV_NW><<<G.n1, 64 * GDSW_GEMV_NW, 0, st>>>(
      static_cast<const T*>(fs.store), fs.d_off, fs.d_n, fs.d_npad, fs.d_xoff, G.d_items1, w, fs.d_partial, want);
  if (tm) {
    GDSW_HIP(hipEventRecord(tm->ev[2 * tm->used++ + 1], st));
    tm->bytes += (double)fs.alg_bytes;
  }
  gemv_sum_kernel<RB><<<G.n2, 256, 0, st>>>(fs.d_n, fs.d_xoff, G.d_items2, fs.d_partial, w, want);
}

}  // namespace

int gemv_rows(int prec) { return prec == P_FP64 ? 128 : prec == P_FP32 ? 256 : 512; }

void gemv_set(const FactorSet& fs, double* w, hipStream_t st, int slot, const int32_t* want) {
  if (fs.count == 0 || slot >= (int)fs.gemv.size()) return;
  if (fs.prec == P_FP64)
    gemv_launch<double>(fs, w, st, slot, want);
  else if (fs.prec == P_FP32)
    gemv_launch<float>(fs, w, st, slot, want);
  else
    gemv_launch<uint16_t>(fs, w, st, slot, want);
  GDSW_HIP(hipGetLastError());
}

void local_solve_set(const FactorSet& fs, double* w, hipStream_t st, int slot, const int32_t* want) {
  if (fs.mode == SOLVE_INVERSE)
    gemv_set(fs, w, st, slot, want);
  else
    trsv_set(fs, w, st, slot, want);
}

}  // namespace gdsw
