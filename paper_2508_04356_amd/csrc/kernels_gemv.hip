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

// Item (f, r0, c0, p): rows [r0, r0 + 64 E) and columns [c0, c0 + CW) of
// matrix D[f]; partial[p * 64 E + row] = sum over those columns of M x.
template <typename T, int NW, int CW>
__global__ __launch_bounds__(64 * NW) void gemv_part_kernel(const GemvDesc* __restrict__ D,
                                                           const int4* __restrict__ items,
                                                           double* __restrict__ partial,
                                                           const int32_t* __restrict__ want) {
  using AT = typename VecW<T>::acc;
  constexpr int E = VecW<T>::W;
  constexpr int RB = 64 * E;
  __shared__ AT xs[CW];
  __shared__ AT red[NW][RB];
  const int4 item = items[blockIdx.x];
  const int f = item.x, r0 = item.y, c0 = item.z, p = item.w;
  if (want && !want[f]) return;  // uniform per work-group
  const GemvDesc d = D[f];
  const int n = d.n;
  const int64_t np = d.np;
  const int ncols = min(CW, n - c0);
  const int tid = threadIdx.x;
  const auto* x = as_global<double>(d.x + c0);
  for (int i = tid; i < CW; i += 64 * NW) xs[i] = i < ncols ? (AT)x[i] : (AT)0;
  const int lane = tid & 63, wave = tid >> 6;
  const int rr = r0 + lane * E;
  const bool active = rr < n;
  const T* col = static_cast<const T*>(d.a) + (int64_t)c0 * np + rr;
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

// Item (f, r0, p0, cnt): x_f[r0 + t] = sum_{q < cnt} partial[(p0 + q) * RB + t].
template <int RB>
__global__ __launch_bounds__(256) void gemv_sum_kernel(const GemvDesc* __restrict__ D,
                                                       const int4* __restrict__ items,
                                                       const double* __restrict__ partial,
                                                       const int32_t* __restrict__ want) {
  const int4 item = items[blockIdx.x];
  const int f = item.x, r0 = item.y, p0 = item.z, cnt = item.w;
  if (want && !want[f]) return;
  const int n = D[f].n;
  double* x = D[f].x;
  for (int t = threadIdx.x; t < RB; t += 256) {
    if (r0 + t >= n) break;
    double s = 0.0;
    for (int q = 0; q < cnt; ++q) s += partial[(int64_t)(p0 + q) * RB + t];
    x[r0 + t] = s;
  }
}

template <typename T>
void gemv_launch(const GemvDesc* desc, const FactorSet::GemvPlan& G, int cw, double* partial, hipStream_t st,
                 const int32_t* want, KernelTimer* tm, double bytes) {
  if (G.n1 == 0) return;
  constexpr int RB = 64 * VecW<T>::W;
  constexpr int NW = GDSW_GEMV_NW;
  auto* k = cw == 512 ? gemv_part_kernel<T, NW, 512>
            : cw == 2048 ? gemv_part_kernel<T, NW, 2048> : gemv_part_kernel<T, NW, 1024>;
  timed_launch(tm, bytes, k, dim3(G.n1), dim3(64 * NW), st, desc, G.d_items1, partial, want);
  gemv_sum_kernel<RB><<<G.n2, 256, 0, st>>>(desc, G.d_items2, partial, want);
}

}  // namespace

int gemv_rows(int prec) { return prec == P_FP64 ? 128 : prec == P_FP32 ? 256 : 512; }

void gemv_desc_launch(int prec, const GemvDesc* desc, const FactorSet::GemvPlan& G, int cw, double* partial,
                      hipStream_t st, const int32_t* want, KernelTimer* tm, double bytes) {
  if (cw != 512 && cw != 1024 && cw != 2048) throw StatusError{1, "column chunk must be 512, 1024 or 2048"};
  if (tm && (!tm->on || tm->used >= KernelTimer::CAP)) tm = nullptr;
  if (prec == P_FP64)
    gemv_launch<double>(desc, G, cw, partial, st, want, tm, bytes);
  else if (prec == P_FP32)
    gemv_launch<float>(desc, G, cw, partial, st, want, tm, bytes);
  else
    gemv_launch<uint16_t>(desc, G, cw, partial, st, want, tm, bytes);
  GDSW_HIP(hipGetLastError());
}

void gemv_set(const FactorSet& fs, double* w, hipStream_t st, int slot, const int32_t* want) {
  (void)w;  // the descriptors address the set's own work vector segments
  if (fs.count == 0 || slot >= (int)fs.gemv.size()) return;
  if (!fs.d_desc) throw StatusError{5, "inverse set used before its descriptors were built"};
  gemv_desc_launch(fs.prec, fs.d_desc, fs.gemv[slot], fs.cw, fs.d_partial, st, want,
                   slot == 0 ? fs.timer : nullptr, (double)fs.alg_bytes);
}

void local_solve_set(const FactorSet& fs, double* w, hipStream_t st, int slot, const int32_t* want) {
  if (fs.mode == SOLVE_INVERSE)
    gemv_set(fs, w, st, slot, want);
  else if (fs.mode == SOLVE_SYM)
    symv_set(fs, w, st, slot, want);
  else
    trsv_set(fs, w, st, slot, want);
}

}  // namespace gdsw
