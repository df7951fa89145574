// Dense factorisation and triangular-solve kernels for the local and coarse
// problems of eqs. (2.2)-(2.5) on gfx950.
//
// * lu_nopiv: blocked right-looking LU without pivoting (64-wide blocks):
//   diagonal block in LDS, row/column panels by triangular solves in LDS,
//   trailing update as a 64x64-tile FP64 product.  No pivoting is needed for
//   the monolithic saddle-point matrices ordered velocity first: the velocity
//   block is SPD and the Schur complement is negative definite.
// * factor_finalize: inverts the diagonal tiles of L and U and scales every
//   off-diagonal tile by its block row's diagonal inverse, so that
//     L y = r  becomes  y_J = L_JJ^-1 r_J - sum_{K<J} (L_JJ^-1 L_JK) y_K,
//     U x = y  becomes  x_J = U_JJ^-1 y_J - sum_{K>J} (U_JJ^-1 U_JK) x_K,
//   then converts the factors to the storage precision.
// * trsv_set: the forward-backward solve as a sequence of launches in which
//   every work-group streams exactly one tile (16-byte loads issued first)
//   and updates one block of its factor's vector.  Factors are interleaved
//   with phase offsets so that every launch moves a similar number of bytes.
//   No work-group ever waits on another; every reduction has a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "kernels.h"
#include "vec16.h"

namespace gdsw {
namespace {

constexpr int LB = 64;  // LU block

__device__ inline void track_pivot(double piv, double& mn) {
  const double a = fabs(piv);
  if (!(a > 0.0) || !isfinite(piv)) {
    mn = 0.0;
  } else if (a < mn) {
    mn = a;
  }
}

__global__ __launch_bounds__(256) void lu_diag_kernel(double* __restrict__ base, const int32_t* __restrict__ N,
                                                      const int32_t* __restrict__ LD,
                                                      const int64_t* __restrict__ OFF, int k,
                                                      unsigned long long* __restrict__ minpiv) {
  const int f = blockIdx.x;
  const int n = N[f];
  const int k0 = k * LB;
  if (k0 >= n) return;
  const int64_t ld = LD[f];
  double* A = base + OFF[f];
  const int bs = min(LB, n - k0);
  __shared__ double a[LB][LB + 1];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < bs * bs; idx += blockDim.x) {
    const int r = idx % bs, c = idx / bs;
    a[r][c] = A[(int64_t)(k0 + c) * ld + k0 + r];
  }
  __syncthreads();
  double mn = 1.0e308;
  for (int j = 0; j < bs; ++j) {
    const double piv = a[j][j];
    if (tid == 0) track_pivot(piv, mn);
    for (int i = j + 1 + tid; i < bs; i += blockDim.x) a[i][j] /= piv;
    __syncthreads();
    const int rem = bs - j - 1;
    for (int idx = tid; idx < rem * rem; idx += blockDim.x) {
      const int i = j + 1 + idx % rem, c = j + 1 + idx / rem;
      a[i][c] -= a[i][j] * a[j][c];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < bs * bs; idx += blockDim.x) {
    const int r = idx % bs, c = idx / bs;
    A[(int64_t)(k0 + c) * ld + k0 + r] = a[r][c];
  }
  if (tid == 0) atomicMin(&minpiv[f], (unsigned long long)__double_as_longlong(mn));
}

// Row panel (L21 = A21 U11^-1) and column panel (U12 = L11^-1 A12) tiles.
__global__ __launch_bounds__(64) void lu_panel_kernel(double* __restrict__ base, const int32_t* __restrict__ N,
                                                     const int32_t* __restrict__ LD,
                                                     const int64_t* __restrict__ OFF, int k) {
  const int f = blockIdx.y;
  const int n = N[f];
  const int k0 = k * LB;
  if (k0 + LB >= n) return;
  const int nrem = (n - k0 - LB + LB - 1) / LB;
  const int t = blockIdx.x;
  if (t >= 2 * nrem) return;
  const int64_t ld = LD[f];
  double* A = base + OFF[f];
  __shared__ double D[LB][LB + 1];
  __shared__ double T[LB][LB + 1];
  const int tid = threadIdx.x;
  for (int c = 0; c < LB; ++c) D[tid][c] = A[(int64_t)(k0 + c) * ld + k0 + tid];
  if (t < nrem) {
    const int r0 = k0 + LB + t * LB;
    const int rb = min(LB, n - r0);
    for (int c = 0; c < LB; ++c) T[tid][c] = tid < rb ? A[(int64_t)(k0 + c) * ld + r0 + tid] : 0.0;
    __syncthreads();
    if (tid < rb) {
      for (int j = 0; j < LB; ++j) {
        double s = T[tid][j];
        for (int l = 0; l < j; ++l) s -= T[tid][l] * D[l][j];
        T[tid][j] = s / D[j][j];
      }
    }
    __syncthreads();
    if (tid < rb)
      for (int c = 0; c < LB; ++c) A[(int64_t)(k0 + c) * ld + r0 + tid] = T[tid][c];
  } else {
    const int c0 = k0 + LB + (t - nrem) * LB;
    const int cb = min(LB, n - c0);
    for (int c = 0; c < cb; ++c) T[tid][c] = A[(int64_t)(c0 + c) * ld + k0 + tid];
    __syncthreads();
    if (tid < cb) {
      for (int j = 0; j < LB; ++j) {
        double s = T[j][tid];
        for (int l = 0; l < j; ++l) s -= D[j][l] * T[l][tid];
        T[j][tid] = s;
      }
    }
    __syncthreads();
    for (int c = 0; c < cb; ++c) A[(int64_t)(c0 + c) * ld + k0 + tid] = T[tid][c];
  }
}

// Trailing update A22 -= L21 U12, one 64x64 tile per work-group.
__global__ __launch_bounds__(256) void lu_update_kernel(double* __restrict__ base, const int32_t* __restrict__ N,
                                                       const int32_t* __restrict__ LD,
                                                       const int64_t* __restrict__ OFF, int k) {
  const int f = blockIdx.y;
  const int n = N[f];
  const int k0 = k * LB;
  const int s0 = k0 + LB;
  if (s0 >= n) return;
  const int nt = (n - s0 + LB - 1) / LB;
  const int t = blockIdx.x;
  if (t >= nt * nt) return;
  const int ti = t % nt, tj = t / nt;
  const int r0 = s0 + ti * LB, c0 = s0 + tj * LB;
  const int rb = min(LB, n - r0), cb = min(LB, n - c0);
  const int64_t ld = LD[f];
  double* A = base + OFF[f];
  // The tile's own entries are loaded first (their latency overlaps the
  // staging) and the update is written as old - product; the 64-deep product
  // runs in two halves of 32 (l ascending, as in one pass), so the staged
  // panels take 33 KB of LDS and four work-groups fit a CU.
  constexpr int KH = LB / 2;
  __shared__ double Ls[LB][KH + 1];  // [row][l]
  __shared__ double Us[KH][LB + 1];  // [l][col]
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  double cur[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int r = tx + 16 * a, c = ty + 16 * b;
      cur[a][b] = (r < rb && c < cb) ? A[(int64_t)(c0 + c) * ld + r0 + r] : 0.0;
    }
  double acc[4][4] = {};
  for (int h = 0; h < 2; ++h) {
    for (int idx = tid; idx < LB * KH; idx += 256) {
      // L panel: rows fastest; U panel: k fastest (both column-major)
      const int r = idx % LB, l = idx / LB;
      Ls[r][l] = r < rb ? A[(int64_t)(k0 + h * KH + l) * ld + r0 + r] : 0.0;
      const int lk = idx % KH, c = idx / KH;
      Us[lk][c] = c < cb ? A[(int64_t)(c0 + c) * ld + k0 + h * KH + lk] : 0.0;
    }
    __syncthreads();
    for (int l = 0; l < KH; ++l) {
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = Ls[tx + 16 * a][l];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Us[l][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int c = ty + 16 * b;
    if (c >= cb) continue;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int r = tx + 16 * a;
      if (r < rb) A[(int64_t)(c0 + c) * ld + r0 + r] = cur[a][b] - acc[a][b];
    }
  }
}

// Forward (unit L) and backward (U) substitution, column oriented, with
// the right-hand sides resident in LDS.
__global__ __launch_bounds__(256) void lu_solve_multi_kernel(const double* __restrict__ base,
                                                            const int32_t* __restrict__ N,
                                                            const int32_t* __restrict__ LD,
                                                            const int64_t* __restrict__ OFF,
                                                            double* __restrict__ rhs,
                                                            const int64_t* __restrict__ roff,
                                                            const int32_t* __restrict__ nrhs, int rg) {
  const int f = blockIdx.y;
  const int n = N[f];
  const int nr = nrhs[f];
  const int c0 = blockIdx.x * rg;
  if (c0 >= nr || n == 0) return;
  const int nc = min(rg, nr - c0);
  const int64_t ld = LD[f];
  const double* A = base + OFF[f];
  double* R = rhs + roff[f] + (int64_t)c0 * n;
  extern __shared__ double b[];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < nc * n; idx += blockDim.x) b[idx] = R[idx];
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    for (int r = j + 1 + tid; r < n; r += blockDim.x) {
      const double l = A[(int64_t)j * ld + r];
      for (int c = 0; c < nc; ++c) b[c * n + r] -= l * b[c * n + j];
    }
    __syncthreads();
  }
  for (int j = n - 1; j >= 0; --j) {
    if (tid < nc) b[tid * n + j] /= A[(int64_t)j * ld + j];
    __syncthreads();
    for (int r = tid; r < j; r += blockDim.x) {
      const double u = A[(int64_t)j * ld + r];
      for (int c = 0; c < nc; ++c) b[c * n + r] -= u * b[c * n + j];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < nc * n; idx += blockDim.x) R[idx] = b[idx];
}

// Inverses of the diagonal tiles: strictly lower part holds (unit L)^-1,
// upper part U^-1.  Rows/columns beyond n are treated as identity.
template <typename DT>
__global__ __launch_bounds__(256) void dinv_kernel(const double* __restrict__ lu, const int32_t* __restrict__ N,
                                                  const int32_t* __restrict__ NP,
                                                  const int64_t* __restrict__ OFF,
                                                  const int32_t* __restrict__ NBLK, DT* __restrict__ dinv,
                                                  const int64_t* __restrict__ DOFF, int nb) {
  const int f = blockIdx.y;
  const int s = blockIdx.x;
  if (s >= NBLK[f]) return;
  const int n = N[f];
  const int64_t np = NP[f];
  const double* A = lu + OFF[f];
  const int o = s * nb;
  extern __shared__ double t[];
  double* colbuf = t + nb * (nb + 1);
  const int P = nb + 1;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < nb * nb; idx += blockDim.x) {
    const int r = idx % nb, c = idx / nb;
    double v;
    if (o + r < n && o + c < n)
      v = A[(int64_t)(o + c) * np + o + r];
    else
      v = (r == c) ? 1.0 : 0.0;
    t[c * P + r] = v;
  }
  __syncthreads();
  for (int j = nb - 2; j >= 0; --j) {
    for (int r = tid; r < nb; r += blockDim.x) colbuf[r] = t[j * P + r];
    __syncthreads();
    for (int i = j + 1 + tid; i < nb; i += blockDim.x) {
      double acc = colbuf[i];
      for (int kk = j + 1; kk < i; ++kk) acc += t[kk * P + i] * colbuf[kk];
      t[j * P + i] = -acc;
    }
    __syncthreads();
  }
  for (int j = 0; j < nb; ++j) {
    for (int r = tid; r <= j; r += blockDim.x) colbuf[r] = t[j * P + r];
    __syncthreads();
    const double dj = 1.0 / colbuf[j];
    for (int i = tid; i <= j; i += blockDim.x) {
      if (i == j) {
        t[j * P + j] = dj;
      } else {
        double acc = 0.0;
        for (int kk = i; kk < j; ++kk) acc += t[kk * P + i] * colbuf[kk];
        t[j * P + i] = -acc * dj;
      }
    }
    __syncthreads();
  }
  DT* out = dinv + DOFF[f] + (int64_t)s * nb * nb;
  for (int idx = tid; idx < nb * nb; idx += blockDim.x) {
    const int r = idx % nb, c = idx / nb;
    out[idx] = (DT)t[c * P + r];
  }
}

__device__ inline uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__global__ void convert_kernel_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}
__global__ void convert_kernel_bf16(const double* __restrict__ src, uint16_t* __restrict__ dst, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = f2bf((float)src[i]);
}

// ---- blocked triangular solve ---------------------------------------------

// part[(wave * GPL + g) * NB + row] = sum over this lane's columns of A[row, c] v[c]
// MODE 0: full tile, 1: strictly lower (c < row), 2: upper (c >= row).
// The tile is loaded into registers first; v (NB entries at vsrc) and the
// current values (NB entries at csrc) are staged in LDS meanwhile.
template <typename T, int NB, int MODE, int NW = 4>
__device__ inline void tile_gemv_split(const T* __restrict__ A, int64_t ld, const double* __restrict__ vsrc,
                                       const double* __restrict__ csrc, double* vbuf, double* cur, int row_lim,
                                       int col_lim, typename VecW<T>::acc* part) {
  using AT = typename VecW<T>::acc;
  constexpr int W = VecW<T>::W;
  constexpr int LPC = NB / W;
  constexpr int GPL = 64 / LPC;
  constexpr int CPW = NB / NW;
  constexpr int IT = CPW / GPL;
  static_assert(GPL >= 1 && IT >= 1, "tile shape");
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int g = lane / LPC, rr = (lane % LPC) * W;
  AT a[IT][W];
  const bool rows_ok = rr < row_lim;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int c = wave * CPW + it * GPL + g;
    // triangular modes load only the columns this lane's rows use
    const bool needed = MODE == 0 || (MODE == 1 && c < rr + W - 1) || (MODE == 2 && c >= rr);
    if (rows_ok && c < col_lim && needed) {
      load16(A + (int64_t)c * ld + rr, a[it]);
    } else {
#pragma unroll
      for (int e = 0; e < W; ++e) a[it][e] = 0;
    }
  }
  if (tid < NB) {
    vbuf[tid] = vsrc[tid];
    cur[tid] = csrc[tid];
  }
  __syncthreads();
  AT acc[W];
#pragma unroll
  for (int e = 0; e < W; ++e) acc[e] = 0;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int c = wave * CPW + it * GPL + g;
    const AT vc = (AT)vbuf[c];
#pragma unroll
    for (int e = 0; e < W; ++e) {
      const bool use = MODE == 0 || (MODE == 1 && c < rr + e) || (MODE == 2 && c >= rr + e);
      if (use) acc[e] = fma(a[it][e], vc, acc[e]);
    }
  }
#pragma unroll
  for (int e = 0; e < W; ++e) part[(wave * GPL + g) * NB + rr + e] = acc[e];
  __syncthreads();
}

template <typename T, int NB, int NW = 4>
__device__ inline typename VecW<T>::acc part_sum(const typename VecW<T>::acc* part, int row) {
  constexpr int GPL = 64 / (NB / VecW<T>::W);
  typename VecW<T>::acc s = 0;
#pragma unroll
  for (int q = 0; q < NW * GPL; ++q) s += part[q * NB + row];
  return s;
}

template <typename T>
struct DinvT {
  using type = float;
};
template <>
struct DinvT<double> {
  using type = double;
};

// One launch of the blocked solve.  Every work item is one tile:
//   mode 0:  x_J -= T_{J,K} x_K   (T = L_JJ^-1 L_JK below, U_JJ^-1 U_JK above the diagonal)
//   mode 1:  x_J  = L_JJ^-1 x_J   (start of the forward sweep)
//   mode 2:  x_J  = U_JJ^-1 x_J   (start of the backward sweep)
// The tile loads are issued before anything else, so a work-group's only
// serial dependence is one tile read.
template <typename T, int NB, int NW>
__global__ __launch_bounds__(64 * NW) void trsv_step_kernel(const T* __restrict__ store,
                                                       const typename DinvT<T>::type* __restrict__ dinv,
                                                       const int32_t* __restrict__ N, const int32_t* __restrict__ NP,
                                                       const int64_t* __restrict__ OFF,
                                                       const int64_t* __restrict__ DOFF,
                                                       const int64_t* __restrict__ XOFF,
                                                       const int4* __restrict__ items, double* __restrict__ w,
                                                       const int32_t* __restrict__ want) {
  using AT = typename VecW<T>::acc;
  using DT = typename DinvT<T>::type;
  using ADT = typename VecW<DT>::acc;
  constexpr int GPLm = 64 / (NB / VecW<T>::W);
  constexpr int GPLd = 64 / (NB / VecW<DT>::W);
  constexpr int PSZ = NW * (GPLm > GPLd ? GPLm : GPLd) * NB;
  __shared__ double vbuf[NB];
  __shared__ double cur[NB];
  __shared__ double part_d[PSZ];
  const int4 item = items[blockIdx.x];
  const int f = item.x, J = item.y, K = item.z, mode = item.w;
  if (want && !want[f]) return;  // uniform per work-group: factor not selected for this pass
  const int n = N[f];
  const int64_t np = NP[f];
  double* x = w + XOFF[f];
  const int tid = threadIdx.x;
  const int r0 = J * NB;
  if (mode == 0) {
    const int c0 = K * NB;
    AT* part = reinterpret_cast<AT*>(part_d);
    tile_gemv_split<T, NB, 0, NW>(store + OFF[f] + (int64_t)c0 * np + r0, np, x + c0, x + r0, vbuf, cur,
                                  min(NB, n - r0), min(NB, n - c0), part);
    if (tid < NB) x[r0 + tid] = cur[tid] - (double)part_sum<T, NB, NW>(part, tid);
  } else {
    ADT* part = reinterpret_cast<ADT*>(part_d);
    const DT* D = dinv + DOFF[f] + (int64_t)J * NB * NB;
    if (mode == 1) {
      tile_gemv_split<DT, NB, 1, NW>(D, NB, x + r0, x + r0, vbuf, cur, NB, NB, part);
      if (tid < NB) x[r0 + tid] = cur[tid] + (double)part_sum<DT, NB, NW>(part, tid);
    } else {
      tile_gemv_split<DT, NB, 2, NW>(D, NB, x + r0, x + r0, vbuf, cur, NB, NB, part);
      if (tid < NB) x[r0 + tid] = (double)part_sum<DT, NB, NW>(part, tid);
    }
  }
}

template <typename T, int NB, int NW>
void trsv_launch(const FactorSet& fs, double* w, hipStream_t st, int slot, const int32_t* want) {
  using DT = typename DinvT<T>::type;
  const T* store = static_cast<const T*>(fs.store);
  const DT* dinv = static_cast<const DT*>(fs.dinv);
  const FactorSet::Schedule& S = fs.sched[slot];
  for (size_t g = 0; g + 1 < S.step_start.size(); ++g) {
    const int cnt = S.step_start[g + 1] - S.step_start[g];
    if (cnt == 0) continue;
    KernelTimer* tm =
        (slot == 0 && fs.timer && fs.timer->on && fs.timer->used < KernelTimer::CAP) ? fs.timer : nullptr;
    // bytes: the average share of one sweep step
    timed_launch(tm, (double)fs.alg_bytes / (double)fs.launches(), trsv_step_kernel<T, NB, NW>, dim3(cnt),
                 dim3(64 * NW), st, store, dinv, fs.d_n, fs.d_npad, fs.d_off, fs.d_doff, fs.d_xoff,
                 S.d_items + S.step_start[g], w, want);
  }
}

// Left-multiplies every off-diagonal tile of block row J by the inverse of
// the diagonal block: L_JK <- L_JJ^-1 L_JK (J > K), U_JK <- U_JJ^-1 U_JK
// (J < K).  One work-group per tile, the tile resident in LDS.
template <int NBT>
__global__ __launch_bounds__(256) void row_scale_kernel(double* __restrict__ lu, const int32_t* __restrict__ NP,
                                                       const int64_t* __restrict__ OFF,
                                                       const int32_t* __restrict__ NBLK,
                                                       const double* __restrict__ dinv,
                                                       const int64_t* __restrict__ DOFF, int64_t dbase) {
  constexpr int nb = NBT;
  const int f = blockIdx.y;
  const int nblk = NBLK[f];
  const int J = blockIdx.x % nblk, K = blockIdx.x / nblk;
  if (K >= nblk || J == K) return;
  const int64_t np = NP[f];
  double* T = lu + OFF[f] + (int64_t)K * nb * np + (int64_t)J * nb;
  const double* S = dinv + (DOFF[f] - dbase) + (int64_t)J * nb * nb;
  extern __shared__ double t[];
  const int P = nb + 1;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < nb * nb; idx += blockDim.x) {
    const int r = idx % nb, c = idx / nb;
    t[c * P + r] = T[(int64_t)c * np + r];
  }
  __syncthreads();
  const bool lower = J > K;
  // each thread: 8 rows x 8 columns (nb = 128) or 4 x 4 (nb = 64)
  constexpr int RB = nb / 16;
  const int tr = tid % 16, tc = tid / 16;
  double acc[RB][RB];
#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int b = 0; b < RB; ++b) acc[a][b] = 0.0;
  for (int k = 0; k < nb; ++k) {
    double sv[RB], tv[RB];
#pragma unroll
    for (int a = 0; a < RB; ++a) {
      const int r = tr * RB + a;
      const double sk = S[(int64_t)k * nb + r];
      sv[a] = lower ? (k < r ? sk : (k == r ? 1.0 : 0.0)) : (k >= r ? sk : 0.0);
    }
#pragma unroll
    for (int b = 0; b < RB; ++b) tv[b] = t[(tc * RB + b) * P + k];
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
      for (int b = 0; b < RB; ++b) acc[a][b] = fma(sv[a], tv[b], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int b = 0; b < RB; ++b) T[(int64_t)(tc * RB + b) * np + tr * RB + a] = acc[a][b];
}

// ---- batched FP64 GEMM (setup only) ----------------------------------------
__global__ __launch_bounds__(256) void gemm_kernel(const GemmDesc* __restrict__ D, double alpha, double beta) {
  const GemmDesc d = D[blockIdx.z];
  const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  if (r0 >= d.m || c0 >= d.n) return;
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  // the next 16-deep chunk of both operands is loaded into registers while
  // the current one is multiplied (op(A) along its rows, or its k when
  // transposed; B along k), then stored to LDS
  double pa[4], pb[4];
  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int i = d.transA ? idx / 16 : idx % 64, kk = d.transA ? idx % 16 : idx / 64;
      const int r = r0 + i, kx = k0 + kk;
      pa[q] = (r < d.m && kx < d.k) ? (d.transA ? d.A[(int64_t)r * d.lda + kx] : d.A[(int64_t)kx * d.lda + r]) : 0.0;
      const int ib = idx / 16, kb = idx % 16;
      const int c = c0 + ib, ky = k0 + kb;
      pb[q] = (c < d.n && ky < d.k) ? d.B[(int64_t)c * d.ldb + ky] : 0.0;
    }
  };
  double acc[4][4] = {};
  load_chunk(0);
  for (int k0 = 0; k0 < d.k; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      As[d.transA ? idx % 16 : idx / 64][d.transA ? idx / 16 : idx % 64] = pa[q];
      Bs[idx % 16][idx / 16] = pb[q];
    }
    __syncthreads();
    if (k0 + 16 < d.k) load_chunk(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[kk][tx + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int c = c0 + ty + 16 * b;
    if (c >= d.n) continue;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int r = r0 + tx + 16 * a;
      if (r >= d.m) continue;
      double* cp = d.C + (int64_t)c * d.ldc + r;
      *cp = alpha * acc[a][b] + (beta == 0.0 ? 0.0 : beta * *cp);
    }
  }
}

}  // namespace

double minpiv_decode(unsigned long long bits) {
  double d;
  std::memcpy(&d, &bits, sizeof d);
  return d;
}

void lu_nopiv(const DenseBatch& B, unsigned long long* minpiv, hipStream_t st) {
  if (B.count == 0 || B.max_n == 0) return;
  const int nblk = (B.max_n + LB - 1) / LB;
  for (int k = 0; k < nblk; ++k) {
    lu_diag_kernel<<<B.count, 256, 0, st>>>(B.base, B.n, B.ld, B.off, k, minpiv);
    const int rem = nblk - k - 1;
    if (rem <= 0) continue;
    lu_panel_kernel<<<dim3(2 * rem, B.count), 64, 0, st>>>(B.base, B.n, B.ld, B.off, k);
    lu_update_kernel<<<dim3(rem * rem, B.count), 256, 0, st>>>(B.base, B.n, B.ld, B.off, k);
  }
  GDSW_HIP(hipGetLastError());
}

void lu_solve_multi(const DenseBatch& B, double* rhs, const int64_t* roff, const int32_t* nrhs, int max_nrhs,
                    hipStream_t st) {
  if (B.count == 0 || max_nrhs == 0 || B.max_n == 0) return;
  int rg = (int)std::max<int64_t>(1, (48 * 1024) / (8 * (int64_t)B.max_n));
  rg = std::min(rg, 8);
  const size_t shm = (size_t)rg * B.max_n * sizeof(double);
  if (shm > 160 * 1024) throw StatusError{6, "local interior block too large for the LDS solve"};
  GDSW_HIP(hipFuncSetAttribute((const void*)lu_solve_multi_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)shm));
  const int groups = (max_nrhs + rg - 1) / rg;
  lu_solve_multi_kernel<<<dim3(groups, B.count), 256, shm, st>>>(B.base, B.n, B.ld, B.off, rhs, roff, nrhs, rg);
  GDSW_HIP(hipGetLastError());
}

__global__ void convert_dinv_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

void factor_finalize(FactorSet& fs, double* lu, int64_t dbase, hipStream_t st) {
  if (fs.count == 0) return;
  const size_t shm = ((size_t)fs.nb * (fs.nb + 1) + fs.nb) * sizeof(double);
  double* d64 = nullptr;
  if (fs.prec == P_FP64) {
    d64 = static_cast<double*>(fs.dinv) + dbase;
  } else {
    GDSW_HIP(hipStreamSynchronize(st));
    GDSW_HIP(hipMalloc((void**)&d64, (size_t)fs.total_dinv * sizeof(double)));
  }
  // diagonal-tile inverses (FP64), written relative to dbase
  GDSW_HIP(hipFuncSetAttribute((const void*)dinv_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)shm));
  dinv_kernel<double><<<dim3(fs.max_nblk, fs.count), 256, shm, st>>>(lu, fs.d_n, fs.d_npad, fs.d_off, fs.d_nblk,
                                                                    d64 - dbase, fs.d_doff, fs.nb);
  // row scaling of the off-diagonal tiles
  const size_t shm2 = (size_t)fs.nb * (fs.nb + 1) * sizeof(double);
  const dim3 grid(fs.max_nblk * fs.max_nblk, fs.count);
  if (fs.nb == 128) {
    GDSW_HIP(hipFuncSetAttribute((const void*)row_scale_kernel<128>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)shm2));
    row_scale_kernel<128><<<grid, 256, shm2, st>>>(lu, fs.d_npad, fs.d_off, fs.d_nblk, d64, fs.d_doff, dbase);
  } else {
    GDSW_HIP(hipFuncSetAttribute((const void*)row_scale_kernel<64>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)shm2));
    row_scale_kernel<64><<<grid, 256, shm2, st>>>(lu, fs.d_npad, fs.d_off, fs.d_nblk, d64, fs.d_doff, dbase);
  }
  if (fs.prec != P_FP64) {
    const int blocks = 4096;
    convert_dinv_f32<<<blocks, 256, 0, st>>>(d64, static_cast<float*>(fs.dinv) + dbase, fs.total_dinv);
    if (fs.prec == P_FP32)
      convert_kernel_f32<<<blocks, 256, 0, st>>>(lu, static_cast<float*>(fs.store), fs.total_elems);
    else
      convert_kernel_bf16<<<blocks, 256, 0, st>>>(lu, static_cast<uint16_t*>(fs.store), fs.total_elems);
    GDSW_HIP(hipStreamSynchronize(st));
    GDSW_HIP(hipFree(d64));
  }
  GDSW_HIP(hipGetLastError());
}

void trsv_set(const FactorSet& fs, double* w, hipStream_t st, int slot, const int32_t* want) {
  if (fs.count == 0 || slot >= (int)fs.sched.size()) return;
  const bool w8 = fs.waves == 8;
  if (fs.nb == 128) {
    if (fs.prec == P_FP64) w8 ? trsv_launch<double, 128, 8>(fs, w, st, slot, want) : trsv_launch<double, 128, 4>(fs, w, st, slot, want);
    else if (fs.prec == P_FP32) w8 ? trsv_launch<float, 128, 8>(fs, w, st, slot, want) : trsv_launch<float, 128, 4>(fs, w, st, slot, want);
    else w8 ? trsv_launch<uint16_t, 128, 8>(fs, w, st, slot, want) : trsv_launch<uint16_t, 128, 4>(fs, w, st, slot, want);
  } else {
    if (fs.prec == P_FP64) trsv_launch<double, 64, 4>(fs, w, st, slot, want);
    else if (fs.prec == P_FP32) trsv_launch<float, 64, 4>(fs, w, st, slot, want);
    else trsv_launch<uint16_t, 64, 4>(fs, w, st, slot, want);
  }
  GDSW_HIP(hipGetLastError());
}

void gemm_batched(const GemmDesc* d_desc, int count, int max_m, int max_n, double alpha, double beta,
                  hipStream_t st) {
  if (count == 0 || max_m == 0 || max_n == 0) return;
  dim3 grid((max_m + 63) / 64, (max_n + 63) / 64, count);
  gemm_kernel<<<grid, 256, 0, st>>>(d_desc, alpha, beta);
  GDSW_HIP(hipGetLastError());
}

}  // namespace gdsw
