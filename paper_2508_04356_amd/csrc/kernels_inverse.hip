// Explicit inverses of the local and coarse matrices (setup).
//
// The preconditioner of eq. (2.2) / (2.5) needs A_i^-1 R_i r for every local
// matrix A_i, and the same for the coarse matrices.  Instead of a forward and
// backward substitution, whose 2 * nblk dependent steps are latency bound on
// a 256-CU device, the setup forms A_i^-1 once (Gauss-Jordan elimination
// without pivoting, in the velocity-first order whose pivots are the pivots
// of the no-pivoting LU), symmetrises it (A_i is symmetric, eq. 2.1) and
// stores it in the precision of the set.  Every apply then streams the same
// n^2 entries per matrix as the triangular solves would, with no dependency
// chain (kernels_gemv.hip, kernels_gemm.hip).
//
// gj_invert: blocked in-place Gauss-Jordan with 64-wide blocks.  Step k
// inverts the pivot block P = A_kk^-1 (one work-group per matrix, in LDS),
// forms T = P A_k* (row panel), updates A_ij -= A_ik T_j for every i, j != k
// (64 x 64 tiles), then sets A_ik <- -A_ik P and A_kj <- T_j.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kernels.h"
#include "vec16.h"

namespace gdsw {
namespace {

constexpr int GB = 64;  // Gauss-Jordan block
typedef double mf64x4 __attribute__((ext_vector_type(4)));

__device__ inline void track_min_pivot(double piv, double& mn) {
  const double a = fabs(piv);
  if (!(a > 0.0) || !isfinite(piv)) {
    mn = 0.0;
  } else if (a < mn) {
    mn = a;
  }
}

// P = A_kk^-1 by Gauss-Jordan without pivoting in LDS; rows and columns
// beyond n are identity.  Writes P (64 x 64, column-major) and A_kk <- P.
__global__ __launch_bounds__(256) void gj_diag_kernel(double* __restrict__ base, const int32_t* __restrict__ N,
                                                      const int32_t* __restrict__ LD,
                                                      const int64_t* __restrict__ OFF, int k,
                                                      double* __restrict__ Pbuf,
                                                      unsigned long long* __restrict__ minpiv) {
  const int f = blockIdx.x;
  const int n = N[f];
  const int k0 = k * GB;
  if (k0 >= n) return;
  const int64_t ld = LD[f];
  double* A = base + OFF[f];
  const int bs = min(GB, n - k0);
  __shared__ double a[GB][GB + 1];
  __shared__ double prow[GB];
  __shared__ double pcol[GB];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < GB * GB; idx += blockDim.x) {
    const int r = idx % GB, c = idx / GB;
    a[r][c] = (r < bs && c < bs) ? A[(int64_t)(k0 + c) * ld + k0 + r] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  double mn = 1.0e308;
  for (int j = 0; j < GB; ++j) {
    const double piv = a[j][j];
    if (tid == 0 && j < bs) track_min_pivot(piv, mn);
    const double p = 1.0 / piv;
    // scaled pivot row and the pivot column, copied so that the update reads
    // values no thread is writing
    if (tid < GB) {
      prow[tid] = tid == j ? p : a[j][tid] * p;
      pcol[tid] = a[tid][j];
    }
    __syncthreads();
    for (int idx = tid; idx < GB * GB; idx += blockDim.x) {
      const int i = idx % GB, c = idx / GB;
      if (i == j) {
        a[i][c] = prow[c];
      } else if (c == j) {
        a[i][c] = -pcol[i] * p;
      } else {
        a[i][c] -= pcol[i] * prow[c];
      }
    }
    __syncthreads();
  }
  double* P = Pbuf + (int64_t)f * GB * GB;
  for (int idx = tid; idx < GB * GB; idx += blockDim.x) {
    const int r = idx % GB, c = idx / GB;
    P[idx] = a[r][c];
    if (r < bs && c < bs) A[(int64_t)(k0 + c) * ld + k0 + r] = a[r][c];
  }
  if (tid == 0) atomicMin(&minpiv[f], (unsigned long long)__double_as_longlong(mn));
}

// 64 x 64 x 64 product in a work-group: acc = X Y with X[r][l] and Y[l][c]
// staged in LDS.  Thread (tx, ty) owns rows tx + 16 a, columns ty + 16 b.
__device__ inline void tile_mm64(const double (*X)[GB + 1], const double (*Y)[GB + 1], int tx, int ty,
                                 double (&acc)[4][4]) {
  for (int l = 0; l < GB; ++l) {
    double av[4], bv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) av[a] = X[tx + 16 * a][l];
#pragma unroll
    for (int b = 0; b < 4; ++b) bv[b] = Y[l][ty + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
  }
}

// T_j = P A_kj for every column tile j != k (T: 64 rows, column-major, ld 64).
__global__ __launch_bounds__(256) void gj_row_kernel(const double* __restrict__ base, const int32_t* __restrict__ N,
                                                     const int32_t* __restrict__ LD,
                                                     const int64_t* __restrict__ OFF, int k,
                                                     const double* __restrict__ Pbuf, double* __restrict__ Tbuf,
                                                     int64_t tstride) {
  const int f = blockIdx.y;
  const int n = N[f];
  const int k0 = k * GB;
  if (k0 >= n) return;
  const int nt = (n + GB - 1) / GB;
  const int j = blockIdx.x;
  if (j >= nt || j == k) return;
  const int c0 = j * GB;
  const int cb = min(GB, n - c0);
  const int bs = min(GB, n - k0);
  const int64_t ld = LD[f];
  const double* A = base + OFF[f];
  const double* P = Pbuf + (int64_t)f * GB * GB;
  __shared__ double Xs[GB][GB + 1];
  __shared__ double Ys[GB][GB + 1];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < GB * GB; idx += 256) {
    const int r = idx % GB, c = idx / GB;
    Xs[r][c] = P[idx];
    Ys[r][c] = (r < bs && c < cb) ? A[(int64_t)(c0 + c) * ld + k0 + r] : 0.0;
  }
  __syncthreads();
  const int tx = tid & 15, ty = tid >> 4;
  double acc[4][4] = {};
  tile_mm64(Xs, Ys, tx, ty, acc);
  double* T = Tbuf + (int64_t)f * tstride;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int c = ty + 16 * b;
    if (c >= cb) continue;
#pragma unroll
    for (int a = 0; a < 4; ++a) T[(int64_t)(c0 + c) * GB + tx + 16 * a] = acc[a][b];
  }
}

// A_ij -= A_ik T_j for every tile with i != k and j != k.
__global__ __launch_bounds__(256) void gj_update_kernel(double* __restrict__ base, const int32_t* __restrict__ N,
                                                        const int32_t* __restrict__ LD,
                                                        const int64_t* __restrict__ OFF, int k,
                                                        const double* __restrict__ Tbuf, int64_t tstride) {
  const int f = blockIdx.y;
  const int n = N[f];
  const int k0 = k * GB;
  if (k0 >= n) return;
  const int nt = (n + GB - 1) / GB;
  const int t = blockIdx.x;
  if (t >= nt * nt) return;
  const int ti = t % nt, tj = t / nt;
  if (ti == k || tj == k) return;
  const int r0 = ti * GB, c0 = tj * GB;
  const int rb = min(GB, n - r0), cb = min(GB, n - c0);
  const int bs = min(GB, n - k0);
  const int64_t ld = LD[f];
  double* A = base + OFF[f];
  const double* T = Tbuf + (int64_t)f * tstride;
  // The 64-deep product runs in two halves of 32 (the same k order), so the
  // staged panels take 33 KB of LDS and four work-groups fit a CU; the
  // tile's own entries are loaded first, their latency overlapping the
  // staging, and the update is written as old - product.
  constexpr int KH = GB / 2;
  __shared__ double Xs[GB][KH + 1];  // [row][l]
  __shared__ double Ys[KH][GB + 1];  // [l][col]
  const int tid = threadIdx.x;
  // 64 x 64 x 64 product on the matrix cores (v_mfma_f64_16x16x4), computed
  // transposed, D = (X Y)^T, so that a lane's results are consecutive rows
  // of the column-major tile: wave w owns the 32 x 32 quadrant (w / 2, w % 2)
  // as 2 x 2 blocks of 16 x 16; lane (i, kq) feeds A[i][kq] = Y[kq][col i]
  // and B[kq][i] = X[row i][kq] of every 4-deep step.  Accumulator register
  // t of a lane: D row kq + 4 t = tile column, D column i = tile row.
  const int lane = tid & 63, wave = tid >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  double cur[2][2][4];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int t4 = 0; t4 < 4; ++t4) {
        const int r = wr + 16 * bi + i, c = wc + 16 * bj + kq + 4 * t4;
        cur[bi][bj][t4] = (r < rb && c < cb) ? A[(int64_t)(c0 + c) * ld + r0 + r] : 0.0;
      }
  mf64x4 acc[2][2];  // [row block][column block]
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = mf64x4{0, 0, 0, 0};
  for (int h = 0; h < 2; ++h) {
    for (int idx = tid; idx < GB * KH; idx += 256) {
      // X: rows fastest (A is column-major); Y: k fastest (T is column-major)
      const int r = idx % GB, l = idx / GB;
      Xs[r][l] = (r < rb && h * KH + l < bs) ? A[(int64_t)(k0 + h * KH + l) * ld + r0 + r] : 0.0;
      const int lk = idx % KH, c = idx / KH;
      Ys[lk][c] = (c < cb && h * KH + lk < bs) ? T[(int64_t)(c0 + c) * GB + h * KH + lk] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int l0 = 0; l0 < KH; l0 += 4) {
      const double x0 = Xs[wr + i][l0 + kq], x1 = Xs[wr + 16 + i][l0 + kq];
      const double y0 = Ys[l0 + kq][wc + i], y1 = Ys[l0 + kq][wc + 16 + i];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(y0, x0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(y1, x0, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(y0, x1, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(y1, x1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi) {
    const int r = wr + 16 * bi + i;
    if (r >= rb) continue;
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int t4 = 0; t4 < 4; ++t4) {
        const int c = wc + 16 * bj + kq + 4 * t4;
        if (c < cb) A[(int64_t)(c0 + c) * ld + r0 + r] = cur[bi][bj][t4] - acc[bi][bj][t4];
      }
  }
}

// Column panel A_ik <- -A_ik P (i != k) and row panel A_kj <- T_j (j != k).
__global__ __launch_bounds__(256) void gj_panel_kernel(double* __restrict__ base, const int32_t* __restrict__ N,
                                                       const int32_t* __restrict__ LD,
                                                       const int64_t* __restrict__ OFF, int k,
                                                       const double* __restrict__ Pbuf,
                                                       const double* __restrict__ Tbuf, int64_t tstride) {
  const int f = blockIdx.y;
  const int n = N[f];
  const int k0 = k * GB;
  if (k0 >= n) return;
  const int nt = (n + GB - 1) / GB;
  const int t = blockIdx.x;
  if (t >= 2 * nt) return;
  const int bs = min(GB, n - k0);
  const int64_t ld = LD[f];
  double* A = base + OFF[f];
  const int tid = threadIdx.x;
  if (t >= nt) {
    const int j = t - nt;
    if (j == k) return;
    const int c0 = j * GB;
    const int cb = min(GB, n - c0);
    const double* T = Tbuf + (int64_t)f * tstride;
    for (int idx = tid; idx < GB * GB; idx += 256) {
      const int r = idx % GB, c = idx / GB;
      if (r < bs && c < cb) A[(int64_t)(c0 + c) * ld + k0 + r] = T[(int64_t)(c0 + c) * GB + r];
    }
    return;
  }
  const int i = t;
  if (i == k) return;
  const int r0 = i * GB;
  const int rb = min(GB, n - r0);
  const double* P = Pbuf + (int64_t)f * GB * GB;
  __shared__ double Xs[GB][GB + 1];
  __shared__ double Ys[GB][GB + 1];
  for (int idx = tid; idx < GB * GB; idx += 256) {
    const int r = idx % GB, c = idx / GB;
    Xs[r][c] = (r < rb && c < bs) ? A[(int64_t)(k0 + c) * ld + r0 + r] : 0.0;
    Ys[r][c] = P[idx];
  }
  __syncthreads();
  const int tx = tid & 15, ty = tid >> 4;
  double acc[4][4] = {};
  tile_mm64(Xs, Ys, tx, ty, acc);
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int c = ty + 16 * b;
    if (c >= bs) continue;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int r = tx + 16 * a;
      if (r < rb) A[(int64_t)(k0 + c) * ld + r0 + r] = -acc[a][b];
    }
  }
}

__global__ void convert_f32_kernel(const double* __restrict__ src, float* __restrict__ dst, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

__global__ void convert_bf16_kernel(const double* __restrict__ src, uint16_t* __restrict__ dst, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = to_bf16((float)src[i]);
}

// M <- (M + M^T) / 2 on the n x n block of every matrix (the inverse of a
// symmetric matrix, freed of the asymmetry left by rounding).  One thread
// per pair (r > c) of a 64 x 64 tile pair.
__global__ void symmetrize_kernel(double* __restrict__ base, const int32_t* __restrict__ N,
                                  const int32_t* __restrict__ LD, const int64_t* __restrict__ OFF) {
  const int f = blockIdx.z;
  const int n = N[f];
  const int r = blockIdx.x * 16 + (threadIdx.x & 15);
  const int c = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (r >= n || c >= n || r <= c) return;
  const int64_t ld = LD[f];
  double* A = base + OFF[f];
  const double a = A[(int64_t)c * ld + r], b = A[(int64_t)r * ld + c];
  const double m = 0.5 * (a + b);
  A[(int64_t)c * ld + r] = m;
  A[(int64_t)r * ld + c] = m;
}

}  // namespace

void gj_invert(const DenseBatch& B, double* Pbuf, double* Tbuf, int64_t tstride, unsigned long long* minpiv,
               hipStream_t st) {
  if (B.count == 0 || B.max_n == 0) return;
  const int nt = (B.max_n + GB - 1) / GB;
  for (int k = 0; k < nt; ++k) {
    gj_diag_kernel<<<B.count, 256, 0, st>>>(B.base, B.n, B.ld, B.off, k, Pbuf, minpiv);
    gj_row_kernel<<<dim3(nt, B.count), 256, 0, st>>>(B.base, B.n, B.ld, B.off, k, Pbuf, Tbuf, tstride);
    gj_update_kernel<<<dim3(nt * nt, B.count), 256, 0, st>>>(B.base, B.n, B.ld, B.off, k, Tbuf, tstride);
    gj_panel_kernel<<<dim3(2 * nt, B.count), 256, 0, st>>>(B.base, B.n, B.ld, B.off, k, Pbuf, Tbuf, tstride);
  }
  GDSW_HIP(hipGetLastError());
}

void convert_store(int prec, const double* src, void* dst, int64_t count, hipStream_t st) {
  if (count == 0) return;
  if (prec == P_FP32)
    convert_f32_kernel<<<4096, 256, 0, st>>>(src, static_cast<float*>(dst), count);
  else if (prec == P_BF16)
    convert_bf16_kernel<<<4096, 256, 0, st>>>(src, static_cast<uint16_t*>(dst), count);
  GDSW_HIP(hipGetLastError());
}

void symmetrize(const DenseBatch& B, hipStream_t st) {
  if (B.count == 0 || B.max_n == 0) return;
  const int t = (B.max_n + 15) / 16;
  symmetrize_kernel<<<dim3(t, t, B.count), 256, 0, st>>>(B.base, B.n, B.ld, B.off);
  GDSW_HIP(hipGetLastError());
}

}  // namespace gdsw
