// Several right-hand sides at once: vector kernels on the interleaved layout.
//
// A block of K <= 32 vectors of length n is stored interleaved: entry (d, j)
// at x[d * K + j], so that the K values of one DOF are contiguous and every
// kernel below reads and writes whole rows of K values.  The ABI's
// column-major blocks are converted at entry and exit (tiled transposes).
// Reductions run in a fixed order per right-hand side, as in the single
// vector kernels, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "kernels_multi.h"

namespace gdsw {
namespace {

inline int grid_for(int64_t n, int bs = 256, int cap = 65536) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (n + bs - 1) / bs));
}

// column-major (ld) <-> interleaved (K), 64 rows x K columns per block via LDS
__global__ __launch_bounds__(256) void cm_to_il_kernel(int64_t n, int K, const double* __restrict__ src, int64_t ld,
                                                       double* __restrict__ dst) {
  __shared__ double t[32][65];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * K; e += 256) {
    const int r = e % 64, j = e / 64;
    t[j][r] = r0 + r < n ? src[(int64_t)j * ld + r0 + r] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * K; e += 256) {
    const int j = e % K, r = e / K;
    if (r0 + r < n) dst[(r0 + r) * K + j] = t[j][r];
  }
}

__global__ __launch_bounds__(256) void il_to_cm_kernel(int64_t n, int K, const double* __restrict__ src,
                                                       double* __restrict__ dst, int64_t ld) {
  __shared__ double t[32][65];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * K; e += 256) {
    const int j = e % K, r = e / K;
    t[j][r] = r0 + r < n ? src[(r0 + r) * K + j] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * K; e += 256) {
    const int r = e % 64, j = e / 64;
    if (r0 + r < n) dst[(int64_t)j * ld + r0 + r] = t[j][r];
  }
}

// w[p, :] = r[idx[p], :] (0 where idx < 0)
__global__ void gather_il_kernel(int64_t count, int K, const int32_t* __restrict__ idx, const double* __restrict__ src,
                                 double* __restrict__ dst) {
  const int64_t total = count * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / K;
    const int j = (int)(e - p * K);
    const int32_t g = idx[p];
    dst[e] = g >= 0 ? src[(int64_t)g * K + j] : 0.0;
  }
}

// w[out_pos[c], :] = (Phi^T r)[c, :]; one block per coarse column, threads
// (8 entry lanes) x (32 right-hand sides), fixed-order combination.
__global__ __launch_bounds__(256) void restrict_il_kernel(int nc, int K, CoarseView cv, const double* __restrict__ r,
                                                          double* __restrict__ w, const int32_t* __restrict__ out_pos) {
  __shared__ double sh[8][32];
  const int c = blockIdx.x;
  const int j = threadIdx.x & 31, el = threadIdx.x >> 5;
  double s = 0.0;
  if (j < K) {
    for (int e = cv.cg_ptr[c] + el; e < cv.cg_ptr[c + 1]; e += 8) s += r[(int64_t)cv.cg_dof[e] * K + j];
    for (int e = cv.cs_ptr[c]; e < cv.cs_ptr[c + 1]; ++e) {
      const int i = cv.cs_sub[e], lc = cv.cs_lc[e];
      const int ib = cv.I_ptr[i], ni = cv.I_ptr[i + 1] - ib;
      const double* ph = cv.phi_cm + cv.phi_off[i] + (int64_t)lc * ni;
      for (int k = el; k < ni; k += 8) s = fma(ph[k], r[(int64_t)cv.I_idx[ib + k] * K + j], s);
    }
  }
  sh[el][j] = s;
  __syncthreads();
  if (el == 0 && j < K) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) t += sh[q][j];
    w[(int64_t)out_pos[c] * K + j] = t;
  }
}

// Per-subdomain pair partials of Phi^T r: tpart[(s * n_pairs + C_ptr[i] + q) * K + j]
// = sum over rows k of split s (ascending) of Phi_I^(i)[k, q] r[I_i[k], j].
// Work-group (split s, subdomain i); rows staged 32 at a time in LDS (the
// gathered right-hand sides and the row-major Phi rows, contiguous when a
// subdomain has at most 128 coarse columns), so each right-hand-side row is
// read once per split instead of once per coarse column.  Every thread
// issues all of its staging loads before its first LDS store.  Columns are
// handled 128 at a time; thread (column group cg, right-hand side j) owns
// columns cg, cg + 8, ...
constexpr int PT_ROWS = 32, PT_COLS = 128;

// ps[kk * PT_COLS + q] = Phi[(k0 + kk) * nc + qb + q] for kk < rows, q < qn,
// zero elsewhere in the 32 x 128 tile (so the products need no predicates)
__device__ inline void stage_phi_rows(double* ps, const double* __restrict__ phi, int k0, int rows, int nc, int qb,
                                      int qn) {
  double v[PT_ROWS * PT_COLS / 256];
#pragma unroll
  for (int u = 0; u < PT_ROWS * PT_COLS / 256; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int kk = e / PT_COLS, q = e % PT_COLS;
    v[u] = (kk < rows && q < qn) ? phi[(int64_t)(k0 + kk) * nc + qb + q] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < PT_ROWS * PT_COLS / 256; ++u) ps[threadIdx.x + 256 * u] = v[u];
}

__global__ __launch_bounds__(256) void phi_t_il_kernel(int K, CoarseView cv, const double* __restrict__ r,
                                                       double* __restrict__ tpart, int n_pairs, int nsplit) {
  __shared__ double rs[PT_ROWS][33];
  __shared__ double ps[PT_ROWS * PT_COLS];
  const int i = blockIdx.y, sp = blockIdx.x;
  const int ib = cv.I_ptr[i], ni = cv.I_ptr[i + 1] - ib;
  const int cb = cv.C_ptr[i], nc = cv.C_ptr[i + 1] - cb;
  const int per = (ni + nsplit - 1) / nsplit;
  const int k0 = min(ni, sp * per), k1 = min(ni, k0 + per);
  const int j = threadIdx.x & 31, cg = threadIdx.x >> 5;
  const double* phi = cv.phi_rm + cv.phi_off[i];
  for (int qb = 0; qb < nc; qb += PT_COLS) {
    const int qn = min(PT_COLS, nc - qb);
    double acc[PT_COLS / 8];
#pragma unroll
    for (int u = 0; u < PT_COLS / 8; ++u) acc[u] = 0.0;
    for (int kc = k0; kc < k1; kc += PT_ROWS) {
      const int rows = min(PT_ROWS, k1 - kc);
      __syncthreads();
      {
        double v[PT_ROWS * 32 / 256];
#pragma unroll
        for (int u = 0; u < PT_ROWS * 32 / 256; ++u) {
          const int e = threadIdx.x + 256 * u, kk = e >> 5, jj = e & 31;
          v[u] = (kk < rows && jj < K) ? r[(int64_t)cv.I_idx[ib + kc + kk] * K + jj] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PT_ROWS * 32 / 256; ++u) {
          const int e = threadIdx.x + 256 * u;
          rs[e >> 5][e & 31] = v[u];
        }
      }
      stage_phi_rows(ps, phi, kc, rows, nc, qb, qn);
      __syncthreads();
      for (int kk = 0; kk < rows; ++kk) {
        const double rv = rs[kk][j];
#pragma unroll
        for (int u = 0; u < PT_COLS / 8; ++u) acc[u] = fma(ps[kk * PT_COLS + cg + 8 * u], rv, acc[u]);
      }
    }
    if (j < K) {
#pragma unroll
      for (int u = 0; u < PT_COLS / 8; ++u)
        if (cg + 8 * u < qn) tpart[((int64_t)sp * n_pairs + cb + qb + cg + 8 * u) * K + j] = acc[u];
    }
  }
}

// w[out_pos[c], j] = sum over the Gamma DOFs of column c of r[d, j] + sum of
// the pair values over its pairs in ascending subdomain order (each pair
// value the sum of its split partials in split order); 8 columns per block.
__global__ __launch_bounds__(256) void restrict_assemble_il_kernel(int nc, int K, CoarseView cv,
                                                                   const double* __restrict__ r,
                                                                   const double* __restrict__ tpart, int n_pairs,
                                                                   int nsplit, double* __restrict__ w,
                                                                   const int32_t* __restrict__ out_pos) {
  const int c = blockIdx.x * 8 + (threadIdx.x >> 5);
  const int j = threadIdx.x & 31;
  if (c >= nc || j >= K) return;
  double s = 0.0;
  for (int e = cv.cg_ptr[c]; e < cv.cg_ptr[c + 1]; ++e) s += r[(int64_t)cv.cg_dof[e] * K + j];
  for (int e = cv.cs_ptr[c]; e < cv.cs_ptr[c + 1]; ++e) {
    const int64_t pe = cv.C_ptr[cv.cs_sub[e]] + cv.cs_lc[e];
    double t = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) t += tpart[((int64_t)sp * n_pairs + pe) * K + j];
    s += t;
  }
  w[(int64_t)out_pos[c] * K + j] = s;
}

// z[I_i[k], j] += sum_q Phi_I^(i)[k, q] y0[C_i[q], j] (ascending q):
// work-group (128-row chunk, subdomain).  The subdomain's coarse values
// (128 columns at a time) and 32 Phi rows at a time are staged in LDS;
// thread (row lane rl, j) owns rows rl, rl + 8, ... of the chunk.
constexpr int PP_ROWS = 128;

__global__ __launch_bounds__(256) void phi_prolong_il_kernel(int K, CoarseView cv, const double* __restrict__ w,
                                                             const int32_t* __restrict__ y0_pos,
                                                             double* __restrict__ z) {
  __shared__ double ys[PT_COLS][33];
  __shared__ double ps[PT_ROWS * PT_COLS];
  const int i = blockIdx.y;
  const int ib = cv.I_ptr[i], ni = cv.I_ptr[i + 1] - ib;
  const int k0 = blockIdx.x * PP_ROWS;
  if (k0 >= ni) return;  // uniform over the work-group
  const int k1 = min(ni, k0 + PP_ROWS);
  const int cb = cv.C_ptr[i], nc = cv.C_ptr[i + 1] - cb;
  const int j = threadIdx.x & 31, rl = threadIdx.x >> 5;
  const double* phi = cv.phi_rm + cv.phi_off[i];
  double c[PP_ROWS / 8];
#pragma unroll
  for (int u = 0; u < PP_ROWS / 8; ++u) c[u] = 0.0;
  for (int qb = 0; qb < nc; qb += PT_COLS) {
    const int qn = min(PT_COLS, nc - qb);
    __syncthreads();
    {
      double v[PT_COLS * 32 / 256];
#pragma unroll
      for (int u = 0; u < PT_COLS * 32 / 256; ++u) {
        const int e = threadIdx.x + 256 * u, q = e >> 5, jj = e & 31;
        v[u] = (q < qn && jj < K) ? w[(int64_t)y0_pos[cv.C_idx[cb + qb + q]] * K + jj] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < PT_COLS * 32 / 256; ++u) {
        const int e = threadIdx.x + 256 * u;
        ys[e >> 5][e & 31] = v[u];
      }
    }
#pragma unroll
    for (int sc = 0; sc < PP_ROWS / PT_ROWS; ++sc) {
      const int kc = k0 + sc * PT_ROWS;
      const int rows = max(0, min(PT_ROWS, k1 - kc));
      __syncthreads();
      stage_phi_rows(ps, phi, kc, rows, nc, qb, qn);
      __syncthreads();
      // the four rows of this thread advance together (independent sums,
      // each in ascending q); rows past the chunk read zero Phi rows
      double a[PT_ROWS / 8];
#pragma unroll
      for (int v = 0; v < PT_ROWS / 8; ++v) a[v] = c[sc * (PT_ROWS / 8) + v];
      for (int q = 0; q < qn; ++q) {
        const double y = ys[q][j];
#pragma unroll
        for (int v = 0; v < PT_ROWS / 8; ++v) a[v] = fma(ps[(rl + 8 * v) * PT_COLS + q], y, a[v]);
      }
#pragma unroll
      for (int v = 0; v < PT_ROWS / 8; ++v) c[sc * (PT_ROWS / 8) + v] = a[v];
    }
  }
  if (j < K) {
#pragma unroll
    for (int sc = 0; sc < PP_ROWS / PT_ROWS; ++sc)
#pragma unroll
      for (int v = 0; v < PT_ROWS / 8; ++v) {
        const int k = k0 + sc * PT_ROWS + rl + 8 * v;
        if (k < k1) z[(int64_t)cv.I_idx[ib + k] * K + j] += c[sc * (PT_ROWS / 8) + v];
      }
  }
}

// z[d, :] = sum of local copies (ascending subdomain) + (Phi y_0)[d, :],
// y_0 read from the work vector at y0_pos (or absent when cv.gamma_col is null).
__global__ void scatter_prolong_il_kernel(int64_t n, int K, const int32_t* __restrict__ inv_ptr,
                                          const int64_t* __restrict__ inv_pos, const double* __restrict__ w,
                                          CoarseView cv, const int32_t* __restrict__ y0_pos, double* __restrict__ z,
                                          int split) {
  const int64_t total = n * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = e / K;
    const int j = (int)(e - d * K);
    double s = 0.0;
    for (int q = inv_ptr[d]; q < inv_ptr[d + 1]; ++q) s += w[inv_pos[q] * K + j];
    double c = 0.0;
    if (y0_pos) {
      const int32_t gc = cv.gamma_col[d];
      if (gc >= 0) {
        c = w[(int64_t)y0_pos[gc] * K + j];
      } else if (!split) {
        const int32_t p = cv.dof_ipos[d];
        if (p >= 0) {
          const int i = cv.I_sub[p];
          const int k = p - cv.I_ptr[i];
          const int cb = cv.C_ptr[i], ncol = cv.C_ptr[i + 1] - cb;
          const double* row = cv.phi_rm + cv.phi_off[i] + (int64_t)k * ncol;
          for (int q = 0; q < ncol; ++q) c = fma(row[q], w[(int64_t)y0_pos[cv.C_idx[cb + q]] * K + j], c);
        }
      }
    }
    z[e] = s + c;
  }
}

// Y = A X for K <= 32 interleaved vectors.  A wave serves ROWS rows; the
// lanes of a row are G groups of LPG = 64 / (ROWS G) lanes, lane l of a group
// holding the RPL = 32 / LPG right-hand sides RPL l .. RPL l + RPL - 1 (one
// 8-, 16- or 32-byte load per nonzero; K must be a multiple of RPL), and
// group g takes the row's nonzeros in batches of eight, batch g, g + G, ...:
// every lane issues the batch's eight column/value loads, then the eight
// gathers of its vector entries (a group reads 256 contiguous bytes per
// nonzero), so a row needs about nnz / (8 G) dependent round trips.  The G
// group sums are combined by a butterfly over the lane exchanges (the same
// tree on every run).  With SPMM_XCD the work-groups take contiguous row
// ranges per XCD (the dispatcher deals work-groups to the 8 XCDs in turn).
// Measured on MI355X at 24^3 x 32 columns (98 launches, rocprofv3): two rows
// per wave with 1 / 2 / 4 groups 923 / 555 / 501 us, one row with 4 / 8
// groups 557 / 518 us (the kernel with one lane per right-hand side and no
// groups took 726 us); XCD-contiguous row ranges 586 / 614 us instead of
// 555 / 557 (the eight XCDs then stream eight far-apart parts of X through
// the shared last-level cache instead of one region).
#ifndef GDSW_SPMM_ROWS
#define GDSW_SPMM_ROWS 2
#endif
#ifndef GDSW_SPMM_G
#define GDSW_SPMM_G 4
#endif
#ifndef GDSW_SPMM_XCD
#define GDSW_SPMM_XCD 0
#endif

template <int RPL>
struct RhsVec;
template <>
struct RhsVec<1> {
  static __device__ inline void load(const double* p, double (&o)[1]) { o[0] = *p; }
};
template <>
struct RhsVec<2> {
  static __device__ inline void load(const double* p, double (&o)[2]) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    o[0] = v.x;
    o[1] = v.y;
  }
};
template <>
struct RhsVec<4> {
  static __device__ inline void load(const double* p, double (&o)[4]) {
    const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
    o[0] = a.x;
    o[1] = a.y;
    o[2] = b.x;
    o[3] = b.y;
  }
};

template <int ROWS, int G>
__global__ __launch_bounds__(256) void spmm_il_kernel(int64_t nrows, int K, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col, const double* __restrict__ val,
                                                      const double* __restrict__ x, double* __restrict__ y) {
  constexpr int LPG = 64 / (ROWS * G);  // lanes per group
  constexpr int RPL = 32 / LPG;         // right-hand sides per lane
  int blk = blockIdx.x;
#if GDSW_SPMM_XCD
  {
    const int nb = gridDim.x, x8 = blockIdx.x % 8, q8 = blockIdx.x / 8, per = nb / 8, rem = nb % 8;
    blk = (x8 < rem ? x8 * (per + 1) : rem * (per + 1) + (x8 - rem) * per) + q8;
  }
#endif
  const int lane = threadIdx.x & 63;
  const int64_t row = ((int64_t)blk * 4 + (threadIdx.x >> 6)) * ROWS + lane / (64 / ROWS);
  const int rl = lane % (64 / ROWS);    // lane within the row
  const int g = rl / LPG, l = rl % LPG;
  const bool live = row < nrows;        // uniform per row's lanes
  const int jb = min(RPL * l, K - RPL); // K % RPL == 0 and K >= RPL
  const int k0 = live ? rowptr[row] : 0, k1 = live ? rowptr[row + 1] : 0;
  double s[RPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) s[q] = 0.0;
  for (int kb = k0 + 8 * g; kb < k1; kb += 8 * G) {
    int32_t c[8];
    double v[8], xv[8][RPL];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = min(kb + u, k1 - 1);
      c[u] = col[k];
      v[u] = kb + u < k1 ? val[k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) RhsVec<RPL>::load(x + (int64_t)c[u] * K + jb, xv[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int q = 0; q < RPL; ++q) s[q] = fma(v[u], xv[u][q], s[q]);
  }
#pragma unroll
  for (int d = LPG; d < LPG * G; d *= 2)
#pragma unroll
    for (int q = 0; q < RPL; ++q) s[q] += __shfl_xor(s[q], d);
  if (live && g == 0)
#pragma unroll
    for (int q = 0; q < RPL; ++q)
      if (RPL * l + q < K) y[row * K + RPL * l + q] = s[q];
}

constexpr int DCH = 256;  // rows per partial block of the dot products

// part[(b * ncols + i) * K + j] = sum over rows of block b of V_i[r, j] * w[r, j]:
// thread (row lane rl, j) sums rows r0 + rl, r0 + rl + 8, ... in ascending
// order, the 8 row lanes are combined in ascending order.  Four columns
// per barrier; every load is unconditional (rows past n read row n - 1
// against a zero w, lanes past K read column K - 1 and are not written), so
// the loads stay in flight together.
constexpr int DCOLS = 4;

__global__ __launch_bounds__(256) void dots_il_partial_kernel(const double* __restrict__ V, int64_t ldv, int ncols,
                                                              const double* __restrict__ w, int64_t n, int K,
                                                              double* __restrict__ part) {
  __shared__ double sh[DCOLS][8][32];
  const int b = blockIdx.x;
  const int j = threadIdx.x & 31, rl = threadIdx.x >> 5;
  const int jj = min(j, K - 1);
  const int64_t r0 = (int64_t)b * DCH;
  double wr[DCH / 8];
#pragma unroll
  for (int q = 0; q < DCH / 8; ++q) {
    const int64_t r = r0 + q * 8 + rl;
    wr[q] = (r < n && j < K) ? w[r * K + j] : 0.0;
  }
  for (int i0 = 0; i0 < ncols; i0 += DCOLS) {
    double s[DCOLS];
#pragma unroll
    for (int c = 0; c < DCOLS; ++c) s[c] = 0.0;
#pragma unroll
    for (int q = 0; q < DCH / 8; ++q) {
      const int64_t rr = min<int64_t>(r0 + q * 8 + rl, n - 1);
#pragma unroll
      for (int c = 0; c < DCOLS; ++c) {
        const int64_t ic = min(i0 + c, ncols - 1);
        s[c] = fma(V[ic * ldv + rr * K + jj], wr[q], s[c]);
      }
    }
    __syncthreads();  // the previous group's sums have been read
#pragma unroll
    for (int c = 0; c < DCOLS; ++c) sh[c][rl][j] = s[c];
    __syncthreads();
    const int c = threadIdx.x >> 5;  // threads (c < DCOLS, j) combine column i0 + c
    if (c < DCOLS && i0 + c < ncols && j < K) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) t += sh[c][q][j];
      part[((int64_t)b * ncols + i0 + c) * K + j] = t;
    }
  }
}

__global__ __launch_bounds__(256) void dots_il_final_kernel(const double* __restrict__ part, int nblocks, int ncols,
                                                            int K, double* __restrict__ out) {
  __shared__ double sh[8][32];
  const int i = blockIdx.x;
  const int j = threadIdx.x & 31, bl = threadIdx.x >> 5;
  double s = 0.0;
  if (j < K)
    for (int b = bl; b < nblocks; b += 8) s += part[((int64_t)b * ncols + i) * K + j];
  sh[bl][j] = s;
  __syncthreads();
  if (bl == 0 && j < K) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) t += sh[q][j];
    out[(int64_t)i * K + j] = t;
  }
}

// w[r, j] -= sum_i V_i[r, j] h[i, j]   (sign = -1)   or   x += ...   (sign = +1),
// summed in ascending i.  The coefficients h (ncols x K) are staged in LDS
// by each work-group, which then strides over many elements.
__global__ __launch_bounds__(256) void gemv_il_kernel(const double* __restrict__ V, int64_t ldv, int ncols,
                                                     const double* __restrict__ h, double* __restrict__ w, int64_t n,
                                                     int K, double sign) {
  extern __shared__ double hs[];
  for (int t = threadIdx.x; t < ncols * K; t += 256) hs[t] = h[t];
  __syncthreads();
  const int64_t total = n * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e % K);
    double s = 0.0;
    int i = 0;
    for (; i + 8 <= ncols; i += 8) {  // eight columns' loads issued together
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = V[(int64_t)(i + u) * ldv + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) s = fma(v[u], hs[(i + u) * K + j], s);
    }
    for (; i < ncols; ++i) s = fma(V[(int64_t)i * ldv + e], hs[i * K + j], s);
    w[e] += sign * s;
  }
}

// v[r, j] = active[j] && s[j] != 0 ? w[r, j] / s[j] : 0
__global__ void scale_il_kernel(int64_t n, int K, const double* __restrict__ w, const double* __restrict__ s,
                                const int32_t* __restrict__ active, double* __restrict__ v) {
  const int64_t total = n * K;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e % K);
    const double d = s[j];
    v[e] = (active[j] && d != 0.0) ? w[e] / d : 0.0;
  }
}

__global__ void sub_il_kernel(int64_t total, const double* __restrict__ b, double* __restrict__ r) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    r[e] = b[e] - r[e];
}

}  // namespace

void cm_to_il(int64_t n, int K, const double* src, int64_t ld, double* dst, hipStream_t st) {
  if (n == 0) return;
  cm_to_il_kernel<<<(unsigned)((n + 63) / 64), 256, 0, st>>>(n, K, src, ld, dst);
}

void il_to_cm(int64_t n, int K, const double* src, double* dst, int64_t ld, hipStream_t st) {
  if (n == 0) return;
  il_to_cm_kernel<<<(unsigned)((n + 63) / 64), 256, 0, st>>>(n, K, src, dst, ld);
}

void gather_il(int64_t count, int K, const int32_t* idx, const double* src, double* dst, hipStream_t st) {
  if (count == 0) return;
  gather_il_kernel<<<grid_for(count * K), 256, 0, st>>>(count, K, idx, src, dst);
}

int phi_t_splits(int nsub) { return nsub > 0 ? std::max(1, std::min(8, (2048 + nsub - 1) / nsub)) : 1; }

void restrict_il(int nc, int K, const CoarseView& cv, const double* r, double* w, const int32_t* out_pos,
                 hipStream_t st, int n_pairs, double* t, int nsub) {
  const int nsplit = phi_t_splits(nsub);
  if (nc == 0) return;
  if (n_pairs > 0 && t && nsub > 0) {
    phi_t_il_kernel<<<dim3(nsplit, nsub), 256, 0, st>>>(K, cv, r, t, n_pairs, nsplit);
    restrict_assemble_il_kernel<<<(nc + 7) / 8, 256, 0, st>>>(nc, K, cv, r, t, n_pairs, nsplit, w, out_pos);
  } else {
    restrict_il_kernel<<<nc, 256, 0, st>>>(nc, K, cv, r, w, out_pos);
  }
}

void scatter_prolong_il(int64_t n, int K, const int32_t* inv_ptr, const int64_t* inv_pos, const double* w,
                        const CoarseView& cv, const int32_t* y0_pos, double* z, hipStream_t st, int nsub,
                        int max_ni) {
  if (n == 0) return;
  const int split = y0_pos && nsub > 0 && max_ni > 0;
  scatter_prolong_il_kernel<<<grid_for(n * K), 256, 0, st>>>(n, K, inv_ptr, inv_pos, w, cv, y0_pos, z, split);
  if (split) phi_prolong_il_kernel<<<dim3((max_ni + PP_ROWS - 1) / PP_ROWS, nsub), 256, 0, st>>>(K, cv, w, y0_pos, z);
}

void spmm_il(int64_t nrows, int K, const int32_t* rowptr, const int32_t* col, const double* val, const double* x,
             double* y, hipStream_t st) {
  if (nrows == 0) return;
  if (K < 1 || K > 32) throw StatusError{1, "interleaved SpMM takes 1 to 32 columns"};
  constexpr int ROWS = GDSW_SPMM_ROWS, G = GDSW_SPMM_G;
  constexpr int RPL = 32 / (64 / (ROWS * G));
  static_assert(ROWS * G >= 2 && ROWS * G <= 8 && 64 % (ROWS * G) == 0, "2 to 8 lane groups per wave");
  const unsigned grid = (unsigned)((nrows + 4 * ROWS - 1) / (4 * ROWS));
  if (K % RPL == 0)
    spmm_il_kernel<ROWS, G><<<grid, 256, 0, st>>>(nrows, K, rowptr, col, val, x, y);
  else  // one right-hand side per lane, two rows per wave
    spmm_il_kernel<2, 1><<<(unsigned)((nrows + 7) / 8), 256, 0, st>>>(nrows, K, rowptr, col, val, x, y);
  GDSW_HIP(hipGetLastError());
}

int dots_il_blocks(int64_t n) { return (int)((n + DCH - 1) / DCH); }

void dots_il(const double* V, int64_t ldv, int ncols, const double* w, int64_t n, int K, double* part, int nblocks,
             double* out, hipStream_t st) {
  dots_il_partial_kernel<<<nblocks, 256, 0, st>>>(V, ldv, ncols, w, n, K, part);
  dots_il_final_kernel<<<ncols, 256, 0, st>>>(part, nblocks, ncols, K, out);
}

void gemv_il(const double* V, int64_t ldv, int ncols, const double* h, double* w, int64_t n, int K, double sign,
             hipStream_t st) {
  if (n == 0 || ncols == 0) return;
  // at most 201 x 32 coefficients (restart <= 200): 51.5 KB of LDS
  gemv_il_kernel<<<grid_for(n * K, 256, 1024), 256, (size_t)ncols * K * sizeof(double), st>>>(V, ldv, ncols, h, w, n,
                                                                                               K, sign);
}

void scale_il(int64_t n, int K, const double* w, const double* s, const int32_t* active, double* v, hipStream_t st) {
  scale_il_kernel<<<grid_for(n * K), 256, 0, st>>>(n, K, w, s, active, v);
}

void sub_il(int64_t total, const double* b, double* r, hipStream_t st) {
  sub_il_kernel<<<grid_for(total), 256, 0, st>>>(total, b, r);
}

}  // namespace gdsw
