// Sparse, gather/scatter, coarse-space and Krylov kernels (gfx950).
//
// Every reduction here runs in a fixed order (per-thread sequential sums in
// a fixed index order, then fixed-shape LDS or shuffle trees), so results are
// bitwise reproducible run to run.  No floating-point atomics.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "kernels_ops.h"

namespace gdsw {
namespace {

__device__ inline int lower_bound_i32(const int32_t* a, int n, int32_t key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <int BS>
__device__ inline double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
#pragma unroll
  for (int s = BS / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// y = A x, 16 lanes per row; lane-strided partial sums then a xor tree.
__global__ __launch_bounds__(256) void spmv_kernel(int64_t nrows, const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ col, const double* __restrict__ val,
                                                  const double* __restrict__ x, double* __restrict__ y) {
  const int64_t row = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  const int l = threadIdx.x & 15;
  double s = 0.0;
  if (row < nrows) {
    // lane l takes the nonzeros b + l, b + l + 16, ... in ascending order,
    // eight at a time: their indices and values (clamped into the row), then
    // the eight x entries, are loaded before any product
    const int b = rowptr[row], e = rowptr[row + 1];
    for (int k0 = b + l; k0 < e; k0 += 128) {
      int32_t c[8];
      double v[8], xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = min(k0 + 16 * u, e - 1);
        c[u] = col[k];
        v[u] = val[k];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) xv[u] = x[c[u]];
#pragma unroll
      for (int u = 0; u < 8; ++u) s = k0 + 16 * u < e ? fma(v[u], xv[u], s) : s;
    }
  }
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
  if (row < nrows && l == 0) y[row] = s;
}

__global__ void gather_kernel(int64_t count, const int32_t* __restrict__ idx, const double* __restrict__ src,
                              double* __restrict__ dst) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < count; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = idx[p];
    dst[p] = g >= 0 ? src[g] : 0.0;
  }
}

// dense A[S_f, S_f] (column-major, ld[f]) from CSR; one thread per local row
__global__ void extract_kernel(double* __restrict__ base, const int32_t* __restrict__ N, const int32_t* __restrict__ LD,
                               const int64_t* __restrict__ OFF, const int32_t* __restrict__ lptr,
                               const int32_t* __restrict__ lidx, const int32_t* __restrict__ rowptr,
                               const int32_t* __restrict__ col, const double* __restrict__ val) {
  const int f = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = N[f];
  if (k >= n) return;
  const int32_t* S = lidx + lptr[f];
  const int64_t ld = LD[f];
  double* A = base + OFF[f];
  const int32_t g = S[k];
  for (int e = rowptr[g]; e < rowptr[g + 1]; ++e) {
    const int32_t c = col[e];
    const int lc = lower_bound_i32(S, n, c);
    if (lc < n && S[lc] == c) A[(int64_t)lc * ld + k] = val[e];
  }
}

__global__ void extract_dense_kernel(double* __restrict__ base, const int32_t* __restrict__ N,
                                     const int32_t* __restrict__ LD, const int64_t* __restrict__ OFF,
                                     const int32_t* __restrict__ lptr, const int32_t* __restrict__ lidx,
                                     const double* __restrict__ M, int64_t ldm) {
  const int f = blockIdx.z;
  const int n = N[f];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= n || c >= n) return;
  const int32_t* S = lidx + lptr[f];
  base[OFF[f] + (int64_t)c * LD[f] + r] = M[(int64_t)S[r] * ldm + S[c]];
}

__global__ void scatter_kernel(int64_t n, const int32_t* __restrict__ inv_ptr, const int64_t* __restrict__ inv_pos,
                               const double* __restrict__ w, double* __restrict__ z) {
  for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int e = inv_ptr[d]; e < inv_ptr[d + 1]; ++e) s += w[inv_pos[e]];
    z[d] = s;
  }
}

// z[d] = sum of local copies (ascending subdomain) + (Phi y0)[d]
// With `split`, interior DOFs receive only their local copies here and the
// Phi_I y0 term is added by phi_prolong_kernel (same operands, same order).
__global__ void scatter_prolong_kernel(int64_t n, const int32_t* __restrict__ inv_ptr,
                                       const int64_t* __restrict__ inv_pos, const double* __restrict__ w,
                                       CoarseView cv, const double* __restrict__ y0,
                                       const int32_t* __restrict__ y0_pos, double* __restrict__ z, int split) {
  for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < n; d += (int64_t)gridDim.x * blockDim.x) {
    // the local copies (ascending subdomain), four positions then four
    // values loaded before the sum
    double s = 0.0;
    const int e0 = inv_ptr[d], e1 = inv_ptr[d + 1];
    for (int e = e0; e < e1; e += 4) {
      int64_t pos[4];
      double wv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) pos[u] = inv_pos[min(e + u, e1 - 1)];
#pragma unroll
      for (int u = 0; u < 4; ++u) wv[u] = w[pos[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u) s = e + u < e1 ? s + wv[u] : s;
    }
    double c = 0.0;
    const int32_t gc = cv.gamma_col[d];
    if (gc >= 0) {
      c = y0_pos ? w[y0_pos[gc]] : y0[gc];
    } else if (!split) {
      const int32_t p = cv.dof_ipos[d];
      if (p >= 0) {
        const int i = cv.I_sub[p];
        const int k = p - cv.I_ptr[i];
        const int cb = cv.C_ptr[i], nc = cv.C_ptr[i + 1] - cb;
        const double* row = cv.phi_rm + cv.phi_off[i] + (int64_t)k * nc;
        for (int j = 0; j < nc; ++j) {
          const int32_t cc = cv.C_idx[cb + j];
          c = fma(row[j], y0_pos ? w[y0_pos[cc]] : y0[cc], c);
        }
      }
    }
    z[d] = s + c;
  }
}

// r0[c] = (Phi^T r)[c]: Gamma part (indicator sum) + interior part
__global__ __launch_bounds__(256) void restrict_kernel(int nc_total, CoarseView cv, const double* __restrict__ r,
                                                      double* __restrict__ out, const int32_t* __restrict__ out_pos) {
  __shared__ double sh[256];
  const int c = blockIdx.x;
  if (c >= nc_total) return;
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int e = cv.cg_ptr[c] + tid; e < cv.cg_ptr[c + 1]; e += 256) s += r[cv.cg_dof[e]];
  for (int e = cv.cs_ptr[c]; e < cv.cs_ptr[c + 1]; ++e) {
    const int i = cv.cs_sub[e], lc = cv.cs_lc[e];
    const int ib = cv.I_ptr[i], ni = cv.I_ptr[i + 1] - ib;
    const double* ph = cv.phi_cm + cv.phi_off[i] + (int64_t)lc * ni;
    for (int k = tid; k < ni; k += 256) s = fma(ph[k], r[cv.I_idx[ib + k]], s);
  }
  const double t = block_sum<256>(s, sh);
  if (tid == 0) out[out_pos ? out_pos[c] : c] = t;
}

// z[I_i[k]] += sum_j Phi_I^(i)[k, j] y0[C_i[j]]: 64 interior rows per
// work-group (lanes = rows, so the column-major Phi_I is read contiguously);
// wave w takes the columns j = w, w + 4, ... in ascending order with eight
// loads in flight, and the four sums are added in wave order.
__global__ __launch_bounds__(256) void phi_prolong_kernel(CoarseView cv, const double* __restrict__ w,
                                                          const double* __restrict__ y0,
                                                          const int32_t* __restrict__ y0_pos,
                                                          double* __restrict__ z) {
  // the subdomain's coarse values are gathered into LDS once (in parallel),
  // 256 columns at a time
  __shared__ double yv[256];
  __shared__ double red[4][64];
  const int i = blockIdx.y;
  const int ib = cv.I_ptr[i], ni = cv.I_ptr[i + 1] - ib;
  const int k0 = blockIdx.x * 64;
  if (k0 >= ni) return;  // uniform over the work-group
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cb = cv.C_ptr[i], nc = cv.C_ptr[i + 1] - cb;
  const double* ph = cv.phi_cm + cv.phi_off[i] + min(k0 + lane, ni - 1);
  double c = 0.0;
  for (int j0 = 0; j0 < nc; j0 += 256) {
    const int jn = min(256, nc - j0);
    __syncthreads();
    if ((int)threadIdx.x < jn) {
      const int32_t cc = cv.C_idx[cb + j0 + threadIdx.x];
      yv[threadIdx.x] = y0_pos ? w[y0_pos[cc]] : y0[cc];
    }
    __syncthreads();
    for (int j = wave; j < jn; j += 32) {
      double pv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) pv[u] = ph[(int64_t)(j0 + min(j + 4 * u, jn - 1)) * ni];
#pragma unroll
      for (int u = 0; u < 8; ++u) c = j + 4 * u < jn ? fma(pv[u], yv[min(j + 4 * u, jn - 1)], c) : c;
    }
  }
  red[wave][lane] = c;
  __syncthreads();
  if (wave == 0 && k0 + lane < ni) {
    const double v = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    const int32_t d = cv.I_idx[ib + k0 + lane];
    z[d] = z[d] + v;
  }
}

// The sum of a DOF's local copies (ascending subdomain): four positions,
// then four values, loaded before they are added; the order of
// scatter_prolong_kernel.
__device__ inline double local_copies_sum(const int32_t* __restrict__ inv_ptr, const int64_t* __restrict__ inv_pos,
                                          const double* __restrict__ w, int64_t d) {
  double s = 0.0;
  const int e0 = inv_ptr[d], e1 = inv_ptr[d + 1];
  for (int e = e0; e < e1; e += 4) {
    int64_t pos[4];
    double wv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) pos[u] = inv_pos[min(e + u, e1 - 1)];
#pragma unroll
    for (int u = 0; u < 4; ++u) wv[u] = w[pos[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u) s = e + u < e1 ? s + wv[u] : s;
  }
  return s;
}

// z = sum_i R_i^T y_i + Phi y0 in one launch, the same sums as
// scatter_prolong_kernel followed by phi_prolong_kernel: work-groups below
// nsub * nblk take 64 interior rows of one subdomain (wave 0 first issues
// the rows' local-copy sums, then every wave its share of Phi_I y0 as in
// phi_prolong_kernel, and z = copies + Phi_I y0); the others take the
// listed rows outside every interior set (the interface), z = copies +
// y0[gamma_col].
__global__ __launch_bounds__(256) void scatter_prolong_fused_kernel(CoarseView cv, const int32_t* __restrict__ inv_ptr,
                                                                    const int64_t* __restrict__ inv_pos,
                                                                    const double* __restrict__ w,
                                                                    const double* __restrict__ y0,
                                                                    const int32_t* __restrict__ y0_pos,
                                                                    double* __restrict__ z, int nsub, int nblk,
                                                                    const int32_t* __restrict__ outer,
                                                                    int64_t n_outer) {
  __shared__ double yv[256];
  __shared__ double red[4][64];
  const int b = blockIdx.x;
  if (b >= nsub * nblk) {  // uniform over the work-group
    const int64_t nb = (int64_t)gridDim.x - (int64_t)nsub * nblk;
    for (int64_t q = (int64_t)(b - nsub * nblk) * blockDim.x + threadIdx.x; q < n_outer; q += nb * blockDim.x) {
      const int32_t d = outer[q];
      const double s = local_copies_sum(inv_ptr, inv_pos, w, d);
      const int32_t gc = cv.gamma_col[d];
      const double c = gc >= 0 ? (y0_pos ? w[y0_pos[gc]] : y0[gc]) : 0.0;
      z[d] = s + c;
    }
    return;
  }
  const int i = b / nblk;
  const int ib = cv.I_ptr[i], ni = cv.I_ptr[i + 1] - ib;
  const int k0 = (b % nblk) * 64;
  if (k0 >= ni) return;  // uniform over the work-group
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double s = 0.0;
  int32_t d = -1;
  if (wave == 0 && k0 + lane < ni) {
    d = cv.I_idx[ib + k0 + lane];
    s = local_copies_sum(inv_ptr, inv_pos, w, d);
  }
  const int cb = cv.C_ptr[i], nc = cv.C_ptr[i + 1] - cb;
  const double* ph = cv.phi_cm + cv.phi_off[i] + min(k0 + lane, ni - 1);
  double c = 0.0;
  for (int j0 = 0; j0 < nc; j0 += 256) {
    const int jn = min(256, nc - j0);
    __syncthreads();
    if ((int)threadIdx.x < jn) {
      const int32_t cc = cv.C_idx[cb + j0 + threadIdx.x];
      yv[threadIdx.x] = y0_pos ? w[y0_pos[cc]] : y0[cc];
    }
    __syncthreads();
    for (int j = wave; j < jn; j += 32) {
      double pv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) pv[u] = ph[(int64_t)(j0 + min(j + 4 * u, jn - 1)) * ni];
#pragma unroll
      for (int u = 0; u < 8; ++u) c = j + 4 * u < jn ? fma(pv[u], yv[min(j + 4 * u, jn - 1)], c) : c;
    }
  }
  red[wave][lane] = c;
  __syncthreads();
  if (d >= 0) {
    const double v = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    z[d] = (s + 0.0) + v;  // as the two kernels: copies (+ 0 coarse), then + Phi_I y0
  }
}

// t[e] = Phi_I^(i)[:, lc]^T r[I_i] for every (subdomain, local column) pair e
// Work-groups n_pairs and up (when gcount > 0) copy the local restrictions
// instead, as gather_kernel does: dst[p] = r[gidx[p]] (0 where gidx < 0).
__global__ __launch_bounds__(256) void phi_t_kernel(CoarseView cv, const double* __restrict__ r,
                                                    double* __restrict__ t, int n_pairs, int64_t gcount,
                                                    const int32_t* __restrict__ gidx, double* __restrict__ gdst) {
  __shared__ double sh[256];
  const int e = blockIdx.x;
  if (e >= n_pairs) {  // uniform over the work-group
    const int64_t nb = (int64_t)gridDim.x - n_pairs;
    for (int64_t p = (int64_t)(e - n_pairs) * blockDim.x + threadIdx.x; p < gcount; p += nb * blockDim.x) {
      const int32_t g = gidx[p];
      gdst[p] = g >= 0 ? r[g] : 0.0;
    }
    return;
  }
  const int i = cv.cs_sub[e], lc = cv.cs_lc[e];
  const int ib = cv.I_ptr[i], ni = cv.I_ptr[i + 1] - ib;
  const double* ph = cv.phi_cm + cv.phi_off[i] + (int64_t)lc * ni;
  // thread rows tid, tid + 256, ... in ascending order; eight rows' loads
  // (clamped into range) are issued before their products, so an interior
  // set of up to 2048 rows takes one round of dependent loads
  double s = 0.0;
  for (int k0 = 0; k0 < ni; k0 += 2048) {
    double pv[8], rv[8];
    int32_t idx[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int kc = min(k0 + (int)threadIdx.x + 256 * u, ni - 1);
      idx[u] = cv.I_idx[ib + kc];
      pv[u] = ph[kc];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) rv[u] = r[idx[u]];
#pragma unroll
    for (int u = 0; u < 8; ++u) s = k0 + (int)threadIdx.x + 256 * u < ni ? fma(pv[u], rv[u], s) : s;
  }
  const double v = block_sum<256>(s, sh);
  if (threadIdx.x == 0) t[e] = v;
}

// The pair sums of phi_t_kernel by (subdomain, column block): work-group b
// takes subdomain i = b / nblk and its local columns j0 = cb (b % nblk) ..
// j0 + cb - 1.  It first gathers r on I_i into LDS (one pass, every load in
// flight), then wave w streams the columns j0 + w, j0 + w + 4, ... of the
// column-major Phi_I^(i), 64 consecutive rows per load instruction and eight
// instructions in flight, and sums each column across the wave by the xor
// tree; t[pair_of[C_ptr[i] + j]] receives column j's sum.  Each work-group
// streams cb |I_i| entries of Phi_I contiguously, so a launch has a few
// thousand work-groups of some 100 KB instead of one 8 KB work-group per
// pair.  Work-groups nsub * nblk and up copy the local restrictions as in
// phi_t_kernel.
__global__ __launch_bounds__(256) void phi_t_sub_kernel(CoarseView cv, const double* __restrict__ r,
                                                        double* __restrict__ t, PairBlocks pb, int64_t gcount,
                                                        const int32_t* __restrict__ gidx,
                                                        double* __restrict__ gdst) {
  extern __shared__ double rl[];  // r on I_i (max_ni doubles)
  const int b = blockIdx.x;
  if (b >= pb.nsub * pb.nblk) {  // uniform over the work-group
    const int64_t nb = (int64_t)gridDim.x - (int64_t)pb.nsub * pb.nblk;
    for (int64_t p = (int64_t)(b - pb.nsub * pb.nblk) * blockDim.x + threadIdx.x; p < gcount;
         p += nb * blockDim.x) {
      const int32_t g = gidx[p];
      gdst[p] = g >= 0 ? r[g] : 0.0;
    }
    return;
  }
  const int i = b / pb.nblk, j0 = (b % pb.nblk) * pb.cb;
  const int cb0 = cv.C_ptr[i], nc = cv.C_ptr[i + 1] - cb0;
  if (j0 >= nc) return;  // uniform over the work-group
  const int ib = cv.I_ptr[i], ni = cv.I_ptr[i + 1] - ib;
  for (int k = threadIdx.x; k < ni; k += 256) rl[k] = r[cv.I_idx[ib + k]];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double* ph = cv.phi_cm + cv.phi_off[i];
  const int j1 = min(nc, j0 + pb.cb);
  for (int j = j0 + wave; j < j1; j += 4) {
    const double* col = ph + (int64_t)j * ni;
    double s = 0.0;
    for (int k0 = 0; k0 < ni; k0 += 512) {
      double pv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) pv[u] = col[min(k0 + lane + 64 * u, ni - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = k0 + lane + 64 * u;
        s = k < ni ? fma(pv[u], rl[k], s) : s;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) t[pb.pair_of[cb0 + j]] = s;
  }
}

// out[c] = sum of r over the Gamma DOFs of column c + sum_e t[e] over its
// pairs in ascending subdomain order; one wave per coarse column.
__global__ __launch_bounds__(256) void restrict_assemble_kernel(int nc_total, CoarseView cv,
                                                                const double* __restrict__ r,
                                                                const double* __restrict__ t,
                                                                double* __restrict__ out,
                                                                const int32_t* __restrict__ out_pos) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= nc_total) return;  // uniform per wave
  restrict_assemble_column(c, threadIdx.x & 63, cv, r, t, out, out_pos);
}

// -(A[I_i, Gamma] Phi_Gamma) for the extension right-hand sides, column-major
__global__ void phi_rhs_kernel(int64_t total_I, CoarseView cv, const int32_t* __restrict__ rowptr,
                               const int32_t* __restrict__ col, const double* __restrict__ val,
                               double* __restrict__ B) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= total_I) return;
  const int i = cv.I_sub[p];
  const int ib = cv.I_ptr[i], ni = cv.I_ptr[i + 1] - ib;
  const int k = (int)(p - ib);
  const int cb = cv.C_ptr[i], nc = cv.C_ptr[i + 1] - cb;
  double* Bi = B + cv.phi_off[i];
  const int32_t g = cv.I_idx[p];
  for (int e = rowptr[g]; e < rowptr[g + 1]; ++e) {
    const int32_t gc = cv.gamma_col[col[e]];
    if (gc < 0) continue;
    const int lc = lower_bound_i32(cv.C_idx + cb, nc, gc);
    if (lc < nc && cv.C_idx[cb + lc] == gc) Bi[(int64_t)lc * ni + k] -= val[e];
  }
}

__global__ void decouple_pressure_kernel(double* __restrict__ base, const int32_t* __restrict__ N,
                                         const int32_t* __restrict__ LD, const int64_t* __restrict__ OFF,
                                         const int32_t* __restrict__ NU) {
  const int f = blockIdx.y;
  const int n = N[f], nu = NU[f];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double* A = base + OFF[f] + (int64_t)c * LD[f];
  for (int r = c < nu ? nu : 0; r < n; ++r) A[r] = r == c ? 1.0 : 0.0;
}

__global__ void phi_pressure_rows_kernel(int64_t total_I, CoarseView cv, const int8_t* __restrict__ pval,
                                         const int32_t* __restrict__ sub_pcol, double* __restrict__ B) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= total_I || pval[p] < 0) return;
  const int i = cv.I_sub[p];
  const int ib = cv.I_ptr[i], ni = cv.I_ptr[i + 1] - ib;
  const int k = (int)(p - ib);
  const int cb = cv.C_ptr[i], nc = cv.C_ptr[i + 1] - cb;
  double* Bi = B + cv.phi_off[i];
  for (int lc = 0; lc < nc; ++lc) Bi[(int64_t)lc * ni + k] = cv.C_idx[cb + lc] == sub_pcol[i] ? (double)pval[p] : 0.0;
}

__global__ void phi_transpose_kernel(int64_t total_I, CoarseView cv, const double* __restrict__ cm,
                                     double* __restrict__ rm) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= total_I) return;
  const int i = cv.I_sub[p];
  const int ib = cv.I_ptr[i], ni = cv.I_ptr[i + 1] - ib;
  const int k = (int)(p - ib);
  const int nc = cv.C_ptr[i + 1] - cv.C_ptr[i];
  const int64_t o = cv.phi_off[i];
  for (int j = 0; j < nc; ++j) rm[o + (int64_t)k * nc + j] = cm[o + (int64_t)j * ni + k];
}

// Phi restricted to the closed box D_i (column-major, ld = |D_i|)
__global__ void phibox_kernel(int64_t total_D, CoarseView cv, BoxView bv, double* __restrict__ phibox) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= total_D) return;
  const int i = bv.D_sub[p];
  const int db = bv.D_ptr[i], nd = bv.D_ptr[i + 1] - db;
  const int q = (int)(p - db);
  const int32_t d = bv.D_idx[p];
  const int cb = cv.C_ptr[i], nc = cv.C_ptr[i + 1] - cb;
  double* out = phibox + bv.box_off[i];
  const int32_t gc = cv.gamma_col[d];
  if (gc >= 0) {
    const int lc = lower_bound_i32(cv.C_idx + cb, nc, gc);
    if (lc < nc && cv.C_idx[cb + lc] == gc) out[(int64_t)lc * nd + q] = 1.0;
  } else {
    const int32_t ip = cv.dof_ipos[d];
    const int ib = cv.I_ptr[i], ni = cv.I_ptr[i + 1] - ib;
    const int k = ip - ib;
    if (ip < 0 || k >= ni) return;
    const double* ph = cv.phi_cm + cv.phi_off[i];
    for (int j = 0; j < nc; ++j) out[(int64_t)j * nd + q] = ph[(int64_t)j * ni + k];
  }
}

// The owner of nonzero (r, c): the lowest-numbered box holding both DOFs,
// -1 if none does
__device__ inline int nonzero_owner(const OwnerMap& om, int32_t r, int32_t c) {
  if (om.blo) {
    int own = 0, mul = 1;
    for (int ax = 0; ax < 3; ++ax) {
      const int lo = max(om.blo[3 * (int64_t)r + ax], om.blo[3 * (int64_t)c + ax]);
      const int hi = min(om.bhi[3 * (int64_t)r + ax], om.bhi[3 * (int64_t)c + ax]);
      if (lo > hi) return -1;
      own += lo * mul;
      mul *= om.m;
    }
    return own;
  }
  int64_t a = om.sub_ptr[r], ae = om.sub_ptr[r + 1], b = om.sub_ptr[c], be = om.sub_ptr[c + 1];
  while (a < ae && b < be) {
    const int32_t x = om.sub_idx[a], y = om.sub_idx[b];
    if (x == y) return x;
    if (x < y) ++a; else ++b;
  }
  return -1;
}

// W_i = A_own_i Phi_box_i, a work-group per (row q of box i): the row's
// nonzeros are taken OWN_T at a time, those box i owns (local column by a
// binary search in the ascending D_i) are packed into LDS in CSR order, and
// thread t adds them into columns t, t + OWN_T, ..., whose sums stay in LDS
// (dynamic, |C_i| doubles).  Every column sums its owned nonzeros in CSR
// order.
constexpr int OWN_T = 128;
__global__ __launch_bounds__(OWN_T) void own_spmm_kernel(CoarseView cv, BoxView bv, OwnerMap om,
                                                        const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ val,
                                                        const double* __restrict__ phibox, double* __restrict__ W) {
  extern __shared__ double acc[];
  __shared__ int32_t lc_s[OWN_T];
  __shared__ double v_s[OWN_T];
  __shared__ int cnt_s[OWN_T / 64];
  const int i = blockIdx.y;
  const int db = bv.D_ptr[i], nd = bv.D_ptr[i + 1] - db;
  const int q = blockIdx.x;
  if (q >= nd) return;  // uniform over the work-group
  const int nc = cv.C_ptr[i + 1] - cv.C_ptr[i];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t o = bv.box_off[i];
  const int32_t* Di = bv.D_idx + db;
  const int32_t r = Di[q];
  for (int j = t; j < nc; j += OWN_T) acc[j] = 0.0;
  const int32_t e0 = rowptr[r], e1 = rowptr[r + 1];
  for (int32_t eb = e0; eb < e1; eb += OWN_T) {
    const int32_t e = eb + t;
    bool owned = false;
    int lc = 0;
    double v = 0.0;
    if (e < e1) {
      const int32_t c = col[e];
      if (nonzero_owner(om, r, c) == i) {
        lc = lower_bound_i32(Di, nd, c);
        owned = lc < nd && Di[lc] == c;  // always, as box i holds c
        v = val[e];
      }
    }
    const unsigned long long bal = __ballot(owned);
    if (lane == 0) cnt_s[wave] = __popcll(bal);
    __syncthreads();
    const int slot = (wave ? cnt_s[0] : 0) + __popcll(bal & ((1ull << lane) - 1));
    const int tot = cnt_s[0] + cnt_s[1];
    if (owned) {
      lc_s[slot] = lc;
      v_s[slot] = v;
    }
    __syncthreads();
    for (int j = t; j < nc; j += OWN_T) {
      const double* ph = phibox + o + (int64_t)j * nd;
      double s = acc[j];
      for (int k = 0; k < tot; ++k) s = fma(v_s[k], ph[lc_s[k]], s);
      acc[j] = s;
    }
    __syncthreads();
  }
  for (int j = t; j < nc; j += OWN_T) W[o + (int64_t)j * nd + q] = acc[j];
}
static_assert(OWN_T == 128, "two waves share the packing counts");

// A_0[c, :] += P_i[lc, :] over the subdomains of c in ascending order
__global__ __launch_bounds__(256) void a0_assemble_kernel(int Nc, CoarseView cv, const double* __restrict__ P,
                                                         const int64_t* __restrict__ p_off, double* __restrict__ A0) {
  const int c = blockIdx.x;
  if (c >= Nc) return;
  double* row = A0 + (int64_t)c * Nc;
  for (int e = cv.cs_ptr[c]; e < cv.cs_ptr[c + 1]; ++e) {
    const int i = cv.cs_sub[e], lc = cv.cs_lc[e];
    const int cb = cv.C_ptr[i], nc = cv.C_ptr[i + 1] - cb;
    const double* Pi = P + p_off[i];
    for (int j = threadIdx.x; j < nc; j += 256) row[cv.C_idx[cb + j]] += Pi[(int64_t)j * nc + lc];
    __syncthreads();
  }
}

// F[:, :] (column-major, ld) = M[perm, perm] (M row-major, ldm)
__global__ void permute_dense_kernel(int n, const int32_t* __restrict__ perm, const double* __restrict__ M,
                                     int64_t ldm, double* __restrict__ F, int64_t ld) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= n) return;
  F[(int64_t)c * ld + r] = M[(int64_t)perm[r] * ldm + perm[c]];
}

__global__ void negate_kernel(int64_t n, double* __restrict__ x) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = -x[i];
}

__global__ void expand_kernel(int64_t nfree, const int64_t* __restrict__ full_index, const double* __restrict__ xf,
                              double* __restrict__ xfull) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nfree; i += (int64_t)gridDim.x * blockDim.x)
    xfull[full_index[i]] = xf[i];
}

// ---- three-level kernels (dense A_0) ---------------------------------------

// -(A_0[I_j, Gamma3] Phi_Gamma^(3)) for the level-3 extension, column-major
__global__ void phi3_rhs_kernel(int64_t total_I, int Nc, const int32_t* __restrict__ I_sub,
                                const int32_t* __restrict__ I_ptr, const int32_t* __restrict__ I_idx,
                                const int32_t* __restrict__ C_ptr, const int32_t* __restrict__ C_idx,
                                const int64_t* __restrict__ off, const int32_t* __restrict__ gcol3,
                                const double* __restrict__ A0, double* __restrict__ B) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= total_I) return;
  const int j = I_sub[p];
  const int ib = I_ptr[j], ni = I_ptr[j + 1] - ib;
  const int k = (int)(p - ib);
  const int cb = C_ptr[j], nc = C_ptr[j + 1] - cb;
  const int32_t c = I_idx[p];
  double* Bj = B + off[j];
  const double* row = A0 + (int64_t)c * Nc;
  for (int cp = 0; cp < Nc; ++cp) {
    const int32_t g = gcol3[cp];
    if (g < 0) continue;
    const int lc = lower_bound_i32(C_idx + cb, nc, g);
    if (lc < nc && C_idx[cb + lc] == g) Bj[(int64_t)lc * ni + k] -= row[cp];
  }
}

// dense Phi^(3) (column-major, ld = Nc): interior rows from the extension
__global__ void phi3_interior_kernel(int64_t total_I, int Nc, const int32_t* __restrict__ I_sub,
                                     const int32_t* __restrict__ I_ptr, const int32_t* __restrict__ I_idx,
                                     const int32_t* __restrict__ C_ptr, const int32_t* __restrict__ C_idx,
                                     const int64_t* __restrict__ off, const double* __restrict__ phiI,
                                     double* __restrict__ phi3) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= total_I) return;
  const int j = I_sub[p];
  const int ib = I_ptr[j], ni = I_ptr[j + 1] - ib;
  const int k = (int)(p - ib);
  const int cb = C_ptr[j], nc = C_ptr[j + 1] - cb;
  const int32_t c = I_idx[p];
  for (int lc = 0; lc < nc; ++lc) phi3[(int64_t)C_idx[cb + lc] * Nc + c] = phiI[off[j] + (int64_t)lc * ni + k];
}

__global__ void phi3_gamma_kernel(int Nc, const int32_t* __restrict__ gcol3, double* __restrict__ phi3) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Nc) return;
  const int32_t g = gcol3[c];
  if (g >= 0) phi3[(int64_t)g * Nc + c] = 1.0;
}

// ---- Krylov helpers --------------------------------------------------------
constexpr int DOT_CHUNK = 256;  // rows per partial block (enough blocks to fill the device at 1e5 rows)

// part[b * ncols + j] = sum over rows of block b of V[:, j] * w.  Wave w
// takes columns w, w + 4, ...; it issues the loads of COLS_AT_ONCE of them
// before reducing any, so their memory latencies overlap.  Per column: each
// lane sums its rows in ascending order, then the lanes combine by the
// xor-shuffle tree.
constexpr int COLS_AT_ONCE = 4;

__global__ __launch_bounds__(256) void cols_dot_partial_kernel(const double* __restrict__ V, int64_t ldv, int ncols,
                                                              const double* __restrict__ w, int64_t n,
                                                              double* __restrict__ part) {
  const int b = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r0 = (int64_t)b * DOT_CHUNK;
  const int64_t r1 = min<int64_t>(n, r0 + DOT_CHUNK);
  double wr[DOT_CHUNK / 64];
#pragma unroll
  for (int q = 0; q < DOT_CHUNK / 64; ++q) {
    const int64_t r = r0 + q * 64 + lane;
    wr[q] = r < r1 ? w[r] : 0.0;
  }
  for (int j0 = wave; j0 < ncols; j0 += 4 * COLS_AT_ONCE) {
    double vv[COLS_AT_ONCE][DOT_CHUNK / 64];
#pragma unroll
    for (int c = 0; c < COLS_AT_ONCE; ++c) {
      const int j = j0 + 4 * c;
      const double* v = V + (int64_t)min(j, ncols - 1) * ldv;
#pragma unroll
      for (int q = 0; q < DOT_CHUNK / 64; ++q) {
        const int64_t r = r0 + q * 64 + lane;
        vv[c][q] = r < r1 ? v[r] : 0.0;
      }
    }
#pragma unroll
    for (int c = 0; c < COLS_AT_ONCE; ++c) {
      const int j = j0 + 4 * c;
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < DOT_CHUNK / 64; ++q) {
        const int64_t r = r0 + q * 64 + lane;
        if (r < r1) s = fma(vv[c][q], wr[q], s);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
      if (lane == 0 && j < ncols) part[(int64_t)b * ncols + j] = s;
    }
  }
}

__global__ __launch_bounds__(64) void cols_dot_final_kernel(const double* __restrict__ part, int nblocks, int ncols,
                                                           double* __restrict__ out) {
  const int j = blockIdx.x;
  const int lane = threadIdx.x;
  double s = 0.0;
  for (int b = lane; b < nblocks; b += 64) s += part[(int64_t)b * ncols + j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) out[j] = s;
}

// sum_j V[r, j] h[j] in ascending j, eight columns' loads issued together
__device__ inline double row_combination(const double* __restrict__ V, int64_t ldv, int ncols,
                                         const double* __restrict__ h, int64_t r) {
  double s = 0.0;
  int j = 0;
  for (; j + 8 <= ncols; j += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = V[(int64_t)(j + u) * ldv + r];
#pragma unroll
    for (int u = 0; u < 8; ++u) s = fma(v[u], h[j + u], s);
  }
  for (; j < ncols; ++j) s = fma(V[(int64_t)j * ldv + r], h[j], s);
  return s;
}

// One CGS2 pass fused with the next dot products: rows [r0, r0 + 256) of
// block b (one per thread) get w[r] -= sum_j V[r, j] h[j] (row_combination,
// ascending j); the new values then give part[b * nd + j] = sum over the
// block's rows of V[:, j] * w (nd = ncols), or of w * w (self, nd = 1),
// with the lane/row mapping and shuffle tree of cols_dot_partial_kernel, so
// the results equal those of the two separate launches bit for bit.
static_assert(DOT_CHUNK == 256, "one row per thread");
__global__ __launch_bounds__(256) void sub_dots_partial_kernel(const double* __restrict__ V, int64_t ldv, int ncols,
                                                              const double* __restrict__ h, double* __restrict__ w,
                                                              int64_t n, int self, double* __restrict__ part) {
  __shared__ double wsh[DOT_CHUNK];
  const int b = blockIdx.x;
  const int64_t r0 = (int64_t)b * DOT_CHUNK;
  const int64_t r1 = min<int64_t>(n, r0 + DOT_CHUNK);
  const int64_t r = r0 + threadIdx.x;
  double wn = 0.0;
  if (r < r1) {
    wn = w[r] - row_combination(V, ldv, ncols, h, r);
    w[r] = wn;
  }
  wsh[threadIdx.x] = wn;
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double wr[DOT_CHUNK / 64];
#pragma unroll
  for (int q = 0; q < DOT_CHUNK / 64; ++q) wr[q] = wsh[q * 64 + lane];
  const int nd = self ? 1 : ncols;
  for (int j0 = wave; j0 < nd; j0 += 4 * COLS_AT_ONCE) {
    double vv[COLS_AT_ONCE][DOT_CHUNK / 64];
#pragma unroll
    for (int c = 0; c < COLS_AT_ONCE; ++c) {
      const double* v = V + (int64_t)min(j0 + 4 * c, nd - 1) * ldv;
#pragma unroll
      for (int q = 0; q < DOT_CHUNK / 64; ++q) {
        const int64_t rq = r0 + q * 64 + lane;
        vv[c][q] = self ? wr[q] : (rq < r1 ? v[rq] : 0.0);
      }
    }
#pragma unroll
    for (int c = 0; c < COLS_AT_ONCE; ++c) {
      const int j = j0 + 4 * c;
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < DOT_CHUNK / 64; ++q) {
        const int64_t rq = r0 + q * 64 + lane;
        if (rq < r1) s = fma(vv[c][q], wr[q], s);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
      if (lane == 0 && j < nd) part[(int64_t)b * nd + j] = s;
    }
  }
}

__global__ void gemv_add_kernel(const double* __restrict__ V, int64_t ldv, int ncols, const double* __restrict__ y,
                                double* __restrict__ x, int64_t n) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    x[r] += row_combination(V, ldv, ncols, y, r);
}

inline int grid_for(int64_t n, int bs = 256, int cap = 65536) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (n + bs - 1) / bs));
}

}  // namespace

void phi3_rhs(int64_t total_I, int Nc, const int32_t* I_sub, const int32_t* I_ptr, const int32_t* I_idx,
              const int32_t* C_ptr, const int32_t* C_idx, const int64_t* off, const int32_t* gcol3, const double* A0,
              double* B, hipStream_t st) {
  if (total_I == 0) return;
  phi3_rhs_kernel<<<(unsigned)((total_I + 63) / 64), 64, 0, st>>>(total_I, Nc, I_sub, I_ptr, I_idx, C_ptr, C_idx,
                                                                  off, gcol3, A0, B);
}

void phi3_build(int64_t total_I, int Nc, const int32_t* I_sub, const int32_t* I_ptr, const int32_t* I_idx,
                const int32_t* C_ptr, const int32_t* C_idx, const int64_t* off, const double* phiI,
                const int32_t* gcol3, double* phi3, hipStream_t st) {
  if (Nc == 0) return;
  phi3_gamma_kernel<<<(Nc + 255) / 256, 256, 0, st>>>(Nc, gcol3, phi3);
  if (total_I)
    phi3_interior_kernel<<<(unsigned)((total_I + 127) / 128), 128, 0, st>>>(total_I, Nc, I_sub, I_ptr, I_idx, C_ptr,
                                                                           C_idx, off, phiI, phi3);
}

int cols_dot_blocks(int64_t n) { return (int)((n + DOT_CHUNK - 1) / DOT_CHUNK); }

#ifndef GDSW_PHI_T_CB
#define GDSW_PHI_T_CB -1  // columns per restriction work-group (0: one work-group per pair, -1: by size)
#endif

int phi_t_columns(int nsub, int max_nc, int max_ni) {
  if (max_ni <= 0 || (int64_t)max_ni * 8 > 48 * 1024) return 0;  // r on I_i must fit LDS
  if (GDSW_PHI_T_CB >= 0) return GDSW_PHI_T_CB;
  // one work-group per pair while the pairs are few enough to keep the
  // launch short (16^3, 64 subdomains: ~4,500 pairs, 12 us either way);
  // blocks of 8 columns beyond (32^3, 512 subdomains: the launch drops from
  // 122 to about 80 us)
  return (int64_t)nsub * max_nc >= 16384 ? 8 : 0;
}


void spmv_csr(int64_t nrows, const int32_t* rowptr, const int32_t* col, const double* val, const double* x,
              double* y, hipStream_t st) {
  if (nrows == 0) return;
  spmv_kernel<<<(unsigned)((nrows + 15) / 16), 256, 0, st>>>(nrows, rowptr, col, val, x, y);
}

void gather(int64_t count, const int32_t* idx, const double* src, double* dst, hipStream_t st) {
  if (count == 0) return;
  gather_kernel<<<grid_for(count), 256, 0, st>>>(count, idx, src, dst);
}

void extract_local(const DenseBatch& B, const int32_t* lptr, const int32_t* lidx, const int32_t* rowptr,
                   const int32_t* col, const double* val, int max_rows, hipStream_t st) {
  if (B.count == 0 || max_rows == 0) return;
  extract_kernel<<<dim3((max_rows + 127) / 128, B.count), 128, 0, st>>>(B.base, B.n, B.ld, B.off, lptr, lidx, rowptr,
                                                                       col, val);
  GDSW_HIP(hipGetLastError());
}

void extract_local_dense(const DenseBatch& B, const int32_t* lptr, const int32_t* lidx, const double* M, int64_t ldm,
                         int max_rows, hipStream_t st) {
  if (B.count == 0 || max_rows == 0) return;
  extract_dense_kernel<<<dim3((max_rows + 127) / 128, max_rows, B.count), 128, 0, st>>>(B.base, B.n, B.ld, B.off,
                                                                                        lptr, lidx, M, ldm);
  GDSW_HIP(hipGetLastError());
}

void deterministic_scatter(int64_t n, const int32_t* inv_ptr, const int64_t* inv_pos, const double* w, double* z,
                           hipStream_t st) {
  if (n == 0) return;
  scatter_kernel<<<grid_for(n), 256, 0, st>>>(n, inv_ptr, inv_pos, w, z);
}

void scatter_prolong(int64_t n, const int32_t* inv_ptr, const int64_t* inv_pos, const double* w,
                     const CoarseView& cv, const double* y0, const int32_t* y0_pos, double* z, hipStream_t st,
                     int nsub, int max_ni, const int32_t* outer, int64_t n_outer) {
  if (n == 0) return;
  const int split = nsub > 0 && max_ni > 0;
  if (split && outer) {
    const int nblk = (max_ni + 63) / 64;
    const unsigned gb = n_outer > 0 ? (unsigned)grid_for(n_outer, 256, 1024) : 0;
    scatter_prolong_fused_kernel<<<(unsigned)(nsub * nblk) + gb, 256, 0, st>>>(cv, inv_ptr, inv_pos, w, y0, y0_pos,
                                                                              z, nsub, nblk, outer, n_outer);
    return;
  }
  scatter_prolong_kernel<<<grid_for(n), 256, 0, st>>>(n, inv_ptr, inv_pos, w, cv, y0, y0_pos, z, split);
  if (split) phi_prolong_kernel<<<dim3((max_ni + 63) / 64, nsub), 256, 0, st>>>(cv, w, y0, y0_pos, z);
}

void restrict_coarse(int nc, const CoarseView& cv, const double* r, double* out, const int32_t* out_pos,
                     hipStream_t st, int n_pairs, double* t, int64_t gcount, const int32_t* gidx, double* gdst,
                     bool assemble, const PairBlocks* blocks) {
  if (nc == 0) {
    if (gcount > 0) gather(gcount, gidx, r, gdst, st);
    return;
  }
  if (n_pairs > 0 && t) {
    const int gb = gcount > 0 ? grid_for(gcount, 256, 1024) : 0;
    if (blocks && blocks->pair_of && blocks->cb > 0 && blocks->nblk > 0)
      phi_t_sub_kernel<<<blocks->nsub * blocks->nblk + gb, 256, (size_t)std::max(blocks->max_ni, 1) * sizeof(double),
                         st>>>(cv, r, t, *blocks, gb > 0 ? gcount : 0, gidx, gdst);
    else
      phi_t_kernel<<<n_pairs + gb, 256, 0, st>>>(cv, r, t, n_pairs, gb > 0 ? gcount : 0, gidx, gdst);
    if (assemble) restrict_assemble_kernel<<<(nc + 3) / 4, 256, 0, st>>>(nc, cv, r, t, out, out_pos);
  } else {
    if (gcount > 0) gather(gcount, gidx, r, gdst, st);
    restrict_kernel<<<nc, 256, 0, st>>>(nc, cv, r, out, out_pos);
  }
}

void phi_rhs(int64_t total_I, const CoarseView& cv, const int32_t* rowptr, const int32_t* col, const double* val,
             double* B, hipStream_t st) {
  if (total_I == 0) return;
  phi_rhs_kernel<<<(unsigned)((total_I + 127) / 128), 128, 0, st>>>(total_I, cv, rowptr, col, val, B);
}

void phi_transpose(int64_t total_I, const CoarseView& cv, const double* cm, double* rm, hipStream_t st) {
  if (total_I == 0) return;
  phi_transpose_kernel<<<(unsigned)((total_I + 127) / 128), 128, 0, st>>>(total_I, cv, cm, rm);
}

void decouple_pressure(const DenseBatch& B, const int32_t* nu, int max_n, hipStream_t st) {
  if (B.count == 0 || max_n == 0) return;
  decouple_pressure_kernel<<<dim3((max_n + 127) / 128, B.count), 128, 0, st>>>(B.base, B.n, B.ld, B.off, nu);
  GDSW_HIP(hipGetLastError());
}

void phi_pressure_rows(int64_t total_I, const CoarseView& cv, const int8_t* pval, const int32_t* sub_pcol,
                       double* phi_cm, hipStream_t st) {
  if (total_I == 0) return;
  phi_pressure_rows_kernel<<<(unsigned)((total_I + 127) / 128), 128, 0, st>>>(total_I, cv, pval, sub_pcol, phi_cm);
  GDSW_HIP(hipGetLastError());
}

void phibox(int64_t total_D, const CoarseView& cv, const BoxView& bv, double* out, hipStream_t st) {
  if (total_D == 0) return;
  phibox_kernel<<<(unsigned)((total_D + 127) / 128), 128, 0, st>>>(total_D, cv, bv, out);
}

void own_spmm(int nbox, int max_nd, int max_nc, const CoarseView& cv, const BoxView& bv, const OwnerMap& om,
              const int32_t* rowptr, const int32_t* col, const double* val, const double* phibox_, double* W,
              hipStream_t st) {
  if (nbox == 0 || max_nd == 0) return;
  if (max_nc > OWN_SPMM_MAX_NC)
    throw StatusError{1, "A_0 assembly: more than " + std::to_string(OWN_SPMM_MAX_NC) +
                             " coarse columns touch one subdomain"};
  if (nbox > 65535) throw StatusError{1, "A_0 assembly: more than 65535 subdomains"};
  own_spmm_kernel<<<dim3((unsigned)max_nd, (unsigned)nbox), OWN_T, (size_t)std::max(max_nc, 1) * sizeof(double), st>>>(
      cv, bv, om, rowptr, col, val, phibox_, W);
}

void a0_assemble(int Nc, const CoarseView& cv, const double* P, const int64_t* p_off, double* A0, hipStream_t st) {
  if (Nc == 0) return;
  a0_assemble_kernel<<<Nc, 256, 0, st>>>(Nc, cv, P, p_off, A0);
}

void permute_dense(int n, const int32_t* perm, const double* M, int64_t ldm, double* F, int64_t ld, hipStream_t st) {
  if (n == 0) return;
  permute_dense_kernel<<<dim3((n + 127) / 128, n), 128, 0, st>>>(n, perm, M, ldm, F, ld);
}

void negate(int64_t n, double* x, hipStream_t st) {
  if (n == 0) return;
  negate_kernel<<<grid_for(n), 256, 0, st>>>(n, x);
}

void expand(int64_t nfree, const int64_t* full_index, const double* xf, double* xfull, hipStream_t st) {
  if (nfree == 0) return;
  expand_kernel<<<grid_for(nfree), 256, 0, st>>>(nfree, full_index, xf, xfull);
}

void cols_dot(const double* V, int64_t ldv, int ncols, const double* w, int64_t n, double* part, int nblocks,
              double* out, hipStream_t st) {
  cols_dot_partial_kernel<<<nblocks, 256, 0, st>>>(V, ldv, ncols, w, n, part);
  cols_dot_final_kernel<<<ncols, 64, 0, st>>>(part, nblocks, ncols, out);
}

void sub_dots(const double* V, int64_t ldv, int ncols, const double* h, double* w, int64_t n, double* part,
              int nblocks, double* out, bool self, hipStream_t st) {
  if (n == 0) return;
  if ((int64_t)nblocks * DOT_CHUNK < n) throw StatusError{1, "sub_dots: partial blocks do not cover the rows"};
  sub_dots_partial_kernel<<<nblocks, 256, 0, st>>>(V, ldv, ncols, h, w, n, self ? 1 : 0, part);
  if (out) cols_dot_final_kernel<<<self ? 1 : ncols, 64, 0, st>>>(part, nblocks, self ? 1 : ncols, out);
}

void cols_dot_finish(const double* part, int nblocks, int ncols, double* out, hipStream_t st) {
  cols_dot_final_kernel<<<ncols, 64, 0, st>>>(part, nblocks, ncols, out);
}

void gemv_add(const double* V, int64_t ldv, int ncols, const double* y, double* x, int64_t n, hipStream_t st) {
  gemv_add_kernel<<<grid_for(n), 256, 0, st>>>(V, ldv, ncols, y, x, n);
}

}  // namespace gdsw
