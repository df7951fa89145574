// Block local solve: A_i^-1 from the saddle-point structure of A_i instead of
// a dense n_i x n_i inverse.  With the gradient form of the viscous term the
// velocity block of every local matrix is K_i = I_3 (x) L_i (the same scalar
// matrix L_i for each component, no coupling between components), so with
// S_i = B_i K_i^-1 B_i^T (SPD) the local solve of [K B^T; B 0] [u; p] = [f; g]
// is
//     U1 = L^-1 F,   p = S^-1 (B U1 - g),   u = U1 - L^-1 (B^T p)
// (F, U1: the velocity right-hand side and solution as three component
// vectors).  An apply reads L_i^-1 twice (upper tiles, three vectors per
// pass), S_i^-1 once and B_i twice: at 16^3 about a quarter of the bytes of
// the dense symmetric inverse, and the same operator up to rounding.  Where
// W_i = K_i^-1 B_i^T (formed at setup for S_i anyway) is smaller than the
// upper tiles of L_i^-1 (a continuous pressure: few pressure DOFs per local
// problem), it is kept and the last step is u = U1 - W p: one pass over
// L_i^-1, one over W_i, B_i once.
#include <hip/hip_runtime.h>

#include "context.h"
#include "kernels.h"
#include "kernels_ops.h"
#include "vec16.h"

namespace gdsw {
namespace {

// Bt of subdomain f (column q = the velocity vector B[q, :]^T in component-
// major order: entry (c, a) at c * npv + a) from the CSR rows of its
// pressure DOFs; velocity columns outside the local set are skipped.
__global__ void fill_bt_kernel(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                               const double* __restrict__ val, int64_t n_u, const int32_t* __restrict__ vx_ptr,
                               const int32_t* __restrict__ vx, const int32_t* __restrict__ pr_ptr,
                               const int32_t* __restrict__ pr, const int32_t* __restrict__ npv,
                               const int64_t* __restrict__ off, int f0, double* __restrict__ bt) {
  const int f = f0 + blockIdx.y;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int np = pr_ptr[f + 1] - pr_ptr[f];
  if (q >= np) return;
  const int nv = vx_ptr[f + 1] - vx_ptr[f];
  const int32_t* v = vx + vx_ptr[f];
  const int64_t ld = 3 * (int64_t)npv[f];
  double* out = bt + off[blockIdx.y] + (int64_t)q * ld;
  const int32_t g = pr[pr_ptr[f] + q];
  for (int32_t e = rowptr[g]; e < rowptr[g + 1]; ++e) {
    const int32_t c = col[e];
    if (c >= n_u) continue;  // pressure columns (the pressure block is zero)
    const int comp = c % 3;
    const int32_t key = c - comp;
    int lo = 0, hi = nv;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (v[mid] < key) lo = mid + 1; else hi = mid;
    }
    if (lo < nv && v[lo] == key) out[(int64_t)comp * npv[f] + lo] = val[e];
  }
}

// dst block f (np x np, ld npad) <- src (np x np, ld np)
__global__ void copy_blocks_kernel(const double* __restrict__ src, const int64_t* __restrict__ soff,
                                   const int32_t* __restrict__ N, double* __restrict__ base,
                                   const int64_t* __restrict__ doff, const int32_t* __restrict__ LD) {
  const int f = blockIdx.y;
  const int n = N[f];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)n * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % n), c = (int)(e / n);
    base[doff[f] + (int64_t)c * LD[f] + r] = src[soff[f] + e];
  }
}

// Sparse row products over the work vector, LPR lanes per row: lane l sums
// the row's entries l, l + LPR, ... in order, the lanes are combined by a
// fixed butterfly (the same sums on every run).
// mode 0: w[row_pos[r]] = sum - w[row_pos[r]]   (t = B U1 - g, pressure rows)
// mode 1: out[row_pos[r]] = sum                 (B^T p, velocity rows)
template <int LPR, int MODE>
__device__ inline void rowprod_rows(int64_t block, int64_t nrows, const int32_t* __restrict__ row_pos,
                                    const int64_t* __restrict__ ptr, const int32_t* __restrict__ pos,
                                    const double* __restrict__ val, double* __restrict__ w,
                                    double* __restrict__ out) {
  const int64_t r = (block * (int64_t)blockDim.x + threadIdx.x) / LPR;
  const int l = threadIdx.x % LPR;
  const bool live = r < nrows;  // uniform over the row's lanes
  double s = 0.0;
  if (live)
    for (int64_t k = ptr[r] + l; k < ptr[r + 1]; k += LPR) s = fma(val[k], w[pos[k]], s);
#pragma unroll
  for (int d = 1; d < LPR; d *= 2) s += __shfl_xor(s, d);
  if (live && l == 0) {
    if (MODE == 0)
      w[row_pos[r]] = s - w[row_pos[r]];
    else
      out[row_pos[r]] = s;
  }
}

template <int LPR, int MODE>
__global__ __launch_bounds__(256) void rowprod_kernel(int64_t nrows, const int32_t* __restrict__ row_pos,
                                                      const int64_t* __restrict__ ptr, const int32_t* __restrict__ pos,
                                                      const double* __restrict__ val, double* __restrict__ w,
                                                      double* __restrict__ out) {
  rowprod_rows<LPR, MODE>(blockIdx.x, nrows, row_pos, ptr, pos, val, w, out);
}

// t = B U1 - g (work-groups below nb_rows, a wave per pressure row) and, in
// the same launch, the coarse restriction's per-column assembly (the other
// work-groups, a wave per coarse column): both read only what earlier
// launches wrote, and the next launch (the Schur complement and coarse
// products) needs both.
__global__ __launch_bounds__(256) void rowprod_assemble_kernel(int64_t nrows, unsigned nb_rows,
                                                               const int32_t* __restrict__ row_pos,
                                                               const int64_t* __restrict__ ptr,
                                                               const int32_t* __restrict__ pos,
                                                               const double* __restrict__ val, double* __restrict__ w,
                                                               int nc, CoarseView cv, const double* __restrict__ r,
                                                               const double* __restrict__ t,
                                                               const int32_t* __restrict__ out_pos) {
  if (blockIdx.x < nb_rows) {  // uniform over the work-group
    rowprod_rows<64, 0>(blockIdx.x, nrows, row_pos, ptr, pos, val, w, nullptr);
    return;
  }
  const int c = (int)(blockIdx.x - nb_rows) * 4 + (threadIdx.x >> 6);
  if (c >= nc) return;  // uniform per wave
  restrict_assemble_column(c, threadIdx.x & 63, cv, r, t, w, out_pos);
}

// u_i -= W_i p_i for every local problem: W_i = K_i^-1 B_i^T (3 npad_i rows
// in the velocity segment's component-major order, np_i columns,
// column-major), p_i the pressure segment of the work vector.  Item: 64 E
// rows of one W_i (E rows per 16-byte piece); lane l of wave q takes rows
// r0 + E l .. + E - 1 and the columns q, q + 4, ..., eight loads in flight;
// the four wave sums are added in wave order, so results repeat bit for bit.
// Rows past 3 npad_i read as zero through the buffer resource.
template <typename T>
__global__ __launch_bounds__(256) void wp_sub_kernel(const T* __restrict__ W, const WItem* __restrict__ items,
                                                     double* __restrict__ w) {
  using Acc = typename VecW<T>::acc;
  constexpr int E = VecW<T>::W;
  constexpr int RW = 64 * E;
  constexpr int U = 8;
  __shared__ double ps[WP_MAX_NP];
  __shared__ Acc red[4][RW];
  const WItem it = items[blockIdx.x];
  const int t = threadIdx.x, lane = t % 64, q0 = t / 64;
  for (int k = t; k < it.np; k += 256) ps[k] = w[it.poff + k];
  __syncthreads();
  const __amdgpu_buffer_rsrc_t rs = buf_rsrc(W + it.woff, (uint32_t)((int64_t)it.rows * it.np * sizeof(T)));
  const int r = it.r0 + E * lane;
  Acc s[E];
#pragma unroll
  for (int e = 0; e < E; ++e) s[e] = 0;
  for (int q = q0; q < it.np; q += 4 * U) {
    Acc v[U][E];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int qq = q + 4 * u;
      const uint32_t off =
          qq < it.np && r < it.rows ? (uint32_t)(((int64_t)qq * it.rows + r) * sizeof(T)) : BUF_SKIP;
      if constexpr (sizeof(T) == 2)
        buf_load16_bf16<true>(rs, off, v[u]);
      else
        buf_load16<true>(rs, off, v[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int qq = q + 4 * u;
      const Acc pv = qq < it.np ? (Acc)ps[qq] : (Acc)0;
#pragma unroll
      for (int e = 0; e < E; ++e) s[e] = fma(v[u][e], pv, s[e]);
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) red[q0][E * lane + e] = s[e];
  __syncthreads();
  for (int k = t; k < RW; k += 256) {
    const int row = it.r0 + k;
    if (row < it.rows) {
      const double x = (((double)red[0][k] + (double)red[1][k]) + (double)red[2][k]) + (double)red[3][k];
      w[it.voff + row] -= x;
    }
  }
}

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65535)); }

}  // namespace

void block_fill_bt(const int32_t* rowptr, const int32_t* col, const double* val, int64_t n_u,
                   const int32_t* vx_ptr, const int32_t* vx, const int32_t* pr_ptr, const int32_t* pr,
                   const int32_t* npv, const int64_t* off, int f0, int cnt, int max_np, double* bt, hipStream_t st) {
  if (cnt == 0 || max_np == 0) return;
  fill_bt_kernel<<<dim3((max_np + 127) / 128, cnt), 128, 0, st>>>(rowptr, col, val, n_u, vx_ptr, vx, pr_ptr, pr, npv,
                                                                   off, f0, bt);
  GDSW_HIP(hipGetLastError());
}

void copy_blocks(const double* src, const int64_t* soff, const int32_t* n, int count, int64_t max_elems,
                 double* base, const int64_t* doff, const int32_t* ld, hipStream_t st) {
  if (count == 0 || max_elems == 0) return;
  copy_blocks_kernel<<<dim3(blocks_for(max_elems), count), 256, 0, st>>>(src, soff, n, base, doff, ld);
  GDSW_HIP(hipGetLastError());
}

bool block_assembles_restriction(const Context& ctx) {
  return ctx.solve_mode == SOLVE_BLOCK && ctx.P.spec.levels == 2 && ctx.Nc > 0 && ctx.n_pairs > 0 &&
         ctx.d_pair_t != nullptr && ctx.L1.count > 0;
}

int wp_rows_per_item(int prec) { return 64 * (prec == P_FP64 ? 2 : prec == P_FP32 ? 4 : 8); }

void wp_sub(int prec, const void* W, const WItem* items, int n_items, double* w, KernelTimer* tm, double bytes,
            hipStream_t st) {
  if (n_items == 0) return;
  if (tm && (!tm->on || tm->used >= KernelTimer::CAP)) tm = nullptr;
  if (prec == P_FP64)
    timed_launch(tm, bytes, wp_sub_kernel<double>, dim3(n_items), dim3(256), st, static_cast<const double*>(W),
                 items, w);
  else if (prec == P_FP32)
    timed_launch(tm, bytes, wp_sub_kernel<float>, dim3(n_items), dim3(256), st, static_cast<const float*>(W),
                 items, w);
  else
    timed_launch(tm, bytes, wp_sub_kernel<uint16_t>, dim3(n_items), dim3(256), st, static_cast<const uint16_t*>(W),
                 items, w);
  GDSW_HIP(hipGetLastError());
}

void block_local_solve(Context& ctx, hipStream_t st, double* part, const double* restrict_r) {
  const BlockSolve& b = ctx.blk;
  FactorSet& L = ctx.L1;
  if (L.count == 0) return;
  // partial sums: the sets' own buffers, or the caller's (the sets run one
  // after the other on st, so they may share it)
  double* pl = part ? part : L.d_partial;
  KernelTimer* tm = part ? nullptr : L.timer;
  // U1 = L^-1 F (three vectors per matrix, in place in the work vector)
  symv_desc_launch(L.prec, L.d_desc, L.gemv[0], pl, L.partial_len, st, nullptr, tm, (double)L.alg_bytes, 3);
  block_local_rest(ctx, st, part, restrict_r);
}

void block_local_rest(Context& ctx, hipStream_t st, double* part, const double* restrict_r) {
  const BlockSolve& b = ctx.blk;
  FactorSet& L = ctx.L1;
  if (L.count == 0) return;
  double* pl = part ? part : L.d_partial;
  KernelTimer* tm = part ? nullptr : L.timer;
  // t = B U1 - g in the pressure segments
  // pressure rows hold hundreds of entries: a wave per row
  const unsigned nb_rows = (unsigned)((b.n_prow * 64 + 255) / 256);
  if (restrict_r) {  // with the coarse restriction's assembly, whose input the caller passes
    const unsigned nb_asm = (unsigned)((ctx.Nc + 3) / 4);
    rowprod_assemble_kernel<<<nb_rows + nb_asm, 256, 0, st>>>(b.n_prow, nb_rows, b.d_prow_pos, b.d_bm_ptr,
                                                               b.d_bm_pos, b.d_bm_val, ctx.d_w, ctx.Nc,
                                                               coarse_view(ctx), restrict_r, ctx.d_pair_t,
                                                               ctx.d_coarse_pinv);
  } else {
    rowprod_kernel<64, 0><<<nb_rows, 256, 0, st>>>(b.n_prow, b.d_prow_pos, b.d_bm_ptr, b.d_bm_pos, b.d_bm_val,
                                                   ctx.d_w, nullptr);
  }
  // p = S^-1 t (and, with two levels, the coarse solve in the same launch)
  if (part) {
    const FactorSet& P = ctx.LP;
    if (P.count > 0 && !P.gemv.empty())
      symv_desc_launch(P.prec, P.d_desc, P.gemv[0], part, P.partial_len, st, nullptr, nullptr, 0.0);
  } else {
    local_solve_set(ctx.LP, ctx.d_w, st);
  }
  if (b.use_w) {  // u = U1 - W p
    wp_sub(L.prec, b.d_W, b.d_witems, b.n_witems, ctx.d_w, nullptr, 0.0, st);
    return;
  }
  // w2 = B^T p, then u = U1 - L^-1 w2 (the block-row sums subtract from U1)
  // velocity rows hold up to a few dozen: eight lanes per row
  rowprod_kernel<8, 1><<<(unsigned)((b.n_vrow * 8 + 255) / 256), 256, 0, st>>>(
      b.n_vrow, b.d_vrow_pos, b.d_bt_ptr, b.d_bt_pos, b.d_bt_val, ctx.d_w, b.d_w2);
  symv_desc_launch(L.prec, b.d_desc2, L.gemv[0], pl, L.partial_len, st, nullptr, tm, (double)L.alg_bytes, 3);
  GDSW_HIP(hipGetLastError());
}

}  // namespace gdsw
