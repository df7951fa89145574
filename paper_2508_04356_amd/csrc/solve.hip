// Preconditioner apply (eq. 2.2) and right-preconditioned FGMRES.
//
// Apply: every local right-hand side R_i r is gathered into one work vector,
// the coarse right-hand side Phi^T r is written next to them, one blocked
// triangular solve runs over all factors (the additive sum of eq. 2.2 makes
// the local and coarse solves independent), and one fixed-order scatter forms
// z = sum_i R_i^T y_i + Phi y_0.
//
// FGMRES follows the stated reading: x_0 = 0, classical Gram-Schmidt applied
// twice, Givens rotations, stop once |g_{j+1}| / ||b|| <= rtol, then
// x = x_0 + Z y and a recomputed true residual; restart from x if needed.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>

#include "context.h"
#include "kernels.h"
#include "kernels_learned.h"
#include "kernels_ops.h"
#include "learned.h"

namespace gdsw {

CoarseView coarse_view(const Context& c) {
  return CoarseView{c.d_gamma_col, c.d_dof_ipos, c.d_I_sub,  c.d_I_ptr,  c.d_I_idx,
                    c.d_C_ptr,     c.d_C_idx,    c.d_phi_off, c.d_phi_cm, c.d_phi_rm,
                    c.d_cg_ptr,    c.d_cg_dof,   c.d_cs_ptr,  c.d_cs_sub, c.d_cs_lc};
}

// (no row-major copy: the pair-sum restriction and the fused scatter read
// only the column-major blocks)
CoarseView coarse_view3(const Context& c) {
  return CoarseView{c.d_gcol3,   c.d_ipos3,   c.d_i2_sub, c.d_i2_ptr,   c.d_i2_idx,
                    c.d_c3_ptr,  c.d_c3_idx,  c.d_off2,   c.d_phi3_cm,  nullptr,
                    c.d_cg3_ptr, c.d_cg3_dof, c.d_cs3_ptr, c.d_cs3_sub, c.d_cs3_lc};
}

namespace {

__global__ void residual_kernel(int64_t n, const double* __restrict__ b, double* __restrict__ r) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    r[i] = b[i] - r[i];
}

// v = w / s[idx]
__global__ void scale_div_kernel(int64_t n, const double* __restrict__ w, const double* __restrict__ s, int idx,
                                 double* __restrict__ v) {
  const double d = s[idx];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = d != 0.0 ? w[i] / d : 0.0;
}

__global__ void sqrt_kernel(double* __restrict__ s, int idx) { s[idx] = sqrt(s[idx]); }

// start of a cycle: g = (beta, 0, ...), beta = sqrt(ss) in scal[1]
__global__ void cycle_start_kernel(double* __restrict__ g, int restart, double* __restrict__ scal) {
  const double beta = sqrt(scal[0]);
  scal[1] = beta;
  for (int i = 0; i <= restart; ++i) g[i] = i == 0 ? beta : 0.0;
}

// Arnoldi column j: H[:j+1, j] = h1 + h2, H[j+1, j] = ||w||, previous rotations,
// new rotation, g update; scal[2] = |g_{j+1}| / ||b||, scal[3] = ||w||.
__global__ void arnoldi_finish_kernel(int j, int restart, const double* __restrict__ h1,
                                      const double* __restrict__ h2, double* __restrict__ H,
                                      double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g,
                                      double* __restrict__ scal) {
  const double bnorm = scal[5];  // ||b||, stored once per solve (a captured graph reads it too)
  const int ldh = restart + 1;
  double* col = H + (int64_t)j * ldh;
  for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
  const double hn = sqrt(scal[4]);
  col[j + 1] = hn;
  scal[3] = hn;
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  const double rho = hypot(col[j], col[j + 1]);
  cs[j] = col[j] / rho;
  sn[j] = col[j + 1] / rho;
  col[j] = rho;
  col[j + 1] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  scal[2] = fabs(g[j + 1]) / bnorm;
}

inline int grid_n(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(65536, (n + 255) / 256)); }

// cols_dot_final_kernel of ||w||^2, arnoldi_finish_kernel and
// scale_div_kernel(n, w, scal, 3, v) in one launch: every work-group sums the
// partial blocks of ||w||^2 (one wave, lane-strided, xor tree: the same sum
// as cols_dot_final_kernel) and scales w into the next basis vector by
// ||w||; the first also stores ||w||^2 in scal[4] and finishes column j of
// H, its threads
// loading the column and the previous rotations into LDS together and one
// thread applying the rotations in order (the same operations as
// arnoldi_finish_kernel).  For restart <= ARN_LDS.
constexpr int ARN_LDS = 512;
__global__ __launch_bounds__(256) void arnoldi_scale_kernel(int j, int restart, const double* __restrict__ h1,
                                                            const double* __restrict__ h2, double* __restrict__ H,
                                                            double* __restrict__ cs, double* __restrict__ sn,
                                                            double* __restrict__ g, double* __restrict__ scal,
                                                            const double* __restrict__ part, int nblocks,
                                                            int64_t n, const double* __restrict__ w,
                                                            double* __restrict__ v, double* __restrict__ host_out) {
  __shared__ double cl[ARN_LDS + 2], cs_l[ARN_LDS], sn_l[ARN_LDS];
  __shared__ double ww;
  if (threadIdx.x < 64) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 64) s += part[b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x == 0) ww = s;
  }
  __syncthreads();
  const double hn = sqrt(ww);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = hn != 0.0 ? w[i] / hn : 0.0;
  if (blockIdx.x != 0) return;  // uniform over the work-group
  const int t = threadIdx.x;
  for (int i = t; i <= j; i += 256) cl[i] = h1[i] + h2[i];
  for (int i = t; i < j; i += 256) {
    cs_l[i] = cs[i];
    sn_l[i] = sn[i];
  }
  __syncthreads();
  if (t == 0) {
    scal[4] = ww;
    cl[j + 1] = hn;
    scal[3] = hn;
    for (int i = 0; i < j; ++i) {
      const double u = cs_l[i] * cl[i] + sn_l[i] * cl[i + 1];
      cl[i + 1] = -sn_l[i] * cl[i] + cs_l[i] * cl[i + 1];
      cl[i] = u;
    }
    const double rho = hypot(cl[j], cl[j + 1]);
    const double c = cl[j] / rho, sj = cl[j + 1] / rho;
    cs[j] = c;
    sn[j] = sj;
    cl[j] = rho;
    cl[j + 1] = 0.0;
    const double gj = g[j];
    g[j + 1] = -sj * gj;
    g[j] = c * gj;
    scal[2] = fabs(g[j + 1]) / scal[5];
    if (host_out) {  // the iteration's record straight into pinned host memory
      host_out[0] = scal[2];
      host_out[1] = hn;
    }
  }
  __syncthreads();
  const int ldh = restart + 1;
  for (int i = t; i <= j + 1; i += 256) H[(int64_t)j * ldh + i] = cl[i];
}

// column j of the Arnoldi process after the projections (part: the
// partial blocks of ||w||^2): H, rotations, g, residual estimate, and the
// next basis vector
// host_out (device view of pinned host memory, or null): the kernel writes
// the residual estimate and ||w|| there itself, so no copy follows
bool arnoldi_step(int j, int restart, const double* h1, const double* h2, double* H, double* cs, double* sn,
                  double* g, double* scal, const double* part, int nblocks, int64_t n, const double* w, double* v,
                  hipStream_t st, double* host_out = nullptr) {
  if (restart <= ARN_LDS) {
    arnoldi_scale_kernel<<<grid_n(n), 256, 0, st>>>(j, restart, h1, h2, H, cs, sn, g, scal, part, nblocks, n, w, v,
                                                    host_out);
    return host_out != nullptr;
  }
  cols_dot_finish(part, nblocks, 1, scal + 4, st);
  arnoldi_finish_kernel<<<1, 1, 0, st>>>(j, restart, h1, h2, H, cs, sn, g, scal);
  scale_div_kernel<<<grid_n(n), 256, 0, st>>>(n, w, scal, 3, v);
  return false;
}

// back substitution y = H[:k,:k]^-1 g[:k] into y (H upper triangular,
// column-major, ld = restart + 1), one thread, row by row
__global__ void back_subst_kernel(int k, int restart, const double* __restrict__ H, const double* __restrict__ g,
                                  double* __restrict__ y) {
  const int ldh = restart + 1;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int l = i + 1; l < k; ++l) s -= H[(int64_t)l * ldh + i] * y[l];
    y[i] = s / H[(int64_t)i * ldh + i];
  }
}

// The same back substitution by columns, for k <= BS_MAX: the work-group
// stages the upper triangle of H[:k,:k] in LDS (packed by columns, every
// load in flight at once), then wave 0 alone runs the k dependent steps
// with the row sums in registers (lane l: rows l and l + 64): at step
// i = k - 1, ..., 0 the owner of row i divides its finished sum by H(i,i),
// the quotient goes to every lane by a shuffle, and each lane subtracts
// H(t,i) y_i from its rows t < i.  Row t thus gets g_t minus the products
// in descending column order, the same on every run.  (One thread walking
// the global H took 88 us for k = 42; the dependent steps here are a
// shuffle, a division and a multiply-add.)
constexpr int BS_MAX = 127;  // the packed triangle fits 64 KB of LDS
__global__ __launch_bounds__(256) void back_subst_lds_kernel(int k, int restart, const double* __restrict__ H,
                                                             const double* __restrict__ g,
                                                             double* __restrict__ y) {
  extern __shared__ double tri[];  // column i at i (i + 1) / 2, rows 0 .. i
  const int ldh = restart + 1;
  const int nt = k * (k + 1) / 2;
  for (int e = threadIdx.x; e < nt; e += 256) {
    // column of packed entry e: the largest i with i (i + 1) / 2 <= e
    int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > e) --i;
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    tri[e] = H[(int64_t)i * ldh + (e - i * (i + 1) / 2)];
  }
  __syncthreads();
  if (threadIdx.x >= 64) return;  // uniform per wave; no barrier follows
  const int l = threadIdx.x;
  double s0 = l < k ? g[l] : 0.0, s1 = l + 64 < k ? g[l + 64] : 0.0;
  double y0 = 0.0, y1 = 0.0;
  for (int i = k - 1; i >= 0; --i) {
    const double* col = tri + i * (i + 1) / 2;
    const double si = __shfl(i < 64 ? s0 : s1, i & 63, 64);
    const double yi = si / col[i];
    if (l == (i & 63)) {
      if (i < 64) y0 = yi; else y1 = yi;
    }
    if (l < i) s0 -= col[l] * yi;
    if (l + 64 < i) s1 -= col[l + 64] * yi;
  }
  if (l < k) y[l] = y0;
  if (l + 64 < k) y[l + 64] = y1;
}

void back_subst(int k, int restart, const double* H, const double* g, double* y, hipStream_t st) {
  if (k <= 0) return;
  if (k <= BS_MAX)
    back_subst_lds_kernel<<<1, 256, (size_t)k * (k + 1) / 2 * sizeof(double), st>>>(k, restart, H, g, y);
  else
    back_subst_kernel<<<1, 1, 0, st>>>(k, restart, H, g, y);
}


void drop_graphs(Context& ctx) {
  for (hipGraphExec_t& e : ctx.graphs.exec)
    if (e) (void)hipGraphExecDestroy(e);
  ctx.graphs.exec.clear();
  ctx.graphs.V = nullptr;
}

void ensure_workspace(Context& ctx, int restart) {
  if (ctx.restart >= restart && ctx.d_V) return;
  drop_graphs(ctx);
  DeviceArena& A = ctx.arena;
  for (void* p : {(void*)ctx.d_V, (void*)ctx.d_Z, (void*)ctx.d_H, (void*)ctx.d_g, (void*)ctx.d_cs,
                  (void*)ctx.d_sn, (void*)ctx.d_hv, (void*)ctx.d_part, (void*)ctx.d_scal, (void*)ctx.d_t1,
                  (void*)ctx.d_t2})
    if (p) A.free(p);
  const int64_t n = ctx.P.n_free;
  ctx.ldv = (n + 63) / 64 * 64;
  ctx.restart = restart;
  ctx.d_V = dalloc<double>(A, ctx.ldv * (restart + 1));
  ctx.d_Z = dalloc<double>(A, ctx.ldv * restart);
  ctx.d_H = dalloc<double>(A, (int64_t)(restart + 1) * restart);
  ctx.d_g = dalloc<double>(A, restart + 1);
  ctx.d_cs = dalloc<double>(A, restart);
  ctx.d_sn = dalloc<double>(A, restart);
  ctx.d_hv = dalloc<double>(A, 2 * (restart + 1));
  ctx.n_part_blocks = cols_dot_blocks(n);
  ctx.d_part = dalloc<double>(A, (int64_t)ctx.n_part_blocks * (restart + 1));
  ctx.d_scal = dalloc<double>(A, 16);
  ctx.d_t1 = dalloc<double>(A, ctx.ldv);
  ctx.d_t2 = dalloc<double>(A, ctx.ldv);
  if (!ctx.h_pinned) {
    GDSW_HIP(hipHostMalloc((void**)&ctx.h_pinned, 16 * sizeof(double), hipHostMallocDefault));
    GDSW_HIP(hipHostGetDevicePointer((void**)&ctx.d_pinned, ctx.h_pinned, 0));
  }
  for (hipEvent_t& e : ctx.it_ev)
    if (!e) GDSW_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

double read_scalar(Context& ctx, int idx, hipStream_t st) {
  GDSW_HIP(hipMemcpyAsync(ctx.h_pinned, ctx.d_scal + idx, sizeof(double), hipMemcpyDeviceToHost, st));
  GDSW_HIP(hipStreamSynchronize(st));
  return ctx.h_pinned[0];
}

}  // namespace

void spmv(Context& ctx, const double* x, double* y, hipStream_t st) {
  spmv_csr(ctx.P.n_free, ctx.d_rowptr, ctx.d_col, ctx.d_val, x, y, st);
}

PairBlocks pair_blocks(const Context& ctx) {
  PairBlocks pb;
  if (ctx.phi_cb > 0) {
    pb.pair_of = ctx.d_pair_of;
    pb.nsub = ctx.P.n_sub;
    pb.nblk = ctx.phi_nblk;
    pb.cb = ctx.phi_cb;
    pb.max_ni = ctx.max_ni;
  }
  return pb;
}

void apply_pre(Context& ctx, const double* r, hipStream_t st) {
  const CoarseView cv = coarse_view(ctx);
  const PairBlocks pb = pair_blocks(ctx);
  const bool three = ctx.P.spec.levels == 3 && ctx.Nc > 0;
  if (three) {
    gather(ctx.n_w1, ctx.d_gidx, r, ctx.d_w, st);
    // r0 = Phi^T r; level-2 copies R_j^(2) r0; level-3 right-hand side Phi3^T r0
    restrict_coarse(ctx.Nc, cv, r, ctx.d_r0, nullptr, st, ctx.n_pairs, ctx.d_pair_t, 0, nullptr, nullptr, true, &pb);
    gather(ctx.HI.total_x, ctx.d_g2idx, ctx.d_r0, ctx.d_w + ctx.n_w1, st);
    // level-3 right-hand side (Phi^(3))^T r0: per-pair sums over the
    // subregion interiors, assembled per level-3 column with its interface
    // part
    restrict_coarse(ctx.Nc3, coarse_view3(ctx), ctx.d_r0, ctx.d_w, ctx.d_c3_pinv, st, ctx.n_pairs3, ctx.d_pair_t3);
  } else if (ctx.Nc > 0) {
    // the local copies are gathered by the same launch as the restriction;
    // the block solve assembles the restriction in its B row launch
    restrict_coarse(ctx.Nc, cv, r, ctx.d_w, ctx.d_coarse_pinv, st, ctx.n_pairs, ctx.d_pair_t, ctx.n_w1, ctx.d_gidx,
                    ctx.d_w, !block_assembles_restriction(ctx), &pb);
  } else {
    gather(ctx.n_w1, ctx.d_gidx, r, ctx.d_w, st);
  }
}

void apply_post(Context& ctx, double* z, hipStream_t st) {
  const CoarseView cv = coarse_view(ctx);
  const bool three = ctx.P.spec.levels == 3 && ctx.Nc > 0;
  if (three) {
    // y0 = sum_j R_j^(2)T y_j + Phi3 y3, then z = sum_i R_i^T y_i + Phi y0
    scatter_prolong(ctx.Nc, ctx.d_inv2_ptr, ctx.d_inv2_pos, ctx.d_w, coarse_view3(ctx), nullptr, ctx.d_c3_pinv,
                    ctx.d_y0, st, ctx.n_sub2, ctx.max_ni2, ctx.d_outer3, ctx.n_outer3);
    scatter_prolong(ctx.P.n_free, ctx.d_inv_ptr, ctx.d_inv_pos, ctx.d_w, cv, ctx.d_y0, nullptr, z, st,
                    ctx.P.n_sub, ctx.max_ni, ctx.d_outer, ctx.n_outer);
  } else if (ctx.Nc > 0) {
    scatter_prolong(ctx.P.n_free, ctx.d_inv_ptr, ctx.d_inv_pos, ctx.d_w, cv, nullptr, ctx.d_coarse_pinv, z, st,
                    ctx.P.n_sub, ctx.max_ni, ctx.d_outer, ctx.n_outer);
  } else {
    deterministic_scatter(ctx.P.n_free, ctx.d_inv_ptr, ctx.d_inv_pos, ctx.d_w, z, st);
  }
}

void apply_precond(Context& ctx, const double* r, double* z, hipStream_t st, hipEvent_t* ev) {
  if (ev) GDSW_HIP(hipEventRecord(ev[0], st));
  apply_pre(ctx, r, st);
  if (ev) GDSW_HIP(hipEventRecord(ev[1], st));
  if (ctx.local_solver != 0 && ctx.learned) {
    // interior subdomains: learned solve (1) or no local correction (2)
    const GridMap gm = learned_gridmap(ctx);
    LearnedSolve* L = ctx.learned;
    copy_segments(gm, L->S, ctx.d_w, L->d_rsave, nullptr, st);
    local_solve_set(ctx.L1, ctx.d_w, st, 1);
    if (ctx.local_solver == 1)
      learned_apply_interior(ctx, st);
    else
      zero_segments(gm, L->S, ctx.d_w, st);
  } else if (ctx.solve_mode == SOLVE_BLOCK) {
    block_local_solve(ctx, st, nullptr, block_assembles_restriction(ctx) ? r : nullptr);
  } else {
    local_solve_set(ctx.L1, ctx.d_w, st);
  }
  if (ev) GDSW_HIP(hipEventRecord(ev[2], st));
  local_solve_set(ctx.HI, ctx.d_w, st);
  if (ev) GDSW_HIP(hipEventRecord(ev[3], st));
  apply_post(ctx, z, st);
  if (ev) GDSW_HIP(hipEventRecord(ev[4], st));
  GDSW_HIP(hipGetLastError());
}

void expand_solution(const Context& ctx, const double* xf, double* xfull, hipStream_t st) {
  GDSW_HIP(hipMemcpyAsync(xfull, ctx.d_dirichlet_full, ctx.P.n_full * sizeof(double), hipMemcpyDeviceToDevice, st));
  expand(ctx.P.n_free, ctx.d_full_index, xf, xfull, st);
  GDSW_HIP(hipGetLastError());
}

namespace {

void put_bnorm(Context& ctx, double bnorm, hipStream_t st) {
  ctx.h_pinned[8] = bnorm;
  GDSW_HIP(hipMemcpyAsync(ctx.d_scal + 5, ctx.h_pinned + 8, sizeof(double), hipMemcpyHostToDevice, st));
  GDSW_HIP(hipStreamSynchronize(st));
}

}  // namespace

void release_graphs(Context& ctx) {
  drop_graphs(ctx);
  if (ctx.graphs.stream) (void)hipStreamDestroy(ctx.graphs.stream);
  ctx.graphs.stream = nullptr;
}

FgmresResult fgmres(Context& ctx, const double* b, double* x, double rtol, int restart, int max_it, bool use_graph,
                    hipStream_t st, double* history, int history_len) {
  ensure_workspace(ctx, restart);
  // Graph mode: the iteration body for basis index j is captured once into a
  // HIP graph (no memset nodes; every argument is fixed for a given j and
  // workspace) and replayed in every later cycle and solve.  Capture needs a
  // stream other than the legacy default one: the context's own stream then
  // carries the whole solve.  The learned solve reads back counts inside the
  // apply and stays eager.
  const bool graph = use_graph && !(ctx.local_solver != 0 && ctx.learned);
  if (graph) {
    // a re-plan (autotuner, schedule, learned subsets) frees and replaces the
    // item arrays and partial buffers the captured kernels point at
    if (ctx.graphs.V != ctx.d_V || ctx.graphs.restart != restart || ctx.graphs.gen1 != ctx.L1.gen ||
        ctx.graphs.gen2 != ctx.HI.gen) {
      drop_graphs(ctx);
      ctx.graphs.V = ctx.d_V;
      ctx.graphs.restart = restart;
      ctx.graphs.gen1 = ctx.L1.gen;
      ctx.graphs.gen2 = ctx.HI.gen;
      ctx.graphs.exec.assign(restart, nullptr);
    }
    if (st == nullptr) {
      if (!ctx.graphs.stream) GDSW_HIP(hipStreamCreateWithFlags(&ctx.graphs.stream, hipStreamNonBlocking));
      GDSW_HIP(hipStreamSynchronize(nullptr));  // the caller's earlier work on the default stream
      st = ctx.graphs.stream;
    }
  }
  const int64_t n = ctx.P.n_free;
  const int64_t ldv = ctx.ldv;
  double* V = ctx.d_V;
  double* Z = ctx.d_Z;
  double* S = ctx.d_scal;
  const int nb = ctx.n_part_blocks;
  FgmresResult res;
  // ||b||
  cols_dot(b, ldv, 1, b, n, ctx.d_part, nb, S + 0, st);
  const double bnorm = std::sqrt(read_scalar(ctx, 0, st));
  GDSW_HIP(hipMemsetAsync(x, 0, n * sizeof(double), st));
  if (bnorm == 0.0) {
    res.converged = true;
    GDSW_HIP(hipStreamSynchronize(st));
    return res;
  }
  put_bnorm(ctx, bnorm, st);
  auto body = [&](int j) {
    double* vj = V + (int64_t)j * ldv;
    double* zj = Z + (int64_t)j * ldv;
    double* w = ctx.d_t2;
    apply_precond(ctx, vj, zj, st);
    spmv(ctx, zj, w, st);
    // CGS2: two projections, each fused with the dot products that follow it
    cols_dot(V, ldv, j + 1, w, n, ctx.d_part, nb, ctx.d_hv, st);
    sub_dots(V, ldv, j + 1, ctx.d_hv, w, n, ctx.d_part, nb, ctx.d_hv + restart + 1, false, st);
    sub_dots(V, ldv, j + 1, ctx.d_hv + restart + 1, w, n, ctx.d_part, nb, nullptr, true, st);
    if (!arnoldi_step(j, restart, ctx.d_hv, ctx.d_hv + restart + 1, ctx.d_H, ctx.d_cs, ctx.d_sn, ctx.d_g, S,
                      ctx.d_part, nb, n, w, V + (int64_t)(j + 1) * ldv, st, ctx.d_pinned + 10 + 2 * (j & 1)))
      GDSW_HIP(hipMemcpyAsync(ctx.h_pinned + 10 + 2 * (j & 1), S + 2, 2 * sizeof(double), hipMemcpyDeviceToHost,
                              st));
  };
  auto launch = [&](int j) {
    if (graph) {
      hipGraphExec_t& e = ctx.graphs.exec[j];
      if (!e) {
        KernelTimer* tm = ctx.L1.timer;
        ctx.L1.timer = nullptr;  // no event nodes in the graph
        hipGraph_t g = nullptr;
        GDSW_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        body(j);
        GDSW_HIP(hipStreamEndCapture(st, &g));
        ctx.L1.timer = tm;
        GDSW_HIP(hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
        GDSW_HIP(hipGraphDestroy(g));
      }
      GDSW_HIP(hipGraphLaunch(e, st));
    } else {
      body(j);
    }
    GDSW_HIP(hipEventRecord(ctx.it_ev[j & 1], st));
  };
  int it = 0;
  int cycles = 0;
  while (true) {
    // r = b - A x
    spmv(ctx, x, ctx.d_t1, st);
    residual_kernel<<<grid_n(n), 256, 0, st>>>(n, b, ctx.d_t1);
    cols_dot(ctx.d_t1, ldv, 1, ctx.d_t1, n, ctx.d_part, nb, S + 0, st);
    cycle_start_kernel<<<1, 1, 0, st>>>(ctx.d_g, restart, S);
    const double beta = read_scalar(ctx, 1, st);
    res.true_rel = beta / bnorm;
    if (res.true_rel <= rtol) {
      res.converged = true;
      break;
    }
    if (it >= max_it) break;
    scale_div_kernel<<<grid_n(n), 256, 0, st>>>(n, ctx.d_t1, S, 1, V);
    // Iteration j + 1 is enqueued before the host waits for iteration j, so
    // the GPU does not idle while the host reads the estimate and launches
    // the next iteration.  If iteration j ends the cycle, iteration j + 1 has
    // run for nothing: it writes only column j + 1 of H, g[j + 1], g[j + 2],
    // rotation j + 1, V_{j+2} and Z_{j+1}, none of which the update with
    // j + 1 columns below reads, and the next cycle starts afresh.  Each
    // iteration writes its estimate to its own pinned slot (j % 2).
    // Iteration j + 1 is not enqueued ahead when the estimates so far,
    // extrapolated geometrically, put iteration j at the tolerance already
    // (saves the wasted iteration at the end of a solve; a wrong guess only
    // costs one host round trip).
    int k = 0;
    bool queued = false;  // iteration j already enqueued
    double rel1 = 0.0, rel2 = 0.0;  // estimates of iterations j - 1 and j - 2 of this cycle
    for (int j = 0; j < restart; ++j) {
      if (!queued) launch(j);
      const bool last = j >= 2 && rel2 > 0.0 && rel1 * (rel1 / rel2) <= rtol;
      queued = j + 1 < restart && it + 1 < max_it && !last;
      if (queued) launch(j + 1);
      GDSW_HIP(hipEventSynchronize(ctx.it_ev[j & 1]));
      const double rel = ctx.h_pinned[10 + 2 * (j & 1)];
      const double hn = ctx.h_pinned[11 + 2 * (j & 1)];
      rel2 = rel1;
      rel1 = rel;
      if (history && it < history_len) history[it] = rel;
      ++it;
      k = j + 1;
      res.rel = rel;
      if (!std::isfinite(rel)) throw StatusError{4, "FGMRES: non-finite residual estimate (NaN in the Arnoldi norm)"};
      if (rel <= rtol || hn == 0.0 || it >= max_it) break;
    }
    back_subst(k, restart, ctx.d_H, ctx.d_g, ctx.d_hv, st);
    gemv_add(Z, ldv, k, ctx.d_hv, x, n, st);
    ++cycles;
    // true residual
    spmv(ctx, x, ctx.d_t1, st);
    residual_kernel<<<grid_n(n), 256, 0, st>>>(n, b, ctx.d_t1);
    cols_dot(ctx.d_t1, ldv, 1, ctx.d_t1, n, ctx.d_part, nb, S + 0, st);
    sqrt_kernel<<<1, 1, 0, st>>>(S, 0);
    res.true_rel = read_scalar(ctx, 0, st) / bnorm;
    if (res.true_rel <= rtol) {
      res.converged = true;
      break;
    }
    if (it >= max_it) break;
  }
  res.iterations = it;
  res.restarts = std::max(0, cycles - 1);
  GDSW_HIP(hipStreamSynchronize(st));
  GDSW_HIP(hipGetLastError());
  return res;
}

// Lockstep FGMRES over the members of a batch: every member runs exactly the
// steps of fgmres() above (same kernels, same order, hence bitwise the same
// iterates as a solve of that member alone); per iteration the members'
// local and coarse solves share one launch pair per level, and the host
// reads every member's residual estimate after one synchronisation.
std::vector<FgmresResult> fgmres_batch(Batch& bt, const double* const* bvec, double* const* xv, double rtol,
                                       int restart, int max_it, hipStream_t st, bool use_graph) {
  const int K = (int)bt.m.size();
  std::vector<FgmresResult> res(K);
  std::vector<double> bnorm(K, 0.0);
  std::vector<char> done(K, 0), in_cycle(K, 0);
  std::vector<int> kc(K, 0), cycles(K, 0);
  double* hp = bt.h_pinned;
  for (int k = 0; k < K; ++k) ensure_workspace(*bt.m[k], restart);
  // Graph mode: the iteration body for basis index j and the set of members
  // in the cycle (the forks onto the lanes, every member's kernels, the
  // merged products and the read-back copies) is captured once and replayed
  // whenever the same (j, set) recurs, in later cycles and solves.  The
  // merged products read their member flags from the device, uploaded by
  // batch_select outside the graph whenever the set changes.  Members with a
  // learned interior solve read back counts inside the iteration and keep
  // the batch eager.
  bool graph = use_graph;
  for (int k = 0; k < K; ++k) graph = graph && !batch_learned(*bt.m[k]);
  if (graph) {
    std::vector<double*> Vs(K);
    for (int k = 0; k < K; ++k) Vs[k] = bt.m[k]->d_V;
    if (Vs != bt.graph_V || bt.graph_restart != restart) {
      batch_drop_graphs(bt);
      bt.graph_V = Vs;
      bt.graph_restart = restart;
    }
    if (st == nullptr) {
      if (!bt.gstream) GDSW_HIP(hipStreamCreateWithFlags(&bt.gstream, hipStreamNonBlocking));
      GDSW_HIP(hipStreamSynchronize(nullptr));  // the caller's earlier work on the default stream
      st = bt.gstream;
    }
  }
  batch_fork(bt, st);
  for (int k = 0; k < K; ++k) {
    Context& c = *bt.m[k];
    const hipStream_t ls = batch_lane(bt, k);
    cols_dot(bvec[k], c.ldv, 1, bvec[k], c.P.n_free, c.d_part, c.n_part_blocks, c.d_scal + 0, ls);
    GDSW_HIP(hipMemcpyAsync(hp + k, c.d_scal + 0, sizeof(double), hipMemcpyDeviceToHost, ls));
    GDSW_HIP(hipMemsetAsync(xv[k], 0, c.P.n_free * sizeof(double), ls));
  }
  batch_join(bt, st);
  GDSW_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < K; ++k) {
    bnorm[k] = std::sqrt(hp[k]);
    if (bnorm[k] == 0.0) {
      res[k].converged = true;
      done[k] = 1;
    } else {
      put_bnorm(*bt.m[k], bnorm[k], st);
    }
  }
  while (true) {
    // r = b - A x and beta for every member still running
    batch_fork(bt, st);
    for (int k = 0; k < K; ++k) {
      if (done[k]) continue;
      Context& c = *bt.m[k];
      const hipStream_t ls = batch_lane(bt, k);
      const int64_t n = c.P.n_free;
      spmv(c, xv[k], c.d_t1, ls);
      residual_kernel<<<grid_n(n), 256, 0, ls>>>(n, bvec[k], c.d_t1);
      cols_dot(c.d_t1, c.ldv, 1, c.d_t1, n, c.d_part, c.n_part_blocks, c.d_scal + 0, ls);
      cycle_start_kernel<<<1, 1, 0, ls>>>(c.d_g, restart, c.d_scal);
      GDSW_HIP(hipMemcpyAsync(hp + k, c.d_scal + 1, sizeof(double), hipMemcpyDeviceToHost, ls));
    }
    batch_join(bt, st);
    GDSW_HIP(hipStreamSynchronize(st));
    int running = 0;
    for (int k = 0; k < K; ++k) {
      in_cycle[k] = 0;
      kc[k] = 0;
      if (done[k]) continue;
      res[k].true_rel = hp[k] / bnorm[k];
      if (res[k].true_rel <= rtol) {
        res[k].converged = true;
        done[k] = 1;
      } else if (res[k].iterations >= max_it) {
        done[k] = 1;
      } else {
        in_cycle[k] = 1;
        ++cycles[k];
        ++running;
        Context& c = *bt.m[k];
        scale_div_kernel<<<grid_n(c.P.n_free), 256, 0, st>>>(c.P.n_free, c.d_t1, c.d_scal, 1, c.d_V);
      }
    }
    if (running == 0) break;
    batch_select(bt, in_cycle, st);
    auto body = [&](int j) {
      batch_fork(bt, st);
      for (int k = 0; k < K; ++k) {
        if (!in_cycle[k]) continue;
        apply_pre(*bt.m[k], bt.m[k]->d_V + (int64_t)j * bt.m[k]->ldv, batch_lane(bt, k));
        if (batch_learned(*bt.m[k])) batch_save_interior(*bt.m[k], batch_lane(bt, k));
      }
      batch_join(bt, st);
      batch_local_solve(bt, st);
      batch_learned_solves(bt, in_cycle, st);
      batch_fork(bt, st);
      for (int k = 0; k < K; ++k) {
        if (!in_cycle[k]) continue;
        Context& c = *bt.m[k];
        const hipStream_t ls = batch_lane(bt, k);
        const int64_t n = c.P.n_free;
        double* V = c.d_V;
        double* zj = c.d_Z + (int64_t)j * c.ldv;
        double* w = c.d_t2;
        batch_block_rest(c, V + (int64_t)j * c.ldv, ls);
        apply_post(c, zj, ls);
        spmv(c, zj, w, ls);
        cols_dot(V, c.ldv, j + 1, w, n, c.d_part, c.n_part_blocks, c.d_hv, ls);
        sub_dots(V, c.ldv, j + 1, c.d_hv, w, n, c.d_part, c.n_part_blocks, c.d_hv + restart + 1, false, ls);
        sub_dots(V, c.ldv, j + 1, c.d_hv + restart + 1, w, n, c.d_part, c.n_part_blocks, nullptr, true, ls);
        arnoldi_step(j, restart, c.d_hv, c.d_hv + restart + 1, c.d_H, c.d_cs, c.d_sn, c.d_g, c.d_scal, c.d_part,
                     c.n_part_blocks, n, w, V + (int64_t)(j + 1) * c.ldv, ls);
        GDSW_HIP(hipMemcpyAsync(hp + 2 * k, c.d_scal + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, ls));
      }
      batch_join(bt, st);
    };
    for (int j = 0; j < restart && running > 0; ++j) {
      if (graph) {
        hipGraphExec_t& e = bt.graphs[std::make_pair(j, in_cycle)];
        if (!e) {
          const bool on = bt.timer.on;
          bt.timer.on = false;  // no event nodes in the graph
          hipGraph_t g = nullptr;
          GDSW_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
          body(j);
          GDSW_HIP(hipStreamEndCapture(st, &g));
          bt.timer.on = on;
          GDSW_HIP(hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
          GDSW_HIP(hipGraphDestroy(g));
        }
        GDSW_HIP(hipGraphLaunch(e, st));
      } else {
        body(j);
      }
      GDSW_HIP(hipStreamSynchronize(st));
      bool changed = false;
      for (int k = 0; k < K; ++k) {
        if (!in_cycle[k]) continue;
        const double rel = hp[2 * k], hn = hp[2 * k + 1];
        if (!std::isfinite(rel))
          throw StatusError{4, "FGMRES: non-finite residual estimate in batch member " + std::to_string(k)};
        res[k].iterations += 1;
        res[k].rel = rel;
        kc[k] = j + 1;
        if (rel <= rtol || hn == 0.0 || res[k].iterations >= max_it) {
          in_cycle[k] = 0;
          changed = true;
          --running;
        }
      }
      if (changed && running > 0) batch_select(bt, in_cycle, st);
    }
    // x += Z y for every member that took part in this cycle
    batch_fork(bt, st);
    for (int k = 0; k < K; ++k) {
      if (kc[k] == 0) continue;
      Context& c = *bt.m[k];
      const hipStream_t ls = batch_lane(bt, k);
      back_subst(kc[k], restart, c.d_H, c.d_g, c.d_hv, ls);
      gemv_add(c.d_Z, c.ldv, kc[k], c.d_hv, xv[k], c.P.n_free, ls);
    }
    batch_join(bt, st);
  }
  for (int k = 0; k < K; ++k) res[k].restarts = std::max(0, cycles[k] - 1);
  GDSW_HIP(hipGetLastError());
  return res;
}

}  // namespace gdsw
