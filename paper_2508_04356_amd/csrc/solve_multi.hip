// Several right-hand sides in lockstep: the two-level preconditioner (eq. 2.2)
// applied to K columns at once and right-preconditioned FGMRES run
// column-wise in lockstep.
//
// Every column follows exactly the steps of the single-vector FGMRES (x_0 = 0,
// classical Gram-Schmidt twice, Givens rotations, stop once
// |g_{j+1}| / ||b|| <= rtol, x = x_0 + Z y, recomputed true residual,
// restart from x if needed); the columns only share kernel launches.  A
// column that has met its stopping test is masked: its next basis vector is
// zero and its Givens state frozen, so it neither changes nor produces NaNs
// while the others continue.  The local solves of all columns are one MFMA
// product per factor set (kernels_gemm.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "context.h"
#include "kernels.h"
#include "kernels_multi.h"
#include "kernels_ops.h"

namespace gdsw {
namespace {

CoarseView coarse_view_m(const Context& c) {
  return CoarseView{c.d_gamma_col, c.d_dof_ipos, c.d_I_sub,  c.d_I_ptr,  c.d_I_idx,
                    c.d_C_ptr,     c.d_C_idx,    c.d_phi_off, c.d_phi_cm, c.d_phi_rm,
                    c.d_cg_ptr,    c.d_cg_dof,   c.d_cs_ptr,  c.d_cs_sub, c.d_cs_lc};
}

// per column j: beta = sqrt(nrm2[j]); g_j = (beta, 0, ...); sv[j] = beta
__global__ void mk_cycle_start_kernel(int K, int restart, const double* __restrict__ nrm2, double* __restrict__ g,
                                      double* __restrict__ sv) {
  const int j = threadIdx.x;
  if (j >= K) return;
  const double beta = sqrt(nrm2[j]);
  sv[j] = beta;
  double* gj = g + (int64_t)j * (restart + 1);
  for (int i = 0; i <= restart; ++i) gj[i] = i == 0 ? beta : 0.0;
}

// Arnoldi column jj of every active column j (same arithmetic as the single
// vector version); out[j] = |g_{jj+1}| / bnorm_j, out[K + j] = ||w_j||,
// sv[j] = ||w_j|| for the normalisation.
__global__ void mk_arnoldi_kernel(int jj, int K, int restart, const double* __restrict__ h1,
                                  const double* __restrict__ h2, const double* __restrict__ nrm2,
                                  const double* __restrict__ bnorm, const int32_t* __restrict__ active,
                                  double* __restrict__ H, double* __restrict__ cs, double* __restrict__ sn,
                                  double* __restrict__ g, double* __restrict__ sv, double* __restrict__ out) {
  const int j = threadIdx.x;
  if (j >= K || !active[j]) return;
  const int ldh = restart + 1;
  double* col = H + (int64_t)j * ldh * restart + (int64_t)jj * ldh;
  double* csj = cs + (int64_t)j * restart;
  double* snj = sn + (int64_t)j * restart;
  double* gj = g + (int64_t)j * ldh;
  for (int i = 0; i <= jj; ++i) col[i] = h1[(int64_t)i * K + j] + h2[(int64_t)i * K + j];
  const double hn = sqrt(nrm2[j]);
  col[jj + 1] = hn;
  for (int i = 0; i < jj; ++i) {
    const double t = csj[i] * col[i] + snj[i] * col[i + 1];
    col[i + 1] = -snj[i] * col[i] + csj[i] * col[i + 1];
    col[i] = t;
  }
  const double rho = hypot(col[jj], col[jj + 1]);
  csj[jj] = col[jj] / rho;
  snj[jj] = col[jj + 1] / rho;
  col[jj] = rho;
  col[jj + 1] = 0.0;
  gj[jj + 1] = -snj[jj] * gj[jj];
  gj[jj] = csj[jj] * gj[jj];
  sv[j] = hn;
  out[j] = fabs(gj[jj + 1]) / bnorm[j];
  out[K + j] = hn;
}

// y[i * K + j] = (H_j[:k_j, :k_j]^-1 g_j[:k_j])_i, zero for k_j <= i < kmax
__global__ void mk_back_subst_kernel(int K, int restart, int kmax, const int32_t* __restrict__ kc,
                                     const double* __restrict__ H, const double* __restrict__ g,
                                     double* __restrict__ y) {
  const int j = threadIdx.x;
  if (j >= K) return;
  const int ldh = restart + 1;
  const double* Hj = H + (int64_t)j * ldh * restart;
  const double* gj = g + (int64_t)j * ldh;
  const int k = kc[j];
  for (int i = kmax - 1; i >= k; --i) y[(int64_t)i * K + j] = 0.0;
  for (int i = k - 1; i >= 0; --i) {
    double s = gj[i];
    for (int l = i + 1; l < k; ++l) s -= Hj[(int64_t)l * ldh + i] * y[(int64_t)l * K + j];
    y[(int64_t)i * K + j] = s / Hj[(int64_t)i * ldh + i];
  }
}


// device scal layout (K each): [0] squared norms, [K] scale values, [2K] bnorm,
// [3K] read-back pair (rel, hn)
void read_back(Context& ctx, const double* dsrc, int count, hipStream_t st) {
  GDSW_HIP(hipMemcpyAsync(ctx.mk.h_pinned, dsrc, count * sizeof(double), hipMemcpyDeviceToHost, st));
  GDSW_HIP(hipStreamSynchronize(st));
}

void upload_ints(Context& ctx, const std::vector<int32_t>& v, int32_t* dst, hipStream_t st) {
  // the previous upload has completed: every caller synchronised the stream since
  for (size_t i = 0; i < v.size(); ++i) ctx.mk.h_active[i] = v[i];
  GDSW_HIP(hipMemcpyAsync(dst, ctx.mk.h_active, v.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
}

}  // namespace

void ensure_multi_workspace(Context& ctx, int restart, int K) {
  Context::MultiKrylov& M = ctx.mk;
  if (M.V && M.restart >= restart && M.K == K) return;
  DeviceArena& A = ctx.arena;
  for (void* p : {(void*)M.V, (void*)M.Z, (void*)M.H, (void*)M.g, (void*)M.cs, (void*)M.sn, (void*)M.h1,
                  (void*)M.h2, (void*)M.part, (void*)M.scal, (void*)M.t1, (void*)M.t2, (void*)M.b, (void*)M.x,
                  (void*)M.y, (void*)M.active})
    if (p) A.free(p);
  const int64_t n = ctx.P.n_free;
  M.restart = restart;
  M.K = K;
  M.ldv = n * K;
  M.nblocks = dots_il_blocks(n);
  M.V = dalloc<double>(A, M.ldv * (restart + 1));
  M.Z = dalloc<double>(A, M.ldv * restart);
  M.H = dalloc<double>(A, (int64_t)K * (restart + 1) * restart);
  M.g = dalloc<double>(A, (int64_t)K * (restart + 1));
  M.cs = dalloc<double>(A, (int64_t)K * restart);
  M.sn = dalloc<double>(A, (int64_t)K * restart);
  M.h1 = dalloc<double>(A, (int64_t)K * (restart + 1));
  M.h2 = dalloc<double>(A, (int64_t)K * (restart + 1));
  M.part = dalloc<double>(A, (int64_t)M.nblocks * (restart + 1) * K);
  M.scal = dalloc<double>(A, 8 * (int64_t)K);
  M.t1 = dalloc<double>(A, M.ldv);
  M.t2 = dalloc<double>(A, M.ldv);
  M.b = dalloc<double>(A, M.ldv);
  M.x = dalloc<double>(A, M.ldv);
  M.y = dalloc<double>(A, (int64_t)K * restart);
  M.active = dalloc<int32_t>(A, K);
  if (!M.h_pinned) GDSW_HIP(hipHostMalloc((void**)&M.h_pinned, 4 * 32 * sizeof(double), hipHostMallocDefault));
  if (!M.h_active) GDSW_HIP(hipHostMalloc((void**)&M.h_active, 2 * 32 * sizeof(int32_t), hipHostMallocDefault));
}

bool multi_supported(const Context& ctx) {
  return ctx.max_rhs > 1 && ctx.d_wm && ctx.P.spec.levels == 2 && ctx.solve_mode == SOLVE_INVERSE &&
         ctx.local_solver == 0;
}

void apply_precond_multi(Context& ctx, const double* r, double* z, int K, hipStream_t st) {
  const CoarseView cv = coarse_view_m(ctx);
  const bool coarse = ctx.Nc > 0;
  gather_il(ctx.n_w1, K, ctx.d_gidx, r, ctx.d_wm, st);
  if (coarse) restrict_il(ctx.Nc, K, cv, r, ctx.d_wm, ctx.d_coarse_pinv, st, ctx.n_pairs, ctx.d_pair_tm,
                          ctx.P.n_sub);
  gemm_set(ctx.L1, ctx.d_wm, K, K, st);
  gemm_set(ctx.HI, ctx.d_wm, K, K, st);
  scatter_prolong_il(ctx.P.n_free, K, ctx.d_inv_ptr, ctx.d_inv_pos, ctx.d_wm, cv,
                     coarse ? ctx.d_coarse_pinv : nullptr, z, st, ctx.P.n_sub, ctx.max_ni);
  GDSW_HIP(hipGetLastError());
}

std::vector<FgmresResult> fgmres_multi(Context& ctx, const double* b_il, double* x_il, int K, double rtol,
                                       int restart, int max_it, hipStream_t st) {
  ensure_multi_workspace(ctx, restart, K);
  Context::MultiKrylov& M = ctx.mk;
  const int64_t n = ctx.P.n_free;
  const int64_t ldv = M.ldv;
  double* nrm2 = M.scal;          // K
  double* sv = M.scal + K;        // K
  double* bn = M.scal + 2 * K;    // K
  double* rb = M.scal + 3 * K;    // 2K
  std::vector<FgmresResult> res(K);
  // ||b_j||
  dots_il(b_il, ldv, 1, b_il, n, K, M.part, M.nblocks, nrm2, st);
  read_back(ctx, nrm2, K, st);
  std::vector<double> bnorm(K);
  for (int j = 0; j < K; ++j) bnorm[j] = std::sqrt(ctx.mk.h_pinned[j]);
  GDSW_HIP(hipMemcpyAsync(bn, bnorm.data(), K * sizeof(double), hipMemcpyHostToDevice, st));
  GDSW_HIP(hipMemsetAsync(x_il, 0, ldv * sizeof(double), st));
  std::vector<int> it(K, 0), done(K, 0), cycles(K, 0);
  for (int j = 0; j < K; ++j)
    if (bnorm[j] == 0.0) {
      res[j].converged = true;
      done[j] = 1;
    }
  std::vector<int32_t> active(K), kc(K);
  GDSW_HIP(hipStreamSynchronize(st));
  while (true) {
    // r = b - A x, true residuals
    spmm_il(n, K, ctx.d_rowptr, ctx.d_col, ctx.d_val, x_il, M.t1, st);
    sub_il(ldv, b_il, M.t1, st);
    dots_il(M.t1, ldv, 1, M.t1, n, K, M.part, M.nblocks, nrm2, st);
    read_back(ctx, nrm2, K, st);
    int n_active = 0;
    for (int j = 0; j < K; ++j) {
      active[j] = 0;
      if (done[j]) continue;
      res[j].true_rel = std::sqrt(ctx.mk.h_pinned[j]) / bnorm[j];
      if (res[j].true_rel <= rtol) {
        res[j].converged = true;
        done[j] = 1;
      } else if (it[j] >= max_it) {
        done[j] = 1;
      } else {
        active[j] = 1;
        ++n_active;
      }
    }
    if (n_active == 0) break;
    upload_ints(ctx, active, M.active, st);
    mk_cycle_start_kernel<<<1, 32, 0, st>>>(K, restart, nrm2, M.g, sv);
    scale_il(n, K, M.t1, sv, M.active, M.V, st);
    for (int j = 0; j < K; ++j) {
      kc[j] = 0;
      if (active[j]) ++cycles[j];
    }
    int kmax = 0;
    for (int jj = 0; jj < restart; ++jj) {
      double* vj = M.V + (int64_t)jj * ldv;
      double* zj = M.Z + (int64_t)jj * ldv;
      apply_precond_multi(ctx, vj, zj, K, st);
      spmm_il(n, K, ctx.d_rowptr, ctx.d_col, ctx.d_val, zj, M.t2, st);
      dots_il(M.V, ldv, jj + 1, M.t2, n, K, M.part, M.nblocks, M.h1, st);
      gemv_il(M.V, ldv, jj + 1, M.h1, M.t2, n, K, -1.0, st);
      dots_il(M.V, ldv, jj + 1, M.t2, n, K, M.part, M.nblocks, M.h2, st);
      gemv_il(M.V, ldv, jj + 1, M.h2, M.t2, n, K, -1.0, st);
      dots_il(M.t2, ldv, 1, M.t2, n, K, M.part, M.nblocks, nrm2, st);
      mk_arnoldi_kernel<<<1, 32, 0, st>>>(jj, K, restart, M.h1, M.h2, nrm2, bn, M.active, M.H, M.cs, M.sn, M.g,
                                          sv, rb);
      scale_il(n, K, M.t2, sv, M.active, M.V + (int64_t)(jj + 1) * ldv, st);
      read_back(ctx, rb, 2 * K, st);
      kmax = jj + 1;
      bool changed = false;
      n_active = 0;
      for (int j = 0; j < K; ++j) {
        if (!active[j]) continue;
        const double rel = ctx.mk.h_pinned[j], hn = ctx.mk.h_pinned[K + j];
        if (!std::isfinite(rel))
          throw StatusError{4, "FGMRES: non-finite residual estimate in column " + std::to_string(j)};
        ++it[j];
        kc[j] = jj + 1;
        res[j].rel = rel;
        if (rel <= rtol || hn == 0.0 || it[j] >= max_it) {
          active[j] = 0;
          changed = true;
        } else {
          ++n_active;
        }
      }
      if (n_active == 0) break;
      if (changed) upload_ints(ctx, active, M.active, st);
    }
    upload_ints(ctx, kc, M.active, st);  // k_j of this cycle (the mask is re-uploaded next cycle)
    mk_back_subst_kernel<<<1, 32, 0, st>>>(K, restart, kmax, M.active, M.H, M.g, M.y);
    gemv_il(M.Z, ldv, kmax, M.y, x_il, n, K, 1.0, st);
    GDSW_HIP(hipStreamSynchronize(st));
  }
  for (int j = 0; j < K; ++j) {
    res[j].iterations = it[j];
    res[j].restarts = std::max(0, cycles[j] - 1);
  }
  GDSW_HIP(hipGetLastError());
  return res;
}

}  // namespace gdsw
