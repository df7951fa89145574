// C ABI entry points (include/gdsw.h).  Exceptions never cross this file:
// every entry point maps them to a gdsw_status and a last-error message.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <new>
#include <stdexcept>
#include <thread>

#include "../../include/gdsw.h"
#include "context.h"
#include "kernels.h"
#include "kernels_multi.h"
#include "learned.h"

using namespace gdsw;

struct gdsw_ctx {
  Context c;
};

struct gdsw_batch {
  std::vector<gdsw_ctx*> members;
  Batch b;
};

namespace {

thread_local std::string g_last_error;

gdsw_status fail(gdsw_ctx* ctx, gdsw_status s, const std::string& msg) {
  g_last_error = msg;
  if (ctx) ctx->c.last_error = msg;
  return s;
}

template <class F>
gdsw_status guarded(gdsw_ctx* ctx, F&& f) {
  try {
    f();
    return GDSW_OK;
  } catch (const StatusError& e) {
    return fail(ctx, (gdsw_status)e.status, e.msg);
  } catch (const HipError& e) {
    return fail(ctx, GDSW_EDEVICE, std::string(hipGetErrorString(e.err)) + " (" + e.where + ")");
  } catch (const std::invalid_argument& e) {
    return fail(ctx, GDSW_EINVAL, e.what());
  } catch (const std::bad_alloc&) {
    return fail(ctx, GDSW_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(ctx, GDSW_EDEVICE, e.what());
  }
}

int host_threads() {
  const unsigned h = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(16u, h));
}

ProblemSpec spec_of(const gdsw_mesh* mesh, const gdsw_decomposition* dec) {
  if (!mesh || !dec) throw std::invalid_argument("mesh and decomposition must not be NULL");
  ProblemSpec s;
  s.n = mesh->n;
  s.mu = mesh->viscosity;
  s.c = mesh->inflow_amplitude;
  s.manufactured = mesh->manufactured_force;
  s.m = dec->subdomains;
  s.overlap = dec->overlap;
  s.levels = dec->levels;
  s.group = dec->group;
  s.local_dirichlet = dec->local_algebraic == 0;
  s.level2_layer = dec->level2_layer != 0;
  s.pressure = mesh->pressure_element;
  s.coarse = dec->coarse_space;
  if (dec->local_precision < 0 || dec->local_precision > 2) throw std::invalid_argument("bad local_precision");
  if (dec->tile != 0 && dec->tile != 64 && dec->tile != 128) throw std::invalid_argument("tile must be 0, 64 or 128");
  if (dec->local_solve != GDSW_SOLVE_INVERSE && dec->local_solve != GDSW_SOLVE_TRIANGULAR &&
      dec->local_solve != GDSW_SOLVE_SYMMETRIC && dec->local_solve != GDSW_SOLVE_BLOCK)
    throw std::invalid_argument("local_solve must be GDSW_SOLVE_INVERSE, _TRIANGULAR, _SYMMETRIC or _BLOCK");
  if ((dec->local_solve == GDSW_SOLVE_SYMMETRIC || dec->local_solve == GDSW_SOLVE_BLOCK) && dec->max_rhs > 1)
    throw std::invalid_argument("GDSW_SOLVE_SYMMETRIC and GDSW_SOLVE_BLOCK take one right-hand side per product "
                                "(max_rhs <= 1)");
  if (dec->max_rhs < 0 || dec->max_rhs > 32) throw std::invalid_argument("max_rhs must be in 0..32");
  return s;
}

gdsw_status check_device_ctx(const gdsw_ctx* ctx) {
  if (!ctx) return fail(nullptr, GDSW_EINVAL, "NULL context");
  if (ctx->c.host_only)
    return fail(const_cast<gdsw_ctx*>(ctx), GDSW_EINVAL, "context was created by gdsw_setup_host (no device data)");
  return GDSW_OK;
}

// Mean time of `reps` calls of `run` on `st` after three untimed ones.
template <class F>
double time_calls(hipStream_t st, int reps, F run) {
  hipEvent_t e0, e1;
  GDSW_HIP(hipEventCreate(&e0));
  GDSW_HIP(hipEventCreate(&e1));
  for (int w = 0; w < 3; ++w) run();
  GDSW_HIP(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r) run();
  GDSW_HIP(hipEventRecord(e1, st));
  GDSW_HIP(hipEventSynchronize(e1));
  float el = 0.f;
  GDSW_HIP(hipEventElapsedTime(&el, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return el / reps;
}

}  // namespace

extern "C" {

gdsw_status gdsw_setup_host(const gdsw_mesh* mesh, const gdsw_decomposition* dec, gdsw_ctx** out) {
  if (!out) return fail(nullptr, GDSW_EINVAL, "out must not be NULL");
  *out = nullptr;
  gdsw_ctx* ctx = nullptr;
  gdsw_status s = guarded(nullptr, [&]() {
    ProblemSpec sp = spec_of(mesh, dec);
    ctx = new gdsw_ctx();
    ctx->c.host_only = true;
    ctx->c.local_prec = dec->local_precision;
    const auto t0 = std::chrono::steady_clock::now();
    build_problem(sp, ctx->c.P, host_threads());
    ctx->c.t_symbolic = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  });
  if (s != GDSW_OK) {
    delete ctx;
    return s;
  }
  *out = ctx;
  return GDSW_OK;
}

gdsw_status gdsw_setup(const gdsw_mesh* mesh, const gdsw_decomposition* dec, void* stream, gdsw_ctx** out) {
  if (!out) return fail(nullptr, GDSW_EINVAL, "out must not be NULL");
  *out = nullptr;
  gdsw_ctx* ctx = nullptr;
  gdsw_status s = guarded(nullptr, [&]() {
    ProblemSpec sp = spec_of(mesh, dec);
    ctx = new gdsw_ctx();
    Context& c = ctx->c;
    c.local_prec = dec->local_precision;
    c.solve_mode = dec->local_solve == GDSW_SOLVE_TRIANGULAR  ? SOLVE_TRSV
                   : dec->local_solve == GDSW_SOLVE_SYMMETRIC ? SOLVE_SYM
                   : dec->local_solve == GDSW_SOLVE_BLOCK     ? SOLVE_BLOCK
                                                              : SOLVE_INVERSE;
    c.max_rhs = std::max(1, dec->max_rhs);
    GDSW_HIP(hipGetDevice(&c.device));
    const auto t0 = std::chrono::steady_clock::now();
    build_problem(sp, c.P, host_threads());
    const auto t1 = std::chrono::steady_clock::now();
    c.t_symbolic = std::chrono::duration<double>(t1 - t0).count();
    uint64_t budget = dec->device_mem_budget;
    if (budget == 0) {
      size_t fr = 0, tot = 0;
      GDSW_HIP(hipMemGetInfo(&fr, &tot));
      budget = (uint64_t)(fr * 0.97);
    }
    const int nb = dec->tile ? dec->tile : 128;
    device_setup(c, (hipStream_t)stream, budget, nb);
    (void)noalloc_scratch(c.device);  // device address of the no-allocation scratch, once per device
    c.t_numeric = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
  });
  if (s != GDSW_OK) {
    if (ctx) {
      ctx->c.arena.release_all();
      if (ctx->c.h_pinned) (void)hipHostFree(ctx->c.h_pinned);
    }
    delete ctx;
    return s;
  }
  *out = ctx;
  return GDSW_OK;
}

namespace {

AlgebraicInput algebraic_input(const gdsw_algebraic_problem* p) {
  if (!p) throw std::invalid_argument("problem must not be NULL");
  AlgebraicInput in;
  in.n = p->n;
  in.row_ptr = p->row_ptr;
  in.col = p->col;
  in.val = p->val;
  in.rhs = p->rhs;
  in.field = p->field;
  in.null_value = p->null_value;
  in.n_sub = p->n_sub;
  in.sub_ptr = p->sub_ptr;
  in.sub_idx = p->sub_idx;
  return in;
}

ProblemSpec algebraic_spec(const gdsw_decomposition* dec) {
  if (!dec) throw std::invalid_argument("decomposition must not be NULL");
  gdsw_mesh dummy{};
  dummy.n = 1;
  dummy.viscosity = 1.0;
  gdsw_decomposition d = *dec;
  d.subdomains = 1;  // not used: the subdomains come with the problem
  ProblemSpec s = spec_of(&dummy, &d);
  s.local_dirichlet = 0;
  return s;
}

}  // namespace

gdsw_status gdsw_setup_algebraic_host(const gdsw_algebraic_problem* prob, const gdsw_decomposition* dec,
                                      gdsw_ctx** out) {
  if (!out) return fail(nullptr, GDSW_EINVAL, "out must not be NULL");
  *out = nullptr;
  gdsw_ctx* ctx = nullptr;
  gdsw_status s = guarded(nullptr, [&]() {
    const AlgebraicInput in = algebraic_input(prob);
    const ProblemSpec sp = algebraic_spec(dec);
    ctx = new gdsw_ctx();
    ctx->c.host_only = true;
    ctx->c.local_prec = dec->local_precision;
    const auto t0 = std::chrono::steady_clock::now();
    build_problem_algebraic(in, sp, ctx->c.P);
    ctx->c.t_symbolic = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  });
  if (s != GDSW_OK) {
    delete ctx;
    return s;
  }
  *out = ctx;
  return GDSW_OK;
}

gdsw_status gdsw_setup_algebraic(const gdsw_algebraic_problem* prob, const gdsw_decomposition* dec, void* stream,
                                 gdsw_ctx** out) {
  if (!out) return fail(nullptr, GDSW_EINVAL, "out must not be NULL");
  *out = nullptr;
  gdsw_ctx* ctx = nullptr;
  gdsw_status s = guarded(nullptr, [&]() {
    const AlgebraicInput in = algebraic_input(prob);
    const ProblemSpec sp = algebraic_spec(dec);
    ctx = new gdsw_ctx();
    Context& c = ctx->c;
    c.local_prec = dec->local_precision;
    c.solve_mode = dec->local_solve == GDSW_SOLVE_TRIANGULAR  ? SOLVE_TRSV
                   : dec->local_solve == GDSW_SOLVE_SYMMETRIC ? SOLVE_SYM
                   : dec->local_solve == GDSW_SOLVE_BLOCK     ? SOLVE_BLOCK
                                                              : SOLVE_INVERSE;
    c.max_rhs = std::max(1, dec->max_rhs);
    GDSW_HIP(hipGetDevice(&c.device));
    const auto t0 = std::chrono::steady_clock::now();
    build_problem_algebraic(in, sp, c.P);
    const auto t1 = std::chrono::steady_clock::now();
    c.t_symbolic = std::chrono::duration<double>(t1 - t0).count();
    uint64_t budget = dec->device_mem_budget;
    if (budget == 0) {
      size_t fr = 0, tot = 0;
      GDSW_HIP(hipMemGetInfo(&fr, &tot));
      budget = (uint64_t)(fr * 0.97);
    }
    device_setup(c, (hipStream_t)stream, budget, dec->tile ? dec->tile : 128);
    (void)noalloc_scratch(c.device);
    c.t_numeric = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
  });
  if (s != GDSW_OK) {
    if (ctx) {
      ctx->c.arena.release_all();
      if (ctx->c.h_pinned) (void)hipHostFree(ctx->c.h_pinned);
    }
    delete ctx;
    return s;
  }
  *out = ctx;
  return GDSW_OK;
}

gdsw_status gdsw_get_sizes(const gdsw_ctx* ctx, gdsw_sizes* out) {
  if (!ctx || !out) return fail(nullptr, GDSW_EINVAL, "NULL argument");
  const Context& c = ctx->c;
  const Problem& P = c.P;
  std::memset(out, 0, sizeof *out);
  out->n_free = P.n_free;
  out->n_full = P.n_full;
  out->n_u_free = P.n_u;
  out->n_p = P.n_p;
  out->nnz = P.nnz();
  out->n_sub = P.n_sub;
  out->n_entities = P.n_ent;
  out->n_coarse = P.n_coarse;
  out->n_subregions = P.spec.levels == 3 ? P.lv2.n_sub : 0;
  out->n_coarse3 = P.spec.levels == 3 ? P.lv2.n_coarse3 : 0;
  int64_t mn = INT64_MAX, mx = 0;
  for (auto& S : P.S) {
    mn = std::min<int64_t>(mn, S.size());
    mx = std::max<int64_t>(mx, S.size());
  }
  out->local_min = P.S.empty() ? 0 : mn;
  out->local_max = mx;
  out->factor_bytes = c.factor_bytes;
  out->coarse_bytes = c.coarse_bytes;
  out->device_bytes = c.arena.used;
  if (!c.host_only) {
    if (c.solve_mode == SOLVE_BLOCK && c.blk.use_w) {  // L_i^-1 once, S_i^-1 once, B and W once
      out->solve_bytes = c.L1.algorithmic_bytes() + c.LP.algorithmic_bytes() + c.HI.algorithmic_bytes() +
                         c.blk.b_bytes + c.blk.w_bytes;
      out->solve_launches = c.L1.launches() + c.LP.launches() + c.HI.launches() + 2;
    } else if (c.solve_mode == SOLVE_BLOCK) {  // two passes over L_i^-1, one over S_i^-1, B twice
      out->solve_bytes = 2 * c.L1.algorithmic_bytes() + c.LP.algorithmic_bytes() + c.HI.algorithmic_bytes() +
                         c.blk.b_bytes;
      out->solve_launches = 2 * c.L1.launches() + c.LP.launches() + c.HI.launches() + 3;
    } else {
      out->solve_bytes = c.L1.algorithmic_bytes() + c.HI.algorithmic_bytes();
      out->solve_launches = c.L1.launches() + c.HI.launches();
    }
  }
  return GDSW_OK;
}

gdsw_status gdsw_dof_map(const gdsw_ctx* ctx, int32_t* field, int32_t* node_abc) {
  if (!ctx || !field || !node_abc) return fail(nullptr, GDSW_EINVAL, "NULL argument");
  const Problem& P = ctx->c.P;
  for (int64_t d = 0; d < P.n_free; ++d) {
    field[d] = P.field[d];
    node_abc[3 * d] = P.abc[3 * d];
    node_abc[3 * d + 1] = P.abc[3 * d + 1];
    node_abc[3 * d + 2] = P.abc[3 * d + 2];
  }
  return GDSW_OK;
}

gdsw_status gdsw_host_matrix(const gdsw_ctx* ctx, int64_t* row_ptr, int32_t* col, double* val) {
  if (!ctx || !row_ptr || !col || !val) return fail(nullptr, GDSW_EINVAL, "NULL argument");
  const Problem& P = ctx->c.P;
  for (int64_t r = 0; r <= P.n_free; ++r) row_ptr[r] = P.row_ptr[r];
  std::memcpy(col, P.col.data(), P.col.size() * sizeof(int32_t));
  std::memcpy(val, P.val.data(), P.val.size() * sizeof(double));
  return GDSW_OK;
}

gdsw_status gdsw_host_rhs(const gdsw_ctx* ctx, double* b) {
  if (!ctx || !b) return fail(nullptr, GDSW_EINVAL, "NULL argument");
  std::memcpy(b, ctx->c.P.rhs.data(), ctx->c.P.rhs.size() * sizeof(double));
  return GDSW_OK;
}

gdsw_status gdsw_rhs(gdsw_ctx* ctx, double* b_dev, void* stream) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (!b_dev) return fail(ctx, GDSW_EINVAL, "NULL vector");
  return guarded(ctx, [&]() {
    GDSW_HIP(hipMemcpyAsync(b_dev, ctx->c.d_rhs, ctx->c.P.n_free * sizeof(double), hipMemcpyDeviceToDevice,
                            (hipStream_t)stream));
  });
}

gdsw_status gdsw_spmv(gdsw_ctx* ctx, const double* x_dev, double* y_dev, void* stream) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (!x_dev || !y_dev) return fail(ctx, GDSW_EINVAL, "NULL vector");
  if (x_dev == y_dev) return fail(ctx, GDSW_EINVAL, "x and y must not overlap");
  return guarded(ctx, [&]() {
    spmv(ctx->c, x_dev, y_dev, (hipStream_t)stream);
    GDSW_HIP(hipGetLastError());
  });
}

gdsw_status gdsw_apply_precond(gdsw_ctx* ctx, const double* r_dev, double* z_dev, int32_t nrhs, int64_t ld,
                               void* stream) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (!r_dev || !z_dev) return fail(ctx, GDSW_EINVAL, "NULL vector");
  if (nrhs < 1 || ld < ctx->c.P.n_free) return fail(ctx, GDSW_EINVAL, "need nrhs >= 1 and ld >= n_free");
  if (r_dev == z_dev) return fail(ctx, GDSW_EINVAL, "r and z must not overlap");
  return guarded(ctx, [&]() {
    Context& c = ctx->c;
    hipStream_t st = (hipStream_t)stream;
    if (nrhs > 1 && multi_supported(c)) {
      const int64_t n = c.P.n_free;
      for (int k0 = 0; k0 < nrhs; k0 += c.max_rhs) {
        const int K = std::min(c.max_rhs, nrhs - k0);
        cm_to_il(n, K, r_dev + (int64_t)k0 * ld, ld, c.d_xin, st);
        apply_precond_multi(c, c.d_xin, c.d_xout, K, st);
        il_to_cm(n, K, c.d_xout, z_dev + (int64_t)k0 * ld, ld, st);
      }
      GDSW_HIP(hipGetLastError());
      return;
    }
    for (int k = 0; k < nrhs; ++k) apply_precond(c, r_dev + (int64_t)k * ld, z_dev + (int64_t)k * ld, st);
  });
}

gdsw_status gdsw_apply_precond_noalloc(gdsw_ctx* ctx, const double* r_dev, double* z_dev, int32_t nrhs, int64_t ld,
                                       void* stream) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (!r_dev || !z_dev) return fail(ctx, GDSW_EINVAL, "NULL vector");
  if (nrhs < 1 || ld < ctx->c.P.n_free) return fail(ctx, GDSW_EINVAL, "need nrhs >= 1 and ld >= n_free");
  if (r_dev == z_dev) return fail(ctx, GDSW_EINVAL, "r and z must not overlap");
  return guarded(ctx, [&]() {
    for (int k = 0; k < nrhs; ++k)
      apply_precond_noalloc(ctx->c, r_dev + (int64_t)k * ld, z_dev + (int64_t)k * ld, (hipStream_t)stream);
  });
}

gdsw_status gdsw_fgmres_solve(gdsw_ctx* ctx, const double* b_dev, double* x_dev, int32_t nrhs, int64_t ld,
                              const gdsw_fgmres_opts* opts, gdsw_fgmres_info* info, void* stream) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (!b_dev || !x_dev || !opts) return fail(ctx, GDSW_EINVAL, "NULL argument");
  if (nrhs < 1 || ld < ctx->c.P.n_free) return fail(ctx, GDSW_EINVAL, "need nrhs >= 1 and ld >= n_free");
  if (opts->restart < 1 || opts->restart > 200 || opts->max_it < 1 || !(opts->rtol > 0.0))
    return fail(ctx, GDSW_EINVAL, "need 1 <= restart <= 200, max_it >= 1, rtol > 0");
  bool all_conv = true;
  gdsw_status s = guarded(ctx, [&]() {
    Context& c = ctx->c;
    hipStream_t st = (hipStream_t)stream;
    if (nrhs > 1 && multi_supported(c)) {
      const int64_t n = c.P.n_free;
      for (int k0 = 0; k0 < nrhs; k0 += c.max_rhs) {
        const int K = std::min(c.max_rhs, nrhs - k0);
        const auto t0 = std::chrono::steady_clock::now();
        GDSW_HIP(hipStreamSynchronize(st));
        ensure_multi_workspace(c, opts->restart, K);  // before the right-hand sides are placed in it
        cm_to_il(n, K, b_dev + (int64_t)k0 * ld, ld, c.mk.b, st);
        std::vector<FgmresResult> r =
            fgmres_multi(c, c.mk.b, c.mk.x, K, opts->rtol, opts->restart, opts->max_it, st);
        il_to_cm(n, K, c.mk.x, x_dev + (int64_t)k0 * ld, ld, st);
        GDSW_HIP(hipStreamSynchronize(st));
        const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int j = 0; j < K; ++j) {
          if (info) {
            info[k0 + j].iterations = r[j].iterations;
            info[k0 + j].restarts = r[j].restarts;
            info[k0 + j].rel_res = r[j].rel;
            info[k0 + j].true_rel_res = r[j].true_rel;
            info[k0 + j].t_solve_s = t;
            info[k0 + j].fallbacks = 0;
            info[k0 + j].learned_solves = 0;
          }
          all_conv = all_conv && r[j].converged;
        }
      }
      return;
    }
    for (int k = 0; k < nrhs; ++k) {
      const auto t0 = std::chrono::steady_clock::now();
      const LearnedSolve* Ls = ctx->c.learned;
      const int64_t fb0 = Ls ? Ls->fallbacks : 0, ls0 = Ls ? Ls->learned_solves : 0;
      FgmresResult r = fgmres(ctx->c, b_dev + (int64_t)k * ld, x_dev + (int64_t)k * ld, opts->rtol, opts->restart,
                              opts->max_it, opts->use_graph != 0, (hipStream_t)stream,
                              k == 0 ? opts->history : nullptr, k == 0 ? opts->history_len : 0);
      GDSW_HIP(hipStreamSynchronize((hipStream_t)stream));
      const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (info) {
        info[k].iterations = r.iterations;
        info[k].restarts = r.restarts;
        info[k].rel_res = r.rel;
        info[k].true_rel_res = r.true_rel;
        info[k].t_solve_s = t;
        info[k].fallbacks = Ls ? Ls->fallbacks - fb0 : 0;
        info[k].learned_solves = Ls ? Ls->learned_solves - ls0 : 0;
      }
      all_conv = all_conv && r.converged;
    }
  });
  if (s != GDSW_OK) return s;
  if (!all_conv) return fail(ctx, GDSW_ENOCONV, "FGMRES reached max_it before rtol");
  return GDSW_OK;
}

gdsw_status gdsw_expand_solution(const gdsw_ctx* ctx, const double* x_free_dev, double* x_full_dev, void* stream) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (!x_free_dev || !x_full_dev) return fail(const_cast<gdsw_ctx*>(ctx), GDSW_EINVAL, "NULL vector");
  return guarded(const_cast<gdsw_ctx*>(ctx), [&]() { expand_solution(ctx->c, x_free_dev, x_full_dev, (hipStream_t)stream); });
}

gdsw_status gdsw_copy_coarse_matrix(const gdsw_ctx* ctx, double* a0_host) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (!a0_host) return fail(const_cast<gdsw_ctx*>(ctx), GDSW_EINVAL, "NULL argument");
  return guarded(const_cast<gdsw_ctx*>(ctx), [&]() {
    const int64_t Nc = ctx->c.Nc;
    if (Nc > 0) GDSW_HIP(hipMemcpy(a0_host, ctx->c.d_A0, Nc * Nc * sizeof(double), hipMemcpyDeviceToHost));
  });
}

gdsw_status gdsw_copy_coarse_basis(const gdsw_ctx* ctx, double* phi) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (!phi) return fail(const_cast<gdsw_ctx*>(ctx), GDSW_EINVAL, "NULL argument");
  return guarded(const_cast<gdsw_ctx*>(ctx), [&]() {
    const Problem& P = ctx->c.P;
    const int64_t n = P.n_free, Nc = ctx->c.Nc;
    std::memset(phi, 0, sizeof(double) * n * Nc);
    for (int64_t d = 0; d < n; ++d)
      if (P.gamma_col[d] >= 0) phi[P.gamma_col[d] * n + d] = 1.0;
    int64_t off = 0;
    for (int i = 0; i < P.n_sub; ++i) {
      const int64_t ni = P.I[i].size(), nc = P.C[i].size();
      std::vector<double> blk(ni * nc);
      if (ni * nc)
        GDSW_HIP(hipMemcpy(blk.data(), ctx->c.d_phi_cm + off, ni * nc * sizeof(double), hipMemcpyDeviceToHost));
      for (int64_t j = 0; j < nc; ++j)
        for (int64_t k = 0; k < ni; ++k) phi[(int64_t)P.C[i][j] * n + P.I[i][k]] = blk[j * ni + k];
      off += ni * nc;
    }
  });
}

gdsw_status gdsw_local_indices(const gdsw_ctx* ctx, int32_t i, int32_t* idx_host, int32_t* size) {
  if (!ctx) return fail(nullptr, GDSW_EINVAL, "NULL context");
  const Problem& P = ctx->c.P;
  if (i < 0 || i >= P.n_sub) return fail(const_cast<gdsw_ctx*>(ctx), GDSW_EINVAL, "subdomain index out of range");
  if (size) *size = (int32_t)P.S[i].size();
  if (idx_host) std::memcpy(idx_host, P.S[i].data(), P.S[i].size() * sizeof(int32_t));
  return GDSW_OK;
}

gdsw_status gdsw_set_schedule(gdsw_ctx* ctx, int32_t phases, int32_t waves, void* stream) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (phases < 1 || phases > 64) return fail(ctx, GDSW_EINVAL, "phases must be in 1..64");
  if (waves != 4 && waves != 8) return fail(ctx, GDSW_EINVAL, "waves must be 4 or 8");
  if (waves == 8 && ctx->c.nb != 128) return fail(ctx, GDSW_EINVAL, "8 waves need tile 128");
  if (ctx->c.solve_mode != SOLVE_TRSV) return GDSW_OK;  // nothing to schedule for the inverse product
  return guarded(ctx, [&]() {
    hipStream_t st = (hipStream_t)stream;
    GDSW_HIP(hipStreamSynchronize(st));
    for (FactorSet* fs : {&ctx->c.L1, &ctx->c.HI}) {
      fs->waves = waves;
      const size_t nsl = fs->sched.size();
      plan_schedule(*fs, phases, ctx->c.arena, st);
      (void)nsl;
    }
    if (ctx->c.learned) {
      std::vector<char> inc(ctx->c.L1.count, 1), only(ctx->c.L1.count, 0);
      for (int32_t f : ctx->c.learned->factors) {
        inc[f] = 0;
        only[f] = 1;
      }
      plan_schedule(ctx->c.L1, phases, ctx->c.arena, st, 1, &inc);
      plan_schedule(ctx->c.L1, phases, ctx->c.arena, st, 2, &only);
    }
    GDSW_HIP(hipStreamSynchronize(st));
  });
}

gdsw_status gdsw_profile_apply(gdsw_ctx* ctx, const double* r_dev, double* z_dev, void* stream, double* ms) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (!r_dev || !z_dev || !ms) return fail(ctx, GDSW_EINVAL, "NULL argument");
  if (r_dev == z_dev) return fail(ctx, GDSW_EINVAL, "r and z must not overlap");
  return guarded(ctx, [&]() {
    hipEvent_t ev[5];
    for (auto& e : ev) GDSW_HIP(hipEventCreate(&e));
    hipStream_t st = (hipStream_t)stream;
    apply_precond(ctx->c, r_dev, z_dev, st, ev);
    GDSW_HIP(hipEventSynchronize(ev[4]));
    for (int k = 0; k < 4; ++k) {
      float t = 0.f;
      GDSW_HIP(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
      ms[k] = t;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
  });
}

gdsw_status gdsw_kernel_timer(gdsw_ctx* ctx, int32_t enable) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  return guarded(ctx, [&]() {
    KernelTimer& T = ctx->c.timer;
    if (enable) {
      if (T.ev.empty()) {
        T.ev.resize(2 * KernelTimer::CAP);
        for (auto& e : T.ev) GDSW_HIP(hipEventCreate(&e));
      }
      T.used = 0;
      T.bytes = 0.0;
      T.on = true;
      ctx->c.L1.timer = &T;
    } else {
      T.on = false;
    }
  });
}

gdsw_status gdsw_kernel_timer_read(gdsw_ctx* ctx, double* total_ms, int64_t* launches, uint64_t* bytes_per_launch) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (!total_ms || !launches || !bytes_per_launch) return fail(ctx, GDSW_EINVAL, "NULL argument");
  return guarded(ctx, [&]() {
    const KernelTimer& T = ctx->c.timer;
    double tot = 0.0;
    if (T.used > 0) GDSW_HIP(hipEventSynchronize(T.ev[2 * T.used - 1]));
    for (int i = 0; i < T.used; ++i) {
      float t = 0.f;
      GDSW_HIP(hipEventElapsedTime(&t, T.ev[2 * i], T.ev[2 * i + 1]));
      tot += t;
    }
    *total_ms = tot;
    *launches = T.used;
    *bytes_per_launch = T.used > 0 ? (uint64_t)(T.bytes / T.used) : 0;
  });
}

gdsw_status gdsw_autotune(gdsw_ctx* ctx, void* stream, int32_t* chosen, double* ms) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  Context& c = ctx->c;
  if (c.solve_mode == SOLVE_TRSV)
    return fail(ctx, GDSW_EUNSUPPORTED, "autotuning applies to the inverse, symmetric and block local solves");
  if (c.learned) return fail(ctx, GDSW_EUNSUPPORTED, "autotune before gdsw_learned_init");
  return guarded(ctx, [&]() {
    hipStream_t st = (hipStream_t)stream;
    FactorSet& fs = c.L1;
    KernelTimer* tm = fs.timer;
    fs.timer = nullptr;
    auto once = [&]() { local_solve_set(fs, c.d_w, st); };
    int best = 0;
    if (c.solve_mode == SOLVE_INVERSE) {
      // column chunk of the partial products
      const int cand[3] = {512, 1024, 2048};
      double t[3];
      for (int q = 0; q < 3; ++q) {
        fs.cw = cand[q];
        plan_schedule(fs, 1, c.arena, st, 0);
        t[q] = time_calls(st, 10, once);
      }
      for (int q = 1; q < 3; ++q)
        if (t[q] < t[best]) best = q;  // argmin over the measured candidates
      fs.cw = cand[best];
      if (chosen) *chosen = fs.cw;
      if (ms)
        for (int q = 0; q < 3; ++q) ms[q] = t[q];
    } else {
      // symmetric tiles (and the block solve's velocity-block tiles): tiles
      // per work item and the work-group order
      const int run[4] = {2, 2, 1, 1}, xcd[4] = {0, 1, 0, 1};
      double t[4];
      for (int q = 0; q < 4; ++q) {
        fs.sym_run = run[q];
        fs.sym_xcd = xcd[q];
        plan_schedule(fs, 1, c.arena, st, 0);
        t[q] = time_calls(st, 10, once);
      }
      for (int q = 1; q < 4; ++q)
        if (t[q] < t[best]) best = q;
      fs.sym_run = run[best];
      fs.sym_xcd = xcd[best];
      if (chosen) *chosen = 10 * run[best] + xcd[best];
      if (ms)
        for (int q = 0; q < 4; ++q) ms[q] = t[q];
    }
    plan_schedule(fs, 1, c.arena, st, 0);
    fs.timer = tm;
    GDSW_HIP(hipMemsetAsync(c.d_w, 0, std::max<int64_t>(c.n_w, 1) * sizeof(double), st));
    GDSW_HIP(hipStreamSynchronize(st));
  });
}

gdsw_status gdsw_autotune_mfma(gdsw_ctx* ctx, void* stream, int32_t* chosen, double* ms) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  Context& c = ctx->c;
  if (c.solve_mode != SOLVE_INVERSE || c.max_rhs < 2 || !c.d_wm)
    return fail(ctx, GDSW_EUNSUPPORTED, "the MFMA autotuner needs GDSW_SOLVE_INVERSE and max_rhs > 1");
  return guarded(ctx, [&]() {
    hipStream_t st = (hipStream_t)stream;
    FactorSet& fs = c.L1;
    KernelTimer* tm = fs.timer;
    fs.timer = nullptr;
    const int K = c.max_rhs;
    auto once = [&]() { gemm_set(fs, c.d_wm, K, K, st); };
    // FP64: the direct kernel with 512 / 1024 / 2048 summation columns per
    // item, then the LDS-staged kernel with 256 / 512 / 1024; FP32 and BF16
    // have one kernel and take the first three
    const int ncand = fs.prec == P_FP64 ? 6 : 3;
    const int cw[6] = {512, 1024, 2048, 256, 512, 1024}, lds[6] = {0, 0, 0, 1, 1, 1};
    double t[6];
    int best = 0;
    for (int q = 0; q < ncand; ++q) {
      fs.gemm_cw_force = cw[q];
      fs.gemm_lds_force = fs.prec == P_FP64 ? lds[q] : -1;
      plan_gemm(fs, c.arena, st);
      t[q] = time_calls(st, 5, once);
      if (t[q] < t[best]) best = q;
    }
    fs.gemm_cw_force = cw[best];
    fs.gemm_lds_force = fs.prec == P_FP64 ? lds[best] : -1;
    plan_gemm(fs, c.arena, st);
    fs.timer = tm;
    GDSW_HIP(hipMemsetAsync(c.d_wm, 0, std::max<int64_t>(c.n_w, 1) * K * sizeof(double), st));
    GDSW_HIP(hipStreamSynchronize(st));
    if (chosen) *chosen = best;
    if (ms)
      for (int q = 0; q < 6; ++q) ms[q] = q < ncand ? t[q] : 0.0;
  });
}

gdsw_status gdsw_learned_init(gdsw_ctx* ctx, uint64_t seed, gdsw_learned_info* info, void* stream) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  return guarded(ctx, [&]() {
    learned_init(ctx->c, seed, (hipStream_t)stream);
    if (info) {
      const LearnedSolve* L = ctx->c.learned;
      info->grid = L->G;
      info->subdomains = L->S;
      info->n_params = L->n_params;
      info->samples = L->N;
      for (int k = 0; k < 4; ++k) info->sigma[k] = L->sigma[k];
    }
  });
}

gdsw_status gdsw_learned_train(gdsw_ctx* ctx, int32_t solves, int32_t steps, int32_t batch, double lr, uint64_t seed,
                               double* loss_history, void* stream) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (!ctx->c.learned) return fail(ctx, GDSW_EINVAL, "call gdsw_learned_init first");
  if (steps < 0 || batch < 1 || !(lr > 0.0)) return fail(ctx, GDSW_EINVAL, "need steps >= 0, batch >= 1, lr > 0");
  return guarded(ctx, [&]() {
    hipStream_t st = (hipStream_t)stream;
    if (solves > 0) learned_generate(ctx->c, solves, seed, st);
    if (steps > 0) learned_train(ctx->c, steps, batch, lr, seed + 1, loss_history, st);
  });
}

gdsw_status gdsw_learned_weights(gdsw_ctx* ctx, const float* set_host, float* get_host, int32_t which, void* stream) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (!ctx->c.learned) return fail(ctx, GDSW_EINVAL, "call gdsw_learned_init first");
  if (which < 0 || which > 2) return fail(ctx, GDSW_EINVAL, "which must be 0, 1 or 2");
  return guarded(ctx, [&]() {
    if (set_host) learned_set_weights(ctx->c, set_host, (hipStream_t)stream);
    if (get_host) learned_get_weights(ctx->c, get_host, which, (hipStream_t)stream);
  });
}

gdsw_status gdsw_learned_loss_grad(gdsw_ctx* ctx, const float* x_host, const float* t_host, int32_t batch,
                                   double* loss, float* grads_host, void* stream) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (!ctx->c.learned) return fail(ctx, GDSW_EINVAL, "call gdsw_learned_init first");
  if (!x_host || !t_host || !loss) return fail(ctx, GDSW_EINVAL, "NULL argument");
  return guarded(ctx, [&]() {
    *loss = learned_loss_grad(ctx->c, x_host, t_host, batch, grads_host, (hipStream_t)stream);
  });
}

gdsw_status gdsw_set_local_solver(gdsw_ctx* ctx, int32_t mode, double tau) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (mode < 0 || mode > 2) return fail(ctx, GDSW_EINVAL, "mode must be 0, 1 or 2");
  if (mode != 0 && !ctx->c.learned) return fail(ctx, GDSW_EINVAL, "call gdsw_learned_init first");
  if (mode == 1 && !(tau > 0.0)) return fail(ctx, GDSW_EINVAL, "tau must be > 0");
  ctx->c.local_solver = mode;
  if (ctx->c.learned && tau > 0.0) ctx->c.learned->tau = tau;
  return GDSW_OK;
}

gdsw_status gdsw_learned_copy(gdsw_ctx* dst, const gdsw_ctx* src, void* stream) {
  if (gdsw_status s = check_device_ctx(dst)) return s;
  if (!src) return fail(dst, GDSW_EINVAL, "NULL source context");
  if (!dst->c.learned || !src->c.learned) return fail(dst, GDSW_EINVAL, "call gdsw_learned_init on both first");
  return guarded(dst, [&]() { learned_copy(dst->c, src->c, (hipStream_t)stream); });
}

gdsw_status gdsw_learned_stats(const gdsw_ctx* ctx, int64_t* learned_solves, int64_t* fallbacks) {
  if (!ctx || !ctx->c.learned) return fail(const_cast<gdsw_ctx*>(ctx), GDSW_EINVAL, "no learned local solve");
  if (learned_solves) *learned_solves = ctx->c.learned->learned_solves;
  if (fallbacks) *fallbacks = ctx->c.learned->fallbacks;
  return GDSW_OK;
}

gdsw_status gdsw_learned_save(const gdsw_ctx* ctx, const char* path, void* stream) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (!path) return fail(const_cast<gdsw_ctx*>(ctx), GDSW_EINVAL, "NULL path");
  return guarded(const_cast<gdsw_ctx*>(ctx), [&]() { learned_save(ctx->c, path, (hipStream_t)stream); });
}

gdsw_status gdsw_learned_load(gdsw_ctx* ctx, const char* path, void* stream) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (!path) return fail(ctx, GDSW_EINVAL, "NULL path");
  if (!ctx->c.learned) return fail(ctx, GDSW_EINVAL, "call gdsw_learned_init first");
  return guarded(ctx, [&]() { learned_load(ctx->c, path, (hipStream_t)stream); });
}

gdsw_status gdsw_train_local_net(gdsw_ctx* ctx, const char* out_weights, int32_t steps, uint64_t seed, void* stream) {
  if (gdsw_status s = check_device_ctx(ctx)) return s;
  if (steps < 1) return fail(ctx, GDSW_EINVAL, "need steps >= 1");
  return guarded(ctx, [&]() {
    hipStream_t st = (hipStream_t)stream;
    learned_init(ctx->c, seed, st);
    if (ctx->c.learned->N == 0) learned_generate(ctx->c, 4, seed, st);
    learned_train(ctx->c, steps, 32, 2e-3, seed + 1, nullptr, st);
    if (out_weights) learned_save(ctx->c, out_weights, st);
  });
}

gdsw_status gdsw_setup_times(const gdsw_ctx* ctx, double* symbolic_s, double* numeric_s) {
  if (!ctx) return fail(nullptr, GDSW_EINVAL, "NULL context");
  if (symbolic_s) *symbolic_s = ctx->c.t_symbolic;
  if (numeric_s) *numeric_s = ctx->c.t_numeric;
  return GDSW_OK;
}

const char* gdsw_last_error(const gdsw_ctx* ctx) {
  if (ctx) return ctx->c.last_error.c_str();
  return g_last_error.c_str();
}

void gdsw_destroy(gdsw_ctx* ctx) {
  if (!ctx) return;
  learned_release(ctx->c);
  for (auto& e : ctx->c.timer.ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->c.it_ev)
    if (e) (void)hipEventDestroy(e);
  release_graphs(ctx->c);
  if (ctx->c.mk.h_pinned) (void)hipHostFree(ctx->c.mk.h_pinned);
  if (ctx->c.mk.h_active) (void)hipHostFree(ctx->c.mk.h_active);
  ctx->c.arena.release_all();
  if (ctx->c.h_pinned) (void)hipHostFree(ctx->c.h_pinned);
  delete ctx;
}

gdsw_status gdsw_setup_batch(const gdsw_mesh* meshes, const gdsw_decomposition* decs, int32_t count, void* stream,
                             gdsw_batch** out) {
  if (!out || !meshes || !decs) return fail(nullptr, GDSW_EINVAL, "NULL argument");
  *out = nullptr;
  if (count < 1) return fail(nullptr, GDSW_EINVAL, "count must be >= 1");
  gdsw_batch* bt = new (std::nothrow) gdsw_batch();
  if (!bt) return fail(nullptr, GDSW_ENOMEM, "host allocation failed");
  for (int k = 0; k < count; ++k) {
    if ((decs[k].local_solve != GDSW_SOLVE_INVERSE && decs[k].local_solve != GDSW_SOLVE_SYMMETRIC &&
         decs[k].local_solve != GDSW_SOLVE_BLOCK) ||
        decs[k].local_solve != decs[0].local_solve) {
      gdsw_destroy_batch(bt);
      return fail(nullptr, GDSW_EINVAL,
                  "batch members need one local_solve, GDSW_SOLVE_INVERSE, GDSW_SOLVE_SYMMETRIC or GDSW_SOLVE_BLOCK");
    }
    gdsw_ctx* c = nullptr;
    const gdsw_status s = gdsw_setup(&meshes[k], &decs[k], stream, &c);
    if (s != GDSW_OK) {
      const std::string msg = "batch member " + std::to_string(k) + ": " + g_last_error;
      gdsw_destroy_batch(bt);
      return fail(nullptr, s, msg);
    }
    bt->members.push_back(c);
    bt->b.m.push_back(&c->c);
  }
  const gdsw_status s = guarded(nullptr, [&]() { batch_build(bt->b, (hipStream_t)stream); });
  if (s != GDSW_OK) {
    gdsw_destroy_batch(bt);
    return s;
  }
  *out = bt;
  return GDSW_OK;
}

gdsw_status gdsw_batch_member(gdsw_batch* batch, int32_t k, gdsw_ctx** member) {
  if (!batch || !member) return fail(nullptr, GDSW_EINVAL, "NULL argument");
  if (k < 0 || k >= (int32_t)batch->members.size()) return fail(nullptr, GDSW_EINVAL, "member index out of range");
  *member = batch->members[k];
  return GDSW_OK;
}

gdsw_status gdsw_apply_precond_batch(gdsw_batch* batch, const double* const* r_dev, double* const* z_dev,
                                     void* stream) {
  if (!batch || !r_dev || !z_dev) return fail(nullptr, GDSW_EINVAL, "NULL argument");
  for (size_t k = 0; k < batch->members.size(); ++k)
    if (!r_dev[k] || !z_dev[k] || r_dev[k] == z_dev[k]) return fail(nullptr, GDSW_EINVAL, "bad vector for a member");
  return guarded(nullptr, [&]() { apply_precond_batch(batch->b, r_dev, z_dev, (hipStream_t)stream); });
}

gdsw_status gdsw_fgmres_solve_batch(gdsw_batch* batch, const double* const* b_dev, double* const* x_dev,
                                    const gdsw_fgmres_opts* opts, gdsw_fgmres_info* info, void* stream) {
  if (!batch || !b_dev || !x_dev || !opts) return fail(nullptr, GDSW_EINVAL, "NULL argument");
  if (opts->restart < 1 || opts->restart > 200 || opts->max_it < 1 || !(opts->rtol > 0.0))
    return fail(nullptr, GDSW_EINVAL, "need 1 <= restart <= 200, max_it >= 1, rtol > 0");
  for (size_t k = 0; k < batch->members.size(); ++k)
    if (!b_dev[k] || !x_dev[k]) return fail(nullptr, GDSW_EINVAL, "NULL vector for a member");
  bool all_conv = true;
  const gdsw_status s = guarded(nullptr, [&]() {
    const auto t0 = std::chrono::steady_clock::now();
    const size_t nm = batch->members.size();
    std::vector<int64_t> fb0(nm, 0), ls0(nm, 0);
    for (size_t k = 0; k < nm; ++k)
      if (const LearnedSolve* L = batch->members[k]->c.learned) {
        fb0[k] = L->fallbacks;
        ls0[k] = L->learned_solves;
      }
    std::vector<FgmresResult> r =
        fgmres_batch(batch->b, b_dev, x_dev, opts->rtol, opts->restart, opts->max_it, (hipStream_t)stream,
                     opts->use_graph != 0);
    GDSW_HIP(hipStreamSynchronize((hipStream_t)stream));
    const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (size_t k = 0; k < r.size(); ++k) {
      if (info) {
        info[k].iterations = r[k].iterations;
        info[k].restarts = r[k].restarts;
        info[k].rel_res = r[k].rel;
        info[k].true_rel_res = r[k].true_rel;
        info[k].t_solve_s = t;
        const LearnedSolve* L = batch->members[k]->c.learned;
        info[k].fallbacks = L ? L->fallbacks - fb0[k] : 0;
        info[k].learned_solves = L ? L->learned_solves - ls0[k] : 0;
      }
      all_conv = all_conv && r[k].converged;
    }
  });
  if (s != GDSW_OK) return s;
  if (!all_conv) return fail(nullptr, GDSW_ENOCONV, "a batch member reached max_it before rtol");
  return GDSW_OK;
}

gdsw_status gdsw_batch_kernel_timer(gdsw_batch* batch, int32_t enable) {
  if (!batch) return fail(nullptr, GDSW_EINVAL, "NULL batch");
  return guarded(nullptr, [&]() {
    KernelTimer& T = batch->b.timer;
    if (enable) {
      if (T.ev.empty()) {
        T.ev.resize(2 * KernelTimer::CAP);
        for (auto& e : T.ev) GDSW_HIP(hipEventCreate(&e));
      }
      T.used = 0;
      T.bytes = 0.0;
      T.on = true;
    } else {
      T.on = false;
    }
  });
}

gdsw_status gdsw_batch_kernel_timer_read(gdsw_batch* batch, double* total_ms, int64_t* launches,
                                         uint64_t* bytes_per_launch) {
  if (!batch || !total_ms || !launches || !bytes_per_launch) return fail(nullptr, GDSW_EINVAL, "NULL argument");
  return guarded(nullptr, [&]() {
    const KernelTimer& T = batch->b.timer;
    double tot = 0.0;
    if (T.used > 0) GDSW_HIP(hipEventSynchronize(T.ev[2 * T.used - 1]));
    for (int i = 0; i < T.used; ++i) {
      float t = 0.f;
      GDSW_HIP(hipEventElapsedTime(&t, T.ev[2 * i], T.ev[2 * i + 1]));
      tot += t;
    }
    *total_ms = tot;
    *launches = T.used;
    *bytes_per_launch = T.used > 0 ? (uint64_t)(T.bytes / T.used) : 0;
  });
}

void gdsw_destroy_batch(gdsw_batch* batch) {
  if (!batch) return;
  batch_release(batch->b);
  for (gdsw_ctx* c : batch->members) gdsw_destroy(c);
  delete batch;
}

}  // extern "C"
