// Learned local solve (host driver): a 4-layer 3x3x3 convolution network
// replaces A_i^-1 of eq. (2.2) on interior subdomains; FGMRES tolerates the
// resulting variable preconditioner.  Training pairs (r_i, A_i^-1 r_i) come
// from the method itself: the Krylov vectors of LU-preconditioned FGMRES
// solves, restricted to the interior subdomains and solved with their LU
// factors.  In the apply the LU factors stay the fallback: a subdomain whose
// local residual ||r_i - A_i N(r_i)|| exceeds tau ||r_i|| is re-solved by LU.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <fstream>
#include <random>

#include "context.h"
#include "kernels.h"
#include "kernels_learned.h"
#include "learned.h"

namespace gdsw {

static const int kCh[5] = {4, 32, 32, 32, 4};

int64_t learned_param_count() {
  int64_t n = 0;
  for (int l = 0; l < 4; ++l) n += (int64_t)kCh[l + 1] * kCh[l] * 27 + kCh[l + 1];
  return n;
}

namespace {

void zero(void* p, size_t bytes, hipStream_t st) { GDSW_HIP(hipMemsetAsync(p, 0, bytes, st)); }

}  // namespace

void learned_init(Context& ctx, uint64_t seed, hipStream_t st) {
  if (ctx.learned) return;
  Problem& P = ctx.P;
  const int m = P.spec.m;
  if (P.algebraic) throw StatusError{6, "the learned local solve needs the structured cube's node grids"};
  if (ctx.solve_mode == SOLVE_BLOCK) throw StatusError{6, "the learned local solve takes dense local inverses"};
  if (m < 3) throw StatusError{6, "the learned local solve needs interior subdomains (m >= 3)"};
  if (P.spec.pressure != 0) throw StatusError{6, "the learned local solve is built for the Q1 pressure"};
  auto L = new LearnedSolve();
  ctx.learned = L;
  DeviceArena& A = ctx.arena;
  // interior subdomains: every local DOF on a full G^3 node grid
  std::vector<int32_t> map_ptr(1, 0), map;
  std::vector<int8_t> field;
  int G = -1;
  for (int K = 1; K < m - 1; ++K)
    for (int J = 1; J < m - 1; ++J)
      for (int I = 1; I < m - 1; ++I) {
        const int i = I + m * (J + m * K);
        const auto& S = P.S[i];
        int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {0, 0, 0};
        for (int32_t d : S)
          for (int ax = 0; ax < 3; ++ax) {
            lo[ax] = std::min(lo[ax], P.abc[3 * (int64_t)d + ax]);
            hi[ax] = std::max(hi[ax], P.abc[3 * (int64_t)d + ax]);
          }
        const int g = hi[0] - lo[0] + 1;
        if (G < 0) G = g;
        if (g != G || hi[1] - lo[1] + 1 != G || hi[2] - lo[2] + 1 != G)
          throw StatusError{6, "interior subdomains do not share one node grid"};
        for (int32_t d : S) {
          const int x = P.abc[3 * (int64_t)d] - lo[0], y = P.abc[3 * (int64_t)d + 1] - lo[1],
                    z = P.abc[3 * (int64_t)d + 2] - lo[2];
          const int ch = P.field[d];
          map.push_back(ch * G * G * G + (z * G + y) * G + x);
          field.push_back((int8_t)ch);
        }
        map_ptr.push_back((int32_t)map.size());
        L->factors.push_back(i);
      }
  L->G = G;
  L->S = (int)L->factors.size();
  const int G3 = G * G * G;
  // loss mask: velocity everywhere, pressure on the Q1 nodes of the grid
  std::vector<float> mask(4 * G3, 0.f);
  for (size_t k = map_ptr[0]; k < (size_t)map_ptr[1]; ++k) mask[map[k]] = 1.f;
  L->d_mask = dupload(A, mask, st);
  L->d_factor = dupload(A, L->factors, st);
  L->d_map_ptr = dupload(A, map_ptr, st);
  L->d_map = dupload(A, map, st);
  L->d_field = dupload(A, field, st);
  std::vector<int32_t> S_ptr, S_idx;
  S_ptr.push_back(0);
  for (int i = 0; i < P.n_sub; ++i) {
    S_idx.insert(S_idx.end(), P.S[i].begin(), P.S[i].end());
    S_ptr.push_back((int32_t)S_idx.size());
  }
  L->d_S_ptr = dupload(A, S_ptr, st);
  L->d_S_idx = dupload(A, S_idx, st);
  // local CSR of every interior matrix A_s = A[S_s, S_s] (local column indices)
  {
    std::vector<int64_t> row_off, lrow(1, 0);
    std::vector<int32_t> lcol;
    std::vector<double> lval;
    L->max_n = 0;
    for (int32_t f : L->factors) {
      const std::vector<int32_t>& Sf = P.S[f];
      const int n = (int)Sf.size();
      L->max_n = std::max(L->max_n, n);
      row_off.push_back((int64_t)lrow.size() - 1);
      for (int k = 0; k < n; ++k) {
        const int32_t g = Sf[k];
        for (int32_t e = P.row_ptr[g]; e < P.row_ptr[g + 1]; ++e) {
          const auto it = std::lower_bound(Sf.begin(), Sf.end(), P.col[e]);
          if (it != Sf.end() && *it == P.col[e]) {
            lcol.push_back((int32_t)(it - Sf.begin()));
            lval.push_back(P.val[e]);
          }
        }
        lrow.push_back((int64_t)lcol.size());
      }
    }
    L->d_lrow_off = dupload(A, row_off, st);
    L->d_lrow = dupload(A, lrow, st);
    L->d_lcol = dupload(A, lcol, st);
    L->d_lval = dupload(A, lval, st);
    L->d_rpart = dalloc<double>(A, std::max<int64_t>(1, 2 * (int64_t)L->factors.size() * ((L->max_n + 255) / 256)));
  }
  // parameters (flat: W0 b0 W1 b1 W2 b2 W3 b3), He-normal init
  const int64_t np = learned_param_count();
  L->n_params = np;
  std::mt19937_64 rng(seed);
  std::vector<float> h(np, 0.f);
  int64_t o = 0;
  for (int l = 0; l < 4; ++l) {
    std::normal_distribution<float> nd(0.f, std::sqrt(2.f / (27.f * kCh[l])));
    const int64_t nw = (int64_t)kCh[l + 1] * kCh[l] * 27;
    for (int64_t k = 0; k < nw; ++k) h[o + k] = nd(rng);
    L->woff[l] = o;
    L->boff[l] = o + nw;
    o += nw + kCh[l + 1];
  }
  L->d_master = dupload(A, h, st);
  L->d_work = dalloc<float>(A, np);
  L->d_wb = dalloc<uint16_t>(A, 4 * 27 * 32 * 32);
  L->d_grad = dalloc<float>(A, np);
  L->d_m = dalloc<float>(A, np);
  L->d_v = dalloc<float>(A, np);
  zero(L->d_m, np * 4, st);
  zero(L->d_v, np * 4, st);
  round_bf16(L->d_master, L->d_work, np, st);
  std::vector<float> sig(4, 1.f);
  L->d_sigma = dupload(A, sig, st);
  L->max_b = std::max(L->S, 32);
  for (int l = 0; l < 5; ++l) {
    L->act[l] = dalloc<float>(A, (int64_t)L->max_b * kCh[l] * G3);
    L->gact[l] = dalloc<float>(A, (int64_t)L->max_b * kCh[l] * G3);
  }
  L->d_target = dalloc<float>(A, (int64_t)L->max_b * 4 * G3);
  L->d_norms = dalloc<double>(A, L->max_b);
  L->d_lossb = dalloc<float>(A, L->max_b);
  L->d_rsave = dalloc<double>(A, std::max<int64_t>(ctx.n_w1, 1));
  L->d_flags = dalloc<int32_t>(A, ctx.L1.count);
  zero(L->d_flags, ctx.L1.count * 4, st);
  L->d_count = dalloc<int32_t>(A, 1);
  L->d_bidx = dalloc<int32_t>(A, L->max_b);
  L->d_sign = dalloc<float>(A, L->max_b);
  GDSW_HIP(hipHostMalloc((void**)&L->h_count, sizeof(int32_t), hipHostMallocDefault));
  // schedules without / with only the interior factors
  std::vector<char> inc(ctx.L1.count, 1), only(ctx.L1.count, 0);
  for (int32_t f : L->factors) {
    inc[f] = 0;
    only[f] = 1;
  }
  plan_schedule(ctx.L1, ctx.L1.phases, A, st, 1, &inc);
  plan_schedule(ctx.L1, ctx.L1.phases, A, st, 2, &only);
  GDSW_HIP(hipStreamSynchronize(st));
}

GridMap learned_gridmap(const Context& ctx) {
  const LearnedSolve* L = ctx.learned;
  return GridMap{L->d_factor, ctx.L1.d_xoff, ctx.L1.d_n, L->d_map_ptr, L->d_map, L->d_field};
}

// forward pass of B samples in act[0] -> act[4]
void learned_forward(Context& ctx, int B, hipStream_t st) {
  LearnedSolve* L = ctx.learned;
  // every layer runs on the matrix cores (channels zero-padded to 32 in, 16 out)
  for (int l = 0; l < 4; ++l) conv_weights_bf16(L->d_work + L->woff[l], kCh[l], kCh[l + 1], L->d_wb + l * 27 * 32 * 32, st);
  for (int l = 0; l < 4; ++l)
    conv_fwd(L->act[l], kCh[l], L->d_work + L->woff[l], L->d_work + L->boff[l], L->act[l + 1], kCh[l + 1], L->G, l < 3,
             B, st, L->d_wb + l * 27 * 32 * 32);
}

// loss of act[4] against d_target and gradients into d_grad; returns the loss
double learned_backward(Context& ctx, int B, hipStream_t st) {
  LearnedSolve* L = ctx.learned;
  const int G3 = L->G * L->G * L->G;
  masked_loss(L->act[4], L->d_target, L->d_mask, 4 * G3, B, L->gact[4], L->d_lossb, st);
  for (int l = 3; l >= 0; --l) {
    if (l < 3) relu_bwd(L->gact[l + 1], L->act[l + 1], (int64_t)B * kCh[l + 1] * G3, st);
    conv_bwd(L->act[l], kCh[l], L->d_work + L->woff[l], L->gact[l + 1], kCh[l + 1], L->G, B, l > 0 ? L->gact[l] : nullptr,
             L->d_grad + L->woff[l], L->d_grad + L->boff[l], st);
  }
  std::vector<float> lb(B);
  GDSW_HIP(hipMemcpyAsync(lb.data(), L->d_lossb, B * sizeof(float), hipMemcpyDeviceToHost, st));
  GDSW_HIP(hipStreamSynchronize(st));
  double s = 0.0;
  for (int b = 0; b < B; ++b) s += lb[b];
  return s / B;
}

void learned_generate(Context& ctx, int nsolves, uint64_t seed, hipStream_t st) {
  LearnedSolve* L = ctx.learned;
  DeviceArena& A = ctx.arena;
  const int G3 = L->G * L->G * L->G;
  const int64_t n = ctx.P.n_free;
  const int keep_mode = ctx.local_solver;
  ctx.local_solver = 0;  // pairs come from the LU-preconditioned method
  const int restart = 100;
  const int per_col = L->S;
  const int max_samples = 8192;
  const int cap = std::min<int64_t>(max_samples, (int64_t)nsolves * (restart + 1) * per_col);
  if (L->Xd) {
    A.free(L->Xd);
    A.free(L->Td);
  }
  L->Xd = dalloc<float>(A, (int64_t)cap * 4 * G3);
  L->Td = dalloc<float>(A, (int64_t)cap * 4 * G3);
  double* b = dalloc<double>(A, n);
  double* x = dalloc<double>(A, n);
  double* norms = dalloc<double>(A, per_col);
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  GridMap gm = learned_gridmap(ctx);
  const double mu = ctx.P.spec.mu;
  int N = 0;
  for (int sidx = 0; sidx < nsolves && N + per_col <= cap; ++sidx) {
    if (sidx == 0) {
      GDSW_HIP(hipMemcpyAsync(b, ctx.d_rhs, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    } else {
      std::vector<double> h(n);
      for (auto& v : h) v = nd(rng);
      GDSW_HIP(hipMemcpyAsync(b, h.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
    }
    FgmresResult r = fgmres(ctx, b, x, 1e-8, restart, restart, false, st);
    const int kcols = std::min(r.iterations + 1, restart + 1);
    for (int j = 0; j < kcols && N + per_col <= cap; ++j) {
      const double* vj = ctx.d_V + (int64_t)j * ctx.ldv;
      gather(ctx.n_w1, ctx.d_gidx, vj, ctx.d_w, st);
      to_grid(gm, per_col, L->G, ctx.d_w, L->Xd + (int64_t)N * 4 * G3, norms, mu, st);
      local_solve_set(ctx.L1, ctx.d_w, st);
      to_grid(gm, per_col, L->G, ctx.d_w, L->Td + (int64_t)N * 4 * G3, norms, mu, st, /*given_norms=*/true);
      N += per_col;
    }
  }
  GDSW_HIP(hipStreamSynchronize(st));
  // channel scales of the targets (root mean square over the data)
  std::vector<float> T((int64_t)N * 4 * G3);
  GDSW_HIP(hipMemcpy(T.data(), L->Td, T.size() * sizeof(float), hipMemcpyDeviceToHost));
  std::vector<float> mask(4 * G3);
  GDSW_HIP(hipMemcpy(mask.data(), L->d_mask, mask.size() * sizeof(float), hipMemcpyDeviceToHost));
  float sig[4];
  for (int ch = 0; ch < 4; ++ch) {
    double ss = 0.0, cnt = 0.0;
    for (int s = 0; s < N; ++s)
      for (int v = 0; v < G3; ++v)
        if (mask[ch * G3 + v] > 0.f) {
          const double t = T[((int64_t)s * 4 + ch) * G3 + v];
          ss += t * t;
          cnt += 1.0;
        }
    sig[ch] = cnt > 0 ? (float)std::sqrt(ss / cnt) : 1.f;
    if (!(sig[ch] > 0.f)) sig[ch] = 1.f;
  }
  for (int s = 0; s < N; ++s)
    for (int ch = 0; ch < 4; ++ch)
      for (int v = 0; v < G3; ++v) {
        float& t = T[((int64_t)s * 4 + ch) * G3 + v];
        t = (float)(t / sig[ch]);
      }
  GDSW_HIP(hipMemcpy(L->Td, T.data(), T.size() * sizeof(float), hipMemcpyHostToDevice));
  GDSW_HIP(hipMemcpy(L->d_sigma, sig, sizeof sig, hipMemcpyHostToDevice));
  for (int ch = 0; ch < 4; ++ch) L->sigma[ch] = sig[ch];
  L->N = N;
  A.free(b);
  A.free(x);
  A.free(norms);
  ctx.local_solver = keep_mode;
}

void learned_train(Context& ctx, int steps, int batch, double lr, uint64_t seed, double* history, hipStream_t st) {
  LearnedSolve* L = ctx.learned;
  if (L->N == 0) throw StatusError{1, "no training pairs: generate them first"};
  batch = std::max(1, std::min(batch, L->max_b));
  const int G3 = L->G * L->G * L->G;
  std::mt19937_64 rng(seed);
  std::uniform_int_distribution<int> pick(0, L->N - 1);
  std::vector<int32_t> idx(batch);
  std::vector<float> sign(batch);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int it = 0; it < steps; ++it) {
    for (int k = 0; k < batch; ++k) {
      idx[k] = pick(rng);
      sign[k] = (rng() & 1) ? 1.f : -1.f;  // A^-1 is linear: (-r, -y) is a pair too
    }
    GDSW_HIP(hipMemcpyAsync(L->d_bidx, idx.data(), batch * sizeof(int32_t), hipMemcpyHostToDevice, st));
    GDSW_HIP(hipMemcpyAsync(L->d_sign, sign.data(), batch * sizeof(float), hipMemcpyHostToDevice, st));
    gather_batch(L->Xd, L->Td, L->d_bidx, L->d_sign, batch, 4 * G3, L->act[0], L->d_target, st);
    learned_forward(ctx, batch, st);
    const double loss = learned_backward(ctx, batch, st);
    if (history) history[it] = loss;
    ++L->adam_t;
    const float c1 = 1.f - std::pow(b1, (float)L->adam_t), c2 = 1.f - std::pow(b2, (float)L->adam_t);
    adam_step(L->d_master, L->d_work, L->d_grad, L->d_m, L->d_v, L->n_params, (float)lr, b1, b2, c1, c2, eps, st);
  }
  GDSW_HIP(hipStreamSynchronize(st));
  L->trained = true;
}

// interior local solves in the apply: network, residual check, LU fallback
void learned_interior_begin(Context& ctx, hipStream_t st) {
  LearnedSolve* L = ctx.learned;
  GridMap gm = learned_gridmap(ctx);
  const double mu = ctx.P.spec.mu;
  to_grid(gm, L->S, L->G, L->d_rsave, L->act[0], L->d_norms, mu, st);
  learned_forward(ctx, L->S, st);
  from_grid(gm, L->S, L->G, L->act[4], L->d_sigma, L->d_norms, mu, ctx.d_w, st);
  GDSW_HIP(hipMemsetAsync(L->d_count, 0, sizeof(int32_t), st));
  local_residual_check_csr(gm, L->S, L->max_n, L->d_rsave, ctx.d_w, L->d_lrow_off, L->d_lrow, L->d_lcol, L->d_lval,
                           L->tau, L->d_rpart, L->d_flags, L->d_count, st);
  GDSW_HIP(hipMemcpyAsync(L->h_count, L->d_count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
}

void learned_interior_finish(Context& ctx, hipStream_t st) {
  LearnedSolve* L = ctx.learned;
  const int nfb = *L->h_count;
  L->learned_solves += L->S - nfb;
  L->fallbacks += nfb;
  if (nfb > 0) {
    copy_segments(learned_gridmap(ctx), L->S, L->d_rsave, ctx.d_w, L->d_flags, st);
    local_solve_set(ctx.L1, ctx.d_w, st, 2, L->d_flags);
  }
}

void learned_apply_interior(Context& ctx, hipStream_t st) {
  learned_interior_begin(ctx, st);
  GDSW_HIP(hipStreamSynchronize(st));
  learned_interior_finish(ctx, st);
}

void learned_copy(Context& dst, const Context& src, hipStream_t st) {
  LearnedSolve* D = dst.learned;
  const LearnedSolve* S = src.learned;
  if (!D || !S) throw StatusError{1, "both contexts need gdsw_learned_init"};
  if (D->G != S->G || D->n_params != S->n_params) throw StatusError{1, "the interior local grids differ"};
  GDSW_HIP(hipMemcpyAsync(D->d_master, S->d_master, D->n_params * sizeof(float), hipMemcpyDeviceToDevice, st));
  round_bf16(D->d_master, D->d_work, D->n_params, st);
  GDSW_HIP(hipMemcpyAsync(D->d_sigma, S->d_sigma, 4 * sizeof(float), hipMemcpyDeviceToDevice, st));
  for (int ch = 0; ch < 4; ++ch) D->sigma[ch] = S->sigma[ch];
  GDSW_HIP(hipMemsetAsync(D->d_m, 0, D->n_params * 4, st));
  GDSW_HIP(hipMemsetAsync(D->d_v, 0, D->n_params * 4, st));
  D->adam_t = 0;
  D->trained = S->trained;
  GDSW_HIP(hipStreamSynchronize(st));
}

// File layout (little-endian): "GDSWNET1", int32 grid, int32 reserved,
// int64 n_params, float sigma[4], float master[n_params].
void learned_save(const Context& ctx, const char* path, hipStream_t st) {
  const LearnedSolve* L = ctx.learned;
  if (!L) throw StatusError{1, "no learned local solve (call gdsw_learned_init)"};
  std::vector<float> w(L->n_params);
  GDSW_HIP(hipMemcpyAsync(w.data(), L->d_master, L->n_params * sizeof(float), hipMemcpyDeviceToHost, st));
  GDSW_HIP(hipStreamSynchronize(st));
  FILE* f = std::fopen(path, "wb");
  if (!f) throw StatusError{1, std::string("cannot open ") + path + " for writing"};
  const int32_t hdr[2] = {L->G, 0};
  const int64_t np = L->n_params;
  bool ok = std::fwrite("GDSWNET1", 1, 8, f) == 8 && std::fwrite(hdr, sizeof hdr, 1, f) == 1 &&
            std::fwrite(&np, sizeof np, 1, f) == 1 && std::fwrite(L->sigma, sizeof(float), 4, f) == 4 &&
            std::fwrite(w.data(), sizeof(float), w.size(), f) == w.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) throw StatusError{1, std::string("writing ") + path + " failed"};
}

void learned_load(Context& ctx, const char* path, hipStream_t st) {
  LearnedSolve* L = ctx.learned;
  if (!L) throw StatusError{1, "no learned local solve (call gdsw_learned_init)"};
  FILE* f = std::fopen(path, "rb");
  if (!f) throw StatusError{1, std::string("cannot open ") + path};
  char magic[8] = {};
  int32_t hdr[2] = {};
  int64_t np = 0;
  float sigma[4] = {};
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "GDSWNET1", 8) == 0 &&
            std::fread(hdr, sizeof hdr, 1, f) == 1 && std::fread(&np, sizeof np, 1, f) == 1;
  if (ok && (hdr[0] != L->G || np != L->n_params)) {
    std::fclose(f);
    throw StatusError{1, std::string(path) + ": the network was trained for another interior node grid"};
  }
  std::vector<float> w(ok ? (size_t)np : 0);
  ok = ok && std::fread(sigma, sizeof(float), 4, f) == 4 && std::fread(w.data(), sizeof(float), w.size(), f) == w.size();
  std::fclose(f);
  if (!ok) throw StatusError{1, std::string(path) + " is not a network file of this library"};
  learned_set_weights(ctx, w.data(), st);
  for (int ch = 0; ch < 4; ++ch) L->sigma[ch] = sigma[ch];
  GDSW_HIP(hipMemcpyAsync(L->d_sigma, L->sigma, 4 * sizeof(float), hipMemcpyHostToDevice, st));
  GDSW_HIP(hipStreamSynchronize(st));
  L->trained = true;
}

void learned_release(Context& ctx) {
  if (!ctx.learned) return;
  if (ctx.learned->h_count) (void)hipHostFree(ctx.learned->h_count);
  delete ctx.learned;
  ctx.learned = nullptr;
}

void learned_set_weights(Context& ctx, const float* host, hipStream_t st) {
  LearnedSolve* L = ctx.learned;
  GDSW_HIP(hipMemcpyAsync(L->d_master, host, L->n_params * sizeof(float), hipMemcpyHostToDevice, st));
  round_bf16(L->d_master, L->d_work, L->n_params, st);
  GDSW_HIP(hipMemsetAsync(L->d_m, 0, L->n_params * 4, st));
  GDSW_HIP(hipMemsetAsync(L->d_v, 0, L->n_params * 4, st));
  L->adam_t = 0;
  GDSW_HIP(hipStreamSynchronize(st));
}

void learned_get_weights(Context& ctx, float* host, int which, hipStream_t st) {
  LearnedSolve* L = ctx.learned;
  const float* src = which == 0 ? L->d_master : (which == 1 ? L->d_work : L->d_grad);
  GDSW_HIP(hipMemcpyAsync(host, src, L->n_params * sizeof(float), hipMemcpyDeviceToHost, st));
  GDSW_HIP(hipStreamSynchronize(st));
}

double learned_loss_grad(Context& ctx, const float* X, const float* T, int B, float* grads, hipStream_t st) {
  LearnedSolve* L = ctx.learned;
  if (B < 1 || B > L->max_b) throw StatusError{1, "batch size out of range"};
  const int G3 = L->G * L->G * L->G;
  GDSW_HIP(hipMemcpyAsync(L->act[0], X, (size_t)B * 4 * G3 * sizeof(float), hipMemcpyHostToDevice, st));
  GDSW_HIP(hipMemcpyAsync(L->d_target, T, (size_t)B * 4 * G3 * sizeof(float), hipMemcpyHostToDevice, st));
  learned_forward(ctx, B, st);
  const double loss = learned_backward(ctx, B, st);
  if (grads) learned_get_weights(ctx, grads, 2, st);
  return loss;
}

}  // namespace gdsw
