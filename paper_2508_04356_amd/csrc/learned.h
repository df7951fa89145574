// Learned local solve state (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "context.h"
#include "kernels_learned.h"

namespace gdsw {

struct LearnedSolve {
  int G = 0;                      // grid nodes per axis of an interior local problem
  int S = 0;                      // interior subdomains
  std::vector<int32_t> factors;   // their level-1 factor indices
  int32_t *d_factor = nullptr, *d_map_ptr = nullptr, *d_map = nullptr;
  int8_t* d_field = nullptr;
  int32_t *d_S_ptr = nullptr, *d_S_idx = nullptr;
  float* d_mask = nullptr;
  int64_t n_params = 0;
  int64_t woff[4] = {}, boff[4] = {};
  float *d_master = nullptr, *d_work = nullptr, *d_grad = nullptr, *d_m = nullptr, *d_v = nullptr;
  uint16_t* d_wb = nullptr;       // BF16 [27][32][32] weights of the 4 layers (matrix-core path)
  int64_t* d_lrow_off = nullptr;  // local CSR of the interior matrices (residual check)
  int64_t* d_lrow = nullptr;
  int32_t* d_lcol = nullptr;
  double* d_lval = nullptr;
  double* d_rpart = nullptr;
  int max_n = 0;
  int adam_t = 0;
  float* d_sigma = nullptr;
  float sigma[4] = {1.f, 1.f, 1.f, 1.f};
  int max_b = 0;
  float* act[5] = {};
  float* gact[5] = {};
  float* d_target = nullptr;
  double* d_norms = nullptr;
  float* d_lossb = nullptr;
  double* d_rsave = nullptr;
  int32_t* d_flags = nullptr;
  int32_t* d_count = nullptr;
  int32_t* h_count = nullptr;
  int32_t* d_bidx = nullptr;
  float* d_sign = nullptr;
  float *Xd = nullptr, *Td = nullptr;
  int N = 0;
  double tau = 0.7;
  bool trained = false;
  int64_t fallbacks = 0, learned_solves = 0;
};

int64_t learned_param_count();
void learned_init(Context& ctx, uint64_t seed, hipStream_t st);
GridMap learned_gridmap(const Context& ctx);
void learned_forward(Context& ctx, int B, hipStream_t st);
double learned_backward(Context& ctx, int B, hipStream_t st);
void learned_generate(Context& ctx, int nsolves, uint64_t seed, hipStream_t st);
void learned_train(Context& ctx, int steps, int batch, double lr, uint64_t seed, double* history, hipStream_t st);
void learned_apply_interior(Context& ctx, hipStream_t st);
// The two halves of learned_apply_interior: the network's solves and their
// residual check (the fallback count is copied to pinned memory), then,
// once the caller has synchronised, the exact re-solve of flagged ones.
void learned_interior_begin(Context& ctx, hipStream_t st);
void learned_interior_finish(Context& ctx, hipStream_t st);
// dst's network (weights and output scales) <- src's; same interior grid.
void learned_copy(Context& dst, const Context& src, hipStream_t st);
void learned_release(Context& ctx);
// the trained network (FP32 master weights and output scales) to / from a file
void learned_save(const Context& ctx, const char* path, hipStream_t st);
void learned_load(Context& ctx, const char* path, hipStream_t st);
void learned_set_weights(Context& ctx, const float* host, hipStream_t st);
void learned_get_weights(Context& ctx, float* host, int which, hipStream_t st);
double learned_loss_grad(Context& ctx, const float* X, const float* T, int B, float* grads, hipStream_t st);

}  // namespace gdsw
