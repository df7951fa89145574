// Launchers of the learned-local-solve kernels (conv net, training, mapping).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gdsw {

// Wb (optional): the layer's weights as BF16 [27][32][32] (tap, out, in,
// zero-padded) for the matrix-core path (Cin and Cout each 4 or 32)
void conv_fwd(const float* X, int Cin, const float* W, const float* bias, float* Y, int Cout, int G, bool relu, int B,
              hipStream_t st, const uint16_t* Wb = nullptr);
// Wb[t][co][ci] = W[co][ci][t] as BF16 bits, zero-padded to 32 x 32 channels
void conv_weights_bf16(const float* W, int Cin, int Cout, uint16_t* Wb, hipStream_t st);
// dX may be null (first layer)
void conv_bwd(const float* X, int Cin, const float* W, const float* dY, int Cout, int G, int B, float* dX, float* dW,
              float* db, hipStream_t st);
void relu_bwd(float* dY, const float* Y, int64_t n, hipStream_t st);
void masked_loss(const float* out, const float* target, const float* mask, int per_sample, int B, float* grad,
                 float* loss_b, hipStream_t st);
void adam_step(float* master, float* work, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
               float c1, float c2, float eps, hipStream_t st);
void round_bf16(const float* src, float* dst, int64_t n, hipStream_t st);

// local vectors (segments of the work vector) <-> network grids
struct GridMap {
  const int32_t* factor;  // per sample: factor index in the level-1 set
  const int64_t* xoff;    // level-1 work offsets (per factor)
  const int32_t* n;       // per factor size
  const int32_t* map_ptr; // per sample: range into map
  const int32_t* map;     // grid index (ch * G^3 + voxel) of each local DOF
  const int8_t* field;    // field of each local DOF (0..3)
};
// X[s] = grid(r~_s) / ||r~_s|| with r~_s = r_s, velocity divided by mu (the
// right-hand side of the unit-viscosity problem); norms[s] = ||r~_s||.
// With given_norms the norms are read instead and the pressure, not the
// velocity, is divided by mu: targets A_i^-1 r_s share their inputs' scale
// and are mapped to the unit-viscosity problem (mu K u + B^T p = f is
// K u + B^T (p / mu) = f / mu).
void to_grid(const GridMap& gm, int S, int G, const double* src, float* X, double* norms, double mu, hipStream_t st,
             bool given_norms = false);
// dst segment of sample s = ungrid(Y[s]) * sigma[ch] * norms[s] (pressure times mu)
void from_grid(const GridMap& gm, int S, int G, const float* Y, const float* sigma, const double* norms, double mu,
               double* dst, hipStream_t st);
// flags[s] = ||r_s - A_s y_s|| > tau ||r_s||; count += flags.  r from rsave (copy of the inputs)
// ||r_s - A_s y_s|| > tau ||r_s|| per interior subdomain s, with A_s in CSR
// (local rows from row_off[s] in lrow, local column indices in lcol); part:
// 2 * S * ceil(max_n / 256) doubles.
void local_residual_check_csr(const GridMap& gm, int S, int max_n, const double* rsave, const double* w,
                              const int64_t* row_off, const int64_t* lrow, const int32_t* lcol, const double* lval,
                              double tau, double* part, int32_t* flags, int32_t* count, hipStream_t st);
void local_residual_check(const GridMap& gm, int S, const double* rsave, const double* w, const int32_t* S_ptr,
                          const int32_t* S_idx, const int32_t* rowptr, const int32_t* col, const double* val,
                          double tau, int32_t* flags, int32_t* count, hipStream_t st);
void copy_segments(const GridMap& gm, int S, const double* src, double* dst, const int32_t* only_flags, hipStream_t st);
void zero_segments(const GridMap& gm, int S, double* dst, hipStream_t st);
// gather a batch: Xb[k] = sign_k * Xd[idx_k], Tb[k] = sign_k * Td[idx_k]
void gather_batch(const float* Xd, const float* Td, const int32_t* idx, const float* sign, int B, int per_sample,
                  float* Xb, float* Tb, hipStream_t st);

}  // namespace gdsw
