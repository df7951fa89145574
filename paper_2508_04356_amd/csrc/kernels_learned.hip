// Learned local solve: a small 3-D convolution network N with BF16 weights
// and activations (values rounded to BF16, FP32 accumulation) that stands in
// for A_i^-1 on interior subdomains, and its training kernels.
//
// Tensors are [B][C][G][G][G] in FP32 arrays holding BF16-rounded values;
// weights are [Cout][Cin][27] (taps dz, dy, dx, dx fastest).  Convolutions are
// 3x3x3 with zero padding 1.  Every reduction has a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels_learned.h"

#define GDSW_HIP_LEARNED(call) (void)(call)

namespace gdsw {
namespace {

__device__ inline float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

constexpr int COB = 8;  // output channels per thread

// Y[b][co][v] = bias[co] + sum_{ci,t} W[co][ci][t] X[b][ci][v + t - 1]
__global__ __launch_bounds__(256) void conv_fwd_kernel(const float* __restrict__ X, int Cin,
                                                      const float* __restrict__ W, const float* __restrict__ bias,
                                                      float* __restrict__ Y, int Cout, int G, int relu, int B) {
  extern __shared__ float wl[];  // [COB][Cin][27]
  const int G3 = G * G * G;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int co0 = blockIdx.y * COB;
  const int b = blockIdx.z;
  const int ncb = min(COB, Cout - co0);
  for (int idx = threadIdx.x; idx < ncb * Cin * 27; idx += blockDim.x)
    wl[idx] = W[(int64_t)co0 * Cin * 27 + idx];
  __syncthreads();
  if (v >= G3 || b >= B) return;
  const int x = v % G, y = (v / G) % G, z = v / (G * G);
  float acc[COB];
#pragma unroll
  for (int c = 0; c < COB; ++c) acc[c] = c < ncb ? bias[co0 + c] : 0.f;
  const float* Xb = X + (int64_t)b * Cin * G3;
  for (int ci = 0; ci < Cin; ++ci) {
    const float* Xc = Xb + (int64_t)ci * G3;
    for (int t = 0; t < 27; ++t) {
      const int zz = z + t / 9 - 1, yy = y + (t / 3) % 3 - 1, xx = x + t % 3 - 1;
      if (zz < 0 || zz >= G || yy < 0 || yy >= G || xx < 0 || xx >= G) continue;
      const float xv = Xc[(zz * G + yy) * G + xx];
#pragma unroll
      for (int c = 0; c < COB; ++c)
        if (c < ncb) acc[c] = fmaf(wl[(c * Cin + ci) * 27 + t], xv, acc[c]);
    }
  }
  for (int c = 0; c < ncb; ++c) {
    float o = acc[c];
    if (relu) o = fmaxf(o, 0.f);
    Y[((int64_t)b * Cout + co0 + c) * G3 + v] = bf16_round(o);
  }
}

// ---- 32 -> 32 channel layers on the matrix cores ---------------------------
//
// Implicit GEMM per tap: for tap t, D[co][v] += sum_ci W[co][ci][t] X[ci][v + t]
// as v_mfma_f32_16x16x32_bf16 (16 output channels x 16 voxels x 32 input
// channels), FP32 accumulation.  A block takes 256 consecutive voxels of one
// sample; their neighbourhood (the voxels within one z-plane, one row and
// one node of them) is staged in LDS channel-last as BF16 so that a lane's
// 8 consecutive input channels are one 16-byte read.  Weights come
// pre-arranged as Wb[t][co][ci] BF16 (conv_weights_bf16).
typedef __bf16 lbf8 __attribute__((ext_vector_type(8)));
typedef float lf4 __attribute__((ext_vector_type(4)));
typedef uint32_t lu4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t bits_bf16(float x) { return (uint16_t)(__float_as_uint(bf16_round(x)) >> 16); }

// Wb[t][co][ci] (co < 32, ci < 32) = W[co][ci][t] for co < Cout, ci < Cin, else 0
__global__ void conv_weights_bf16_kernel(const float* __restrict__ W, int Cin, int Cout, uint16_t* __restrict__ Wb) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // (t, co, ci)
  if (idx >= 27 * 32 * 32) return;
  const int ci = idx % 32, co = (idx / 32) % 32, t = idx / 1024;
  Wb[idx] = (ci < Cin && co < Cout) ? bits_bf16(W[(co * Cin + ci) * 27 + t]) : (uint16_t)0;
}

constexpr int CV_TILE = 256;

// CIN input channels (4 or 32, zero-padded to 32 in LDS), COUT output
// channels (4 or 32; 16-row output blocks, the padded rows are not written).
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv_fwd_mfma_kernel(const float* __restrict__ X,
                                                           const uint16_t* __restrict__ Wb,
                                                           const float* __restrict__ bias, float* __restrict__ Y,
                                                           int G, int relu) {
  constexpr int NCB = (COUT + 15) / 16;
  extern __shared__ uint16_t xs[];  // [(CV_TILE + 2 H) voxels][32 channels]
  const int G3 = G * G * G;
  const int H = G * G + G + 1;
  const int nr = CV_TILE + 2 * H;
  const int b = blockIdx.y;
  const int v0 = blockIdx.x * CV_TILE;
  const float* Xb = X + (int64_t)b * CIN * G3;
  for (int idx = threadIdx.x; idx < nr * 32; idx += 256) {
    const int vr = idx % nr, ci = idx / nr;  // consecutive threads: consecutive voxels of one channel
    const int v = v0 - H + vr;
    const float val = (ci < CIN && v >= 0 && v < G3) ? Xb[(int64_t)ci * G3 + v] : 0.f;
    xs[vr * 32 + ci] = bits_bf16(val);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  lf4 acc[4][NCB];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[q][cb] = lf4{0.f, 0.f, 0.f, 0.f};
  int vx[4], vy[4], vz[4];
  bool vin[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int v = v0 + 64 * wave + 16 * q + i;
    vin[q] = v < G3;
    vx[q] = v % G;
    vy[q] = (v / G) % G;
    vz[q] = v / (G * G);
  }
  for (int t = 0; t < 27; ++t) {
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const int off = (dz * G + dy) * G + dx;
    lbf8 a[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
      a[cb] = __builtin_bit_cast(lbf8, *reinterpret_cast<const lu4*>(Wb + ((t * 32 + cb * 16 + i) * 32 + 8 * kq)));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool ok = vin[q] && vz[q] + dz >= 0 && vz[q] + dz < G && vy[q] + dy >= 0 && vy[q] + dy < G &&
                      vx[q] + dx >= 0 && vx[q] + dx < G;
      lu4 raw = {0u, 0u, 0u, 0u};
      if (ok) {
        const int vr = 64 * wave + 16 * q + i + H + off;
        raw = *reinterpret_cast<const lu4*>(xs + vr * 32 + 8 * kq);
      }
      const lbf8 bx = __builtin_bit_cast(lbf8, raw);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        acc[q][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[cb], bx, acc[q][cb], 0, 0, 0);
    }
  }
  // lane holds D[co = 16 cb + 4 kq + r][voxel i]
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int v = v0 + 64 * wave + 16 * q + i;
    if (!vin[q]) continue;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int co = 16 * cb + 4 * kq + r;
        if (co >= COUT) continue;
        float o = acc[q][cb][r] + bias[co];
        if (relu) o = fmaxf(o, 0.f);
        Y[((int64_t)b * COUT + co) * G3 + v] = bf16_round(o);
      }
  }
}

// dX[b][ci][v] = sum_{co,t} W[co][ci][t] dY[b][co][v - t + 1]
__global__ __launch_bounds__(256) void conv_bwd_data_kernel(const float* __restrict__ dY, int Cout,
                                                           const float* __restrict__ W, float* __restrict__ dX,
                                                           int Cin, int G, int B) {
  extern __shared__ float wl[];  // [CIB][Cout][27]
  const int G3 = G * G * G;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int ci0 = blockIdx.y * COB;
  const int b = blockIdx.z;
  const int ncb = min(COB, Cin - ci0);
  for (int idx = threadIdx.x; idx < ncb * Cout * 27; idx += blockDim.x) {
    const int c = idx / (Cout * 27), rem = idx % (Cout * 27), co = rem / 27, t = rem % 27;
    wl[idx] = W[((int64_t)co * Cin + ci0 + c) * 27 + t];
  }
  __syncthreads();
  if (v >= G3 || b >= B) return;
  const int x = v % G, y = (v / G) % G, z = v / (G * G);
  float acc[COB];
#pragma unroll
  for (int c = 0; c < COB; ++c) acc[c] = 0.f;
  const float* dYb = dY + (int64_t)b * Cout * G3;
  for (int co = 0; co < Cout; ++co) {
    const float* dYc = dYb + (int64_t)co * G3;
    for (int t = 0; t < 27; ++t) {
      const int zz = z - (t / 9 - 1), yy = y - ((t / 3) % 3 - 1), xx = x - (t % 3 - 1);
      if (zz < 0 || zz >= G || yy < 0 || yy >= G || xx < 0 || xx >= G) continue;
      const float g = dYc[(zz * G + yy) * G + xx];
#pragma unroll
      for (int c = 0; c < COB; ++c)
        if (c < ncb) acc[c] = fmaf(wl[(c * Cout + co) * 27 + t], g, acc[c]);
    }
  }
  for (int c = 0; c < ncb; ++c) dX[((int64_t)b * Cin + ci0 + c) * G3 + v] = acc[c];
}

// dW[co][ci][t] = sum_{b,v} dY[b][co][v] X[b][ci][v + t - 1]; one work-group per (ci, co)
__global__ __launch_bounds__(256) void conv_bwd_weight_kernel(const float* __restrict__ dY, int Cout,
                                                             const float* __restrict__ X, int Cin,
                                                             float* __restrict__ dW, int G, int B) {
  __shared__ float red[27][257];
  const int ci = blockIdx.x, co = blockIdx.y;
  const int G3 = G * G * G;
  float acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = 0.f;
  for (int idx = threadIdx.x; idx < B * G3; idx += blockDim.x) {
    const int b = idx / G3, v = idx % G3;
    const float g = dY[((int64_t)b * Cout + co) * G3 + v];
    if (g == 0.f) continue;
    const int x = v % G, y = (v / G) % G, z = v / (G * G);
    const float* Xc = X + ((int64_t)b * Cin + ci) * G3;
#pragma unroll
    for (int t = 0; t < 27; ++t) {
      const int zz = z + t / 9 - 1, yy = y + (t / 3) % 3 - 1, xx = x + t % 3 - 1;
      if (zz < 0 || zz >= G || yy < 0 || yy >= G || xx < 0 || xx >= G) continue;
      acc[t] = fmaf(g, Xc[(zz * G + yy) * G + xx], acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < 27; ++t) red[t][threadIdx.x] = acc[t];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int t = 0; t < 27; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 27) dW[((int64_t)co * Cin + ci) * 27 + threadIdx.x] = red[threadIdx.x][0];
}

// db[co] = sum_{b,v} dY[b][co][v]
__global__ __launch_bounds__(256) void conv_bwd_bias_kernel(const float* __restrict__ dY, int Cout, int G3, int B,
                                                           float* __restrict__ db) {
  __shared__ float red[256];
  const int co = blockIdx.x;
  float s = 0.f;
  for (int idx = threadIdx.x; idx < B * G3; idx += blockDim.x) {
    const int b = idx / G3, v = idx % G3;
    s += dY[((int64_t)b * Cout + co) * G3 + v];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[co] = red[0];
}

// dY *= (Y > 0)
__global__ void relu_bwd_kernel(float* __restrict__ dY, const float* __restrict__ Y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!(Y[i] > 0.f)) dY[i] = 0.f;
}

// per sample: loss_b = 0.5 sum mask*(out-target)^2; grad = mask*(out-target)/B
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ out, const float* __restrict__ target,
                                                  const float* __restrict__ mask, int per_sample, int B,
                                                  float* __restrict__ grad, float* __restrict__ loss_b) {
  __shared__ float red[256];
  const int b = blockIdx.x;
  float s = 0.f;
  for (int i = threadIdx.x; i < per_sample; i += blockDim.x) {
    const int64_t k = (int64_t)b * per_sample + i;
    const float d = (out[k] - target[k]) * mask[i];
    s += d * d;
    grad[k] = d * mask[i] / (float)B;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_b[b] = 0.5f * red[0];
}

__global__ void adam_kernel(float* __restrict__ master, float* __restrict__ work, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int64_t n, float lr, float b1, float b2,
                            float c1, float c2, float eps) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float p = master[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    master[i] = p;
    work[i] = bf16_round(p);
  }
}

__global__ void round_bf16_kernel(const float* __restrict__ src, float* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = bf16_round(src[i]);
}

inline int g1(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + 255) / 256)); }

}  // namespace

void conv_weights_bf16(const float* W, int Cin, int Cout, uint16_t* Wb, hipStream_t st) {
  conv_weights_bf16_kernel<<<(27 * 32 * 32 + 255) / 256, 256, 0, st>>>(W, Cin, Cout, Wb);
}

void conv_fwd(const float* X, int Cin, const float* W, const float* bias, float* Y, int Cout, int G, bool relu, int B,
              hipStream_t st, const uint16_t* Wb) {
  const int G3 = G * G * G;
  const size_t shm = (size_t)(CV_TILE + 2 * (G * G + G + 1)) * 32 * sizeof(uint16_t);
  if (Wb && shm <= 64 * 1024) {
    const dim3 grid((G3 + CV_TILE - 1) / CV_TILE, B);
    const int rl = relu ? 1 : 0;
    if (Cin == 32 && Cout == 32) {
      conv_fwd_mfma_kernel<32, 32><<<grid, 256, shm, st>>>(X, Wb, bias, Y, G, rl);
      return;
    }
    if (Cin == 4 && Cout == 32) {
      conv_fwd_mfma_kernel<4, 32><<<grid, 256, shm, st>>>(X, Wb, bias, Y, G, rl);
      return;
    }
    if (Cin == 32 && Cout == 4) {
      conv_fwd_mfma_kernel<32, 4><<<grid, 256, shm, st>>>(X, Wb, bias, Y, G, rl);
      return;
    }
  }
  const size_t shm_w = (size_t)COB * Cin * 27 * sizeof(float);
  dim3 grid((G3 + 255) / 256, (Cout + COB - 1) / COB, B);
  conv_fwd_kernel<<<grid, 256, shm_w, st>>>(X, Cin, W, bias, Y, Cout, G, relu ? 1 : 0, B);
}

void conv_bwd(const float* X, int Cin, const float* W, const float* dY, int Cout, int G, int B, float* dX, float* dW,
              float* db, hipStream_t st) {
  const int G3 = G * G * G;
  if (dX) {
    const size_t shm = (size_t)COB * Cout * 27 * sizeof(float);
    dim3 grid((G3 + 255) / 256, (Cin + COB - 1) / COB, B);
    conv_bwd_data_kernel<<<grid, 256, shm, st>>>(dY, Cout, W, dX, Cin, G, B);
  }
  conv_bwd_weight_kernel<<<dim3(Cin, Cout), 256, 0, st>>>(dY, Cout, X, Cin, dW, G, B);
  conv_bwd_bias_kernel<<<Cout, 256, 0, st>>>(dY, Cout, G3, B, db);
}

void relu_bwd(float* dY, const float* Y, int64_t n, hipStream_t st) { relu_bwd_kernel<<<g1(n), 256, 0, st>>>(dY, Y, n); }

void masked_loss(const float* out, const float* target, const float* mask, int per_sample, int B, float* grad,
                 float* loss_b, hipStream_t st) {
  loss_kernel<<<B, 256, 0, st>>>(out, target, mask, per_sample, B, grad, loss_b);
}

void adam_step(float* master, float* work, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
               float c1, float c2, float eps, hipStream_t st) {
  adam_kernel<<<g1(n), 256, 0, st>>>(master, work, g, m, v, n, lr, b1, b2, c1, c2, eps);
}

void round_bf16(const float* src, float* dst, int64_t n, hipStream_t st) {
  round_bf16_kernel<<<g1(n), 256, 0, st>>>(src, dst, n);
}

}  // namespace gdsw

namespace gdsw {
namespace {

__global__ __launch_bounds__(256) void to_grid_kernel(GridMap gm, int G, const double* __restrict__ src,
                                                     float* __restrict__ X, double* __restrict__ norms, double mu,
                                                     int given) {
  __shared__ double red[256];
  const int s = blockIdx.x;
  const int f = gm.factor[s];
  const int n = gm.n[f];
  const double* r = src + gm.xoff[f];
  const int8_t* fl = gm.field + gm.map_ptr[s];
  // the norm of the input as the unit-viscosity problem sees it, (f / mu, g)
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) {
    const double v = fl[k] < 3 ? r[k] / mu : r[k];
    acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int q = 128; q > 0; q >>= 1) {
    if ((int)threadIdx.x < q) red[threadIdx.x] += red[threadIdx.x + q];
    __syncthreads();
  }
  const double nr = given ? norms[s] : sqrt(red[0]);
  const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
  __syncthreads();
  if (threadIdx.x == 0 && !given) norms[s] = nr;
  const int G3 = G * G * G;
  float* Xs = X + (int64_t)s * 4 * G3;
  const int32_t* mp = gm.map + gm.map_ptr[s];
  // inputs r = (f, g): the unit-viscosity problem sees (f / mu, g); targets
  // A_i^-1 r = (u, p): its solution is (u, p / mu)
  for (int k = threadIdx.x; k < n; k += 256) {
    const double scale = given ? (fl[k] < 3 ? inv : inv / mu) : (fl[k] < 3 ? inv / mu : inv);
    Xs[mp[k]] = bf16_round((float)(r[k] * scale));
  }
}

__global__ void from_grid_kernel(GridMap gm, int G, const float* __restrict__ Y, const float* __restrict__ sigma,
                                 const double* __restrict__ norms, double mu, double* __restrict__ dst) {
  const int s = blockIdx.y;
  const int f = gm.factor[s];
  const int n = gm.n[f];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int G3 = G * G * G;
  const int32_t* mp = gm.map + gm.map_ptr[s];
  const int8_t* fl = gm.field + gm.map_ptr[s];
  const int ch = fl[k];
  const double scale = norms[s] * (double)sigma[ch] * (ch == 3 ? mu : 1.0);
  dst[gm.xoff[f] + k] = (double)Y[(int64_t)s * 4 * G3 + mp[k]] * scale;
}

__device__ inline int lb32(const int32_t* a, int n, int32_t key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Per interior subdomain s and row block: partial sums of |r|^2 and
// |r - A_s y|^2 with the local matrix A_s in CSR (local column indices).
__global__ __launch_bounds__(256) void residual_part_kernel(GridMap gm, const double* __restrict__ rsave,
                                                           const double* __restrict__ w,
                                                           const int64_t* __restrict__ row_off,
                                                           const int64_t* __restrict__ lrow,
                                                           const int32_t* __restrict__ lcol,
                                                           const double* __restrict__ lval,
                                                           double* __restrict__ part) {
  __shared__ double red0[256], red1[256];
  const int s = blockIdx.y;
  const int f = gm.factor[s];
  const int n = gm.n[f];
  const double* y = w + gm.xoff[f];
  const double* r = rsave + gm.xoff[f];
  const int k = blockIdx.x * 256 + threadIdx.x;
  double rr = 0.0, ee = 0.0;
  if (k < n) {
    const int64_t ro = row_off[s] + k;
    double ay = 0.0;
    for (int64_t e = lrow[ro]; e < lrow[ro + 1]; ++e) ay = fma(lval[e], y[lcol[e]], ay);
    const double d = r[k] - ay;
    rr = r[k] * r[k];
    ee = d * d;
  }
  red0[threadIdx.x] = rr;
  red1[threadIdx.x] = ee;
  __syncthreads();
  for (int q = 128; q > 0; q >>= 1) {
    if ((int)threadIdx.x < q) {
      red0[threadIdx.x] += red0[threadIdx.x + q];
      red1[threadIdx.x] += red1[threadIdx.x + q];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((int64_t)s * gridDim.x + blockIdx.x) * 2] = red0[0];
    part[((int64_t)s * gridDim.x + blockIdx.x) * 2 + 1] = red1[0];
  }
}

// flags[f] = 1 where ||r - A y|| > tau ||r||, summing the row blocks in order
__global__ void residual_flag_kernel(GridMap gm, int S, int nblk, const double* __restrict__ part, double tau,
                                     int32_t* __restrict__ flags, int32_t* __restrict__ count) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  double rr = 0.0, ee = 0.0;
  for (int q = 0; q < nblk; ++q) {
    rr += part[((int64_t)s * nblk + q) * 2];
    ee += part[((int64_t)s * nblk + q) * 2 + 1];
  }
  const bool bad = !(sqrt(ee) <= tau * sqrt(rr));
  flags[gm.factor[s]] = bad ? 1 : 0;
  if (bad) atomicAdd(count, 1);
}

__global__ __launch_bounds__(256) void residual_check_kernel(GridMap gm, const double* __restrict__ rsave,
                                                            const double* __restrict__ w,
                                                            const int32_t* __restrict__ S_ptr,
                                                            const int32_t* __restrict__ S_idx,
                                                            const int32_t* __restrict__ rowptr,
                                                            const int32_t* __restrict__ col,
                                                            const double* __restrict__ val, double tau,
                                                            int32_t* __restrict__ flags, int32_t* __restrict__ count) {
  __shared__ double red0[256], red1[256];
  const int s = blockIdx.x;
  const int f = gm.factor[s];
  const int n = gm.n[f];
  const int32_t* S = S_idx + S_ptr[f];
  const double* y = w + gm.xoff[f];
  const double* r = rsave + gm.xoff[f];
  double rr = 0.0, ee = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) {
    const int32_t g = S[k];
    double ay = 0.0;
    for (int e = rowptr[g]; e < rowptr[g + 1]; ++e) {
      const int lc = lb32(S, n, col[e]);
      if (lc < n && S[lc] == col[e]) ay = fma(val[e], y[lc], ay);
    }
    const double d = r[k] - ay;
    rr += r[k] * r[k];
    ee += d * d;
  }
  red0[threadIdx.x] = rr;
  red1[threadIdx.x] = ee;
  __syncthreads();
  for (int q = 128; q > 0; q >>= 1) {
    if ((int)threadIdx.x < q) {
      red0[threadIdx.x] += red0[threadIdx.x + q];
      red1[threadIdx.x] += red1[threadIdx.x + q];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const bool bad = !(sqrt(red1[0]) <= tau * sqrt(red0[0]));
    flags[f] = bad ? 1 : 0;
    if (bad) atomicAdd(count, 1);
  }
}

__global__ void copy_segments_kernel(GridMap gm, const double* __restrict__ src, double* __restrict__ dst,
                                     const int32_t* __restrict__ only_flags) {
  const int s = blockIdx.y;
  const int f = gm.factor[s];
  if (only_flags && !only_flags[f]) return;
  const int n = gm.n[f];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[gm.xoff[f] + k] = src[gm.xoff[f] + k];
}

__global__ void zero_segments_kernel(GridMap gm, double* __restrict__ dst) {
  const int s = blockIdx.y;
  const int f = gm.factor[s];
  const int n = gm.n[f];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[gm.xoff[f] + k] = 0.0;
}

__global__ void gather_batch_kernel(const float* __restrict__ Xd, const float* __restrict__ Td,
                                    const int32_t* __restrict__ idx, const float* __restrict__ sign, int per_sample,
                                    float* __restrict__ Xb, float* __restrict__ Tb) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= per_sample) return;
  const int64_t src = (int64_t)idx[b] * per_sample + i;
  Xb[(int64_t)b * per_sample + i] = sign[b] * Xd[src];
  Tb[(int64_t)b * per_sample + i] = sign[b] * Td[src];
}

}  // namespace

void to_grid(const GridMap& gm, int S, int G, const double* src, float* X, double* norms, double mu, hipStream_t st,
             bool given_norms) {
  if (S == 0) return;
  GDSW_HIP_LEARNED(hipMemsetAsync(X, 0, (size_t)S * 4 * G * G * G * sizeof(float), st));
  to_grid_kernel<<<S, 256, 0, st>>>(gm, G, src, X, norms, mu, given_norms ? 1 : 0);
}

void from_grid(const GridMap& gm, int S, int G, const float* Y, const float* sigma, const double* norms, double mu,
               double* dst, hipStream_t st) {
  if (S == 0) return;
  const int maxn = 4 * G * G * G;
  from_grid_kernel<<<dim3((maxn + 255) / 256, S), 256, 0, st>>>(gm, G, Y, sigma, norms, mu, dst);
}

void local_residual_check_csr(const GridMap& gm, int S, int max_n, const double* rsave, const double* w,
                              const int64_t* row_off, const int64_t* lrow, const int32_t* lcol, const double* lval,
                              double tau, double* part, int32_t* flags, int32_t* count, hipStream_t st) {
  if (S == 0) return;
  const int nblk = (max_n + 255) / 256;
  residual_part_kernel<<<dim3(nblk, S), 256, 0, st>>>(gm, rsave, w, row_off, lrow, lcol, lval, part);
  residual_flag_kernel<<<(S + 255) / 256, 256, 0, st>>>(gm, S, nblk, part, tau, flags, count);
}

void local_residual_check(const GridMap& gm, int S, const double* rsave, const double* w, const int32_t* S_ptr,
                          const int32_t* S_idx, const int32_t* rowptr, const int32_t* col, const double* val,
                          double tau, int32_t* flags, int32_t* count, hipStream_t st) {
  if (S == 0) return;
  residual_check_kernel<<<S, 256, 0, st>>>(gm, rsave, w, S_ptr, S_idx, rowptr, col, val, tau, flags, count);
}

void copy_segments(const GridMap& gm, int S, const double* src, double* dst, const int32_t* only_flags,
                   hipStream_t st) {
  if (S == 0) return;
  copy_segments_kernel<<<dim3(64, S), 256, 0, st>>>(gm, src, dst, only_flags);
}

void zero_segments(const GridMap& gm, int S, double* dst, hipStream_t st) {
  if (S == 0) return;
  zero_segments_kernel<<<dim3(64, S), 256, 0, st>>>(gm, dst);
}

void gather_batch(const float* Xd, const float* Td, const int32_t* idx, const float* sign, int B, int per_sample,
                  float* Xb, float* Tb, hipStream_t st) {
  gather_batch_kernel<<<dim3((per_sample + 255) / 256, B), 256, 0, st>>>(Xd, Td, idx, sign, per_sample, Xb, Tb);
}

}  // namespace gdsw
