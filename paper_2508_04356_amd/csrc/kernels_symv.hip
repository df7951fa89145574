// x_f <- M_f x_f for symmetric explicit inverses stored as the upper
// triangle of 64 x 64 tiles: the inverse of a symmetric local (or coarse)
// saddle-point matrix of eq. (2.1) is symmetric, so only the tiles (I, J)
// with J >= I are kept (each tile column-major and contiguous), which halves
// the bytes of the HBM-bound product.  A stored tile with J > I contributes
// M_IJ x_J to block row I and M_IJ^T x_I to block row J; a diagonal tile
// (stored whole) contributes M_II x_I.  A work-group stages a tile in LDS
// (one contiguous 32 KB read for FP64) and writes both partial blocks
// (runs of several tiles per work-group measured slower on MI355X: 1 tile
// 503 us, 2: 507 us, 4: 520 us, 8: 536 us at 16^3); a second launch sums
// them per block row in a fixed order
// (tiles (I, I), (I, I+1), ... then the transposed tiles (0, I), (1, I), ...),
// so results are repeatable bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "vec16.h"

namespace gdsw {
namespace {

constexpr int ST = 64;        // tile edge
constexpr int SPAD = ST + 1;  // LDS column stride

__host__ __device__ inline int64_t tile_index(int I, int J, int nt) {
  return (int64_t)I * nt - (int64_t)I * (I - 1) / 2 + (J - I);
}

// Item (f, I, J0, p0): tiles (I, J0 .. J0 + SYMV_RUN - 1) (those with
// J < nt) of matrix f; partial slots p0 + (J - J0).  The work-group walks
// the run with the next tile's loads in flight while the current one is
// multiplied.  Rows and columns past n meet zero vector entries (the padded
// inverse is block-diagonal, so those tile entries only feed outputs that
// are never read).
#ifndef GDSW_SYMV_RUN
#define GDSW_SYMV_RUN 1
#endif
constexpr int SYMV_RUN = GDSW_SYMV_RUN;

template <typename T>
__global__ __launch_bounds__(256) void symv_part_kernel(const T* __restrict__ store, const int64_t* __restrict__ OFF,
                                                        const int32_t* __restrict__ N, const int32_t* __restrict__ NP,
                                                        const int64_t* __restrict__ XOFF,
                                                        const int4* __restrict__ items, const double* __restrict__ w,
                                                        double* __restrict__ prow, double* __restrict__ pcol) {
  using Acc = typename VecW<T>::acc;
  constexpr int E = VecW<T>::W;  // entries per 16-byte load
  constexpr int PER = ST * ST / E / 256;
  __shared__ Acc Ms[ST * SPAD];
  __shared__ Acc xi[ST], xj[ST];
  __shared__ Acc red[4][ST];
  const int4 item = items[blockIdx.x];
  const int f = item.x, I = item.y, J0 = item.z, p0 = item.w;
  const int n = N[f];
  const int nt = NP[f] / ST;
  const int J1 = min(nt, J0 + SYMV_RUN);
  const double* x = w + XOFF[f];
  const T* tiles = store + OFF[f] + tile_index(I, J0, nt) * (ST * ST);  // the run is contiguous
  const int l = threadIdx.x & 63, q = threadIdx.x >> 6;
  if (threadIdx.x < ST) {
    const int ri = ST * I + threadIdx.x;
    xi[threadIdx.x] = ri < n ? (Acc)x[ri] : (Acc)0;
  }
  Acc v[PER][E];
#pragma unroll
  for (int u = 0; u < PER; ++u) load16_nt(tiles + (threadIdx.x + 256 * u) * E, v[u]);
  for (int J = J0; J < J1; ++J) {
    __syncthreads();  // the previous tile's products are done with LDS
#pragma unroll
    for (int u = 0; u < PER; ++u)
#pragma unroll
      for (int t = 0; t < E; ++t) {
        const int e = (threadIdx.x + 256 * u) * E + t;  // column-major: row e % 64, column e / 64
        Ms[(e >> 6) * SPAD + (e & 63)] = v[u][t];
      }
    if (threadIdx.x < ST) {
      const int rj = ST * J + threadIdx.x;
      xj[threadIdx.x] = rj < n ? (Acc)x[rj] : (Acc)0;
    }
    __syncthreads();
    if (J + 1 < J1) {  // uniform: the next tile of the run
      const T* nxt = tiles + (int64_t)(J + 1 - J0) * (ST * ST);
#pragma unroll
      for (int u = 0; u < PER; ++u) load16_nt(nxt + (threadIdx.x + 256 * u) * E, v[u]);
    }
    const int p = p0 + (J - J0);
    // block row I: thread (row l, quarter q) sums columns 16 q .. 16 q + 15
    Acc s = 0;
#pragma unroll
    for (int c = 16 * q; c < 16 * q + 16; ++c) s = fma(Ms[c * SPAD + l], xj[c], s);
    red[q][l] = s;
    __syncthreads();
    if (q == 0)
      prow[(int64_t)p * ST + l] = (double)red[0][l] + (double)red[1][l] + (double)red[2][l] + (double)red[3][l];
    if (J > I) {  // uniform: block row J gets the transposed tile
      __syncthreads();
      Acc s2 = 0;
#pragma unroll
      for (int r = 16 * q; r < 16 * q + 16; ++r) s2 = fma(Ms[l * SPAD + r], xi[r], s2);
      red[q][l] = s2;
      __syncthreads();
      if (q == 0)
        pcol[(int64_t)p * ST + l] = (double)red[0][l] + (double)red[1][l] + (double)red[2][l] + (double)red[3][l];
    }
  }
}

// Item (f, I, P0, nt): x_f[64 I + l] = sum_{J >= I} prow(I, J)[l] + sum_{K < I} pcol(K, I)[l].
__global__ __launch_bounds__(64) void symv_sum_kernel(const int32_t* __restrict__ N, const int64_t* __restrict__ XOFF,
                                                      const int4* __restrict__ items,
                                                      const double* __restrict__ prow,
                                                      const double* __restrict__ pcol, double* __restrict__ w) {
  const int4 item = items[blockIdx.x];
  const int f = item.x, I = item.y, P0 = item.z, nt = item.w;
  const int l = threadIdx.x;
  double s = 0.0;
  for (int J = I; J < nt; ++J) s += prow[(P0 + tile_index(I, J, nt)) * ST + l];
  for (int K = 0; K < I; ++K) s += pcol[(P0 + tile_index(K, I, nt)) * ST + l];
  const int r = ST * I + l;
  if (r < N[f]) w[XOFF[f] + r] = s;
}

// Upper tiles of npad x npad column-major FP64 matrices, converted to the
// storage type: block (tile t of matrix k) copies one 64 x 64 tile.
template <typename T>
__global__ __launch_bounds__(256) void pack_upper_kernel(const double* __restrict__ src, const int64_t* __restrict__ soff,
                                                         const int32_t* __restrict__ NP,
                                                         const int64_t* __restrict__ doff, T* __restrict__ dst) {
  const int k = blockIdx.y;
  const int nt = NP[k] / ST;
  const int64_t t = blockIdx.x;
  if (t >= (int64_t)nt * (nt + 1) / 2) return;  // uniform over the work-group
  int I = 0;
  while (tile_index(I + 1, I + 1, nt) <= t) ++I;  // block row of tile t
  const int J = I + (int)(t - tile_index(I, I, nt));
  const int64_t np = NP[k];
  const double* s = src + soff[k] + (int64_t)ST * J * np + (int64_t)ST * I;
  T* d = dst + doff[k] + t * (ST * ST);
  for (int e = threadIdx.x; e < ST * ST; e += 256) {
    const int r = e & 63, c = e >> 6;
    const double v = s[(int64_t)c * np + r];
    if constexpr (sizeof(T) == 2)
      d[e] = to_bf16((float)v);
    else
      d[e] = (T)v;
  }
}

template <typename T>
void symv_launch(const FactorSet& fs, double* w, hipStream_t st) {
  const FactorSet::GemvPlan& G = fs.gemv[0];
  if (G.n1 == 0) return;
  double* prow = fs.d_partial;
  double* pcol = fs.d_partial + fs.partial_len / 2;
  KernelTimer* tm = (fs.timer && fs.timer->on && fs.timer->used < KernelTimer::CAP) ? fs.timer : nullptr;
  if (tm) GDSW_HIP(hipEventRecord(tm->ev[2 * tm->used], st));
  symv_part_kernel<T><<<G.n1, 256, 0, st>>>(static_cast<const T*>(fs.store), fs.d_off, fs.d_n, fs.d_npad, fs.d_xoff,
                                            G.d_items1, w, prow, pcol);
  if (tm) {
    GDSW_HIP(hipEventRecord(tm->ev[2 * tm->used++ + 1], st));
    tm->bytes += (double)fs.alg_bytes;
  }
  symv_sum_kernel<<<G.n2, 64, 0, st>>>(fs.d_n, fs.d_xoff, G.d_items2, prow, pcol, w);
}

}  // namespace

int64_t symv_tiles(int npad) {
  const int64_t nt = npad / ST;
  return nt * (nt + 1) / 2;
}

void symv_items(int f, int npad, int64_t p0, std::vector<int4>& it1, std::vector<int4>& it2) {
  const int nt = npad / ST;
  for (int I = 0; I < nt; ++I) {
    for (int J = I; J < nt; J += SYMV_RUN) it1.push_back(make_int4(f, I, J, (int)(p0 + tile_index(I, J, nt))));
    it2.push_back(make_int4(f, I, (int)p0, nt));
  }
}

void pack_upper(int prec, const double* src, const int64_t* soff, const int32_t* npad, int count, int max_npad,
                const int64_t* doff, void* dst, hipStream_t st) {
  if (count == 0) return;
  const int64_t nt = max_npad / ST;
  const dim3 grid((unsigned)(nt * (nt + 1) / 2), count);
  if (prec == P_FP64)
    pack_upper_kernel<double><<<grid, 256, 0, st>>>(src, soff, npad, doff, static_cast<double*>(dst));
  else if (prec == P_FP32)
    pack_upper_kernel<float><<<grid, 256, 0, st>>>(src, soff, npad, doff, static_cast<float*>(dst));
  else
    pack_upper_kernel<uint16_t><<<grid, 256, 0, st>>>(src, soff, npad, doff, static_cast<uint16_t*>(dst));
  GDSW_HIP(hipGetLastError());
}

void symv_set(const FactorSet& fs, double* w, hipStream_t st) {
  if (fs.count == 0) return;
  if (fs.prec == P_FP64)
    symv_launch<double>(fs, w, st);
  else if (fs.prec == P_FP32)
    symv_launch<float>(fs, w, st);
  else
    symv_launch<uint16_t>(fs, w, st);
  GDSW_HIP(hipGetLastError());
}

}  // namespace gdsw
