// X_i <- A_i^-1 X_i for several right-hand sides (up to 32 per launch) on
// the matrix cores: v_mfma_f64_16x16x4 (FP64 storage), v_mfma_f32_16x16x4f32
// (FP32) and v_mfma_f32_16x16x32_bf16 (BF16, right-hand sides rounded to
// BF16, FP32 accumulation).  Still HBM bound at 32 right-hand sides
// (8 / 16 / 32 flop per byte of FP64 / FP32 / BF16 storage).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "kernels.h"
#include "vec16.h"

namespace gdsw {
namespace {

// ---- several right-hand sides: MFMA products with the stored inverses ------
//
// Item (f, r0, c0, p) of a multi-RHS plan: output rows [r0, r0 + RB) and
// summation columns [c0, c0 + GEMM_CW) of matrix f for up to 32 right-hand
// sides (two groups of 16).  partial layout: partial[(p * RB + row) * 32 + j].
// FP64/FP32 storage: each wave owns RB / 4 output rows and reads its MFMA
// operands straight from memory (no LDS, no barriers): the matrix fragments
// with non-temporal 16-byte loads (each instruction covers 4 columns x 16
// consecutive row pairs/quads), the right-hand-side fragments (re-read by
// every row block of the matrix, so cached) from the work vectors; the
// loads of the next step are issued before the products of the current one.
// BF16 storage: tiles staged through LDS (gemm_part_bf16_lds_kernel), with
// the right-hand sides from a BF16 copy made once per launch.  Summation
// entries past n meet zero right-hand sides, so padded entries never
// contribute; rows and right-hand sides past n and nrhs give outputs that
// are never read.
typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef double mf_d2 __attribute__((ext_vector_type(2)));
typedef __bf16 mf_bf8 __attribute__((ext_vector_type(8)));

#ifndef GDSW_GEMM_HD
#define GDSW_GEMM_HD 4    // FP64: row groups of 32 rows per wave
#endif
#ifndef GDSW_GEMM_H
#define GDSW_GEMM_H 1     // FP32: row groups of 64 rows per wave
#endif
#ifndef GDSW_GEMM_Q
#define GDSW_GEMM_Q 2     // FP64/FP32: groups of 4 summation columns per step
#endif
#ifndef GDSW_GEMM_CW
#define GDSW_GEMM_CW 2048 // summation columns per work item
#endif
#ifndef GDSW_GEMM_SBL
#define GDSW_GEMM_SBL 256 // BF16: summation entries per staged step
#endif

constexpr int GEMM_CW = GDSW_GEMM_CW;

template <typename T>
struct MultiShape;
template <>
struct MultiShape<double> {  // v_mfma_f64_16x16x4: a lane's 16-byte load = 2 rows of one column
  static constexpr int H = GDSW_GEMM_HD, RB = 4 * H * 32;  // direct kernel (the LDS one: DL_RB)
  using P = double;
};
template <>
struct MultiShape<float> {  // v_mfma_f32_16x16x4f32: 4 rows of one column
  static constexpr int H = GDSW_GEMM_H, RB = 4 * H * 64;
  using P = float;
};
template <>
struct MultiShape<uint16_t> {  // v_mfma_f32_16x16x32_bf16, staged through LDS (gemm_part_bf16_lds_kernel)
  static constexpr int RB = 64;
  using P = float;
};

// FP64 and FP32 storage.  One step covers 4 Q summation columns.  For each
// of H row groups h, lane l loads E = 16 / sizeof(T) consecutive rows
// (Rw + 16 E h + E (l % 16) + v) of column c + 4 q + l / 16; MFMA (h, v)
// uses A[i][k] = M[Rw + 16 E h + E i + v][c + 4 q + k] and
// B[k][j] = x[c + 4 q + k][16 g + j] (rounded to T).
template <typename T, int G>
struct StepRegs {
  static constexpr int E = 16 / sizeof(T), H = MultiShape<T>::H, Q = GDSW_GEMM_Q;
  T a[Q][H][E];
  double b[Q][G];  // right-hand sides as loaded; rounded to T at the product
};

// Every load is unconditional (addresses clamped into the matrix and the
// work vector), so that the loads of the next step stay in flight while the
// products of the current one run; rows and right-hand sides beyond n and
// nrhs produce outputs that are never read, and summation columns beyond
// the chunk get a zero right-hand side.
template <typename T, int G>
__device__ inline void load_step(StepRegs<T, G>& R, const T* const (&arow)[MultiShape<T>::H], int64_t np,
                                 const double* const (&xj)[G], int64_t ldk, int c, int cend) {
  using S = StepRegs<T, G>;
#pragma unroll
  for (int q = 0; q < S::Q; ++q) {
    const int col = c + 4 * q;  // + l / 16, folded into the pointers
#pragma unroll
    for (int h = 0; h < S::H; ++h) load16_nt(arow[h] + (int64_t)col * np, R.a[q][h]);
#pragma unroll
    for (int g = 0; g < G; ++g) R.b[q][g] = xj[g][(int64_t)col * ldk];
  }
}

template <typename T, int G, typename ACC>
__device__ inline void mma_step(ACC (&acc)[MultiShape<T>::H][16 / sizeof(T)][G], const StepRegs<T, G>& R) {
  using S = StepRegs<T, G>;
#pragma unroll
  for (int q = 0; q < S::Q; ++q)
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int h = 0; h < S::H; ++h)
#pragma unroll
        for (int v = 0; v < S::E; ++v) {
          if constexpr (sizeof(T) == 8)
            acc[h][v][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(R.a[q][h][v], R.b[q][g], acc[h][v][g], 0, 0, 0);
          else
            acc[h][v][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(R.a[q][h][v], (float)R.b[q][g], acc[h][v][g], 0, 0, 0);
        }
}

template <typename T, int G>
__global__ __launch_bounds__(256) void gemm_part_kernel(const T* __restrict__ store, const int64_t* __restrict__ OFF,
                                                        const int32_t* __restrict__ N, const int32_t* __restrict__ NP,
                                                        const int64_t* __restrict__ XOFF,
                                                        const int4* __restrict__ items, const double* __restrict__ w,
                                                        int64_t ldk, int nrhs, int cw,
                                                        typename MultiShape<T>::P* __restrict__ partial) {
  using S = MultiShape<T>;
  using P = typename S::P;
  using ACC = typename std::conditional<sizeof(T) == 8, mf_d4, mf_f4>::type;
  constexpr int E = 16 / sizeof(T);
  constexpr int H = S::H, RB = S::RB, SK = 4 * GDSW_GEMM_Q;
  const int4 item = items[blockIdx.x];
  const int f = item.x, r0 = item.y, c0 = item.z, p = item.w;
  const int n = N[f];
  const int64_t np = NP[f];
  const int cend = min(c0 + cw, n);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const int Rw = r0 + wave * (RB / 4);
  const T* arow[H];
#pragma unroll
  for (int h = 0; h < H; ++h)
    arow[h] = store + OFF[f] + min<int64_t>(Rw + 16 * E * h + E * i, np - E) + (int64_t)kq * np;
  const double* xj[G];
#pragma unroll
  for (int g = 0; g < G; ++g) xj[g] = w + (XOFF[f] + kq) * ldk + min(16 * g + i, nrhs - 1);
  ACC acc[H][E][G];
#pragma unroll
  for (int h = 0; h < H; ++h)
#pragma unroll
    for (int v = 0; v < E; ++v)
#pragma unroll
      for (int g = 0; g < G; ++g) acc[h][v][g] = ACC{0, 0, 0, 0};
  // steps of SK columns; the last one may run past n into the padding
  // (zero right-hand side there, columns < np)
  const int nstep = (cend - c0 + SK - 1) / SK;
  const int clast = c0 + (nstep - 1) * SK;
  const bool tail = cend % SK != 0;  // only the last step can be partial
  StepRegs<T, G> R0, R1;
  int c = c0;
  auto fix_tail = [&](StepRegs<T, G>& R, int cs) {
    if (tail && cs == clast) {
#pragma unroll
      for (int q = 0; q < GDSW_GEMM_Q; ++q)
#pragma unroll
        for (int g = 0; g < G; ++g)
          if (cs + 4 * q + kq >= cend) R.b[q][g] = 0.0;
    }
  };
  if (nstep & 1) {
    load_step(R0, arow, np, xj, ldk, c, cend);
    fix_tail(R0, c);
    mma_step<T, G>(acc, R0);
    c += SK;
  }
  if (c < cend) {
    load_step(R0, arow, np, xj, ldk, c, cend);
    for (; c < cend; c += 2 * SK) {
      // the scheduling barriers keep the next step's loads ahead of the
      // current step's products (the scheduler would otherwise sink them)
      load_step(R1, arow, np, xj, ldk, c + SK, cend);
      __builtin_amdgcn_sched_barrier(0);
      mma_step<T, G>(acc, R0);
      __builtin_amdgcn_sched_barrier(0);
      load_step(R0, arow, np, xj, ldk, min(c + 2 * SK, clast), cend);
      __builtin_amdgcn_sched_barrier(0);
      fix_tail(R1, c + SK);
      mma_step<T, G>(acc, R1);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // D_(h,v)[i'][j] = y[Rw + 16 E h + E i' + v][16 g + j], j = i.  Accumulator
  // register t of a lane holds output row i' = 4 kq + t for the f32 shape and
  // i' = kq + 4 t for the f64 shape (groups of one row strided by 4).
  P* out = partial + (int64_t)p * RB * 32;
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int v = 0; v < E; ++v)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int ip = sizeof(T) == 8 ? kq + 4 * t : 4 * kq + t;
          out[(int64_t)(wave * (RB / 4) + 16 * E * h + E * ip + v) * 32 + g * 16 + i] = (P)acc[h][v][g][t];
        }
}

// BF16 right-hand sides for the BF16 products, stored right-hand side by
// right-hand side per matrix: xb[32 XP_f + j np_f + d] = bf16(x_f[d][j]),
// zero for d >= n_f and j >= nrhs.  One work-group per (64 rows, matrix),
// transposed through LDS.
__global__ __launch_bounds__(256) void stage_bf16_kernel(const int32_t* __restrict__ N, const int32_t* __restrict__ NP,
                                                         const int64_t* __restrict__ XOFF,
                                                         const int64_t* __restrict__ XPOFF,
                                                         const double* __restrict__ w, int64_t ldk, int nrhs,
                                                         uint16_t* __restrict__ xb) {
  const int f = blockIdx.y;
  const int n = N[f];
  const int64_t np = NP[f];
  const int d0 = blockIdx.x * 64;
  if (d0 >= np) return;  // uniform over the work-group
  __shared__ double t[64][33];
  const double* x = w + XOFF[f] * ldk;
  for (int e = threadIdx.x; e < 64 * 32; e += 256) {
    const int d = e >> 5, j = e & 31;
    t[d][j] = (d0 + d < n && j < nrhs) ? x[(int64_t)(d0 + d) * ldk + j] : 0.0;
  }
  __syncthreads();
  uint16_t* o = xb + XPOFF[f] * 32 + d0;
  for (int e = threadIdx.x; e < 64 * 32; e += 256) {
    const int j = e >> 6, d = e & 63;
    o[(int64_t)j * np + d] = to_bf16((float)t[d][j]);
  }
}

// BF16 storage, tiles staged through LDS.  Item (f, r0, c0, p): 64 output
// rows (= storage columns r0.., the inverse being symmetric) and GEMM_CW
// summation entries.  Each step stages SB entries of those 64 columns
// (each column's SB entries are contiguous: 2 SB bytes per column, read by
// consecutive lanes, so every load instruction covers whole runs of a
// column) and the same SB entries of the 32 BF16 right-hand sides; wave w
// then runs the MFMAs of output rows 16 w .. 16 w + 15 from LDS.  The next
// step's loads are issued before the current step's products.  Columns
// past n read a clamped column (outputs never used); entries past np read
// clamped addresses and get zero right-hand sides.
constexpr int BL_RB = 64, BL_SB = GDSW_GEMM_SBL, BL_PAD = BL_SB + 8;
constexpr int BL_APIECES = BL_RB * BL_SB / 8 / 256;  // 16-byte pieces per thread per step (A)
constexpr int BL_BPIECES = 32 * BL_SB / 8 / 256;     // (right-hand sides)
static_assert(BL_APIECES >= 1 && BL_BPIECES >= 1 && 256 % BL_SB == 0, "BF16 LDS step shape: chunks are multiples of 256");

struct BlRegs {
  gdsw_u4 a[BL_APIECES];
  gdsw_u4 b[BL_BPIECES];
};

__device__ inline void bl_load(BlRegs& R, const uint16_t* __restrict__ A, const uint16_t* __restrict__ X, int r0,
                               int n, int64_t np, int c) {
  constexpr int PPC = BL_SB / 8;  // pieces per column
#pragma unroll
  for (int u = 0; u < BL_APIECES; ++u) {
    const int e = threadIdx.x + 256 * u, cc = e / PPC, pc = e % PPC;
    const int64_t col = min(r0 + cc, n - 1);
    const int64_t ent = min<int64_t>(c + 8 * pc, np - 8);
    R.a[u] = *reinterpret_cast<const gdsw_u4*>(A + col * np + ent);
  }
#pragma unroll
  for (int u = 0; u < BL_BPIECES; ++u) {
    const int e = threadIdx.x + 256 * u, j = e / PPC, pc = e % PPC;
    const int64_t ent = c + 8 * pc;
    const gdsw_u4 v = *reinterpret_cast<const gdsw_u4*>(X + j * np + min<int64_t>(ent, np - 8));
    const gdsw_u4 z = {0, 0, 0, 0};
    R.b[u] = ent < np ? v : z;
  }
}

__device__ inline void bl_store(const BlRegs& R, uint16_t* As, uint16_t* Bs) {
  constexpr int PPC = BL_SB / 8;
#pragma unroll
  for (int u = 0; u < BL_APIECES; ++u) {
    const int e = threadIdx.x + 256 * u, cc = e / PPC, pc = e % PPC;
    *reinterpret_cast<gdsw_u4*>(As + cc * BL_PAD + 8 * pc) = R.a[u];
  }
#pragma unroll
  for (int u = 0; u < BL_BPIECES; ++u) {
    const int e = threadIdx.x + 256 * u, j = e / PPC, pc = e % PPC;
    *reinterpret_cast<gdsw_u4*>(Bs + j * BL_PAD + 8 * pc) = R.b[u];
  }
}

template <int G>
__global__ __launch_bounds__(256) void gemm_part_bf16_lds_kernel(const uint16_t* __restrict__ store,
                                                                 const int64_t* __restrict__ OFF,
                                                                 const int32_t* __restrict__ N,
                                                                 const int32_t* __restrict__ NP,
                                                                 const int64_t* __restrict__ XPOFF,
                                                                 const int4* __restrict__ items,
                                                                 const uint16_t* __restrict__ xb, int cw,
                                                                 float* __restrict__ partial) {
  __shared__ __attribute__((aligned(16))) uint16_t As[BL_RB * BL_PAD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[32 * BL_PAD];
  const int4 item = items[blockIdx.x];
  const int f = item.x, r0 = item.y, c0 = item.z, p = item.w;
  const int n = N[f];
  const int64_t np = NP[f];
  const int cend = min(c0 + cw, n);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const uint16_t* A = store + OFF[f];
  const uint16_t* X = xb + XPOFF[f] * 32;
  const int nstep = (cend - c0 + BL_SB - 1) / BL_SB;
  const int clast = c0 + (nstep - 1) * BL_SB;
  mf_f4 acc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) acc[g] = mf_f4{0, 0, 0, 0};
  auto products = [&]() {
    const uint16_t* arow = As + (16 * wave + i) * BL_PAD + 8 * kq;
#pragma unroll
    for (int t = 0; t < BL_SB / 32; ++t) {
      const mf_bf8 a = *reinterpret_cast<const mf_bf8*>(arow + 32 * t);
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const mf_bf8 b = *reinterpret_cast<const mf_bf8*>(Bs + (16 * g + i) * BL_PAD + 8 * kq + 32 * t);
        acc[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[g], 0, 0, 0);
      }
    }
  };
  BlRegs R;
  bl_load(R, A, X, r0, n, np, c0);
  for (int c = c0; c < cend; c += BL_SB) {
    __syncthreads();  // the previous step's products are done with LDS
    bl_store(R, As, Bs);
    __syncthreads();
    bl_load(R, A, X, r0, n, np, min(c + BL_SB, clast));  // next step (the last one reloads, unused)
    products();
  }
  float* out = partial + (int64_t)p * BL_RB * 32;
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int t = 0; t < 4; ++t) out[(int64_t)(16 * wave + 4 * kq + t) * 32 + g * 16 + i] = acc[g][t];
}

// FP64 storage, tiles staged through LDS.  Item (f, r0, c0, p): 128 output
// rows and GEMM_CW summation columns.  Each step stages 32 columns of those
// rows (1 KB contiguous per column, read by 64 consecutive lanes) and the
// 32 x 32 right-hand-side block of the same columns; wave w then runs the
// MFMAs of rows 32 w .. 32 w + 31 (two 16-row tiles) from LDS.  The next
// step's loads are issued before the current step's products.  Rows past np
// read a clamped row (outputs never used); columns past the chunk get zero
// right-hand sides; right-hand sides past nrhs read a clamped one (outputs
// never used).
constexpr int DL_RB = 128, DL_SK = 32, DL_APAD = DL_RB + 4, DL_BPAD = 32 + 1;
constexpr int DL_APIECES = DL_SK * DL_RB / 2 / 256;  // 16-byte pieces per thread per step
constexpr int DL_BVALS = DL_SK * 32 / 256;           // right-hand-side values per thread per step
static_assert(256 % DL_SK == 0, "FP64 LDS step shape: chunks are multiples of 256");

struct DlRegs {
  mf_d2 a[DL_APIECES];
  double b[DL_BVALS];
};

__device__ inline void dl_load(DlRegs& R, const double* __restrict__ A, const double* __restrict__ x, int64_t ldk,
                               int nrhs, int r0, int64_t np, int c, int cend) {
#pragma unroll
  for (int u = 0; u < DL_APIECES; ++u) {
    const int e = threadIdx.x + 256 * u, col = e / (DL_RB / 2), pc = e % (DL_RB / 2);
    const int64_t row = min<int64_t>(r0 + 2 * pc, np - 2);
    R.a[u] = __builtin_nontemporal_load(reinterpret_cast<const mf_d2*>(A + (int64_t)(c + col) * np + row));
  }
#pragma unroll
  for (int u = 0; u < DL_BVALS; ++u) {
    const int e = threadIdx.x + 256 * u, kk = e / 32, j = e % 32;
    const double v = x[(int64_t)(c + kk) * ldk + min(j, nrhs - 1)];
    R.b[u] = c + kk < cend ? v : 0.0;
  }
}

__device__ inline void dl_store(const DlRegs& R, double* As, double* Bs) {
#pragma unroll
  for (int u = 0; u < DL_APIECES; ++u) {
    const int e = threadIdx.x + 256 * u, col = e / (DL_RB / 2), pc = e % (DL_RB / 2);
    As[col * DL_APAD + 2 * pc] = R.a[u].x;
    As[col * DL_APAD + 2 * pc + 1] = R.a[u].y;
  }
#pragma unroll
  for (int u = 0; u < DL_BVALS; ++u) {
    const int e = threadIdx.x + 256 * u;
    Bs[(e / 32) * DL_BPAD + e % 32] = R.b[u];
  }
}

template <int G>
__global__ __launch_bounds__(256) void gemm_part_f64_lds_kernel(const double* __restrict__ store,
                                                                const int64_t* __restrict__ OFF,
                                                                const int32_t* __restrict__ N,
                                                                const int32_t* __restrict__ NP,
                                                                const int64_t* __restrict__ XOFF,
                                                                const int4* __restrict__ items,
                                                                const double* __restrict__ w, int64_t ldk, int nrhs,
                                                                int cw, double* __restrict__ partial) {
  __shared__ double As[DL_SK * DL_APAD];
  __shared__ double Bs[DL_SK * DL_BPAD];
  const int4 item = items[blockIdx.x];
  const int f = item.x, r0 = item.y, c0 = item.z, p = item.w;
  const int n = N[f];
  const int64_t np = NP[f];
  const int cend = min(c0 + cw, n);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const double* A = store + OFF[f];
  const double* x = w + XOFF[f] * ldk;
  const int nstep = (cend - c0 + DL_SK - 1) / DL_SK;
  const int clast = c0 + (nstep - 1) * DL_SK;
  mf_d4 acc[2][G];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int g = 0; g < G; ++g) acc[t][g] = mf_d4{0, 0, 0, 0};
  DlRegs R;
  dl_load(R, A, x, ldk, nrhs, r0, np, c0, cend);
  for (int c = c0; c < cend; c += DL_SK) {
    __syncthreads();  // the previous step's products are done with LDS
    dl_store(R, As, Bs);
    __syncthreads();
    const int cn = min(c + DL_SK, clast);  // next step (the last one reloads, unused)
    dl_load(R, A, x, ldk, nrhs, r0, np, cn, cn == c + DL_SK ? cend : cn + DL_SK);
#pragma unroll
    for (int s4 = 0; s4 < DL_SK / 4; ++s4) {
      const int col = 4 * s4 + kq;
      double a[2], b[G];
#pragma unroll
      for (int t = 0; t < 2; ++t) a[t] = As[col * DL_APAD + 32 * wave + 16 * t + i];
#pragma unroll
      for (int g = 0; g < G; ++g) b[g] = Bs[col * DL_BPAD + 16 * g + i];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int g = 0; g < G; ++g) acc[t][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[g], acc[t][g], 0, 0, 0);
    }
  }
  // accumulator register q of a lane holds output row kq + 4 q of its tile
  double* out = partial + (int64_t)p * DL_RB * 32;
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        out[(int64_t)(32 * wave + 16 * t + kq + 4 * q) * 32 + 16 * g + i] = acc[t][g][q];
}

// Item (f, r0, p0, cnt): w[(XOFF + r0 + t) * ldk + j] = sum_q partial[((p0 + q) * RB + t) * 32 + j].
template <typename P, int RB>
__global__ __launch_bounds__(256) void gemm_sum_kernel(const int32_t* __restrict__ N, const int64_t* __restrict__ XOFF,
                                                       const int4* __restrict__ items, const P* __restrict__ partial,
                                                       double* __restrict__ w, int64_t ldk, int nrhs) {
  const int4 item = items[blockIdx.x];
  const int f = item.x, r0 = item.y, p0 = item.z, cnt = item.w;
  const int n = N[f];
  const int rows = min(RB, n - r0);
  for (int e = threadIdx.x; e < rows * nrhs; e += 256) {
    const int t = e / nrhs, j = e % nrhs;
    double s = 0.0;
    for (int q = 0; q < cnt; ++q) s += (double)partial[((int64_t)(p0 + q) * RB + t) * 32 + j];
    w[(XOFF[f] + r0 + t) * ldk + j] = s;
  }
}

template <typename T>
void gemm_launch(const FactorSet& fs, double* w, int64_t ldk, int nrhs, hipStream_t st) {
  using S = MultiShape<T>;
  using P = typename S::P;
  const FactorSet::GemvPlan& G = fs.gemm;
  if (G.n1 == 0) return;
  P* part = static_cast<P*>(fs.d_partial_m);
  for (int j0 = 0; j0 < nrhs; j0 += 32) {
    const int nr = std::min(32, nrhs - j0);
    double* wj = w + j0;
    KernelTimer* tm = (fs.timer && fs.timer->on && fs.timer->used < KernelTimer::CAP) ? fs.timer : nullptr;
    const int cw = fs.gemm_cw;
    if constexpr (sizeof(T) == 2)
      stage_bf16_kernel<<<dim3((fs.max_np + 63) / 64, fs.count), 256, 0, st>>>(fs.d_n, fs.d_npad, fs.d_xoff,
                                                                            fs.d_xpoff, wj, ldk, nr, fs.d_xb);
    const double bytes = (double)fs.alg_bytes;
    if constexpr (sizeof(T) == 2) {
      const uint16_t* store = static_cast<const uint16_t*>(fs.store);
      timed_launch(tm, bytes, nr > 16 ? gemm_part_bf16_lds_kernel<2> : gemm_part_bf16_lds_kernel<1>, dim3(G.n1),
                   dim3(256), st, store, fs.d_off, fs.d_n, fs.d_npad, fs.d_xpoff, G.d_items1, fs.d_xb, cw, part);
    } else if (sizeof(T) == 8 && fs.gemm_lds) {
      const double* store = reinterpret_cast<const double*>(fs.store);
      double* pd = reinterpret_cast<double*>(part);
      timed_launch(tm, bytes, nr > 16 ? gemm_part_f64_lds_kernel<2> : gemm_part_f64_lds_kernel<1>, dim3(G.n1),
                   dim3(256), st, store, fs.d_off, fs.d_n, fs.d_npad, fs.d_xoff, G.d_items1, wj, ldk, nr, cw, pd);
    } else {
      timed_launch(tm, bytes, nr > 16 ? gemm_part_kernel<T, 2> : gemm_part_kernel<T, 1>, dim3(G.n1), dim3(256), st,
                   static_cast<const T*>(fs.store), fs.d_off, fs.d_n, fs.d_npad, fs.d_xoff, G.d_items1, wj, ldk, nr,
                   cw, part);
    }
    if (sizeof(T) == 8 && fs.gemm_lds)
      gemm_sum_kernel<P, DL_RB><<<G.n2, 256, 0, st>>>(fs.d_n, fs.d_xoff, G.d_items2, part, wj, ldk, nr);
    else
      gemm_sum_kernel<P, S::RB><<<G.n2, 256, 0, st>>>(fs.d_n, fs.d_xoff, G.d_items2, part, wj, ldk, nr);
  }
}

}  // namespace

void gemm_choose(FactorSet& fs) {
  // items of a shape: sum over matrices of row blocks x column chunks
  auto items = [&](int rb, int cw) {
    int64_t t = 0;
    for (int f = 0; f < fs.count; ++f) t += (int64_t)((fs.n[f] + rb - 1) / rb) * ((fs.n[f] + cw - 1) / cw);
    return t;
  };
  fs.gemm_lds = false;
  fs.gemm_cw = GEMM_CW;
  if (fs.prec == P_FP32) {
    fs.gemm_rb = MultiShape<float>::RB;
  } else if (fs.prec == P_BF16) {
    fs.gemm_rb = MultiShape<uint16_t>::RB;
  } else if (fs.gemm_lds_force == 0 || (fs.gemm_lds_force < 0 && items(MultiShape<double>::RB, GEMM_CW) >= 2048)) {
    fs.gemm_rb = MultiShape<double>::RB;  // many matrices: direct fragments, long rows per wave
  } else {
    // few matrices (a coarse level): 128-row LDS tiles and narrower
    // column chunks, so that the launch still fills the device
    fs.gemm_lds = true;
    fs.gemm_rb = DL_RB;
    while (fs.gemm_cw > 256 && items(DL_RB, fs.gemm_cw) < 2048) fs.gemm_cw /= 2;
  }
  if (fs.gemm_cw_force > 0) fs.gemm_cw = fs.gemm_cw_force;
}

void gemm_set(const FactorSet& fs, double* w, int64_t ldk, int nrhs, hipStream_t st) {
  if (fs.count == 0 || nrhs == 0) return;
  if (fs.prec == P_FP64)
    gemm_launch<double>(fs, w, ldk, nrhs, st);
  else if (fs.prec == P_FP32)
    gemm_launch<float>(fs, w, ldk, nrhs, st);
  else
    gemm_launch<uint16_t>(fs, w, ldk, nrhs, st);
  GDSW_HIP(hipGetLastError());
}

}  // namespace gdsw
