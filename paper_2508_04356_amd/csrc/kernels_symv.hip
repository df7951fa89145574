// x_f <- M_f x_f for symmetric explicit inverses stored as the upper
// triangle of 64 x 64 tiles: the inverse of a symmetric local (or coarse)
// saddle-point matrix of eq. (2.1) is symmetric, so only the tiles (I, J)
// with J >= I are kept (each tile column-major and contiguous), which halves
// the bytes of the HBM-bound product.  A stored tile with J > I contributes
// M_IJ x_J to block row I and M_IJ^T x_I to block row J; a diagonal tile,
// stored as its upper triangle U with half the diagonal, contributes
// U x_I + U^T x_I = M_II x_I.  Pieces that hold no needed entry are not read
// (rows or columns past n in the last tile row and column, the part of a
// diagonal tile below the diagonal): the tiles fetched are the upper
// triangle, not the padded square.  A work-group reads a run of one or two
// tiles of one block row (each a contiguous 32 KB read for FP64; two by
// default, gdsw_autotune may pick one) and writes one row partial for the
// run (block row I) and one column partial per off-diagonal tile (block rows
// J); a second launch sums them per block row in a fixed order (the runs of
// row I from the diagonal on, then the transposed tiles (0, I), (1, I), ...),
// so results are repeatable bit for bit.  Tried and measured slower at 16^3
// on MI355X: runs of 3 or 4 tiles (also in FP32 and BF16), staging tiles in
// LDS, a gap between stored tiles (off the 32 KB stride), and fewer resident
// work-groups that each walk many items.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "vec16.h"

namespace gdsw {
namespace {

constexpr int ST = 64;        // tile edge

__host__ __device__ inline int64_t tile_index(int I, int J, int nt) {
  return (int64_t)I * nt - (int64_t)I * (I - 1) / 2 + (J - I);
}

// Item (f, I, J0, p0): tiles (I, J0 .. J0 + SYMV_RUN - 1) (those with
// J < nt, contiguous in the store) of matrix f, partial slots p0 + J - J0.
// Thread t loads 16-byte pieces of E consecutive rows: rows r0 = E (t % PPC)
// .. r0 + E - 1 of columns t / PPC + CPT u (PPC pieces per column, CPT
// columns per 256 pieces), so a tile is read once, contiguously, straight
// into registers, the next tile's pieces in flight while the current one is
// multiplied.  The thread's share of the row product (E rows over its
// columns) and of the column product (its columns over E rows) go through
// small LDS reductions in a fixed order.  Rows and columns past n meet zero
// vector entries (the padded inverse is block-diagonal, so those tile
// entries only feed outputs that are never read).
#ifndef GDSW_SYMV_NT
#define GDSW_SYMV_NT 1  // non-temporal tile loads
#endif
#ifndef GDSW_SYMV_KB
// vectors reduced per barrier round when a tile serves several: one per
// round measured 61.4 us against 67.1 us for all three at once (16^3, the
// velocity-block inverses, MI355X; the larger LDS footprint halves occupancy)
#define GDSW_SYMV_KB 1
#endif

template <typename T, typename A>
__device__ inline void tile_load16(__amdgpu_buffer_rsrc_t r, uint32_t off, A (&o)[VecW<T>::W]) {
  if constexpr (sizeof(T) == 2)
    buf_load16_bf16<GDSW_SYMV_NT != 0>(r, off, o);
  else
    buf_load16<GDSW_SYMV_NT != 0>(r, off, o);
}

// NC > 1: the tile is applied to NC vectors (x + k vs, k < NC) while it sits
// in registers; the partial slots hold NC blocks of 64 per item slot.
template <typename T, int NC, int SYMV_RUN>
__global__ __launch_bounds__(256) void symv_part_kernel(const GemvDesc* __restrict__ desc,
                                                        const int4* __restrict__ items, double* __restrict__ prow,
                                                        double* __restrict__ pcol, const int32_t* __restrict__ want,
                                                        int xcd) {
  using Acc = typename VecW<T>::acc;
  constexpr int E = VecW<T>::W;        // rows per 16-byte piece
  constexpr int PPC = ST / E;          // pieces per column
  constexpr int CPT = 256 / PPC;       // columns covered by one piece per thread
  constexpr int PER = ST / CPT;        // pieces per thread
  __shared__ Acc xi[NC][ST], xj[NC][SYMV_RUN][ST];  // the vector blocks of row I and of every tile of the run
  // the NC vectors are reduced KB at a time (one pair of barriers per round)
  constexpr int KB = GDSW_SYMV_KB < NC ? GDSW_SYMV_KB : NC;
  static_assert(NC % KB == 0, "rounds of equal size");
  __shared__ Acc rred[KB][CPT][ST];    // row partials per column group
  __shared__ Acc cred[KB][ST][PPC + 1];  // column partials per row group
  // work-groups are dealt to the 8 XCDs in turn; with xcd set XCD x takes
  // the x-th contiguous eighth of the items instead (a permutation of the
  // grid: 1032 -> 999 us for FP32 tiles at 24^3 on MI355X, while FP64 lost
  // 1.5% and BF16 did not change; the default is on for FP32 only)
  int it = blockIdx.x;
  if (xcd) {
    const int nb = gridDim.x, x8 = blockIdx.x % 8, q8 = blockIdx.x / 8, per = nb / 8, rem = nb % 8;
    it = (x8 < rem ? x8 * (per + 1) : rem * (per + 1) + (x8 - rem) * per) + q8;
  }
  const int4 item = items[it];
  const int g = item.x, I = item.y, J0 = item.z, p0 = item.w;
  if (want && !want[g]) return;  // uniform: a matrix left out of this launch
  const GemvDesc d = desc[g];
  const int n = d.n;
  const int nt = d.np / ST;
  const int J1 = min(nt, J0 + SYMV_RUN);
  const T* tiles = static_cast<const T*>(d.a) + tile_index(I, J0, nt) * (ST * ST);
  const double* x = d.x;
  const int t = threadIdx.x;
  const int rg = t % PPC, cg = t / PPC, r0 = E * rg;
  // the vector entries first (every thread loads, clamped to the np entries
  // the work vector holds for this matrix, so that no load sits in a
  // branch), then the first tile; they reach LDS only once the next tile's
  // loads are issued too
  static_assert(SYMV_RUN * ST <= 256, "one vector entry per thread");
  const auto* xg = as_global<double>(x);
  const int ri = ST * I + (t % ST), rj = ST * J0 + (t % (SYMV_RUN * ST));
  double xiv[NC], xjv[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    xiv[k] = xg[(int64_t)k * d.vs + min(ri, d.np - 1)];
    xjv[k] = xg[(int64_t)k * d.vs + min(rj, d.np - 1)];
  }
  Acc v[PER][E], vn[PER][E];
  // piece u of tile J holds a needed entry: inside n x n, and for a
  // diagonal tile on or above the diagonal (the packed zeros below it are
  // not read)
  auto need = [&](int J, int u) {
    const int c = cg + CPT * u;
    return ST * J + c < n && ST * I + r0 < n && (J > I || r0 <= c);
  };
  // the run's tiles as one buffer resource: a piece that is not needed gets
  // an offset past its end and reads as zero without a memory access
  const __amdgpu_buffer_rsrc_t rs = buf_rsrc(tiles, (uint32_t)((J1 - J0) * ST * ST * sizeof(T)));
  auto load_piece = [&](int J, int u, Acc (&o)[E]) {
    const uint32_t off = need(J, u) ? (uint32_t)(((J - J0) * ST * ST + (t + 256 * u) * E) * sizeof(T)) : BUF_SKIP;
    tile_load16<T>(rs, off, o);
  };
#pragma unroll
  for (int u = 0; u < PER; ++u) load_piece(J0, u, v[u]);
  auto store_x = [&]() {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      if (t < ST) xi[k][t] = ri < n ? (Acc)xiv[k] : (Acc)0;
      if (t < SYMV_RUN * ST) xj[k][t / ST][t % ST] = rj < n ? (Acc)xjv[k] : (Acc)0;
    }
  };
  // products of tile J held in v: row part into rred, transposed part into
  // cred, one vector at a time; the row parts of the run's tiles all belong
  // to block row I and are summed here (in tile order), written once, to the
  // run's first slot
  double racc[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) racc[k] = 0.0;
  auto products = [&](int J) {
    const int b = J - J0;
#pragma unroll
    for (int k0 = 0; k0 < NC; k0 += KB) {
      __syncthreads();  // xi / xj written; the previous round's reductions read
#pragma unroll
      for (int kk = 0; kk < KB; ++kk) {
        const int k = k0 + kk;
        Acc rs[E];
#pragma unroll
        for (int e = 0; e < E; ++e) rs[e] = 0;
#pragma unroll
        for (int u = 0; u < PER; ++u) {  // block row I: rows r0 .. r0 + E - 1 over columns cg + CPT u
          const Acc xc = xj[k][b][cg + CPT * u];
#pragma unroll
          for (int e = 0; e < E; ++e) rs[e] = fma(v[u][e], xc, rs[e]);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) rred[kk][cg][r0 + e] = rs[e];
        // block row J gets the transposed tile (for the diagonal tile, row I)
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          Acc cs = 0;
#pragma unroll
          for (int e = 0; e < E; ++e) cs = fma(v[u][e], xi[k][r0 + e], cs);
          cred[kk][cg + CPT * u][rg] = cs;
        }
      }
      __syncthreads();
      // 2 KB sums of 64 entries (row sums of each vector of the round, then
      // column sums), dealt to the four waves: wave q takes sums q, q + 4, ...
      const int p = p0 + b;
      const int l = t % ST, wq = t / ST;
#pragma unroll
      for (int it = 0; it < 2 * KB; ++it) {
        if (it % 4 != wq) continue;  // uniform per wave
        if (it < KB) {
          const int k = k0 + it;
          double sr = 0.0;
#pragma unroll
          for (int g = 0; g < CPT; ++g) sr += (double)rred[it][g][l];
          if (J == I) {  // uniform: the diagonal tile's transposed part belongs to row I too
            double sc = 0.0;
#pragma unroll
            for (int g = 0; g < PPC; ++g) sc += (double)cred[it][l][g];
            sr += sc;
          }
          racc[k] += sr;
          if (J == J1 - 1) prow[((int64_t)p0 * NC + k) * ST + l] = racc[k];
        } else if (J > I) {
          const int k = k0 + it - KB;
          double sc = 0.0;
#pragma unroll
          for (int g = 0; g < PPC; ++g) sc += (double)cred[it - KB][l][g];
          pcol[((int64_t)p * NC + k) * ST + l] = sc;
        }
      }
    }
  };
  for (int J = J0; J + 1 < J1; ++J) {
    // the next tile's pieces, issued before this tile's products (unconditional
    // inside the loop, so that they stay in flight meanwhile)
#pragma unroll
    for (int u = 0; u < PER; ++u) load_piece(J + 1, u, vn[u]);
    if (J == J0) store_x();
    products(J);
#pragma unroll
    for (int u = 0; u < PER; ++u)
#pragma unroll
      for (int e = 0; e < E; ++e) v[u][e] = vn[u][e];
  }
  if (J1 - 1 == J0) store_x();
  products(J1 - 1);
}

// Item (g, I, P0, nt): x_g[64 I + l] = sum over the runs of block row I of
// their row partial + sum_{K < I} pcol(K, I)[l] (with a descriptor output y:
// y_g[64 I + l] -= that sum instead).  The terms, in the order (runs of row I
// from the diagonal on, then K = 0 .. I - 1), are dealt to the four waves in
// turn; each wave sums its terms in order and the four sums are added in
// wave order, so the result is repeatable bit for bit.  All NC vectors are
// summed in the same pass (their loads in flight together).
template <int NC>
__global__ __launch_bounds__(256) void symv_sum_kernel(const GemvDesc* __restrict__ desc,
                                                       const int4* __restrict__ items,
                                                       const double* __restrict__ prow,
                                                       const double* __restrict__ pcol, const int32_t* __restrict__ want,
                                                       int run) {
  static_assert(NC <= 4, "one wave per vector for the last step");
  __shared__ double red[4][NC][ST];
  const int4 item = items[blockIdx.x];
  const int g = item.x, I = item.y, P0 = item.z, nt = item.w;
  if (want && !want[g]) return;  // uniform over the work-group
  const int l = threadIdx.x % ST, w = threadIdx.x / ST;
  const int na = (nt - I + run - 1) / run;  // runs of row I
  double s[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) s[k] = 0.0;
  for (int q = w; q < na + I; q += 4) {
    const int64_t slot = q < na ? P0 + tile_index(I, I + run * q, nt) : P0 + tile_index(q - na, I, nt);
    const double* src = (q < na ? prow : pcol) + slot * NC * ST + l;
#pragma unroll
    for (int k = 0; k < NC; ++k) s[k] += src[k * ST];
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) red[w][k][l] = s[k];
  __syncthreads();
  if (w < NC) {  // wave k finishes vector k
    const double x = ((red[0][w][l] + red[1][w][l]) + red[2][w][l]) + red[3][w][l];
    const GemvDesc& d = desc[g];
    const int r = ST * I + l;
    if (r < d.n) {
      const int64_t e = (int64_t)w * d.vs + r;
      if (d.y)
        d.y[e] -= x;
      else
        d.x[e] = x;
    }
  }
}

// Upper tiles of npad x npad column-major FP64 matrices, converted to the
// storage type: block (tile t of matrix k) copies one 64 x 64 tile.  A
// diagonal tile keeps its strict upper triangle, half its diagonal and zeros
// below, so that its row and column products together give M_II x_I.
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
    double v = s[(int64_t)c * np + r];
    if (I == J) v = r < c ? v : r == c ? 0.5 * v : 0.0;  // U with U + U^T = M_II (halving is exact)
    if constexpr (sizeof(T) == 2)
      d[e] = to_bf16((float)v);
    else
      d[e] = (T)v;
  }
}

template <typename T, int NC>
void symv_launch(const GemvDesc* desc, const FactorSet::GemvPlan& G, double* partial, int64_t partial_len,
                 hipStream_t st, const int32_t* want, KernelTimer* tm, double bytes) {
  if (G.n1 == 0) return;
  double* prow = partial;
  double* pcol = partial + partial_len / 2;
  if (G.run == 1)
    timed_launch(tm, bytes, symv_part_kernel<T, NC, 1>, dim3(G.n1), dim3(256), st, desc, G.d_items1, prow, pcol,
                 want, G.xcd);
  else
    timed_launch(tm, bytes, symv_part_kernel<T, NC, 2>, dim3(G.n1), dim3(256), st, desc, G.d_items1, prow, pcol,
                 want, G.xcd);
  symv_sum_kernel<NC><<<G.n2, 256, 0, st>>>(desc, G.d_items2, prow, pcol, want, G.run);
}

}  // namespace

int64_t symv_tiles(int npad) {
  const int64_t nt = npad / ST;
  return nt * (nt + 1) / 2;
}

void symv_items(int f, int npad, int64_t p0, int run, std::vector<int4>& it1, std::vector<int4>& it2) {
  if (run != 1 && run != 2) throw StatusError{1, "symmetric tile runs of 1 or 2 tiles"};
  const int nt = npad / ST;
  for (int I = 0; I < nt; ++I) {
    for (int J = I; J < nt; J += run) it1.push_back(make_int4(f, I, J, (int)(p0 + tile_index(I, J, nt))));
    it2.push_back(make_int4(f, I, (int)p0, nt));
  }
}

int symv_default_xcd(int prec) { return prec == P_FP32 ? 1 : 0; }

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

void symv_desc_launch(int prec, const GemvDesc* desc, const FactorSet::GemvPlan& G, double* partial,
                      int64_t partial_len, hipStream_t st, const int32_t* want, KernelTimer* tm, double bytes,
                      int nc) {
  if (tm && (!tm->on || tm->used >= KernelTimer::CAP)) tm = nullptr;
  if (nc != 1 && nc != 3) throw StatusError{1, "symmetric products take 1 or 3 vectors"};
  if (nc == 3) {
    if (prec == P_FP64)
      symv_launch<double, 3>(desc, G, partial, partial_len, st, want, tm, bytes);
    else if (prec == P_FP32)
      symv_launch<float, 3>(desc, G, partial, partial_len, st, want, tm, bytes);
    else
      symv_launch<uint16_t, 3>(desc, G, partial, partial_len, st, want, tm, bytes);
  } else if (prec == P_FP64) {
    symv_launch<double, 1>(desc, G, partial, partial_len, st, want, tm, bytes);
  } else if (prec == P_FP32) {
    symv_launch<float, 1>(desc, G, partial, partial_len, st, want, tm, bytes);
  } else {
    symv_launch<uint16_t, 1>(desc, G, partial, partial_len, st, want, tm, bytes);
  }
  GDSW_HIP(hipGetLastError());
}

void symv_set(const FactorSet& fs, double* w, hipStream_t st, int slot, const int32_t* want) {
  (void)w;  // the descriptors address the set's own work vector segments
  if (fs.count == 0 || slot >= (int)fs.gemv.size()) return;
  if (!fs.d_desc) throw StatusError{5, "symmetric set used before its descriptors were built"};
  symv_desc_launch(fs.prec, fs.d_desc, fs.gemv[slot], fs.d_partial, fs.partial_len, st, want,
                   slot == 0 ? fs.timer : nullptr, (double)fs.alg_bytes, fs.nc);
}

}  // namespace gdsw
