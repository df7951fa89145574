// Numeric setup on the device: local matrices and their LU factors, the
// coarse basis Phi (eq. 2.4), A_0 = Phi^T A Phi (eq. 2.3) and its factors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <numeric>
#include <stdexcept>
#include <string>
#include <thread>

#include "context.h"
#include "kernels.h"
#include "kernels_multi.h"
#include "kernels_ops.h"

namespace gdsw {

void* DeviceArena::alloc(uint64_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~uint64_t(255);
  if (budget && used + bytes > budget)
    throw StatusError{2, "device memory budget exceeded: need " + std::to_string(used + bytes) + " bytes, budget " +
                             std::to_string(budget)};
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw StatusError{2, "hipMalloc of " + std::to_string(bytes) + " bytes failed (" + hipGetErrorString(e) + ")"};
  }
  used += bytes;
  ptrs.push_back(p);
  sizes.push_back(bytes);
  return p;
}

void DeviceArena::free(void* p) {
  for (size_t k = 0; k < ptrs.size(); ++k)
    if (ptrs[k] == p) {
      (void)hipFree(p);
      used -= sizes[k];
      ptrs.erase(ptrs.begin() + k);
      sizes.erase(sizes.begin() + k);
      return;
    }
}

void DeviceArena::release_all() {
  for (void* p : ptrs) (void)hipFree(p);
  ptrs.clear();
  sizes.clear();
  used = 0;
}


uint64_t FactorSet::algorithmic_bytes() const {
  uint64_t b = 0;
  for (int f = 0; f < count; ++f)
    b += (mode == SOLVE_SYM ? (uint64_t)n[f] * (n[f] + 1) / 2 : (uint64_t)n[f] * n[f]) * elem_size(prec);
  return b;
}

std::vector<GemvDesc> gemv_descs(const FactorSet& fs, double* w) {
  std::vector<GemvDesc> d(fs.count);
  const size_t es = elem_size(fs.prec);
  for (int f = 0; f < fs.count; ++f)
    d[f] = GemvDesc{static_cast<const char*>(fs.store) + (size_t)fs.off[f] * es, w + fs.xoff[f], fs.n[f], fs.npad[f]};
  return d;
}

int64_t FactorSet::launches() const {
  if (count == 0) return 0;
  if (mode == SOLVE_INVERSE || mode == SOLVE_SYM) return gemv.empty() || gemv[0].n1 == 0 ? 0 : 2;
  int64_t l = 0;
  if (!sched.empty())
    for (size_t k = 0; k + 1 < sched[0].step_start.size(); ++k) l += sched[0].step_start[k + 1] > sched[0].step_start[k];
  return l;
}

namespace {

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

}  // namespace

// Launch schedule with `phases` groups of factors whose sweeps start
// ceil(max_nblk / phases) launches apart.  Local step l of a factor with nblk
// tiles: 0 = forward start (x_J = L_JJ^-1 x_J for all J); 1 .. nblk-1 =
// forward updates with block s = l-1 (J > s); nblk = backward start
// (x_J = U_JJ^-1 x_J); nblk+1 .. 2 nblk-1 = backward updates with block
// s = 2 nblk - l (J < s), i.e. s = nblk-1 down to 1.
namespace {

// Work items of the explicit-inverse product for the factors selected by
// `include`: partial items in (factor, column chunk, row block) order, so
// that consecutive work-groups stream consecutive rows of the same columns;
// partial index p in (factor, row block, column chunk) order, so that the
// partials of one row block are contiguous for the summation kernel.
void plan_gemv(FactorSet& fs, DeviceArena& A, hipStream_t st, int slot, const std::vector<char>* include) {
  const int RB = gemv_rows(fs.prec);
  const int CW = fs.cw;
  std::vector<int4> it1, it2;
  int p = 0;
  for (int f = 0; f < fs.count; ++f) {
    if (include && !(*include)[f]) continue;
    const int n = fs.n[f];
    const int nr = (n + RB - 1) / RB, nc = (n + CW - 1) / CW;
    for (int c = 0; c < nc; ++c)
      for (int J = 0; J < nr; ++J) it1.push_back(make_int4(f, J * RB, c * CW, p + J * nc + c));
    for (int J = 0; J < nr; ++J) it2.push_back(make_int4(f, J * RB, p + J * nc, nc));
    p += nr * nc;
  }
  if ((int)fs.gemv.size() <= slot) fs.gemv.resize(slot + 1);
  FactorSet::GemvPlan& G = fs.gemv[slot];
  if (G.d_items1) A.free(G.d_items1);
  if (G.d_items2) A.free(G.d_items2);
  G.n1 = (int)it1.size();
  G.n2 = (int)it2.size();
  G.d_items1 = it1.empty() ? nullptr : dupload(A, it1, st);
  G.d_items2 = it2.empty() ? nullptr : dupload(A, it2, st);
  const int64_t need = (int64_t)p * RB;
  if (need > fs.partial_len) {
    if (fs.d_partial) A.free(fs.d_partial);
    fs.d_partial = dalloc<double>(A, need);
    fs.partial_len = need;
  }
}

}  // namespace

void plan_gemm(FactorSet& fs, DeviceArena& A, hipStream_t st) {
  if (fs.mode != SOLVE_INVERSE || fs.count == 0) return;
  ++fs.gen;
  gemm_choose(fs);
  const int RB = fs.gemm_rb, CW = fs.gemm_cw;
  std::vector<int4> it1, it2;
  int p = 0;
  for (int f = 0; f < fs.count; ++f) {
    const int n = fs.n[f];
    const int nr = (n + RB - 1) / RB, nc = (n + CW - 1) / CW;
    for (int c = 0; c < nc; ++c)
      for (int J = 0; J < nr; ++J) it1.push_back(make_int4(f, J * RB, c * CW, p + J * nc + c));
    for (int J = 0; J < nr; ++J) it2.push_back(make_int4(f, J * RB, p + J * nc, nc));
    p += nr * nc;
  }
  FactorSet::GemvPlan& G = fs.gemm;
  if (G.d_items1) A.free(G.d_items1);
  if (G.d_items2) A.free(G.d_items2);
  if (fs.d_partial_m) A.free(fs.d_partial_m);
  G.n1 = (int)it1.size();
  G.n2 = (int)it2.size();
  G.d_items1 = it1.empty() ? nullptr : dupload(A, it1, st);
  G.d_items2 = it2.empty() ? nullptr : dupload(A, it2, st);
  const size_t psz = fs.prec == P_FP64 ? 8 : 4;
  fs.d_partial_m = A.alloc((uint64_t)std::max(p, 1) * RB * 32 * psz);
  // BF16 products read their right-hand sides as BF16, right-hand side by
  // right-hand side per matrix (32 * sum of padded sizes entries)
  if (fs.prec == P_BF16 && !fs.d_xb) {
    std::vector<int64_t> xp(fs.count + 1, 0);
    fs.max_np = 0;
    for (int f = 0; f < fs.count; ++f) {
      xp[f + 1] = xp[f] + fs.npad[f];
      fs.max_np = std::max(fs.max_np, fs.npad[f]);
    }
    fs.d_xpoff = dupload(A, xp, st);
    fs.d_xb = static_cast<uint16_t*>(A.alloc((uint64_t)std::max<int64_t>(xp.back(), 1) * 32 * sizeof(uint16_t)));
  }
}

void plan_schedule(FactorSet& fs, int phases, DeviceArena& A, hipStream_t st, int slot,
                   const std::vector<char>* include) {
  ++fs.gen;  // captured graphs that hold the old item arrays must be re-captured
  if (fs.mode == SOLVE_INVERSE) {
    plan_gemv(fs, A, st, slot, include);
    return;
  }
  if (fs.mode == SOLVE_SYM) {
    // slots (learned solve) cover subsets of the matrices; partial slots
    // stay the global tile indices
    std::vector<int4> it1, it2;
    for (int f = 0; f < fs.count; ++f)
      if (!include || (*include)[f]) symv_items(f, fs.npad[f], fs.off[f] / (64 * 64), fs.sym_run, it1, it2);
    if ((int)fs.gemv.size() <= slot) fs.gemv.resize(slot + 1);
    FactorSet::GemvPlan& G = fs.gemv[slot];
    G.run = fs.sym_run;
    G.xcd = fs.sym_xcd >= 0 ? fs.sym_xcd : symv_default_xcd(fs.prec);
    if (G.d_items1) A.free(G.d_items1);
    if (G.d_items2) A.free(G.d_items2);
    G.n1 = (int)it1.size();
    G.n2 = (int)it2.size();
    G.d_items1 = it1.empty() ? nullptr : dupload(A, it1, st);
    G.d_items2 = it2.empty() ? nullptr : dupload(A, it2, st);
    const int64_t need = 2 * fs.nc * (fs.total_elems / 64);  // 64 row and 64 column partials per tile and vector
    if (need > fs.partial_len) {
      if (fs.d_partial) A.free(fs.d_partial);
      fs.d_partial = dalloc<double>(A, std::max<int64_t>(need, 2));
      fs.partial_len = std::max<int64_t>(need, 2);
    }
    return;
  }
  phases = std::max(1, std::min(phases, std::max(1, fs.count)));
  if (slot == 0) fs.phases = phases;
  const int P = (fs.max_nblk + phases - 1) / phases;
  std::vector<int> o(fs.count);
  int total = 0;
  for (int f = 0; f < fs.count; ++f) {
    o[f] = (f % phases) * P;
    total = std::max(total, o[f] + 2 * fs.nblk[f]);
  }
  if ((int)fs.sched.size() <= slot) fs.sched.resize(slot + 1);
  FactorSet::Schedule& S = fs.sched[slot];
  std::vector<int4> items;
  S.step_start.assign(1, 0);
  for (int g = 0; g < total; ++g) {
    for (int f = 0; f < fs.count; ++f) {
      if (include && !(*include)[f]) continue;
      const int nb = fs.nblk[f];
      const int l = g - o[f];
      if (l < 0 || l >= 2 * nb) continue;
      if (l == 0) {
        for (int J = 0; J < nb; ++J) items.push_back(make_int4(f, J, J, 1));
      } else if (l < nb) {
        const int s = l - 1;
        for (int J = s + 1; J < nb; ++J) items.push_back(make_int4(f, J, s, 0));
      } else if (l == nb) {
        for (int J = 0; J < nb; ++J) items.push_back(make_int4(f, J, J, 2));
      } else {
        const int s = 2 * nb - l;
        for (int J = 0; J < s; ++J) items.push_back(make_int4(f, J, s, 0));
      }
    }
    S.step_start.push_back((int32_t)items.size());
  }
  if (S.d_items) A.free(S.d_items);
  S.d_items = dupload(A, items, st);
}

namespace {

// Host metadata of a factor set for the given sizes; device arrays uploaded.
void plan_factor_set(FactorSet& fs, const std::vector<int32_t>& sizes, int prec, int nb, int64_t xbase,
                     int mode, DeviceArena& A, hipStream_t st) {
  fs.mode = mode;
  fs.prec = prec;
  fs.nb = nb;
  fs.count = (int)sizes.size();
  fs.n = sizes;
  fs.npad.resize(fs.count);
  fs.nblk.resize(fs.count);
  fs.off.resize(fs.count);
  fs.doff.resize(fs.count);
  fs.xoff.resize(fs.count);
  int64_t o = 0, d = 0, x = xbase;
  fs.max_nblk = 0;
  for (int f = 0; f < fs.count; ++f) {
    const int64_t np = std::max<int64_t>(nb, round_up(sizes[f], nb));
    fs.npad[f] = (int32_t)np;
    fs.nblk[f] = (int32_t)(np / nb);
    fs.off[f] = o;
    fs.doff[f] = d;
    fs.xoff[f] = x;
    o += mode == SOLVE_SYM ? symv_tiles((int)np) * 64 * 64 : np * np;
    if (mode == SOLVE_TRSV) d += (int64_t)fs.nblk[f] * nb * nb;
    x += np;
    fs.max_nblk = std::max(fs.max_nblk, fs.nblk[f]);
  }
  fs.total_elems = o;
  fs.total_dinv = d;
  fs.total_x = x - xbase;
  fs.d_n = dupload(A, fs.n, st);
  fs.d_npad = dupload(A, fs.npad, st);
  fs.d_nblk = dupload(A, fs.nblk, st);
  fs.d_off = dupload(A, fs.off, st);
  fs.d_doff = dupload(A, fs.doff, st);
  fs.d_xoff = dupload(A, fs.xoff, st);
  fs.alg_bytes = fs.algorithmic_bytes();
  plan_schedule(fs, 1, A, st);
}

struct PivotCheck {
  std::vector<std::string> names;
};

void check_pivots(const unsigned long long* d_minpiv, int count, double tol, const std::string& what, hipStream_t st) {
  std::vector<unsigned long long> mp(count);
  GDSW_HIP(hipMemcpyAsync(mp.data(), d_minpiv, count * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  GDSW_HIP(hipStreamSynchronize(st));
  for (int f = 0; f < count; ++f) {
    const double v = minpiv_decode(mp[f]);
    if (!(v > tol) || !std::isfinite(v))
      throw StatusError{3, what + " " + std::to_string(f) + ": pivot " + std::to_string(v) +
                               " below tolerance " + std::to_string(tol)};
  }
}

unsigned long long* minpiv_buffer(DeviceArena& A, int count, hipStream_t st) {
  auto* p = dalloc<unsigned long long>(A, std::max(count, 1));
  std::vector<unsigned long long> init(std::max(count, 1), 0x7fefffffffffffffULL);  // largest finite double
  GDSW_HIP(hipMemcpyAsync(p, init.data(), init.size() * sizeof(unsigned long long), hipMemcpyHostToDevice, st));
  return p;
}

// Factor the matrices of `fs` in chunks: fill (callback writes the FP64
// matrices into a zeroed staging batch laid out like the set), LU, checks,
// diagonal-tile inverses and conversion to the storage precision.
// Offset of matrix f in a factorisation chunk starting at f0: the staging
// buffer holds full npad x npad matrices back to back in every mode.
int64_t staging_offset(const FactorSet& fs, int f0, int f) {
  int64_t o = 0;
  for (int k = f0; k < f; ++k) o += (int64_t)fs.npad[k] * fs.npad[k];
  return o;
}

template <class Fill, class Post>
void factor_set(Context& ctx, FactorSet& fs, uint64_t staging_cap, double pivot_tol, const std::string& what,
                hipStream_t st, Fill&& fill, Post&& post) {
  DeviceArena& A = ctx.arena;
  const size_t es = elem_size(fs.prec);
  fs.store = A.alloc((uint64_t)fs.total_elems * es);
  if (fs.mode == SOLVE_TRSV) fs.dinv = A.alloc((uint64_t)fs.total_dinv * (fs.prec == P_FP64 ? 8 : 4));
  int f0 = 0;
  while (f0 < fs.count) {
    // chunk [f0, f1) within the staging cap
    int f1 = f0;
    uint64_t bytes = 0;
    while (f1 < fs.count) {
      const uint64_t b = (uint64_t)fs.npad[f1] * fs.npad[f1] * 8;
      if (f1 > f0 && bytes + b > staging_cap) break;
      bytes += b;
      ++f1;
    }
    const int cnt = f1 - f0;
    double* staging;
    bool own_staging = fs.prec != P_FP64 || fs.mode == SOLVE_SYM;
    if (own_staging) {
      staging = static_cast<double*>(A.alloc(bytes));
    } else {
      staging = static_cast<double*>(fs.store) + fs.off[f0];
    }
    GDSW_HIP(hipMemsetAsync(staging, 0, bytes, st));
    // chunk-relative descriptors
    FactorSet ch = fs;
    ch.count = cnt;
    ch.n.assign(fs.n.begin() + f0, fs.n.begin() + f1);
    ch.npad.assign(fs.npad.begin() + f0, fs.npad.begin() + f1);
    ch.nblk.assign(fs.nblk.begin() + f0, fs.nblk.begin() + f1);
    std::vector<int64_t> off_rel(cnt), doff(cnt);
    int max_n = 0, max_nblk = 0;
    int64_t orel = 0;  // staging layout: full npad x npad matrices back to back
    for (int k = 0; k < cnt; ++k) {
      off_rel[k] = orel;
      orel += (int64_t)ch.npad[k] * ch.npad[k];
      doff[k] = fs.doff[f0 + k];
      max_n = std::max(max_n, ch.n[k]);
      max_nblk = std::max(max_nblk, ch.nblk[k]);
    }
    ch.max_nblk = max_nblk;
    int32_t* d_n = dupload(A, ch.n, st);
    int32_t* d_np = dupload(A, ch.npad, st);
    int32_t* d_nblk = dupload(A, ch.nblk, st);
    int64_t* d_off = dupload(A, off_rel, st);
    int64_t* d_doff = dupload(A, doff, st);
    DenseBatch B;
    B.base = staging;
    B.n = d_n;
    B.ld = d_np;
    B.off = d_off;
    B.count = cnt;
    B.max_n = max_n;
    fill(B, f0, f1);
    unsigned long long* mp = minpiv_buffer(A, cnt, st);
    if (fs.mode == SOLVE_INVERSE || fs.mode == SOLVE_SYM) {
      int64_t max_np = 0;
      for (int k = 0; k < cnt; ++k) max_np = std::max<int64_t>(max_np, ch.npad[k]);
      const int64_t tstride = 64 * max_np;
      double* Pbuf = dalloc<double>(A, (int64_t)cnt * 64 * 64);
      double* Tbuf = dalloc<double>(A, (int64_t)cnt * tstride);
      gj_invert(B, Pbuf, Tbuf, tstride, mp, st);
      check_pivots(mp, cnt, pivot_tol, what, st);
      symmetrize(B, st);
      post(B, f0, f1);  // the FP64 inverses of the chunk, before they are stored
      if (fs.mode == SOLVE_SYM) {
        // full staging matrices -> upper tiles of the store (chunk-relative offsets)
        std::vector<int64_t> doff_t(cnt);
        for (int k = 0; k < cnt; ++k) doff_t[k] = fs.off[f0 + k] - fs.off[f0];
        int64_t* d_doff_t = dupload(A, doff_t, st);
        pack_upper(fs.prec, staging, d_off, d_np, cnt, (int)max_np, d_doff_t,
                   static_cast<char*>(fs.store) + (size_t)fs.off[f0] * es, st);
        GDSW_HIP(hipStreamSynchronize(st));
        A.free(d_doff_t);
      } else if (fs.prec != P_FP64) {
        convert_store(fs.prec, staging, static_cast<char*>(fs.store) + (size_t)fs.off[f0] * es, (int64_t)(bytes / 8),
                      st);
      }
      GDSW_HIP(hipStreamSynchronize(st));
      A.free(Tbuf);
      A.free(Pbuf);
      A.free(mp);
      A.free(d_n);
      A.free(d_np);
      A.free(d_nblk);
      A.free(d_off);
      A.free(d_doff);
      if (own_staging) A.free(staging);
      f0 = f1;
      continue;
    }
    lu_nopiv(B, mp, st);
    check_pivots(mp, cnt, pivot_tol, what, st);
    // finalize: dinv + conversion on the chunk
    ch.d_n = d_n;
    ch.d_npad = d_np;
    ch.d_nblk = d_nblk;
    ch.d_off = d_off;
    ch.d_doff = d_doff;
    ch.total_elems = (int64_t)(bytes / 8);
    ch.store = static_cast<char*>(fs.store) + (size_t)fs.off[f0] * es;
    ch.dinv = fs.dinv;
    const int64_t dbase = fs.doff[f0];
    ch.total_dinv = (f1 < fs.count ? fs.doff[f1] : fs.total_dinv) - dbase;
    factor_finalize(ch, staging, dbase, st);
    GDSW_HIP(hipStreamSynchronize(st));
    A.free(mp);
    A.free(d_n);
    A.free(d_np);
    A.free(d_nblk);
    A.free(d_off);
    A.free(d_doff);
    if (own_staging) A.free(staging);
    f0 = f1;
  }
}

template <class Fill>
void factor_set(Context& ctx, FactorSet& fs, uint64_t staging_cap, double pivot_tol, const std::string& what,
                hipStream_t st, Fill&& fill) {
  factor_set(ctx, fs, staging_cap, pivot_tol, what, st, fill, [](DenseBatch&, int, int) {});
}

// Block local solve: the velocity block must be I_3 (x) L -- velocity DOFs
// numbered 3 node + component, every velocity row coupling only to its own
// component with the values of the x-component row of the same node.
void block_check(const Problem& P) {
  for (int64_t d = 0; d < P.n_u; ++d)
    if (P.field[d] != d % 3)
      throw StatusError{1, "the block local solve needs velocity DOFs numbered 3 node + component"};
  for (int64_t r = 0; r < P.n_u; r += 3) {
    const int32_t b0 = P.row_ptr[r], e0 = P.row_ptr[r + 1];
    for (int c = 1; c < 3; ++c) {
      const int32_t b = P.row_ptr[r + c], e = P.row_ptr[r + c + 1];
      int32_t i = b0, j = b;
      while (i < e0 && P.col[i] < P.n_u) {
        if (j >= e || P.col[j] != P.col[i] + c || P.val[j] != P.val[i])
          throw StatusError{1, "the block local solve needs a velocity block I_3 (x) L (row " +
                                   std::to_string(r + c) + " differs from row " + std::to_string(r) + ")"};
        ++i;
        ++j;
      }
      if (j < e && P.col[j] < P.n_u)
        throw StatusError{1, "the block local solve needs a velocity block I_3 (x) L"};
    }
    for (int32_t i = b0; i < e0 && P.col[i] < P.n_u; ++i)
      if (P.col[i] % 3 != 0) throw StatusError{1, "the block local solve needs uncoupled velocity components"};
  }
}

// fn(i) for every i in [0, count) on up to 16 host threads (the calling
// thread among them); an exception thrown for an item is rethrown here, that
// of the lowest item first
template <class F>
void parallel_items(int count, F&& fn) {
  const int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::exception_ptr> err(std::max(count, 0));
  std::atomic<int> next{0};
  auto work = [&]() {
    for (int i = next++; i < count; i = next++) {
      try {
        fn(i);
      } catch (...) {
        err[i] = std::current_exception();
      }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < std::min(nt, count); ++t) pool.emplace_back(work);
  work();
  for (auto& th : pool) th.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}

template <class T>
void concat(const std::vector<std::vector<T>>& lists, std::vector<int32_t>& ptr, std::vector<T>& idx) {
  ptr.assign(lists.size() + 1, 0);
  for (size_t i = 0; i < lists.size(); ++i) ptr[i + 1] = ptr[i] + (int32_t)lists[i].size();
  idx.clear();
  idx.reserve(ptr.back());
  for (auto& l : lists) idx.insert(idx.end(), l.begin(), l.end());
}

}  // namespace

void device_setup(Context& ctx, hipStream_t st, uint64_t budget, int nb) {
  Problem& P = ctx.P;
  DeviceArena& A = ctx.arena;
  A.budget = budget;
  ctx.nb = nb;
  const int64_t n = P.n_free;
  const int levels = P.spec.levels;
  ctx.Nc = P.n_coarse;
  const int Nc = ctx.Nc;

  const bool blockm = ctx.solve_mode == SOLVE_BLOCK;
  // block local solve: x-component DOFs (one per local velocity node) and
  // pressure DOFs of every overlapping set
  std::vector<std::vector<int32_t>> bvx(blockm ? P.n_sub : 0), bpr(blockm ? P.n_sub : 0);
  if (blockm) {
    block_check(P);
    for (int i = 0; i < P.n_sub; ++i) {
      const auto& S = P.S[i];
      for (size_t k = 0; k < S.size(); ++k) {
        const int32_t d = S[k];
        if (P.field[d] == 3) {
          bpr[i].push_back(d);
        } else if (P.field[d] == 0) {
          if (k + 2 >= S.size() || S[k + 1] != d + 1 || S[k + 2] != d + 2)
            throw StatusError{1, "the block local solve needs all three velocity components of a node in a set"};
          bvx[i].push_back(d);
        }
      }
      if (3 * bvx[i].size() + bpr[i].size() != S.size())
        throw StatusError{1, "the block local solve needs all three velocity components of a node in a set"};
    }
  }

  // ---- budget pre-check (dominant terms) --------------------------------
  {
    uint64_t need = 0;
    const size_t es = elem_size(ctx.local_prec);
    for (int i = 0; i < P.n_sub; ++i) {
      if (blockm) {
        const uint64_t nv = round_up(std::max<int64_t>(1, (int64_t)bvx[i].size()), 64);
        const uint64_t np = round_up(std::max<int64_t>(1, (int64_t)bpr[i].size()), 64);
        need += (nv * nv * es + np * np * 8) / 2 + 2 * 3 * nv * np * 8 / 4;
        continue;
      }
      const uint64_t np = std::max<int64_t>(nb, round_up((int64_t)P.S[i].size(), nb));
      need += np * np * es + np * nb * (ctx.local_prec == P_FP64 ? 8 : 4);
    }
    need += (uint64_t)Nc * Nc * 8 * 2;
    need += (uint64_t)P.nnz() * 12;
    if (budget && need > budget)
      throw StatusError{2, "device memory budget exceeded: need at least " + std::to_string(need) +
                               " bytes for factors and coarse matrix, budget " + std::to_string(budget) +
                               (levels == 2 ? " (try levels=3 or a lower local precision)" : "")};
  }

  // ---- system matrix ------------------------------------------------------
  ctx.d_rowptr = dupload(A, P.row_ptr, st);
  ctx.d_col = dupload(A, P.col, st);
  ctx.d_val = dupload(A, P.val, st);
  ctx.d_rhs = dupload(A, P.rhs, st);
  ctx.d_full_index = dupload(A, P.full_index, st);
  ctx.d_dirichlet_full = dupload(A, P.dirichlet_full, st);
  double amax = 0.0;
  for (double v : P.val) amax = std::max(amax, std::fabs(v));

  // ---- factor sets and work vector layout ---------------------------------
  // level-1 work positions of every overlapping set's DOFs (P.S order)
  std::vector<std::vector<int64_t>> lpos(P.n_sub);
  if (blockm) {
    // L1: L_i^-1 (three component vectors each), LP: S_i^-1 and, with two
    // levels, the coarse inverse; per subdomain [x | y | z | p] segments
    std::vector<int32_t> nv(P.n_sub), npr(P.n_sub);
    for (int i = 0; i < P.n_sub; ++i) {
      nv[i] = (int32_t)bvx[i].size();
      npr[i] = (int32_t)bpr[i].size();
    }
    if (levels == 2 && Nc > 0) npr.push_back(Nc);
    ctx.L1.nc = 3;
    plan_factor_set(ctx.L1, nv, ctx.local_prec, 64, 0, SOLVE_SYM, A, st);
    plan_factor_set(ctx.LP, npr, P_FP64, 64, 0, SOLVE_SYM, A, st);
    int64_t cur = 0;
    for (int i = 0; i < P.n_sub; ++i) {
      ctx.L1.xoff[i] = cur;
      cur += 3 * (int64_t)ctx.L1.npad[i];
      ctx.LP.xoff[i] = cur;
      cur += ctx.LP.npad[i];
    }
    if ((int)npr.size() > P.n_sub) {
      ctx.LP.xoff[P.n_sub] = cur;
      cur += ctx.LP.npad[P.n_sub];
    }
    ctx.n_w1 = cur;
    GDSW_HIP(hipMemcpyAsync(ctx.L1.d_xoff, ctx.L1.xoff.data(), ctx.L1.count * sizeof(int64_t),
                            hipMemcpyHostToDevice, st));
    GDSW_HIP(hipMemcpyAsync(ctx.LP.d_xoff, ctx.LP.xoff.data(), ctx.LP.count * sizeof(int64_t),
                            hipMemcpyHostToDevice, st));
    ctx.merged = false;
    for (int i = 0; i < P.n_sub; ++i) {
      const int64_t vb = ctx.L1.xoff[i], npv = ctx.L1.npad[i], pb = ctx.LP.xoff[i];
      int64_t a = 0, q = 0;
      for (int32_t d : P.S[i]) {
        if (P.field[d] == 3)
          lpos[i].push_back(pb + q++);
        else
          lpos[i].push_back(vb + (int64_t)P.field[d] * npv + (P.field[d] == 2 ? a++ : a));
      }
    }
  } else {
    std::vector<int32_t> l1_sizes(P.n_sub);
    for (int i = 0; i < P.n_sub; ++i) l1_sizes[i] = (int32_t)P.S[i].size();
    ctx.merged = (levels == 2 && ctx.local_prec == P_FP64 && Nc > 0);
    if (ctx.merged) l1_sizes.push_back(Nc);
    plan_factor_set(ctx.L1, l1_sizes, ctx.local_prec, nb, 0, ctx.solve_mode, A, st);
    ctx.n_w1 = ctx.L1.total_x;
    for (int i = 0; i < P.n_sub; ++i)
      for (size_t k = 0; k < P.S[i].size(); ++k) lpos[i].push_back(ctx.L1.xoff[i] + (int64_t)k);
  }
  std::vector<int32_t> hi_sizes;
  const Level2& L2 = P.lv2;
  // level-2 index sets in factor order: velocity-type coarse DOFs first
  std::vector<std::vector<int32_t>> S2(L2.n_sub), I2(L2.n_sub);
  auto vfirst = [&](const std::vector<int32_t>& v) {
    std::vector<int32_t> o;
    for (int32_t c : v)
      if (P.coarse_field[c] < 3) o.push_back(c);
    for (int32_t c : v)
      if (P.coarse_field[c] == 3) o.push_back(c);
    return o;
  };
  if (levels == 2 && !ctx.merged && !blockm && Nc > 0) hi_sizes.push_back(Nc);
  if (levels == 3) {
    ctx.n_sub2 = L2.n_sub;
    ctx.Nc3 = L2.n_coarse3;
    for (int j = 0; j < L2.n_sub; ++j) {
      S2[j] = vfirst(L2.S[j]);
      I2[j] = vfirst(L2.I[j]);
      hi_sizes.push_back((int32_t)S2[j].size());
    }
    if (ctx.Nc3 > 0) hi_sizes.push_back(ctx.Nc3);
  }
  plan_factor_set(ctx.HI, hi_sizes, P_FP64, nb, ctx.n_w1, blockm ? SOLVE_SYM : ctx.solve_mode, A, st);
  ctx.n_w = ctx.n_w1 + ctx.HI.total_x;
  ctx.d_w = dalloc<double>(A, std::max<int64_t>(ctx.n_w, 1));
  GDSW_HIP(hipMemsetAsync(ctx.d_w, 0, std::max<int64_t>(ctx.n_w, 1) * 8, st));

  // gather map and inverse (scatter) map of the level-1 local copies
  {
    std::vector<int32_t> gidx(ctx.n_w1, -1);
    std::vector<int32_t> cnt(n + 1, 0);
    for (int i = 0; i < P.n_sub; ++i) {
      for (size_t k = 0; k < P.S[i].size(); ++k) {
        gidx[lpos[i][k]] = P.S[i][k];
        cnt[P.S[i][k] + 1]++;
      }
    }
    std::vector<int32_t> inv_ptr(n + 1, 0);
    for (int64_t d = 0; d < n; ++d) inv_ptr[d + 1] = inv_ptr[d] + cnt[d + 1];
    std::vector<int64_t> inv_pos(inv_ptr[n]);
    std::vector<int32_t> fill(n, 0);
    for (int i = 0; i < P.n_sub; ++i) {  // ascending i: fixed summation order
      for (size_t k = 0; k < P.S[i].size(); ++k) {
        const int32_t d = P.S[i][k];
        inv_pos[inv_ptr[d] + fill[d]++] = lpos[i][k];
      }
    }
    ctx.d_gidx = dupload(A, gidx, st);
    ctx.d_inv_ptr = dupload(A, inv_ptr, st);
    ctx.d_inv_pos = dupload(A, inv_pos, st);
  }

  // ---- coarse basis Phi (eq. 2.4) ------------------------------------------
  std::vector<int32_t> I_ptr, I_idx, C_ptr, C_idx;
  concat(P.I, I_ptr, I_idx);
  concat(P.C, C_ptr, C_idx);
  const int64_t total_I = I_idx.size();
  std::vector<int32_t> I_sub(total_I), dof_ipos(n, -1);
  std::vector<int64_t> phi_off(P.n_sub + 1, 0);
  for (int i = 0; i < P.n_sub; ++i) {
    for (int32_t p = I_ptr[i]; p < I_ptr[i + 1]; ++p) {
      I_sub[p] = i;
      dof_ipos[I_idx[p]] = p;
    }
    phi_off[i + 1] = phi_off[i] + (int64_t)P.I[i].size() * P.C[i].size();
  }
  // per coarse column: Gamma DOFs and (subdomain, local column) pairs
  std::vector<std::vector<int32_t>> cg(Nc), cs_sub(Nc), cs_lc(Nc);
  for (int64_t d = 0; d < n; ++d)
    if (P.gamma_col[d] >= 0) cg[P.gamma_col[d]].push_back((int32_t)d);
  for (int i = 0; i < P.n_sub; ++i)
    for (size_t j = 0; j < P.C[i].size(); ++j) {
      cs_sub[P.C[i][j]].push_back(i);
      cs_lc[P.C[i][j]].push_back((int32_t)j);
    }
  std::vector<int32_t> cg_ptr, cg_dof, cs_ptr, cs_s, cs_ptr2, cs_l;
  concat(cg, cg_ptr, cg_dof);
  concat(cs_sub, cs_ptr, cs_s);
  concat(cs_lc, cs_ptr2, cs_l);
  ctx.d_gamma_col = dupload(A, P.gamma_col, st);
  ctx.d_I_ptr = dupload(A, I_ptr, st);
  ctx.d_I_idx = dupload(A, I_idx, st);
  ctx.d_I_sub = dupload(A, I_sub, st);
  ctx.d_dof_ipos = dupload(A, dof_ipos, st);
  ctx.d_C_ptr = dupload(A, C_ptr, st);
  ctx.d_C_idx = dupload(A, C_idx, st);
  ctx.d_phi_off = dupload(A, phi_off, st);
  ctx.d_cg_ptr = dupload(A, cg_ptr, st);
  ctx.d_cg_dof = dupload(A, cg_dof, st);
  ctx.d_cs_ptr = dupload(A, cs_ptr, st);
  ctx.d_cs_sub = dupload(A, cs_s, st);
  ctx.d_cs_lc = dupload(A, cs_l, st);
  ctx.n_pairs = (int)cs_s.size();
  ctx.d_pair_t = dalloc<double>(A, std::max(ctx.n_pairs, 1));
  ctx.max_ni = 0;
  for (int i = 0; i < P.n_sub; ++i) ctx.max_ni = std::max(ctx.max_ni, I_ptr[i + 1] - I_ptr[i]);
  {
    // pair index of every (subdomain, local column), for the restriction
    // by (subdomain, column block)
    std::vector<int32_t> pair_of(C_ptr.back(), -1);
    int32_t e = 0;
    for (int c = 0; c < Nc; ++c)
      for (size_t q = 0; q < cs_sub[c].size(); ++q) pair_of[C_ptr[cs_sub[c][q]] + cs_lc[c][q]] = e++;
    ctx.d_pair_of = dupload(A, pair_of, st);
    int max_nc = 0;
    for (int i = 0; i < P.n_sub; ++i) max_nc = std::max(max_nc, C_ptr[i + 1] - C_ptr[i]);
    ctx.phi_cb = phi_t_columns(P.n_sub, max_nc, ctx.max_ni);
    ctx.phi_nblk = ctx.phi_cb > 0 ? (max_nc + ctx.phi_cb - 1) / ctx.phi_cb : 0;
  }
  {
    std::vector<int32_t> outer;
    for (int64_t d = 0; d < n; ++d)
      if (dof_ipos[d] < 0) outer.push_back((int32_t)d);
    ctx.n_outer = (int64_t)outer.size();
    ctx.d_outer = dupload(A, outer, st);
  }
  ctx.d_phi_cm = dalloc<double>(A, std::max<int64_t>(phi_off.back(), 1));
  ctx.d_phi_rm = dalloc<double>(A, std::max<int64_t>(phi_off.back(), 1));
  CoarseView cv{ctx.d_gamma_col, ctx.d_dof_ipos, ctx.d_I_sub, ctx.d_I_ptr, ctx.d_I_idx, ctx.d_C_ptr,
                ctx.d_C_idx, ctx.d_phi_off, ctx.d_phi_cm, ctx.d_phi_rm, ctx.d_cg_ptr, ctx.d_cg_dof,
                ctx.d_cs_ptr, ctx.d_cs_sub, ctx.d_cs_lc};

  if (Nc > 0) {
    // A_II^(i) dense, LU, and Phi_I = -A_II^-1 A_IGamma Phi_Gamma
    std::vector<int32_t> ni(P.n_sub), nr(P.n_sub);
    std::vector<int64_t> aoff(P.n_sub);
    int64_t tot = 0;
    int max_ni = 0, max_nr = 0;
    for (int i = 0; i < P.n_sub; ++i) {
      ni[i] = (int32_t)P.I[i].size();
      nr[i] = (int32_t)P.C[i].size();
      aoff[i] = tot;
      tot += (int64_t)ni[i] * ni[i];
      max_ni = std::max(max_ni, ni[i]);
      max_nr = std::max(max_nr, nr[i]);
    }
    double* aii = dalloc<double>(A, std::max<int64_t>(tot, 1));
    GDSW_HIP(hipMemsetAsync(aii, 0, std::max<int64_t>(tot, 1) * 8, st));
    int32_t* d_ni = dupload(A, ni, st);
    int32_t* d_nr = dupload(A, nr, st);
    int64_t* d_aoff = dupload(A, aoff, st);
    DenseBatch B;
    B.base = aii;
    B.n = d_ni;
    B.ld = d_ni;
    B.off = d_aoff;
    B.count = P.n_sub;
    B.max_n = max_ni;
    extract_local(B, ctx.d_I_ptr, ctx.d_I_idx, ctx.d_rowptr, ctx.d_col, ctx.d_val, max_ni, st);
    // discontinuous pressure: the velocity columns are extended with the
    // velocity block alone and the pressure rows of Phi_I are fixed (the
    // subdomain's constant pressure column), so the pressure part of A_II
    // becomes the identity
    const bool disc = !P.sub_pcol.empty();
    int32_t* d_nu = nullptr;
    int8_t* d_pval = nullptr;
    int32_t* d_sub_pcol = nullptr;
    if (disc) {
      std::vector<int32_t> nu(P.n_sub, 0);
      std::vector<int8_t> pval(total_I, -1);
      for (int i = 0; i < P.n_sub; ++i)
        for (int32_t q = I_ptr[i]; q < I_ptr[i + 1]; ++q) {
          const int32_t d = I_idx[q];
          if (P.field[d] < 3)
            ++nu[i];
          else
            pval[q] = P.pnull[d];
        }
      d_nu = dupload(A, nu, st);
      d_pval = dupload(A, pval, st);
      d_sub_pcol = dupload(A, P.sub_pcol, st);
      decouple_pressure(B, d_nu, max_ni, st);
    }
    unsigned long long* mp = minpiv_buffer(A, P.n_sub, st);
    lu_nopiv(B, mp, st);
    check_pivots(mp, P.n_sub, 1e-14 * amax, "interior block", st);
    GDSW_HIP(hipMemsetAsync(ctx.d_phi_cm, 0, std::max<int64_t>(phi_off.back(), 1) * 8, st));
    phi_rhs(total_I, cv, ctx.d_rowptr, ctx.d_col, ctx.d_val, ctx.d_phi_cm, st);
    if (disc) phi_pressure_rows(total_I, cv, d_pval, d_sub_pcol, ctx.d_phi_cm, st);
    lu_solve_multi(B, ctx.d_phi_cm, ctx.d_phi_off, d_nr, max_nr, st);
    phi_transpose(total_I, cv, ctx.d_phi_cm, ctx.d_phi_rm, st);
    GDSW_HIP(hipStreamSynchronize(st));
    for (void* q : {(void*)d_nu, (void*)d_pval, (void*)d_sub_pcol})
      if (q) A.free(q);
    A.free(aii);
    A.free(d_ni);
    A.free(d_nr);
    A.free(d_aoff);
    A.free(mp);

    // ---- A_0 = Phi^T A Phi via box-owned nonzeros -------------------------
    const int m = P.spec.m, s = P.s;
    std::vector<int32_t> D_ptr, D_idx;
    concat(P.D, D_ptr, D_idx);
    const int64_t total_D = D_idx.size();
    std::vector<int32_t> D_sub(total_D);
    std::vector<int64_t> box_off(P.n_sub + 1, 0), p_off(P.n_sub + 1, 0);
    int max_nd = 0, max_nc = 0;
    for (int i = 0; i < P.n_sub; ++i) {
      for (int32_t p = D_ptr[i]; p < D_ptr[i + 1]; ++p) D_sub[p] = i;
      box_off[i + 1] = box_off[i] + (int64_t)P.D[i].size() * P.C[i].size();
      p_off[i + 1] = p_off[i] + (int64_t)P.C[i].size() * P.C[i].size();
      max_nd = std::max(max_nd, (int)P.D[i].size());
      max_nc = std::max(max_nc, (int)P.C[i].size());
    }
    // owner of a nonzero: the lowest-numbered box holding both DOFs, found
    // on the device from each DOF's boxes (structured problems: per axis the
    // range of box indices holding its node; algebraic problems: the
    // subdomain lists, whose nonzeros were checked to share one)
    OwnerMap om{nullptr, nullptr, m, nullptr, nullptr};
    std::vector<void*> om_bufs;
    if (!P.algebraic) {
      std::vector<int32_t> blo(3 * (size_t)n), bhi(3 * (size_t)n);
      const int two_s = 2 * s;
      for (int64_t d = 0; d < n; ++d)
        for (int ax = 0; ax < 3; ++ax) {
          const int coord = P.abc[3 * d + ax];
          blo[3 * d + ax] = (coord % two_s == 0) ? std::max(coord / two_s - 1, 0) : coord / two_s;
          bhi[3 * d + ax] = std::min(coord / two_s, m - 1);
        }
      om.blo = dupload(A, blo, st);
      om.bhi = dupload(A, bhi, st);
      om_bufs = {(void*)om.blo, (void*)om.bhi};
      GDSW_HIP(hipStreamSynchronize(st));  // the host vectors go out of scope
    } else {
      om.sub_ptr = dupload(A, P.sub_ptr, st);
      om.sub_idx = dupload(A, P.sub_idx, st);
      om_bufs = {(void*)om.sub_ptr, (void*)om.sub_idx};
    }
    int32_t* d_D_ptr = dupload(A, D_ptr, st);
    int32_t* d_D_idx = dupload(A, D_idx, st);
    int32_t* d_D_sub = dupload(A, D_sub, st);
    int64_t* d_box_off = dupload(A, box_off, st);
    int64_t* d_p_off = dupload(A, p_off, st);
    BoxView bv{d_D_ptr, d_D_idx, d_D_sub, d_box_off};
    double* pbox = dalloc<double>(A, std::max<int64_t>(box_off.back(), 1));
    double* W = dalloc<double>(A, std::max<int64_t>(box_off.back(), 1));
    double* Pm = dalloc<double>(A, std::max<int64_t>(p_off.back(), 1));
    GDSW_HIP(hipMemsetAsync(pbox, 0, std::max<int64_t>(box_off.back(), 1) * 8, st));
    phibox(total_D, cv, bv, pbox, st);
    own_spmm(P.n_sub, max_nd, max_nc, cv, bv, om, ctx.d_rowptr, ctx.d_col, ctx.d_val, pbox, W, st);
    std::vector<GemmDesc> gd(P.n_sub);
    for (int i = 0; i < P.n_sub; ++i) {
      const int nd = (int)P.D[i].size(), nci = (int)P.C[i].size();
      gd[i] = GemmDesc{pbox + box_off[i], W + box_off[i], Pm + p_off[i], nci, nci, nd, nd, nd, nci, 1, 0};
    }
    GemmDesc* d_gd = dupload(A, gd, st);
    gemm_batched(d_gd, P.n_sub, max_nc, max_nc, 1.0, 0.0, st);
    ctx.d_A0 = dalloc<double>(A, (int64_t)Nc * Nc);
    GDSW_HIP(hipMemsetAsync(ctx.d_A0, 0, (int64_t)Nc * Nc * 8, st));
    a0_assemble(Nc, cv, Pm, d_p_off, ctx.d_A0, st);
    GDSW_HIP(hipStreamSynchronize(st));
    for (void* p : {(void*)d_D_ptr, (void*)d_D_idx, (void*)d_D_sub, (void*)d_box_off, (void*)d_p_off,
                    (void*)pbox, (void*)W, (void*)Pm, (void*)d_gd})
      A.free(p);
    for (void* p : om_bufs) A.free(p);

    // coarse factor order: velocity-type columns first, then pressure-type
    ctx.coarse_perm.clear();
    for (int c = 0; c < Nc; ++c)
      if (P.coarse_field[c] < 3) ctx.coarse_perm.push_back(c);
    for (int c = 0; c < Nc; ++c)
      if (P.coarse_field[c] == 3) ctx.coarse_perm.push_back(c);
  }

  // ---- three levels: Phi^(3) on A_0 (eq. 2.4 applied to A_0) and A_0^(3) ----
  std::vector<int32_t> perm3;
  if (levels == 3 && Nc > 0) {
    const int Nc3 = ctx.Nc3;
    std::vector<int32_t> i2_ptr, i2_idx, c3_ptr, c3_idx;
    concat(I2, i2_ptr, i2_idx);
    concat(L2.C, c3_ptr, c3_idx);
    const int64_t total_I2 = i2_idx.size();
    std::vector<int32_t> i2_sub(total_I2), ni2(L2.n_sub), nr2(L2.n_sub);
    std::vector<int64_t> off2(L2.n_sub + 1, 0), aoff2(L2.n_sub);
    int64_t atot = 0;
    int max_ni2 = 0, max_nr2 = 0;
    for (int j = 0; j < L2.n_sub; ++j) {
      for (int32_t q = i2_ptr[j]; q < i2_ptr[j + 1]; ++q) i2_sub[q] = j;
      ni2[j] = (int32_t)I2[j].size();
      nr2[j] = (int32_t)L2.C[j].size();
      off2[j + 1] = off2[j] + (int64_t)ni2[j] * nr2[j];
      aoff2[j] = atot;
      atot += (int64_t)ni2[j] * ni2[j];
      max_ni2 = std::max(max_ni2, ni2[j]);
      max_nr2 = std::max(max_nr2, nr2[j]);
    }
    int32_t* d_i2_ptr = dupload(A, i2_ptr, st);
    int32_t* d_i2_idx = dupload(A, i2_idx, st);
    int32_t* d_i2_sub = dupload(A, i2_sub, st);
    int32_t* d_c3_ptr = dupload(A, c3_ptr, st);
    int32_t* d_c3_idx = dupload(A, c3_idx, st);
    int64_t* d_off2 = dupload(A, off2, st);
    int64_t* d_aoff2 = dupload(A, aoff2, st);
    int32_t* d_ni2 = dupload(A, ni2, st);
    int32_t* d_nr2 = dupload(A, nr2, st);
    int32_t* d_gcol3 = dupload(A, L2.gamma_col3, st);
    double* aii = dalloc<double>(A, std::max<int64_t>(atot, 1));
    double* phiI = dalloc<double>(A, std::max<int64_t>(off2.back(), 1));
    GDSW_HIP(hipMemsetAsync(phiI, 0, std::max<int64_t>(off2.back(), 1) * 8, st));
    DenseBatch B;
    B.base = aii;
    B.n = d_ni2;
    B.ld = d_ni2;
    B.off = d_aoff2;
    B.count = L2.n_sub;
    B.max_n = max_ni2;
    extract_local_dense(B, d_i2_ptr, d_i2_idx, ctx.d_A0, Nc, max_ni2, st);
    unsigned long long* mp = minpiv_buffer(A, L2.n_sub, st);
    lu_nopiv(B, mp, st);
    check_pivots(mp, L2.n_sub, 0.0, "level-2 interior block", st);
    phi3_rhs(total_I2, Nc, d_i2_sub, d_i2_ptr, d_i2_idx, d_c3_ptr, d_c3_idx, d_off2, d_gcol3, ctx.d_A0, phiI, st);
    lu_solve_multi(B, phiI, d_off2, d_nr2, max_nr2, st);
    // the dense Phi^(3) only for forming A_0^(3) here; the apply reads the
    // subregion blocks phiI and the interface indicator (coarse_view3)
    double* phi3 = dalloc<double>(A, std::max<int64_t>((int64_t)Nc * Nc3, 1));
    GDSW_HIP(hipMemsetAsync(phi3, 0, std::max<int64_t>((int64_t)Nc * Nc3, 1) * 8, st));
    phi3_build(total_I2, Nc, d_i2_sub, d_i2_ptr, d_i2_idx, d_c3_ptr, d_c3_idx, d_off2, phiI, d_gcol3, phi3, st);
    // A_0^(3) = Phi3^T (A_0 Phi3): A_0 is row-major, i.e. A_0^T column-major
    double* T = dalloc<double>(A, std::max<int64_t>((int64_t)Nc * Nc3, 1));
    ctx.d_A03 = dalloc<double>(A, std::max<int64_t>((int64_t)Nc3 * Nc3, 1));
    std::vector<GemmDesc> gd = {GemmDesc{ctx.d_A0, phi3, T, Nc, Nc3, Nc, Nc, Nc, Nc, 1, 0}};
    GemmDesc* d_gd = dupload(A, gd, st);
    gemm_batched(d_gd, 1, Nc, Nc3, 1.0, 0.0, st);
    std::vector<GemmDesc> gd2 = {GemmDesc{phi3, T, ctx.d_A03, Nc3, Nc3, Nc, Nc, Nc, Nc3, 1, 0}};
    GemmDesc* d_gd2 = dupload(A, gd2, st);
    gemm_batched(d_gd2, 1, Nc3, Nc3, 1.0, 0.0, st);
    GDSW_HIP(hipStreamSynchronize(st));
    for (void* q : {(void*)d_aoff2, (void*)d_ni2, (void*)d_nr2, (void*)aii, (void*)phi3, (void*)T, (void*)d_gd,
                    (void*)d_gd2, (void*)mp})
      A.free(q);
    // the level-3 view: the level-1 layout with subregions for subdomains
    ctx.d_gcol3 = d_gcol3;
    ctx.d_i2_sub = d_i2_sub;
    ctx.d_i2_ptr = d_i2_ptr;
    ctx.d_i2_idx = d_i2_idx;
    ctx.d_c3_ptr = d_c3_ptr;
    ctx.d_c3_idx = d_c3_idx;
    ctx.d_off2 = d_off2;
    ctx.d_phi3_cm = phiI;
    ctx.max_ni2 = max_ni2;
    {
      std::vector<int32_t> ipos3(Nc, -1);
      for (int64_t q = 0; q < total_I2; ++q) ipos3[i2_idx[q]] = (int32_t)q;
      std::vector<std::vector<int32_t>> cg3(Nc3), cs3s(Nc3), cs3l(Nc3);
      for (int c = 0; c < Nc; ++c)
        if (L2.gamma_col3[c] >= 0) cg3[L2.gamma_col3[c]].push_back(c);
      for (int j = 0; j < L2.n_sub; ++j)
        for (size_t q = 0; q < L2.C[j].size(); ++q) {
          cs3s[L2.C[j][q]].push_back(j);
          cs3l[L2.C[j][q]].push_back((int32_t)q);
        }
      std::vector<int32_t> cg_ptr3, cg_dof3, cs_ptr3, cs_sub3, cs_ptr3b, cs_lc3, outer3;
      concat(cg3, cg_ptr3, cg_dof3);
      concat(cs3s, cs_ptr3, cs_sub3);
      concat(cs3l, cs_ptr3b, cs_lc3);
      for (int c = 0; c < Nc; ++c)
        if (ipos3[c] < 0) outer3.push_back(c);
      ctx.d_ipos3 = dupload(A, ipos3, st);
      ctx.d_cg3_ptr = dupload(A, cg_ptr3, st);
      ctx.d_cg3_dof = dupload(A, cg_dof3, st);
      ctx.d_cs3_ptr = dupload(A, cs_ptr3, st);
      ctx.d_cs3_sub = dupload(A, cs_sub3, st);
      ctx.d_cs3_lc = dupload(A, cs_lc3, st);
      ctx.n_pairs3 = (int)cs_sub3.size();
      ctx.d_pair_t3 = dalloc<double>(A, std::max(ctx.n_pairs3, 1));
      ctx.n_outer3 = (int64_t)outer3.size();
      ctx.d_outer3 = dupload(A, outer3, st);
    }
    // level-3 factor order: velocity-type columns first
    std::vector<int32_t> f3(Nc3, 0);
    for (int c = 0; c < Nc; ++c)
      if (L2.gamma_col3[c] >= 0) f3[L2.gamma_col3[c]] = P.coarse_field[c];
    for (int k = 0; k < Nc3; ++k)
      if (f3[k] < 3) perm3.push_back(k);
    for (int k = 0; k < Nc3; ++k)
      if (f3[k] == 3) perm3.push_back(k);
    // work-vector maps of the level-2 copies and the level-3 segment
    const int64_t hx = ctx.HI.total_x;
    std::vector<int32_t> g2(hx, -1), cnt(Nc + 1, 0);
    for (int j = 0; j < L2.n_sub; ++j) {
      const int64_t xo = ctx.HI.xoff[j] - ctx.n_w1;
      for (size_t k = 0; k < S2[j].size(); ++k) {
        g2[xo + k] = S2[j][k];
        cnt[S2[j][k] + 1]++;
      }
    }
    std::vector<int32_t> inv2_ptr(Nc + 1, 0);
    for (int c = 0; c < Nc; ++c) inv2_ptr[c + 1] = inv2_ptr[c] + cnt[c + 1];
    std::vector<int64_t> inv2_pos(inv2_ptr[Nc]);
    std::vector<int32_t> fill(Nc, 0);
    // ascending subregion index: for each c, positions in increasing j
    for (int j = 0; j < L2.n_sub; ++j)
      for (size_t k = 0; k < S2[j].size(); ++k) {
        const int32_t c = S2[j][k];
        inv2_pos[inv2_ptr[c] + fill[c]++] = ctx.HI.xoff[j] + (int64_t)k;
      }
    ctx.d_g2idx = dupload(A, g2, st);
    ctx.d_inv2_ptr = dupload(A, inv2_ptr, st);
    ctx.d_inv2_pos = dupload(A, inv2_pos, st);
    std::vector<int32_t> p3(Nc3);
    if (Nc3 > 0) {
      const int64_t x3 = ctx.HI.xoff[L2.n_sub];
      for (int q = 0; q < Nc3; ++q) p3[perm3[q]] = (int32_t)(x3 + q);
    }
    ctx.d_c3_pinv = dupload(A, p3, st);
    ctx.d_r0 = dalloc<double>(A, Nc);
    ctx.d_y0 = dalloc<double>(A, Nc);
  }

  // ---- level-1 local factors (and the coarse factor when merged) -----------
  std::vector<int32_t> S_ptr, S_idx;
  concat(P.S, S_ptr, S_idx);
  int32_t* d_S_ptr = dupload(A, S_ptr, st);
  int32_t* d_S_idx = dupload(A, S_idx, st);
  int32_t* d_perm = ctx.coarse_perm.empty() ? nullptr : dupload(A, ctx.coarse_perm, st);
  const uint64_t staging_cap = std::max<uint64_t>(1ull << 30, std::min<uint64_t>(32ull << 30, budget / 4));
  if (blockm) {
    // L_i^-1 by Gauss-Jordan; from each chunk's FP64 inverses, before they are
    // stored, S_i = B_i K_i^-1 B_i^T = Bt^T (L^-1 Bt) with Bt the velocity
    // columns of B_i^T in component-major blocks (3 npad_v x np_i)
    std::vector<int32_t> vx_ptr, vx_idx, pr_ptr, pr_idx;
    concat(bvx, vx_ptr, vx_idx);
    concat(bpr, pr_ptr, pr_idx);
    int32_t* d_vx_ptr = dupload(A, vx_ptr, st);
    int32_t* d_vx = dupload(A, vx_idx, st);
    int32_t* d_pr_ptr = dupload(A, pr_ptr, st);
    int32_t* d_pr = dupload(A, pr_idx, st);
    std::vector<int64_t> soff(P.n_sub + 1, 0);
    for (int i = 0; i < P.n_sub; ++i) soff[i + 1] = soff[i] + (int64_t)bpr[i].size() * bpr[i].size();
    double* Sbuf = dalloc<double>(A, std::max<int64_t>(soff.back(), 1));
    int64_t* d_soff = dupload(A, soff, st);
    // keep W_i = K_i^-1 B_i^T for the last step where it is the smaller read
    // (its bytes against one pass over the upper tiles of L_i^-1)
    BlockSolve& b = ctx.blk;
    const size_t les = elem_size(ctx.local_prec);
    std::vector<int64_t> woff(P.n_sub + 1, 0);
    uint64_t tile_bytes = 0;
    bool fits = true;
    for (int i = 0; i < P.n_sub; ++i) {
      const int64_t wi = 3 * (int64_t)ctx.L1.npad[i] * (int64_t)bpr[i].size();
      woff[i + 1] = woff[i] + wi;
      tile_bytes += (uint64_t)symv_tiles(ctx.L1.npad[i]) * 64 * 64 * les;
      fits = fits && bpr[i].size() <= (size_t)WP_MAX_NP && (uint64_t)wi * les < (1ull << 31);
    }
    b.use_w = fits && woff.back() > 0 && (uint64_t)woff.back() * les < tile_bytes;
    if (b.use_w) {
      b.d_W = A.alloc((uint64_t)woff.back() * les);
      b.w_bytes = (uint64_t)woff.back() * les;
    }
    factor_set(
        ctx, ctx.L1, staging_cap, 1e-14 * amax, "velocity block", st,
        [&](DenseBatch& B, int f0, int f1) {
          int mx = 0;
          for (int f = f0; f < f1; ++f) mx = std::max(mx, (int)bvx[f].size());
          extract_local(B, d_vx_ptr + f0, d_vx, ctx.d_rowptr, ctx.d_col, ctx.d_val, mx, st);
        },
        [&](DenseBatch& B, int f0, int f1) {
          const int cnt = f1 - f0;
          std::vector<int64_t> boff(cnt + 1, 0);
          std::vector<int32_t> npv(cnt);
          int max_np = 0, max_nv = 0;
          for (int k = 0; k < cnt; ++k) {
            npv[k] = ctx.L1.npad[f0 + k];
            boff[k + 1] = boff[k] + 3 * (int64_t)npv[k] * bpr[f0 + k].size();
            max_np = std::max(max_np, (int)bpr[f0 + k].size());
            max_nv = std::max(max_nv, (int)bvx[f0 + k].size());
          }
          if (boff.back() == 0) return;
          double* Bt = dalloc<double>(A, boff.back());
          double* W = dalloc<double>(A, boff.back());
          GDSW_HIP(hipMemsetAsync(Bt, 0, boff.back() * 8, st));
          GDSW_HIP(hipMemsetAsync(W, 0, boff.back() * 8, st));
          int32_t* d_npv = dupload(A, std::vector<int32_t>(ctx.L1.npad.begin(), ctx.L1.npad.end()), st);
          int64_t* d_boff = dupload(A, boff, st);
          block_fill_bt(ctx.d_rowptr, ctx.d_col, ctx.d_val, P.n_u, d_vx_ptr, d_vx, d_pr_ptr, d_pr, d_npv, d_boff, f0,
                        cnt, max_np, Bt, st);
          // staging offsets of the chunk's inverses (full npad x npad matrices)
          std::vector<GemmDesc> g1, g2;
          int64_t so = 0;
          for (int k = 0; k < cnt; ++k) {
            const int f = f0 + k, nvf = (int)bvx[f].size(), npf = (int)bpr[f].size(), ld = npv[k];
            if (npf > 0 && nvf > 0) {
              g1.push_back(GemmDesc{B.base + so, Bt + boff[k], W + boff[k], nvf, 3 * npf, nvf, ld, ld, ld, 0, 0});
              g2.push_back(GemmDesc{Bt + boff[k], W + boff[k], Sbuf + soff[f], npf, npf, 3 * ld, 3 * ld, 3 * ld, npf,
                                    1, 0});
            }
            so += (int64_t)ld * ld;
          }
          GemmDesc* d_g1 = dupload(A, g1, st);
          GemmDesc* d_g2 = dupload(A, g2, st);
          gemm_batched(d_g1, (int)g1.size(), max_nv, 3 * max_np, 1.0, 0.0, st);
          gemm_batched(d_g2, (int)g2.size(), max_np, max_np, 1.0, 0.0, st);
          if (b.use_w) {  // the chunk's W_i, contiguous in the store as in W
            char* dst = static_cast<char*>(b.d_W) + (size_t)woff[f0] * les;
            if (ctx.local_prec == P_FP64)
              GDSW_HIP(hipMemcpyAsync(dst, W, boff.back() * 8, hipMemcpyDeviceToDevice, st));
            else
              convert_store(ctx.local_prec, W, dst, boff.back(), st);
          }
          GDSW_HIP(hipStreamSynchronize(st));
          for (void* q : {(void*)Bt, (void*)W, (void*)d_npv, (void*)d_boff, (void*)d_g1, (void*)d_g2}) A.free(q);
        });
    int32_t* d_perm_b = ctx.coarse_perm.empty() ? nullptr : dupload(A, ctx.coarse_perm, st);
    factor_set(ctx, ctx.LP, staging_cap, 0.0, "pressure Schur complement", st, [&](DenseBatch& B, int f0, int f1) {
      const int nloc = std::min(f1, P.n_sub) - f0;
      int64_t mx = 0;
      for (int f = f0; f < f0 + nloc; ++f) mx = std::max<int64_t>(mx, (int64_t)bpr[f].size() * bpr[f].size());
      copy_blocks(Sbuf, d_soff + f0, B.n, nloc, mx, B.base, B.off, B.ld, st);
      if (f1 == ctx.LP.count && ctx.LP.count > P.n_sub) {
        double* dst = B.base + staging_offset(ctx.LP, f0, ctx.LP.count - 1);
        permute_dense(Nc, d_perm_b, ctx.d_A0, Nc, dst, ctx.LP.npad[ctx.LP.count - 1], st);
      }
    });
    GDSW_HIP(hipStreamSynchronize(st));
    for (void* q : {(void*)d_vx_ptr, (void*)d_vx, (void*)d_pr_ptr, (void*)d_pr, (void*)Sbuf, (void*)d_soff})
      A.free(q);
    if (d_perm_b) A.free(d_perm_b);
    // B_i as row lists over work positions: pressure rows (velocity positions)
    // and, without W, velocity rows (pressure positions), each subdomain in
    // order.  The subdomains are listed in parallel and joined in order.
    struct BRows {
      std::vector<int32_t> prow_pos, bm_pos, vrow_pos, bt_pos;
      std::vector<int64_t> bm_end, bt_end;  // row ends within the subdomain's lists
      std::vector<double> bm_val, bt_val;
    };
    std::vector<BRows> br(P.n_sub);
    parallel_items(P.n_sub, [&](int i) {
      BRows& o = br[i];
      const int64_t vb = ctx.L1.xoff[i], npv = ctx.L1.npad[i], pb = ctx.LP.xoff[i];
      const auto& vx = bvx[i];
      for (size_t q = 0; q < bpr[i].size(); ++q) {
        const int32_t g = bpr[i][q];
        o.prow_pos.push_back((int32_t)(pb + (int64_t)q));
        for (int32_t e = P.row_ptr[g]; e < P.row_ptr[g + 1]; ++e) {
          const int32_t c = P.col[e];
          if (c >= P.n_u) continue;
          const int comp = c % 3;
          const auto it = std::lower_bound(vx.begin(), vx.end(), c - comp);
          if (it == vx.end() || *it != c - comp) continue;
          o.bm_pos.push_back((int32_t)(vb + comp * npv + (it - vx.begin())));
          o.bm_val.push_back(P.val[e]);
        }
        o.bm_end.push_back((int64_t)o.bm_pos.size());
      }
      if (b.use_w) return;
      // B_i^T: the entries ordered by velocity position with a stable
      // counting sort; the pressure rows were visited in ascending order, so
      // each velocity row lists its pressure positions in ascending order
      const int64_t nvp = 3 * npv;
      std::vector<int64_t> start(nvp + 1, 0);
      for (int32_t vp : o.bm_pos) ++start[vp - vb + 1];
      for (int64_t v = 0; v < nvp; ++v) start[v + 1] += start[v];
      std::vector<int64_t> put(start.begin(), start.end() - 1);
      o.bt_pos.resize(o.bm_pos.size());
      o.bt_val.resize(o.bm_pos.size());
      size_t e = 0;
      for (size_t q = 0; q < bpr[i].size(); ++q)
        for (; e < (size_t)o.bm_end[q]; ++e) {
          const int64_t k = put[o.bm_pos[e] - vb]++;
          o.bt_pos[k] = (int32_t)(pb + (int64_t)q);
          o.bt_val[k] = o.bm_val[e];
        }
      for (int64_t v = 0; v < nvp; ++v)
        if (start[v + 1] > start[v]) {
          o.vrow_pos.push_back((int32_t)(vb + v));
          o.bt_end.push_back(start[v + 1]);
        }
    });
    std::vector<int32_t> prow_pos, bm_pos, vrow_pos, bt_pos;
    std::vector<int64_t> bm_ptr(1, 0), bt_ptr(1, 0);
    std::vector<double> bm_val, bt_val;
    {
      size_t np_tot = 0, nm_tot = 0, nv_tot = 0, nt_tot = 0;
      for (const BRows& o : br) {
        np_tot += o.prow_pos.size();
        nm_tot += o.bm_pos.size();
        nv_tot += o.vrow_pos.size();
        nt_tot += o.bt_pos.size();
      }
      prow_pos.reserve(np_tot);
      bm_ptr.reserve(np_tot + 1);
      bm_pos.reserve(nm_tot);
      bm_val.reserve(nm_tot);
      vrow_pos.reserve(nv_tot);
      bt_ptr.reserve(nv_tot + 1);
      bt_pos.reserve(nt_tot);
      bt_val.reserve(nt_tot);
    }
    for (BRows& o : br) {
      const int64_t m0 = (int64_t)bm_pos.size(), t0 = (int64_t)bt_pos.size();
      prow_pos.insert(prow_pos.end(), o.prow_pos.begin(), o.prow_pos.end());
      for (int64_t x : o.bm_end) bm_ptr.push_back(m0 + x);
      bm_pos.insert(bm_pos.end(), o.bm_pos.begin(), o.bm_pos.end());
      bm_val.insert(bm_val.end(), o.bm_val.begin(), o.bm_val.end());
      vrow_pos.insert(vrow_pos.end(), o.vrow_pos.begin(), o.vrow_pos.end());
      for (int64_t x : o.bt_end) bt_ptr.push_back(t0 + x);
      bt_pos.insert(bt_pos.end(), o.bt_pos.begin(), o.bt_pos.end());
      bt_val.insert(bt_val.end(), o.bt_val.begin(), o.bt_val.end());
      o = BRows();
    }
    b.n_prow = (int64_t)prow_pos.size();
    b.n_vrow = (int64_t)vrow_pos.size();
    b.d_prow_pos = dupload(A, prow_pos, st);
    b.d_bm_ptr = dupload(A, bm_ptr, st);
    b.d_bm_pos = dupload(A, bm_pos, st);
    b.d_bm_val = dupload(A, bm_val, st);
    b.b_bytes = (uint64_t)(bm_pos.size() + bt_pos.size()) * 12 + (uint64_t)(prow_pos.size() + vrow_pos.size()) * 12;
    if (b.use_w) {
      const int rw = wp_rows_per_item(ctx.local_prec);
      std::vector<WItem> items;
      for (int i = 0; i < P.n_sub; ++i) {
        const int32_t rows = 3 * ctx.L1.npad[i], np = (int32_t)bpr[i].size();
        if (np == 0) continue;
        for (int32_t r0 = 0; r0 < rows; r0 += rw)
          items.push_back(WItem{woff[i], ctx.L1.xoff[i], ctx.LP.xoff[i], rows, np, r0, 0});
      }
      b.n_witems = (int)items.size();
      b.d_witems = dupload(A, items, st);
    } else {
      b.d_vrow_pos = dupload(A, vrow_pos, st);
      b.d_bt_ptr = dupload(A, bt_ptr, st);
      b.d_bt_pos = dupload(A, bt_pos, st);
      b.d_bt_val = dupload(A, bt_val, st);
      b.d_w2 = dalloc<double>(A, std::max<int64_t>(ctx.n_w1, 1));
      GDSW_HIP(hipMemsetAsync(b.d_w2, 0, std::max<int64_t>(ctx.n_w1, 1) * 8, st));
    }
  } else
  factor_set(ctx, ctx.L1, staging_cap, 1e-14 * amax, "local factor", st,
             [&](DenseBatch& B, int f0, int f1) {
               const int nloc = std::min(f1, P.n_sub) - f0;
               if (nloc > 0) {
                 DenseBatch Bl = B;
                 Bl.count = nloc;
                 int mx = 0;
                 for (int f = f0; f < f0 + nloc; ++f) mx = std::max(mx, (int)P.S[f].size());
                 Bl.max_n = mx;
                 extract_local(Bl, d_S_ptr + f0, d_S_idx, ctx.d_rowptr, ctx.d_col, ctx.d_val, mx, st);
               }
               if (ctx.merged && f1 == ctx.L1.count) {
                 const int fc = ctx.L1.count - 1 - f0;
                 double* dst = B.base + staging_offset(ctx.L1, f0, ctx.L1.count - 1);
                 permute_dense(Nc, d_perm, ctx.d_A0, Nc, dst, ctx.L1.npad[ctx.L1.count - 1], st);
                 (void)fc;
               }
             });
  if (!ctx.merged && !blockm && ctx.HI.count > 0 && levels == 2) {
    factor_set(ctx, ctx.HI, staging_cap, 0.0, "coarse factor", st, [&](DenseBatch& B, int, int) {
      permute_dense(Nc, d_perm, ctx.d_A0, Nc, B.base, ctx.HI.npad[0], st);
    });
  }
  if (levels == 3 && ctx.HI.count > 0) {
    std::vector<int32_t> s2_ptr, s2_idx;
    concat(S2, s2_ptr, s2_idx);
    int32_t* d_s2_ptr = dupload(A, s2_ptr, st);
    int32_t* d_s2_idx = dupload(A, s2_idx, st);
    int32_t* d_perm3 = dupload(A, perm3, st);
    factor_set(ctx, ctx.HI, staging_cap, 0.0, "level-2/3 factor", st, [&](DenseBatch& B, int f0, int f1) {
      const int nloc = std::min(f1, ctx.n_sub2) - f0;
      if (nloc > 0) {
        DenseBatch Bl = B;
        Bl.count = nloc;
        int mx = 0;
        for (int f = f0; f < f0 + nloc; ++f) mx = std::max(mx, (int)S2[f].size());
        Bl.max_n = mx;
        extract_local_dense(Bl, d_s2_ptr + f0, d_s2_idx, ctx.d_A0, ctx.Nc, mx, st);
      }
      if (ctx.Nc3 > 0 && f1 == ctx.HI.count) {
        double* dst = B.base + staging_offset(ctx.HI, f0, ctx.HI.count - 1);
        permute_dense(ctx.Nc3, d_perm3, ctx.d_A03, ctx.Nc3, dst, ctx.HI.npad[ctx.HI.count - 1], st);
      }
    });
    A.free(d_s2_ptr);
    A.free(d_s2_idx);
    A.free(d_perm3);
  }
  A.free(d_S_ptr);
  A.free(d_S_idx);
  // coarse column -> work-vector position (two levels)
  if (Nc > 0 && levels == 2) {
    const FactorSet& cs = blockm ? ctx.LP : ctx.merged ? ctx.L1 : ctx.HI;
    const int fc = blockm ? ctx.LP.count - 1 : ctx.merged ? ctx.L1.count - 1 : 0;
    ctx.coarse_xoff = cs.xoff[fc];
    std::vector<int32_t> pinv(Nc);
    for (int q = 0; q < Nc; ++q) pinv[ctx.coarse_perm[q]] = (int32_t)(ctx.coarse_xoff + q);
    ctx.d_coarse_pinv = dupload(A, pinv, st);
  }
  if (d_perm) A.free(d_perm);
  ctx.factor_bytes = 0;
  for (int f = 0; f < P.n_sub; ++f)
    ctx.factor_bytes += (ctx.solve_mode == SOLVE_SYM || blockm ? (uint64_t)symv_tiles(ctx.L1.npad[f]) * 64 * 64
                                                               : (uint64_t)ctx.L1.npad[f] * ctx.L1.npad[f]) *
                            elem_size(ctx.local_prec) +
                        (blockm ? (uint64_t)symv_tiles(ctx.LP.npad[f]) * 64 * 64 * 8 : 0);
  ctx.factor_bytes += ctx.blk.w_bytes;
  ctx.coarse_bytes = (uint64_t)Nc * Nc * 8 * 2 + (uint64_t)phi_off.back() * 16;
  // descriptors of the stored inverses against the work vector
  for (FactorSet* fs : {&ctx.L1, &ctx.HI, &ctx.LP})
    if ((fs->mode == SOLVE_INVERSE || fs->mode == SOLVE_SYM) && fs->count > 0) {
      std::vector<GemvDesc> d = gemv_descs(*fs, ctx.d_w);
      if (fs->nc > 1)
        for (int f = 0; f < fs->count; ++f) d[f].vs = fs->npad[f];
      fs->d_desc = dupload(A, d, st);
      if (blockm && fs == &ctx.L1 && !ctx.blk.use_w) {
        // L^-1 (B^T p), read from d_w2 and subtracted from U1 in the work vector
        std::vector<GemvDesc> d2 = gemv_descs(*fs, ctx.blk.d_w2);
        for (int f = 0; f < fs->count; ++f) {
          d2[f].vs = fs->npad[f];
          d2[f].y = ctx.d_w + fs->xoff[f];
        }
        ctx.blk.d_desc2 = dupload(A, d2, st);
      }
    }
  // several right-hand sides: MFMA work plans and interleaved work buffers
  if (ctx.max_rhs > 1 && ctx.solve_mode == SOLVE_INVERSE) {
    plan_gemm(ctx.L1, A, st);
    plan_gemm(ctx.HI, A, st);
    const int K = ctx.max_rhs;
    ctx.d_wm = dalloc<double>(A, std::max<int64_t>(ctx.n_w, 1) * K);
    ctx.d_xin = dalloc<double>(A, std::max<int64_t>(n, 1) * K);
    ctx.d_xout = dalloc<double>(A, std::max<int64_t>(n, 1) * K);
    ctx.d_pair_tm = dalloc<double>(A, (int64_t)phi_t_splits(P.n_sub) * std::max(ctx.n_pairs, 1) * K);
  }
  GDSW_HIP(hipStreamSynchronize(st));
}

}  // namespace gdsw
