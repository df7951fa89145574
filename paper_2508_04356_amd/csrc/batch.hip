// A batch of independent Stokes problems (eq. 2.1 with their own meshes,
// viscosities and inflows), each with its own GDSW preconditioner, whose
// local and coarse solves run together: one partial-product launch and one
// summation launch per level cover the stored inverses of every member.
// The work items are ordered longest matrix first, so the largest members'
// matrices start first and the small ones fill in at the end.  Members that
// have stopped (converged or out of iterations) are masked out of the
// launches through a per-matrix flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>

#include "context.h"
#include "kernels.h"
#include "kernels_learned.h"
#include "learned.h"

namespace gdsw {
namespace {

void build_set(Batch& b, BatchSet& S, bool level1, hipStream_t st) {
  std::vector<GemvDesc> desc;
  S.owner.clear();
  S.fidx.clear();
  S.bytes.clear();
  S.prec = -1;
  for (size_t k = 0; k < b.m.size(); ++k) {
    Context& c = *b.m[k];
    const FactorSet& fs = level1 ? c.L1 : c.HI;
    if (fs.count == 0) continue;
    if (fs.mode != SOLVE_INVERSE && fs.mode != SOLVE_SYM)
      throw StatusError{1, "batched solves need explicit inverses (full or symmetric) or the block solve"};
    if (S.prec >= 0 && S.prec != fs.prec) throw StatusError{1, "batch members must share the local precision"};
    if (S.prec >= 0 && S.sym != (fs.mode == SOLVE_SYM)) throw StatusError{1, "batch members must share the storage"};
    if (S.prec >= 0 && S.nc != fs.nc) throw StatusError{1, "batch members must share the local solve"};
    S.prec = fs.prec;
    S.sym = fs.mode == SOLVE_SYM;
    S.nc = fs.nc;
    std::vector<GemvDesc> d = gemv_descs(fs, c.d_w);
    if (fs.nc > 1)  // the velocity components, npad apart (the member's own descriptors)
      for (int f = 0; f < fs.count; ++f) d[f].vs = fs.npad[f];
    for (int f = 0; f < fs.count; ++f) {
      desc.push_back(d[f]);
      S.owner.push_back((int)k);
      S.fidx.push_back(f);
      S.bytes.push_back((fs.mode == SOLVE_SYM ? (uint64_t)fs.n[f] * (fs.n[f] + 1) / 2 : (uint64_t)fs.n[f] * fs.n[f]) *
                        elem_size(fs.prec));
    }
  }
  S.count = (int)desc.size();
  if (S.count == 0) return;
  // longest matrix first (stable: ties keep member order)
  std::vector<int> order(S.count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return desc[a].n > desc[c].n; });
  std::vector<GemvDesc> sd(S.count);
  std::vector<int> so(S.count), sf(S.count);
  std::vector<uint64_t> sb(S.count);
  for (int g = 0; g < S.count; ++g) {
    sd[g] = desc[order[g]];
    so[g] = S.owner[order[g]];
    sf[g] = S.fidx[order[g]];
    sb[g] = S.bytes[order[g]];
  }
  S.owner = so;
  S.fidx = sf;
  S.bytes = sb;
  const int RB = gemv_rows(S.prec);
  std::vector<int4> it1, it2;
  int64_t p = 0;
  for (int f = 0; f < S.count; ++f) {
    const int n = sd[f].n;
    if (S.sym) {  // the same tile runs and slots as the member's own plan
      symv_items(f, sd[f].np, p, S.plan.run, it1, it2);
      p += symv_tiles(sd[f].np);
      continue;
    }
    const int nr = (n + RB - 1) / RB, nc = (n + GEMV_CW - 1) / GEMV_CW;
    for (int c = 0; c < nc; ++c)
      for (int J = 0; J < nr; ++J) it1.push_back(make_int4(f, J * RB, c * GEMV_CW, (int)(p + J * nc + c)));
    for (int J = 0; J < nr; ++J) it2.push_back(make_int4(f, J * RB, (int)(p + J * nc), nc));
    p += nr * nc;
  }
  DeviceArena& A = b.arena;
  S.d_desc = dupload(A, sd, st);
  S.plan.xcd = symv_default_xcd(S.prec);
  S.plan.n1 = (int)it1.size();
  S.plan.n2 = (int)it2.size();
  S.plan.d_items1 = dupload(A, it1, st);
  S.plan.d_items2 = dupload(A, it2, st);
  S.partial_len = S.sym ? 2 * 64 * S.nc * std::max<int64_t>(p, 1) : std::max<int64_t>(p, 1) * RB;
  S.d_partial = dalloc<double>(A, S.partial_len);
  S.h_want.assign(S.count, 1);
  S.d_want = dupload(A, S.h_want, st);
  S.active_bytes = 0.0;
  for (uint64_t v : S.bytes) S.active_bytes += (double)v;
}

// want[g] = member of matrix g active, and g not an interior matrix of a
// member whose interior solves are learned (or dropped) instead
void select_set(const Batch& b, BatchSet& S, const std::vector<char>& active, bool level1, hipStream_t st) {
  if (S.count == 0) return;
  std::vector<std::vector<char>> skip(b.m.size());
  if (level1)
    for (size_t k = 0; k < b.m.size(); ++k) {
      const Context& c = *b.m[k];
      if (!batch_learned(c)) continue;
      skip[k].assign(c.L1.count, 0);
      for (int32_t f : c.learned->factors) skip[k][f] = 1;
    }
  bool same = true;
  S.active_bytes = 0.0;
  for (int g = 0; g < S.count; ++g) {
    const int k = S.owner[g];
    const bool off = !skip[k].empty() && skip[k][S.fidx[g]];
    const int32_t v = (active[k] && !off) ? 1 : 0;
    same = same && v == S.h_want[g];
    S.h_want[g] = v;
    if (v) S.active_bytes += (double)S.bytes[g];
  }
  if (same) return;
  // the stream is idle here (callers synchronise before selecting), so the
  // host vector may be reused by the next call
  GDSW_HIP(hipMemcpyAsync(S.d_want, S.h_want.data(), S.count * sizeof(int32_t), hipMemcpyHostToDevice, st));
  GDSW_HIP(hipStreamSynchronize(st));
}

}  // namespace

void batch_build(Batch& b, hipStream_t st) {
  build_set(b, b.s1, true, st);
  build_set(b, b.s2, false, st);
  GDSW_HIP(hipHostMalloc((void**)&b.h_pinned, std::max<size_t>(1, 4 * b.m.size()) * sizeof(double),
                         hipHostMallocDefault));
  // four lanes: the number of hardware queues a process gets by default
  const size_t nl = std::max<size_t>(1, std::min<size_t>(4, b.m.size()));
  b.lanes.assign(nl, nullptr);
  b.join.assign(nl, nullptr);
  for (size_t l = 0; l < nl; ++l) {
    GDSW_HIP(hipStreamCreateWithFlags(&b.lanes[l], hipStreamNonBlocking));
    GDSW_HIP(hipEventCreateWithFlags(&b.join[l], hipEventDisableTiming));
  }
  GDSW_HIP(hipEventCreateWithFlags(&b.fork, hipEventDisableTiming));
  GDSW_HIP(hipStreamSynchronize(st));
}

void batch_fork(Batch& b, hipStream_t st) {
  GDSW_HIP(hipEventRecord(b.fork, st));
  for (hipStream_t l : b.lanes) GDSW_HIP(hipStreamWaitEvent(l, b.fork, 0));
}

void batch_join(Batch& b, hipStream_t st) {
  for (size_t l = 0; l < b.lanes.size(); ++l) {
    GDSW_HIP(hipEventRecord(b.join[l], b.lanes[l]));
    GDSW_HIP(hipStreamWaitEvent(st, b.join[l], 0));
  }
}

bool batch_learned(const Context& c) { return c.local_solver != 0 && c.learned && c.learned->S > 0; }

void batch_block_rest(Context& c, const double* r, hipStream_t ls) {
  if (c.solve_mode == SOLVE_BLOCK) block_local_rest(c, ls, nullptr, block_assembles_restriction(c) ? r : nullptr);
}

void batch_save_interior(Context& c, hipStream_t ls) {
  copy_segments(learned_gridmap(c), c.learned->S, c.d_w, c.learned->d_rsave, nullptr, ls);
}

void batch_learned_solves(Batch& b, const std::vector<char>& on, hipStream_t st) {
  bool any = false;
  batch_fork(b, st);
  for (size_t k = 0; k < b.m.size(); ++k) {
    Context& c = *b.m[k];
    if (!on[k] || !batch_learned(c)) continue;
    if (c.local_solver == 1) {
      learned_interior_begin(c, batch_lane(b, k));
      any = true;
    } else {
      zero_segments(learned_gridmap(c), c.learned->S, c.d_w, batch_lane(b, k));
    }
  }
  batch_join(b, st);
  if (!any) return;
  GDSW_HIP(hipStreamSynchronize(st));
  batch_fork(b, st);
  for (size_t k = 0; k < b.m.size(); ++k)
    if (on[k] && batch_learned(*b.m[k]) && b.m[k]->local_solver == 1)
      learned_interior_finish(*b.m[k], batch_lane(b, k));
  batch_join(b, st);
}

void batch_select(Batch& b, const std::vector<char>& member_active, hipStream_t st) {
  select_set(b, b.s1, member_active, true, st);
  select_set(b, b.s2, member_active, false, st);
}

void batch_local_solve(Batch& b, hipStream_t st) {
  for (BatchSet* S : {&b.s1, &b.s2}) {
    if (!S->count) continue;
    KernelTimer* tm = S == &b.s1 ? &b.timer : nullptr;
    const double bytes = S == &b.s1 ? S->active_bytes : 0.0;
    if (S->sym)
      symv_desc_launch(S->prec, S->d_desc, S->plan, S->d_partial, S->partial_len, st, S->d_want, tm, bytes, S->nc);
    else
      gemv_desc_launch(S->prec, S->d_desc, S->plan, GEMV_CW, S->d_partial, st, S->d_want, tm, bytes);
  }
}

void batch_drop_graphs(Batch& b) {
  for (auto& kv : b.graphs)
    if (kv.second) (void)hipGraphExecDestroy(kv.second);
  b.graphs.clear();
  b.graph_V.clear();
}

void batch_release(Batch& b) {
  batch_drop_graphs(b);
  if (b.gstream) (void)hipStreamDestroy(b.gstream);
  b.gstream = nullptr;
  for (auto& e : b.timer.ev) (void)hipEventDestroy(e);
  b.timer.ev.clear();
  for (hipStream_t l : b.lanes) (void)hipStreamSynchronize(l);
  if (b.h_pinned) (void)hipHostFree(b.h_pinned);
  b.h_pinned = nullptr;
  for (hipStream_t l : b.lanes) (void)hipStreamDestroy(l);
  for (hipEvent_t e : b.join) (void)hipEventDestroy(e);
  if (b.fork) (void)hipEventDestroy(b.fork);
  b.lanes.clear();
  b.join.clear();
  b.fork = nullptr;
  b.arena.release_all();
}

void apply_precond_batch(Batch& b, const double* const* r, double* const* z, hipStream_t st) {
  const std::vector<char> all(b.m.size(), 1);
  batch_select(b, all, st);
  batch_fork(b, st);
  for (size_t k = 0; k < b.m.size(); ++k) {
    apply_pre(*b.m[k], r[k], batch_lane(b, k));
    if (batch_learned(*b.m[k])) batch_save_interior(*b.m[k], batch_lane(b, k));
  }
  batch_join(b, st);
  batch_local_solve(b, st);
  batch_learned_solves(b, all, st);
  batch_fork(b, st);
  for (size_t k = 0; k < b.m.size(); ++k) {
    batch_block_rest(*b.m[k], r[k], batch_lane(b, k));
    apply_post(*b.m[k], z[k], batch_lane(b, k));
  }
  batch_join(b, st);
  GDSW_HIP(hipGetLastError());
}

}  // namespace gdsw
