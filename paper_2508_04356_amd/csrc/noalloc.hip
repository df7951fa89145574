// Preconditioner apply that allocates nothing (gdsw_apply_precond_noalloc).
//
// The one- and two-launch products of the explicit inverses (full or upper
// tiles) write partial sums that a second launch adds up per row block; the
// context keeps a buffer for them, allocated at setup.  This variant takes
// that scratch from a file-scope device array instead, so a caller that must
// not allocate (stream capture, serving loops) gets the same kernels, the same
// summation orders and therefore the same results bit for bit.
//
// The array lives once per device for the whole process.  Host code never
// passes its name to a kernel (in host code the name is only a stand-in for
// the device symbol): the device address is looked up once per device with
// hipGetSymbolAddress, at gdsw_setup, and kept in a per-device table.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/gdsw.h"
#include "context.h"
#include "kernels.h"

#ifndef GDSW_NOALLOC_SCRATCH_BYTES
#define GDSW_NOALLOC_SCRATCH_BYTES (128ull << 20)  // 128 MiB per device
#endif

namespace gdsw {
namespace {

constexpr uint64_t SCRATCH_BYTES = GDSW_NOALLOC_SCRATCH_BYTES;
static_assert(SCRATCH_BYTES % 256 == 0, "scratch size must be a multiple of 256 bytes");

static __device__ __align__(256) double scratch[SCRATCH_BYTES / sizeof(double)];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};

}  // namespace

// Looks up the device address of `scratch` on the current device (once per
// device) and returns it; throws on a HIP error.
double* noalloc_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) throw StatusError{6, "device index beyond the scratch table"};
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    int cur = -1;
    GDSW_HIP(hipGetDevice(&cur));
    if (cur != device) throw StatusError{1, "scratch lookup needs the context's device to be current"};
    void* p = nullptr;
    GDSW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw StatusError{5, "hipGetSymbolAddress returned NULL for the scratch array"};
    g_ptr[device] = static_cast<double*>(p);
  }
  return g_ptr[device];
}

uint64_t noalloc_scratch_bytes() { return SCRATCH_BYTES; }

// Partial-sum doubles the product of `fs` needs (0 for an empty set).
static int64_t partial_need(const FactorSet& fs) { return fs.count == 0 ? 0 : fs.partial_len; }

void apply_precond_noalloc(Context& ctx, const double* r, double* z, hipStream_t st) {
  if (ctx.solve_mode != SOLVE_INVERSE && ctx.solve_mode != SOLVE_SYM && ctx.solve_mode != SOLVE_BLOCK)
    throw StatusError{6, "the no-allocation apply covers the inverse, symmetric and block local solves"};
  if (ctx.local_solver != 0)
    throw StatusError{6, "the no-allocation apply covers the exact local solves (local solver 0)"};
  const int64_t need =
      std::max(std::max(partial_need(ctx.L1), partial_need(ctx.HI)),
               ctx.solve_mode == SOLVE_BLOCK ? partial_need(ctx.LP) : (int64_t)0);
  if ((uint64_t)need * sizeof(double) > SCRATCH_BYTES)
    throw StatusError{1, "the no-allocation apply needs " + std::to_string((uint64_t)need * sizeof(double)) +
                             " bytes of scratch; the static buffer holds " + std::to_string(SCRATCH_BYTES)};
  // every partial slot the sums read is written earlier in the same call,
  // so the array needs no clearing between calls
  double* part = noalloc_scratch(ctx.device);
  apply_pre(ctx, r, st);
  // the sets run one after the other on `st`, so they share the scratch
  if (ctx.solve_mode == SOLVE_BLOCK) block_local_solve(ctx, st, part, block_assembles_restriction(ctx) ? r : nullptr);
  for (const FactorSet* fs : {&ctx.L1, &ctx.HI}) {
    if (fs == &ctx.L1 && ctx.solve_mode == SOLVE_BLOCK) continue;
    if (fs->count == 0 || fs->gemv.empty()) continue;
    if (!fs->d_desc) throw StatusError{5, "inverse set used before its descriptors were built"};
    if (fs->mode == SOLVE_INVERSE)
      gemv_desc_launch(fs->prec, fs->d_desc, fs->gemv[0], fs->cw, part, st, nullptr, nullptr, 0.0);
    else
      symv_desc_launch(fs->prec, fs->d_desc, fs->gemv[0], part, fs->partial_len, st, nullptr, nullptr, 0.0);
  }
  apply_post(ctx, z, st);
  GDSW_HIP(hipGetLastError());
}

}  // namespace gdsw
