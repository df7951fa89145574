// Device-side context of one GDSW problem (internal to the library).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "problem.h"

namespace gdsw {

struct HipError {
  hipError_t err;
  std::string where;
};

#define GDSW_HIP(call)                                                          \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) throw ::gdsw::HipError{e_, std::string(#call) + " at " \
                                                  + __FILE__ + ":" + std::to_string(__LINE__)}; \
  } while (0)

struct StatusError {  // a gdsw_status with a message
  int status;
  std::string msg;
};

// Device allocation tracker: every buffer of a context goes through it so
// that the budget check and the reported device footprint are exact.
struct DeviceArena {
  uint64_t budget = 0;
  uint64_t used = 0;
  std::vector<void*> ptrs;
  std::vector<uint64_t> sizes;
  void* alloc(uint64_t bytes);
  void free(void* p);
  void release_all();
  ~DeviceArena() { release_all(); }
};

template <class T>
T* dalloc(DeviceArena& A, uint64_t count) {
  return static_cast<T*>(A.alloc(count * sizeof(T)));
}
template <class T, class Al>
T* dupload(DeviceArena& A, const std::vector<T, Al>& v, hipStream_t st) {
  T* p = dalloc<T>(A, v.empty() ? 1 : v.size());
  if (!v.empty()) GDSW_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return p;
}

enum Precision { P_FP64 = 0, P_FP32 = 1, P_BF16 = 2 };
inline size_t elem_size(int prec) { return prec == P_FP64 ? 8 : (prec == P_FP32 ? 4 : 2); }

// A batch of dense square matrices factored as A = L U without pivoting and
// solved by the blocked triangular-solve kernels.  Each matrix is stored
// column-major in a zero-padded npad x npad block (npad = n rounded up to the
// tile), and the inverses of its diagonal tiles (unit-lower L^-1 strictly
// below the diagonal, U^-1 on and above it) are kept separately in `dinv`.
constexpr int SOLVE_INVERSE = 0;  // explicit inverse, applied as a dense matrix-vector product
constexpr int SOLVE_TRSV = 1;     // LU factors, blocked forward/backward substitution
constexpr int SOLVE_SYM = 2;      // symmetric explicit inverse, upper 64 x 64 tiles only
constexpr int SOLVE_BLOCK = 3;    // velocity block I_3 (x) L and Schur complement (block.hip)
#ifndef GDSW_GEMV_CW
#define GDSW_GEMV_CW 1024
#endif
constexpr int GEMV_CW = GDSW_GEMV_CW;  // columns per matrix-vector work item

// One stored inverse for the matrix-vector kernels: its entries (column-major,
// leading dimension np, in the set's precision) and its segment of a work
// vector (n entries, overwritten with the product).  The symmetric-tile
// kernels can apply the matrix to NC vectors at once: vector k at x + k vs.
struct GemvDesc {
  const void* a;
  double* x;
  int32_t n, np;
  int32_t vs = 0;       // stride between the vectors of a several-vector product
  double* y = nullptr;  // symmetric products: y -= M x instead of x <- M x
};

// HIP events around each launch of a set's dominant solve kernel (slot 0),
// for measuring its average duration inside a timed region.
struct KernelTimer {
  static constexpr int CAP = 16384;  // launch pairs recorded before it stops
  bool on = false;
  int used = 0;
  double bytes = 0.0;                // algorithmic bytes of the recorded launches
  std::vector<hipEvent_t> ev;        // 2 * CAP events, created on first enable
};

// Launches kernel<<<grid, block, 0, st>>>(args...).  With a timer that is on
// and not full, the dispatch itself stamps the kernel's start and end into the
// timer's next event pair (hipExtLaunchKernel): no marker packets go between
// the launches, which cost about 6 us of idle time each on MI355X.
template <typename... P, typename... Args>
void timed_launch(KernelTimer* tm, double bytes, void (*kernel)(P...), dim3 grid, dim3 block, hipStream_t st,
                  Args... args) {
  if (tm && tm->on && tm->used < KernelTimer::CAP) {
    std::tuple<std::decay_t<P>...> a(args...);  // the kernel's own parameter types
    void* ptrs[sizeof...(P) > 0 ? sizeof...(P) : 1];
    std::apply([&](auto&... v) {
      int i = 0;
      ((ptrs[i++] = (void*)&v), ...);
    }, a);
    GDSW_HIP(hipExtLaunchKernel((const void*)kernel, grid, block, ptrs, 0, st, tm->ev[2 * tm->used],
                                tm->ev[2 * tm->used + 1], 0));
    ++tm->used;
    tm->bytes += bytes;
  } else {
    kernel<<<grid, block, 0, st>>>(args...);
  }
}

struct FactorSet {
  int mode = SOLVE_INVERSE;
  KernelTimer* timer = nullptr;      // set while timing is enabled
  int prec = P_FP64;
  int nb = 128;                       // tile
  int count = 0;
  std::vector<int32_t> n, npad, nblk; // host copies
  std::vector<int64_t> off, doff, xoff;
  int64_t total_elems = 0, total_dinv = 0, total_x = 0;
  int max_nblk = 0;
  void* store = nullptr;              // factors (prec)
  void* dinv = nullptr;               // diagonal tile inverses (fp64 or fp32)
  int32_t* d_n = nullptr;
  int32_t* d_npad = nullptr;
  int32_t* d_nblk = nullptr;
  int64_t* d_off = nullptr;
  int64_t* d_doff = nullptr;
  int64_t* d_xoff = nullptr;
  // launch schedules: items (factor, J, K, mode) of every launch; factors run
  // their 2*nblk sweeps with phase offsets so that launches carry similar work.
  // Slot 0 covers every factor; further slots cover subsets (learned solve).
  struct Schedule {
    std::vector<int32_t> step_start;
    int4* d_items = nullptr;
  };
  int phases = 1;
  int waves = 4;                      // work-group size of the solve kernel: 64 * waves
  std::vector<Schedule> sched;
  // explicit-inverse mode: work items of the two matrix-vector kernels per
  // slot (partials: (f, r0, c0, p); sums: (f, r0, p0, count)) and the
  // partial-sum buffer (64 * E doubles per item of the largest slot)
  struct GemvPlan {
    int n1 = 0, n2 = 0;
    int4* d_items1 = nullptr;
    int4* d_items2 = nullptr;
    int run = 2;   // symmetric tiles: stored tiles per work item (1 or 2)
    int xcd = 0;   // symmetric tiles: XCD-contiguous work-group order
  };
  std::vector<GemvPlan> gemv;
  int cw = GEMV_CW;                  // columns per partial-product item (512, 1024 or 2048)
  int sym_run = 2;                   // symmetric tiles per item, and the order (-1: by precision)
  int sym_xcd = -1;
  GemvDesc* d_desc = nullptr;        // per factor, built once the store and work vector exist
  double* d_partial = nullptr;
  int64_t partial_len = 0;
  GemvPlan gemm;                     // several right-hand sides (all factors)
  int gemm_rb = 0, gemm_cw = 0;      // its rows and summation columns per item
  bool gemm_lds = false;             // FP64: LDS-staged kernel (few matrices)
  int gemm_cw_force = 0;             // autotuner's choices (0 / -1: by shape)
  int gemm_lds_force = -1;
  void* d_partial_m = nullptr;       // 32 * rows partial sums per gemm item
  int max_np = 0;                    // BF16 products: right-hand sides as BF16,
  int64_t* d_xpoff = nullptr;        //   xb[32 * xpoff[f] + j * npad[f] + row]
  uint16_t* d_xb = nullptr;
  uint64_t gen = 0;                    // bumped by every re-plan (item arrays, partial buffers)
  int nc = 1;                          // symmetric storage: vectors per matrix (1, or 3 for the
                                       // velocity blocks of the block local solve)
  uint64_t algorithmic_bytes() const;  // sum n^2 * sizeof(prec)
  uint64_t alg_bytes = 0;              // algorithmic_bytes(), set when planned
  int64_t launches() const;            // solve kernel launches per pass (slot 0)
};

struct LearnedSolve;

// Block local solve (SOLVE_BLOCK): the level-1 set L1 holds L_i^-1 (upper
// tiles, three component vectors per matrix: x, y, z at vs = npad apart in
// the work vector), LP holds S_i^-1 (and the coarse inverse with two levels);
// B_i as flat row lists over absolute work-vector positions.
struct BlockSolve {
  int64_t n_prow = 0;                // pressure rows of every local problem
  int32_t* d_prow_pos = nullptr;     // their work positions
  int64_t* d_bm_ptr = nullptr;       // B rows: velocity positions and values
  int32_t* d_bm_pos = nullptr;
  double* d_bm_val = nullptr;
  int64_t n_vrow = 0;                // velocity rows (component, node) of every local problem
  int32_t* d_vrow_pos = nullptr;
  int64_t* d_bt_ptr = nullptr;       // B^T rows: pressure positions and values
  int32_t* d_bt_pos = nullptr;
  double* d_bt_val = nullptr;
  double* d_w2 = nullptr;            // second work vector (B^T p, then L^-1 B^T p), n_w1
  GemvDesc* d_desc2 = nullptr;       // L1's matrices against d_w2
  uint64_t b_bytes = 0;              // bytes of the B row lists an apply reads
  // u = U1 - W p with W_i = K_i^-1 B_i^T kept from the setup (3 npad_i x np_i,
  // column-major, local precision) instead of a second pass over L_i^-1,
  // where W is the smaller read
  bool use_w = false;
  void* d_W = nullptr;
  struct WItem* d_witems = nullptr;  // one per (subdomain, block of rows)
  int n_witems = 0;
  uint64_t w_bytes = 0;              // algorithmic bytes of W
};

// Work item of the W p product: rows r0 .. r0 + 64 E - 1 of W_i.
struct WItem {
  int64_t woff;   // element offset of W_i in the store
  int64_t voff;   // work position of row 0 (velocity segment of subdomain i)
  int64_t poff;   // work position of p_i (pressure segment)
  int32_t rows;   // 3 npad_i
  int32_t np;     // columns
  int32_t r0;
  int32_t pad;
};
constexpr int WP_MAX_NP = 1024;      // pressure DOFs per local problem on the W path

struct Context {
  Problem P;
  bool host_only = false;
  int device = 0;
  DeviceArena arena;
  std::string last_error;
  int local_prec = P_FP64;
  int solve_mode = SOLVE_INVERSE;
  int nb = 128;
  KernelTimer timer;

  // several right-hand sides (two levels, explicit inverses): up to max_rhs
  // columns per pass, interleaved (entry (d, j) at x[d * max_rhs + j])
  // captured FGMRES iterations (one executable graph per basis index)
  struct IterGraphs {
    int restart = 0;
    const double* V = nullptr;       // workspace the graphs were captured against
    uint64_t gen1 = 0, gen2 = 0;     // plan generations of L1 / HI they were captured against
    hipStream_t stream = nullptr;    // own stream when the caller passes the default one
    std::vector<hipGraphExec_t> exec;
  } graphs;

  int max_rhs = 1;
  double* d_wm = nullptr;          // n_w x max_rhs work vectors
  double* d_xin = nullptr;         // n_free x max_rhs (ABI column-major input, interleaved)
  double* d_xout = nullptr;
  double* d_pair_tm = nullptr;     // n_pairs x max_rhs per-pair restriction sums
  struct MultiKrylov {
    int restart = 0, K = 0, nblocks = 0;
    int64_t ldv = 0;               // n_free * K
    double *V = nullptr, *Z = nullptr, *H = nullptr, *g = nullptr, *cs = nullptr, *sn = nullptr;
    double *h1 = nullptr, *h2 = nullptr, *part = nullptr, *scal = nullptr, *t1 = nullptr, *t2 = nullptr;
    double *b = nullptr, *x = nullptr, *y = nullptr;
    int32_t* active = nullptr;
    double* h_pinned = nullptr;    // 4 * K doubles
    int32_t* h_active = nullptr;   // K ints (pinned)
  } mk;

  // system matrix (free DOFs)
  int32_t* d_rowptr = nullptr;
  int32_t* d_col = nullptr;
  double* d_val = nullptr;
  double* d_rhs = nullptr;
  int64_t* d_full_index = nullptr;
  double* d_dirichlet_full = nullptr;

  // level-1 local solves
  FactorSet L1;      // level-1 local factors (local_prec)
  FactorSet HI;      // FP64: coarse (two levels) or level-2 + level-3 factors
  FactorSet LP;      // block local solve: Schur complement inverses (+ coarse with two levels)
  BlockSolve blk;
  bool merged = false;  // true when L1 also holds the coarse factor(s)
  int32_t* d_gidx = nullptr;      // wbuf position -> global DOF (or -1)
  int64_t n_w1 = 0;               // length of the level-1 work segment
  int32_t* d_inv_ptr = nullptr;   // per DOF: range into d_inv_pos
  int64_t* d_inv_pos = nullptr;   // wbuf positions of each DOF's local copies
  double* d_w = nullptr;          // work vector (all factor sets)
  int64_t n_w = 0;

  // coarse space (level 2 of eq. 2.2 / 2.5)
  int Nc = 0;
  int32_t* d_gamma_col = nullptr;  // per DOF: coarse column or -1
  int32_t* d_I_ptr = nullptr;      // interior lists
  int32_t* d_I_idx = nullptr;
  int32_t* d_I_sub = nullptr;      // per interior DOF position: subdomain
  int32_t* d_dof_ipos = nullptr;   // per DOF: position in the concatenated interior list or -1
  int32_t* d_C_ptr = nullptr;      // adjacent coarse columns per subdomain
  int32_t* d_C_idx = nullptr;
  int64_t* d_phi_off = nullptr;    // per subdomain offset of Phi_I (|I_i| x |C_i|)
  double* d_phi_cm = nullptr;      // Phi_I column-major (ld = |I_i|)
  double* d_phi_rm = nullptr;      // Phi_I row-major (ld = |C_i|)
  int32_t* d_cg_ptr = nullptr;     // per coarse column: its Gamma DOFs
  int32_t* d_cg_dof = nullptr;
  int32_t* d_cs_ptr = nullptr;     // per coarse column: (subdomain, local column) pairs
  int32_t* d_cs_sub = nullptr;
  int32_t* d_cs_lc = nullptr;
  double* d_A0 = nullptr;          // dense A_0, row-major Nc x Nc
  std::vector<int32_t> coarse_perm;  // factor position -> coarse column (velocity first)
  int32_t* d_coarse_pinv = nullptr;  // coarse column -> wbuf position
  int64_t coarse_xoff = 0;
  int n_pairs = 0;                 // (subdomain, local coarse column) pairs
  int max_ni = 0;                  // largest interior set |I_i|
  int32_t* d_outer = nullptr;      // DOFs in no interior set (the interface), ascending
  int64_t n_outer = 0;
  double* d_pair_t = nullptr;      // per pair: Phi_I column^T r (restriction)
  int32_t* d_pair_of = nullptr;    // per (subdomain i, local column j) at C_ptr[i] + j: its pair index
  int phi_cb = 0, phi_nblk = 0;    // restriction work-groups per (subdomain, cb columns); 0: one per pair
  double* d_r0 = nullptr;          // coarse vectors (three levels)
  double* d_y0 = nullptr;

  // three levels
  int Nc3 = 0;
  int n_sub2 = 0;
  int32_t* d_g2idx = nullptr;      // level-2 work positions -> coarse index
  int32_t* d_inv2_ptr = nullptr;
  int64_t* d_inv2_pos = nullptr;
  // Phi^(3) in the layout of the level-1 basis, on the coarse DOFs: per
  // subregion j a column-major |I2_j| x |C3_j| block, the interface part an
  // indicator (coarse_view3)
  int32_t* d_gcol3 = nullptr;      // per coarse DOF: its level-3 column (interface), or -1
  int32_t* d_ipos3 = nullptr;      // per coarse DOF: position in the concatenated interiors, or -1
  int32_t* d_i2_sub = nullptr;     // per interior position: subregion
  int32_t* d_i2_ptr = nullptr;     // interior coarse DOFs of each subregion
  int32_t* d_i2_idx = nullptr;
  int32_t* d_c3_ptr = nullptr;     // level-3 columns adjacent to each subregion
  int32_t* d_c3_idx = nullptr;
  int64_t* d_off2 = nullptr;       // offset of each subregion's block
  double* d_phi3_cm = nullptr;
  int32_t* d_cg3_ptr = nullptr;    // per level-3 column: its interface coarse DOFs
  int32_t* d_cg3_dof = nullptr;
  int32_t* d_cs3_ptr = nullptr;    // per level-3 column: (subregion, local column) pairs
  int32_t* d_cs3_sub = nullptr;
  int32_t* d_cs3_lc = nullptr;
  int n_pairs3 = 0, max_ni2 = 0;
  double* d_pair_t3 = nullptr;
  int32_t* d_outer3 = nullptr;     // coarse DOFs in no subregion interior
  int64_t n_outer3 = 0;
  int32_t* d_c3_pinv = nullptr;    // level-3 column -> wbuf position
  double* d_A03 = nullptr;

  // Krylov workspace
  int restart = 0;
  double* d_V = nullptr;
  double* d_Z = nullptr;
  double* d_H = nullptr;
  double* d_g = nullptr;
  double* d_cs = nullptr;
  double* d_sn = nullptr;
  double* d_hv = nullptr;          // CGS coefficients
  double* d_part = nullptr;        // partial sums
  double* d_scal = nullptr;        // scalars: norms, flags
  double* d_t1 = nullptr;          // n-vectors
  double* d_t2 = nullptr;
  double* h_pinned = nullptr;      // pinned host scalars
  double* d_pinned = nullptr;      // their device view (kernels write the FGMRES records there)
  hipEvent_t it_ev[2] = {nullptr, nullptr};  // end of FGMRES iteration j, slot j % 2
  int64_t ldv = 0;
  int n_part_blocks = 0;

  // learned local solve (interior subdomains)
  int local_solver = 0;            // 0 LU, 1 learned with LU fallback, 2 none (ablation)
  LearnedSolve* learned = nullptr;

  // diagnostics
  double t_symbolic = 0, t_numeric = 0;
  uint64_t factor_bytes = 0, coarse_bytes = 0;
};

// numeric setup and operators (setup.hip / solve.hip)
void plan_schedule(FactorSet& fs, int phases, DeviceArena& A, hipStream_t st, int slot = 0,
                   const std::vector<char>* include = nullptr);
void device_setup(Context& ctx, hipStream_t st, uint64_t budget, int nb);
void apply_precond(Context& ctx, const double* r, double* z, hipStream_t st, hipEvent_t* ev = nullptr);
// the two halves of apply_precond around the local and coarse solves:
// right-hand sides into the work vector, and the sum back into z
void apply_pre(Context& ctx, const double* r, hipStream_t st);
void apply_post(Context& ctx, double* z, hipStream_t st);
void spmv(Context& ctx, const double* x, double* y, hipStream_t st);
// apply_precond with the product's partial sums in the library's static
// per-device scratch array instead of the context's buffer (noalloc.hip)
void apply_precond_noalloc(Context& ctx, const double* r, double* z, hipStream_t st);
// block local solve of every level-1 subdomain in the work vector (block.hip)
// part (or null: the sets' own buffers): partial sums for every product;
// restrict_r (or null): the vector whose coarse restriction apply_pre left
// unassembled (two levels), assembled in the launch of the B row products
void block_local_solve(Context& ctx, hipStream_t st, double* part = nullptr, const double* restrict_r = nullptr);
// the block local solve after its velocity-block product (U1 already in the
// work vector): the B row products, the Schur complement and coarse
// products, and u = U1 - W p (or the second pass); for a batch whose merged
// launch formed U1 of every member
void block_local_rest(Context& ctx, hipStream_t st, double* part = nullptr, const double* restrict_r = nullptr);
// two levels with the block solve: the coarse restriction is assembled
// inside block_local_solve
bool block_assembles_restriction(const Context& ctx);
int wp_rows_per_item(int prec);
void wp_sub(int prec, const void* W, const WItem* items, int n_items, double* w, KernelTimer* tm, double bytes,
            hipStream_t st);
void block_fill_bt(const int32_t* rowptr, const int32_t* col, const double* val, int64_t n_u,
                   const int32_t* vx_ptr, const int32_t* vx, const int32_t* pr_ptr, const int32_t* pr,
                   const int32_t* npv, const int64_t* off, int f0, int cnt, int max_np, double* bt, hipStream_t st);
void copy_blocks(const double* src, const int64_t* soff, const int32_t* n, int count, int64_t max_elems,
                 double* base, const int64_t* doff, const int32_t* ld, hipStream_t st);
double* noalloc_scratch(int device);  // device address of the array (looked up once per device)
uint64_t noalloc_scratch_bytes();
struct FgmresResult {
  int iterations = 0, restarts = 0;
  double rel = 0, true_rel = 0;
  bool converged = false;
};
FgmresResult fgmres(Context& ctx, const double* b, double* x, double rtol, int restart, int max_it,
                    bool use_graph, hipStream_t st, double* history = nullptr, int history_len = 0);
void expand_solution(const Context& ctx, const double* xf, double* xfull, hipStream_t st);
void release_graphs(Context& ctx);

// A batch of independent problems (own contexts) whose local and coarse
// inverse products run as one launch pair per level over all members, in
// longest-first order of the matrices (batch.hip).
struct BatchSet {
  int prec = P_FP64;
  int count = 0;                     // matrices over all members
  std::vector<int> owner;            // member of each matrix
  std::vector<int> fidx;             // its factor index within the member
  std::vector<uint64_t> bytes;       // algorithmic bytes of each matrix
  GemvDesc* d_desc = nullptr;
  FactorSet::GemvPlan plan;
  double* d_partial = nullptr;
  int64_t partial_len = 0;
  bool sym = false;                  // symmetric tile storage (symv kernels)
  int nc = 1;                        // vectors per matrix (3: the block solve's velocity-block inverses)
  int32_t* d_want = nullptr;
  std::vector<int32_t> h_want;       // host copy of the last upload
  double active_bytes = 0.0;
};

struct Batch {
  std::vector<Context*> m;
  DeviceArena arena;
  BatchSet s1, s2;                   // level-1 inverses; coarse-level inverses
  KernelTimer timer;                 // times the level-1 partial-product launches
  double* h_pinned = nullptr;        // 4 doubles per member, read-back staging
  // per-member work (gathers, scatters, SpMV, orthogonalisation) runs on
  // lanes[k % lanes.size()], forked from and joined back into the caller's
  // stream around each phase, so that the members' small kernels overlap
  std::vector<hipStream_t> lanes;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  // graph replays of the lockstep iteration, one per (basis index, members
  // in the cycle); dropped when a member's Krylov workspace moves
  std::map<std::pair<int, std::vector<char>>, hipGraphExec_t> graphs;
  std::vector<double*> graph_V;
  int graph_restart = 0;
  hipStream_t gstream = nullptr;     // capture stream when the caller passes the null stream
};

// Make every lane wait for the work queued on st so far / make st wait for
// everything queued on the lanes.
void batch_fork(Batch& b, hipStream_t st);
void batch_join(Batch& b, hipStream_t st);
inline hipStream_t batch_lane(const Batch& b, size_t k) { return b.lanes[k % b.lanes.size()]; }
// Members whose interior subdomains use the learned solve (local_solver 1)
// or none (2): the merged product skips those matrices; their inputs are
// saved after the gathers and the network (or zero) fills them in after it.
bool batch_learned(const Context& c);
// a block-solve member's work after the merged velocity-block product (r:
// the vector being preconditioned); nothing for the other local solves
void batch_block_rest(Context& c, const double* r, hipStream_t ls);
void batch_save_interior(Context& c, hipStream_t ls);
void batch_learned_solves(Batch& b, const std::vector<char>& on, hipStream_t st);

void batch_build(Batch& b, hipStream_t st);
// member_active[k] selects the members whose matrices the next products touch
void batch_select(Batch& b, const std::vector<char>& member_active, hipStream_t st);
void batch_local_solve(Batch& b, hipStream_t st);
void batch_release(Batch& b);
void apply_precond_batch(Batch& b, const double* const* r, double* const* z, hipStream_t st);
std::vector<FgmresResult> fgmres_batch(Batch& b, const double* const* bvec, double* const* x, double rtol,
                                       int restart, int max_it, hipStream_t st, bool use_graph = false);
void batch_drop_graphs(Batch& b);

// several right-hand sides (solve_multi.hip): blocks of K <= max_rhs
// interleaved columns (entry (d, j) at x[d * K + j])
void plan_gemm(FactorSet& fs, DeviceArena& A, hipStream_t st);
// descriptors of the set's inverses against the work vector w (device_setup)
std::vector<GemvDesc> gemv_descs(const FactorSet& fs, double* w);
bool multi_supported(const Context& ctx);
void ensure_multi_workspace(Context& ctx, int restart, int K);
void apply_precond_multi(Context& ctx, const double* r, double* z, int K, hipStream_t st);
std::vector<FgmresResult> fgmres_multi(Context& ctx, const double* b_il, double* x_il, int K, double rtol,
                                       int restart, int max_it, hipStream_t st);

}  // namespace gdsw
