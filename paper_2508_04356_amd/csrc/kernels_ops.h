// Coarse-space kernels: views of the device index structures and launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace gdsw {

// Device index structures of the coarse basis Phi (eq. 2.4), passed by value.
struct CoarseView {
  const int32_t* gamma_col;  // per DOF: coarse column of its interface entity/field, or -1
  const int32_t* dof_ipos;   // per DOF: position in the concatenated interior list, or -1
  const int32_t* I_sub;      // per interior position: subdomain
  const int32_t* I_ptr;      // interior list offsets per subdomain
  const int32_t* I_idx;      // interior DOFs (sorted per subdomain)
  const int32_t* C_ptr;      // adjacent coarse columns per subdomain
  const int32_t* C_idx;
  const int64_t* phi_off;    // offset of Phi_I^(i) (|I_i| x |C_i|)
  const double* phi_cm;      // column-major Phi_I
  const double* phi_rm;      // row-major Phi_I
  const int32_t* cg_ptr;     // per coarse column: its Gamma DOFs
  const int32_t* cg_dof;
  const int32_t* cs_ptr;     // per coarse column: (subdomain, local column) pairs, ascending subdomain
  const int32_t* cs_sub;
  const int32_t* cs_lc;
};

// The coarse-basis arrays of a context.
CoarseView coarse_view(const Context& c);
// Three levels: the level-3 basis Phi^(3) on the coarse DOFs in the same
// layout (subregions for subdomains, coarse DOFs for DOFs).
CoarseView coarse_view3(const Context& c);

// Closed subdomain boxes D_i, used for A_0 = sum_i Phi_box_i^T A_own_i
// Phi_box_i, where A_own_i holds the nonzeros box i owns: a nonzero belongs
// to the lowest-numbered box holding both of its DOFs.
struct BoxView {
  const int32_t* D_ptr;
  const int32_t* D_idx;      // each box's DOFs, ascending
  const int32_t* D_sub;
  const int64_t* box_off;    // offset of the |D_i| x |C_i| blocks
};

// The boxes holding a DOF, from which the owner of a nonzero follows.
// Structured problems (blo != null): per DOF and axis the range of box
// indices holding its node, boxes numbered x + m (y + m z); algebraic
// problems: per DOF the ascending list of subdomains holding it.
struct OwnerMap {
  const int32_t* blo;
  const int32_t* bhi;
  int m;
  const int64_t* sub_ptr;
  const int32_t* sub_idx;
};

// z = sum_i R_i^T y_i + Phi y0.  With nsub > 0 the Phi_I y0 term runs as a
// second, per-subdomain kernel over the column-major Phi_I (max_ni: largest
// interior set); the result is the same either way.
// With outer (the n_outer DOFs in no interior set) both run in one launch.
void scatter_prolong(int64_t n, const int32_t* inv_ptr, const int64_t* inv_pos, const double* w,
                     const CoarseView& cv, const double* y0, const int32_t* y0_pos, double* z, hipStream_t st,
                     int nsub = 0, int max_ni = 0, const int32_t* outer = nullptr, int64_t n_outer = 0);
// out[pos[c]] = (Phi^T r)[c].  With t (n_pairs doubles, one per (subdomain,
// local column) pair) the interior part is first reduced per pair, then
// assembled per column in ascending subdomain order.
// With gcount > 0 the same launch also performs gather(gcount, gidx, r, gdst)
// (before the restriction is assembled).  assemble = false leaves the
// per-column assembly (restrict_assemble_column) to a later launch of the
// caller's.
// Per-subdomain layout of the pair sums (restrict_coarse with t): a
// work-group per (subdomain, block of cb local columns) instead of one per
// pair; pair_of[C_ptr[i] + j] = the pair index of (subdomain i, local column
// j); max_ni: the largest interior set (its r values are staged in LDS).
struct PairBlocks {
  const int32_t* pair_of = nullptr;
  int nsub = 0, nblk = 0, cb = 0, max_ni = 0;
};
void restrict_coarse(int nc, const CoarseView& cv, const double* r, double* out, const int32_t* out_pos,
                     hipStream_t st, int n_pairs = 0, double* t = nullptr, int64_t gcount = 0,
                     const int32_t* gidx = nullptr, double* gdst = nullptr, bool assemble = true,
                     const PairBlocks* blocks = nullptr);

// out[c] = sum of r over the Gamma DOFs of coarse column c + sum_e t[e] over
// its (subdomain, local column) pairs in ascending subdomain order, by one
// wave (lane 0..63; every lane of the wave calls it).
__device__ inline void restrict_assemble_column(int c, int lane, const CoarseView& cv, const double* __restrict__ r,
                                                const double* __restrict__ t, double* __restrict__ out,
                                                const int32_t* __restrict__ out_pos) {
  double s = 0.0;
  for (int e = cv.cg_ptr[c] + lane; e < cv.cg_ptr[c + 1]; e += 64) s += r[cv.cg_dof[e]];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) {
    for (int e = cv.cs_ptr[c]; e < cv.cs_ptr[c + 1]; ++e) s += t[e];
    out[out_pos ? out_pos[c] : c] = s;
  }
}
void phi_rhs(int64_t total_I, const CoarseView& cv, const int32_t* rowptr, const int32_t* col, const double* val,
             double* B, hipStream_t st);
void phi_transpose(int64_t total_I, const CoarseView& cv, const double* cm, double* rm, hipStream_t st);
// Discontinuous pressure (velocity-only extension): in every dense A_II^(i)
// (column-major, ld = |I_i|, the first nu[i] rows/columns velocity) the rows
// and columns of the pressure DOFs become those of the identity; in Phi_I the
// pressure rows are set to their fixed values: pval on the subdomain's own
// pressure column sub_pcol[i], 0 elsewhere (pval per interior position, < 0
// on velocity rows, which are left alone).
void decouple_pressure(const DenseBatch& B, const int32_t* nu, int max_n, hipStream_t st);
void phi_pressure_rows(int64_t total_I, const CoarseView& cv, const int8_t* pval, const int32_t* sub_pcol,
                       double* phi_cm, hipStream_t st);
void phibox(int64_t total_D, const CoarseView& cv, const BoxView& bv, double* out, hipStream_t st);
// W_i = A_own_i Phi_box_i for every box (column-major, ld |D_i|); the owned
// nonzeros of a row are found from the CSR matrix and om on the device.
// max_nc: the largest |C_i| (at most OWN_SPMM_MAX_NC).
constexpr int OWN_SPMM_MAX_NC = 7936;
void own_spmm(int nbox, int max_nd, int max_nc, const CoarseView& cv, const BoxView& bv, const OwnerMap& om,
              const int32_t* rowptr, const int32_t* col, const double* val, const double* phibox_, double* W,
              hipStream_t st);
void a0_assemble(int Nc, const CoarseView& cv, const double* P, const int64_t* p_off, double* A0, hipStream_t st);
void permute_dense(int n, const int32_t* perm, const double* M, int64_t ldm, double* F, int64_t ld, hipStream_t st);
void negate(int64_t n, double* x, hipStream_t st);
// three levels (eq. 2.5) on the dense A_0 (row-major, Nc x Nc)
void phi3_rhs(int64_t total_I, int Nc, const int32_t* I_sub, const int32_t* I_ptr, const int32_t* I_idx,
              const int32_t* C_ptr, const int32_t* C_idx, const int64_t* off, const int32_t* gcol3, const double* A0,
              double* B, hipStream_t st);
void phi3_build(int64_t total_I, int Nc, const int32_t* I_sub, const int32_t* I_ptr, const int32_t* I_idx,
                const int32_t* C_ptr, const int32_t* C_idx, const int64_t* off, const double* phiI,
                const int32_t* gcol3, double* phi3, hipStream_t st);
void expand(int64_t nfree, const int64_t* full_index, const double* xf, double* xfull, hipStream_t st);

}  // namespace gdsw
