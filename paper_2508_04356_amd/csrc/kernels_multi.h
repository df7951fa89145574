// Launchers of the interleaved multi-right-hand-side vector kernels
// (entry (d, j) of a K-column block at x[d * K + j], K <= 32).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels_ops.h"

namespace gdsw {

void cm_to_il(int64_t n, int K, const double* src, int64_t ld, double* dst, hipStream_t st);
void il_to_cm(int64_t n, int K, const double* src, double* dst, int64_t ld, hipStream_t st);
void gather_il(int64_t count, int K, const int32_t* idx, const double* src, double* dst, hipStream_t st);
// with t (phi_t_splits(nsub) * n_pairs * K doubles) and nsub subdomains:
// per-subdomain pair partials first, then assembly
int phi_t_splits(int nsub);
void restrict_il(int nc, int K, const CoarseView& cv, const double* r, double* w, const int32_t* out_pos,
                 hipStream_t st, int n_pairs = 0, double* t = nullptr, int nsub = 0);
// y0_pos == nullptr: no coarse term; nsub > 0: the Phi_I y0 term runs per
// subdomain over the column-major Phi_I (same operands and order)
void scatter_prolong_il(int64_t n, int K, const int32_t* inv_ptr, const int64_t* inv_pos, const double* w,
                        const CoarseView& cv, const int32_t* y0_pos, double* z, hipStream_t st, int nsub = 0,
                        int max_ni = 0);
void spmm_il(int64_t nrows, int K, const int32_t* rowptr, const int32_t* col, const double* val, const double* x,
             double* y, hipStream_t st);
int dots_il_blocks(int64_t n);
// out[i * K + j] = <V_i[:, j], w[:, j]> for i < ncols (V_i at V + i * ldv)
void dots_il(const double* V, int64_t ldv, int ncols, const double* w, int64_t n, int K, double* part, int nblocks,
             double* out, hipStream_t st);
// w[:, j] += sign * sum_i V_i[:, j] h[i * K + j]
void gemv_il(const double* V, int64_t ldv, int ncols, const double* h, double* w, int64_t n, int K, double sign,
             hipStream_t st);
void scale_il(int64_t n, int K, const double* w, const double* s, const int32_t* active, double* v, hipStream_t st);
void sub_il(int64_t total, const double* b, double* r, hipStream_t st);

}  // namespace gdsw
