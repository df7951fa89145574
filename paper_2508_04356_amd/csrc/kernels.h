// Launchers of the HIP kernels (gfx950).  All work is enqueued on `st`.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "context.h"

namespace gdsw {

// ---- dense batches: column-major matrices at base + off[f], leading dim ld[f]
struct DenseBatch {
  double* base = nullptr;
  const int32_t* n = nullptr;
  const int32_t* ld = nullptr;
  const int64_t* off = nullptr;
  int count = 0;
  int max_n = 0;
};

// In-place LU without pivoting (A = L U, L unit lower) of every matrix of the
// batch; right-looking with 64-wide blocks.  minpiv[f] receives the smallest
// |u_kk| / max|a_kk| seen in matrix f (as an ordered bit pattern, see
// minpiv_decode).
void lu_nopiv(const DenseBatch& B, unsigned long long* minpiv, hipStream_t st);
double minpiv_decode(unsigned long long bits);

// Unblocked forward (unit L) and backward (U) substitution for nrhs[f]
// right-hand sides held column-major at rhs + roff[f] (leading dim n[f]).
void lu_solve_multi(const DenseBatch& B, double* rhs, const int64_t* roff, const int32_t* nrhs,
                    int max_nrhs, hipStream_t st);

// From the FP64 LU in `lu` (laid out like the set): inverses of the diagonal
// tiles (into the set's dinv, offsets relative to dbase), every off-diagonal
// tile left-multiplied by its block row's diagonal inverse, and conversion to
// the set's precision when it is not FP64 (lu -> set.store).
void factor_finalize(FactorSet& fs, double* lu, int64_t dbase, hipStream_t st);

// Blocked forward/backward solve, in place on the work vector w, for every
// factor of the set: one launch per schedule step.
// `slot` selects a schedule of the set; `want` (device, per factor, or null)
// skips the work-groups of unselected factors.
void trsv_set(const FactorSet& fs, double* w, hipStream_t st, int slot = 0, const int32_t* want = nullptr);

// In-place inverse of every matrix of the batch by blocked Gauss-Jordan
// elimination without pivoting (64-wide blocks).  Pbuf: count * 64 * 64
// doubles; Tbuf: count * tstride doubles with tstride >= 64 * max ld.
// minpiv as for lu_nopiv (the pivots are those of the no-pivoting LU).
void gj_invert(const DenseBatch& B, double* Pbuf, double* Tbuf, int64_t tstride, unsigned long long* minpiv,
               hipStream_t st);
// FP64 -> FP32 / BF16 (round to nearest even) conversion of count entries.
void convert_store(int prec, const double* src, void* dst, int64_t count, hipStream_t st);
// Rows per matrix-vector work item for a storage precision (64 lanes x 16 bytes).
int gemv_rows(int prec);
// Partial-product and summation launches of the matrix-vector product for
// the inverses in desc (items of plan G built with column chunk cw, partial
// sums in `partial`); `want`
// (per descriptor, or null) skips unselected matrices; tm (or null) times the
// partial-product launch and charges it `bytes`.
void gemv_desc_launch(int prec, const GemvDesc* desc, const FactorSet::GemvPlan& G, int cw, double* partial,
                      hipStream_t st, const int32_t* want, KernelTimer* tm, double bytes);
// x_f <- M_f x_f for every stored inverse M_f of the set, in place on w.
void gemv_set(const FactorSet& fs, double* w, hipStream_t st, int slot = 0, const int32_t* want = nullptr);
// Symmetric inverses stored as upper 64 x 64 tiles (SOLVE_SYM): tiles per
// matrix, the work items of one matrix (tiles (f, I, J, p0 + index); block
// row sums (f, I, p0, tiles per row)), packing of full FP64 npad x npad
// matrices (offsets soff) into tiles at doff (elements), and the product.
int64_t symv_tiles(int npad);
void symv_items(int f, int npad, int64_t p0, int run, std::vector<int4>& it1, std::vector<int4>& it2);
// default work-group order of a precision (XCD-contiguous for FP32 tiles)
int symv_default_xcd(int prec);
void pack_upper(int prec, const double* src, const int64_t* soff, const int32_t* npad, int count, int max_npad,
                const int64_t* doff, void* dst, hipStream_t st);
void symv_set(const FactorSet& fs, double* w, hipStream_t st, int slot = 0, const int32_t* want = nullptr);
// The same product over the matrices of a descriptor list (desc[g].a: the
// tiles of matrix g; items of symv_items with g for f); want (or null)
// skips unselected matrices; tm (or null) times the tile launch.
void symv_desc_launch(int prec, const GemvDesc* desc, const FactorSet::GemvPlan& G, double* partial,
                      int64_t partial_len, hipStream_t st, const int32_t* want, KernelTimer* tm, double bytes,
                      int nc = 1);
// Shape of the set's several-column products: rows and summation columns
// per work item and which kernel (fs.gemm_rb, gemm_cw, gemm_lds).
void gemm_choose(FactorSet& fs);
// M <- (M + M^T) / 2 for every matrix of the batch.
void symmetrize(const DenseBatch& B, hipStream_t st);
// X_f <- M_f X_f for nrhs right-hand sides of the interleaved work buffer
// (entry (row, j) at w[row * ldk + j]), every stored inverse of the set
// (MFMA; FP32 accumulation for FP32 and BF16 storage, the right-hand sides
// rounded to the storage type).
void gemm_set(const FactorSet& fs, double* w, int64_t ldk, int nrhs, hipStream_t st);
// The set's local solve in its mode (inverse product or triangular solves).
void local_solve_set(const FactorSet& fs, double* w, hipStream_t st, int slot = 0, const int32_t* want = nullptr);

// C_b = alpha * op(A_b) * B_b + beta * C_b, FP64, column-major.
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
  int32_t m, n, k, lda, ldb, ldc, transA, pad;
};
void gemm_batched(const GemmDesc* d_desc, int count, int max_m, int max_n, double alpha, double beta,
                  hipStream_t st);

// ---- sparse / vector operations
void spmv_csr(int64_t nrows, const int32_t* rowptr, const int32_t* col, const double* val,
              const double* x, double* y, hipStream_t st);
void gather(int64_t count, const int32_t* idx, const double* src, double* dst, hipStream_t st);
// dense extraction of A[S_f, S_f] for every list f into a zeroed batch
void extract_local(const DenseBatch& B, const int32_t* list_ptr, const int32_t* list_idx,
                   const int32_t* rowptr, const int32_t* col, const double* val, int max_rows,
                   hipStream_t st);
// dense extraction from a dense row-major matrix M (ld = ldm)
void extract_local_dense(const DenseBatch& B, const int32_t* list_ptr, const int32_t* list_idx,
                         const double* M, int64_t ldm, int max_rows, hipStream_t st);

void deterministic_scatter(int64_t n, const int32_t* inv_ptr, const int64_t* inv_pos, const double* w,
                           double* z, hipStream_t st);

// Krylov helpers
void cols_dot(const double* V, int64_t ldv, int ncols, const double* w, int64_t n, double* part,
              int nblocks, double* out, hipStream_t st);
// w -= V h (each row summed in ascending column order) followed by
// cols_dot(V, w) (or, with self, cols_dot(w, w)) into out, in two launches;
// with out null only the partial blocks are written (nblocks x columns in
// part), for a consumer that finishes the sums itself (cols_dot_finish)
void sub_dots(const double* V, int64_t ldv, int ncols, const double* h, double* w, int64_t n, double* part,
              int nblocks, double* out, bool self, hipStream_t st);
void gemv_add(const double* V, int64_t ldv, int ncols, const double* y, double* x, int64_t n,
              hipStream_t st);
int cols_dot_blocks(int64_t n);
// local columns per work-group of the coarse restriction's pair sums for
// nsub subdomains of at most max_nc coarse columns and max_ni interior DOFs
// (0: one work-group per (subdomain, column) pair)
int phi_t_columns(int nsub, int max_nc, int max_ni);
void cols_dot_finish(const double* part, int nblocks, int ncols, double* out, hipStream_t st);

}  // namespace gdsw
