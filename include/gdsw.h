/*
 * gdsw.h -- C ABI of the MI355X (gfx950) monolithic GDSW / FGMRES library.
 *
 * Problem (Section 2 of Koehler & Rheinbach, "Monolithic Multi-level
 * Overlapping Schwarz Solvers for Fluid Problems"): the Stokes saddle-point
 * system of eq. (2.1),
 *
 *     [A  B^T] [u]   [F]
 *     [B  0  ] [p] = [0],
 *
 * discretised with Q2 velocity and Q1 pressure on the unit cube split into
 * n^3 hexahedra, Poiseuille inflow u_x = c y(1-y) z(1-z) on x = 0, no-slip
 * walls on y, z in {0, 1} and a do-nothing outflow on x = 1 (Section 4).
 *
 * Preconditioner: the monolithic two-level GDSW operator of eq. (2.2),
 *     M^-1 = Phi A_0^-1 Phi^T + sum_i R_i^T A_i^-1 R_i,
 * with A_0 = Phi^T A Phi and R_i of eq. (2.3) and the energy-minimising coarse
 * basis Phi of eq. (2.4); or the three-level operator of eq. (2.5).  It is
 * applied inside flexible GMRES (Tables 1-4: FGMRES, relative tolerance).
 *
 * Conventions shared by every entry point
 *   - Vectors live on the FREE degrees of freedom only (Dirichlet velocity
 *     DOFs are eliminated and their data lifted into the right-hand side):
 *     first every free velocity DOF -- Q2 nodes (a, b, c), a, b, c in [0, 2n],
 *     lexicographic with a fastest, then the component x, y, z -- then every
 *     pressure DOF (Q1 nodes (i, j, k) lexicographic with i fastest).
 *     gdsw_dof_map() reports the field and node of each free DOF.
 *   - Vector arguments are DEVICE pointers to FP64 arrays owned by the caller
 *     (for example torch tensors); the library never frees them.  Multi-column
 *     arguments are column-major with leading dimension ld >= n_free.
 *   - The library owns every internal device buffer.  They are allocated in
 *     gdsw_setup() and released in gdsw_destroy(); gdsw_apply_precond() and
 *     gdsw_spmv() allocate nothing.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued on it; calls return without waiting unless stated.
 *   - One context must not be used from two streams at the same time.
 *   - Every function returns a gdsw_status; no exception crosses the ABI.
 *     On failure a message is available from gdsw_last_error().
 *   - Results are bitwise reproducible for the same inputs, build and GPU:
 *     every reduction runs in a fixed order, no floating-point atomics.
 */
#ifndef GDSW_H
#define GDSW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gdsw_ctx gdsw_ctx; /* opaque, owned by the library */

typedef enum {
  GDSW_OK = 0,
  GDSW_EINVAL = 1,       /* bad argument: sizes, pointers, n % m != 0, ... */
  GDSW_ENOMEM = 2,       /* device or host memory (budget) exhausted */
  GDSW_ESINGULAR = 3,    /* a zero or tiny pivot in a local or coarse factor */
  GDSW_ENOCONV = 4,      /* FGMRES reached max_it; x holds the last iterate */
  GDSW_EDEVICE = 5,      /* a HIP runtime error; its text is in last_error */
  GDSW_EUNSUPPORTED = 6  /* valid request this build does not implement */
} gdsw_status;

typedef enum { GDSW_FP64 = 0, GDSW_FP32 = 1, GDSW_BF16 = 2 } gdsw_precision;

/* How the local solves A_i^-1 R_i r of eq. (2.2) / (2.5), and the coarse
 * solves, are carried out.  All give A_i^-1 v up to rounding.
 *   GDSW_SOLVE_BLOCK: the local saddle-point matrix by its blocks, with no
 *     dense n_i x n_i inverse.  The velocity block of A_i is I_3 (x) L_i (one
 *     scalar matrix for the three components: the gradient form of the
 *     viscous term), so with S_i = B_i K_i^-1 B_i^T the local solve is
 *     U1 = L^-1 F, p = S^-1 (B U1 - g), u = U1 - L^-1 B^T p: L_i^-1 and S_i^-1
 *     are formed at setup (Gauss-Jordan, FP64) and stored as upper tiles
 *     (L_i^-1 in the local precision), B_i as sparse rows.  An apply reads
 *     L_i^-1 twice (three vectors per pass), S_i^-1 once and B_i twice.
 *     Where W_i = K_i^-1 B_i^T (formed for S_i) has fewer entries than the
 *     upper triangle of L_i^-1 (the Q1 pressure: few pressure DOFs per local
 *     problem), the setup keeps it (local precision) and the last step is
 *     u = U1 - W p: L_i^-1 once, W_i once, B_i once; with the P1disc pressure
 *     the second pass stays.  At 16^3 an apply reads about a fifth of the
 *     bytes of GDSW_SOLVE_SYMMETRIC.  EINVAL when the
 *     velocity block lacks that structure (numbering 3 node + component,
 *     uncoupled components with equal values) or max_rhs > 1; the learned
 *     interior solve and batches are not offered with it.  Coarse levels use
 *     the symmetric storage.
 *   GDSW_SOLVE_INVERSE (default): the setup forms A_i^-1 explicitly by
 *     Gauss-Jordan elimination without pivoting (velocity DOFs first; its
 *     pivots are those of the no-pivoting LU) and stores it in place of the
 *     factors (same n^2 entries); an apply is one batched dense product.
 *   GDSW_SOLVE_TRIANGULAR: LU factors without pivoting and a blocked
 *     forward/backward substitution (2 * ceil(n / tile) dependent steps).
 *   GDSW_SOLVE_SYMMETRIC: the explicit inverse as above (symmetric, as
 *     A_i is), stored as its upper triangle of 64 x 64 tiles: about half
 *     the bytes per apply.  One right-hand side per product (max_rhs <= 1,
 *     EINVAL otherwise); batches and the learned interior solve accept it. */
typedef enum {
  GDSW_SOLVE_INVERSE = 0,
  GDSW_SOLVE_TRIANGULAR = 1,
  GDSW_SOLVE_SYMMETRIC = 2,
  GDSW_SOLVE_BLOCK = 3
} gdsw_local_solve;

/* The mesh: structured Q2/Q1 Stokes on the unit cube (Section 4). */
typedef struct {
  int32_t n;                  /* n^3 hexahedra, n >= 1 */
  int32_t manufactured_force; /* 0: f = 0 (the paper's workload);
                                 1: f_x = 2 mu c (y(1-y) + z(1-z)), which makes
                                    u = (c y(1-y) z(1-z), 0, 0), p = 0 exact */
  double viscosity;           /* mu > 0 */
  double inflow_amplitude;    /* c */
  int32_t pressure_element;   /* 0 (default): Q1, continuous pressure;
                                 1: P1-discontinuous, the paper's pair
                                 (Section 2): 4 DOFs per hexahedron, the basis
                                 1, 2 xi - 1, 2 eta - 1, 2 zeta - 1 on the
                                 reference cube, numbered 4 e + k after the
                                 velocity DOFs (element e lexicographic, x
                                 fastest).  There is no pressure interface:
                                 the coarse space gets one pressure column per
                                 subdomain, constant over it (Section 3), and
                                 the velocity columns are extended with the
                                 velocity block alone.  Needs local_algebraic
                                 = 1 and two levels (EINVAL otherwise). */
} gdsw_mesh;

/* Decomposition, overlap and levels (Section 2.1 and 2.2). */
typedef struct {
  int32_t subdomains;         /* m subdomains per axis (N = m^3), n % m == 0 */
  int32_t overlap;            /* delta >= 1 element layers: the overlapping set
                                 of subdomain i is its closed box grown by
                                 delta (see local_algebraic) */
  int32_t levels;             /* 2: eq. (2.2);  3: eq. (2.5) */
  int32_t group;              /* levels == 3: subdomains per subregion per axis,
                                 m % group == 0 (N^(2) = (m/group)^3) */
  int32_t local_precision;    /* gdsw_precision of the level-1 local factors
                                 (the coarse levels are always FP64) */
  int32_t tile;               /* tile size of the factor layout and of the
                                 triangular solves: 0 = default (128),
                                 else 64 or 128 */
  int32_t local_algebraic;    /* 0 (default): nodes on the artificial boundary
                                 of the grown box (the faces inside the cube)
                                 are left out for velocity and pressure, i.e.
                                 homogeneous Dirichlet conditions for both on
                                 the local problem (Section 2.1);
                                 1: every node of the grown box (algebraic
                                 overlap, one graph layer for delta = 1) */
  int32_t level2_layer;       /* levels == 3.  0 (default): the level-2 local
                                 set of a subregion holds the coarse DOFs of
                                 its subdomains (neighbouring subregions share
                                 their interface entities); 1: plus one layer
                                 of the A_0 graph */
  uint64_t device_mem_budget; /* bytes the setup may allocate; 0 = the free
                                 device memory reported by HIP */
  int32_t local_solve;        /* gdsw_local_solve: how A_i^-1 (and the coarse
                                 inverses) are applied */
  int32_t max_rhs;            /* 0 or 1: one column at a time.  2..32: the
                                 setup also allocates work buffers for that
                                 many columns, and gdsw_apply_precond /
                                 gdsw_fgmres_solve then process up to max_rhs
                                 columns together (two levels,
                                 GDSW_SOLVE_INVERSE, LU local solver): one
                                 MFMA product per factor set for all of them,
                                 FGMRES in lockstep with per-column stopping.
                                 With BF16 factors the columns are rounded to
                                 BF16 for the products (FP32 accumulation). */
  int32_t coarse_space;       /* 0 (default): full GDSW, every vertex, edge and
                                 face class its own entity; 1: GDSW* (Section
                                 4): each vertex grouped with its adjacent
                                 edges into one entity, an edge between two
                                 vertices joining the one first in entity
                                 order (smallest node id), faces on their own */
} gdsw_decomposition;

typedef struct {
  double rtol;                /* stop when |g_{j+1}| / ||b||_2 <= rtol */
  int32_t restart;            /* Krylov cycle length (1 ... 200) */
  int32_t max_it;             /* total inner iterations */
  int32_t use_graph;          /* 1: replay each iteration as a HIP graph */
  int32_t history_len;        /* entries available in `history` */
  double* history;            /* host array or NULL: |g_{j+1}| / ||b|| after
                                 each iteration (first column only) */
} gdsw_fgmres_opts;

typedef struct {
  int32_t iterations;         /* preconditioner applications */
  int32_t restarts;           /* completed cycles beyond the first */
  double rel_res;             /* last implicit |g_{j+1}| / ||b|| */
  double true_rel_res;        /* ||b - A x|| / ||b|| recomputed at the end */
  double t_solve_s;           /* wall time of the solve (host clock) */
  int64_t learned_solves;     /* interior local solves done by the network in
                                 this solve (learned local solver), else 0 */
  int64_t fallbacks;          /* of those, re-solved exactly because their
                                 local residual exceeded tau */
} gdsw_fgmres_info;

typedef struct {
  int64_t n_free, n_full, n_u_free, n_p;
  int64_t nnz;                /* nonzeros of the free-DOF CSR matrix */
  int64_t n_sub;              /* N = m^3 */
  int64_t n_entities;         /* interface entities (vertices, edges, faces) */
  int64_t n_coarse;           /* columns of Phi = size of A_0 */
  int64_t n_subregions;       /* three levels: N^(2), else 0 */
  int64_t n_coarse3;          /* three levels: size of A_0^(3), else 0 */
  int64_t local_min, local_max; /* smallest / largest overlapping local size */
  uint64_t factor_bytes;      /* level-1 local factors as stored */
  uint64_t coarse_bytes;      /* coarse factors and bases (all levels) */
  uint64_t device_bytes;      /* everything the context holds on the device */
  uint64_t solve_bytes;       /* algorithmic bytes the local and coarse solves
                                 of one apply read: per stored matrix n^2
                                 (inverse, triangular) or n (n + 1) / 2
                                 (symmetric, block) times the element size,
                                 each pass counted; block mode adds B_i and
                                 W_i as read */
  int64_t solve_launches;     /* kernel launches of those solves per apply */
} gdsw_sizes;

/* Setup ------------------------------------------------------------------- */

/* Builds the problem (host: numbering, assembly, decomposition, interface
 * entities; Section 3 calls this the symbolic setup) and the preconditioner
 * (device: local matrices and their inverses, LU factors or block factors
 * as local_solve asks, Phi, A_0 and its inverse; the numeric setup).  Blocks
 * until the setup is complete.
 * Errors: EINVAL for n < 1, m < 1, n % m, overlap < 1, levels not 2/3,
 * m % group (3 levels), bad precision or tile; ENOMEM when the budget check
 * fails (the message gives the bytes needed); ESINGULAR when a pivot of a
 * local or coarse factor is tiny (the message names the factor). */
gdsw_status gdsw_setup(const gdsw_mesh* mesh, const gdsw_decomposition* dec,
                       void* stream, gdsw_ctx** out);

/* Host-only variant: performs the symbolic setup and the assembly but touches
 * no device.  Only gdsw_get_sizes, gdsw_dof_map, gdsw_host_matrix,
 * gdsw_host_rhs, gdsw_last_error and gdsw_destroy accept such a context. */
gdsw_status gdsw_setup_host(const gdsw_mesh* mesh, const gdsw_decomposition* dec,
                            gdsw_ctx** out);

/* Algebraic entry point (Section 3: the implementation needs only the
 * distribution of the velocity and pressure DOFs over the subdomains): any
 * assembled saddle-point matrix of eq. (2.1) and any partition, e.g. an
 * unstructured mesh.  Host arrays, read during the call only:
 *   n                 unknowns (Dirichlet DOFs already eliminated);
 *   row_ptr[n + 1], col[nnz], val[nnz]
 *                     CSR of the matrix, columns sorted and distinct per
 *                     row, nnz < 2^31;
 *   rhs[n]            right-hand side (gdsw_rhs returns it), or NULL (zeros);
 *   field[n]          0, 1, 2 velocity components, 3 pressure; every velocity
 *                     DOF numbered before every pressure DOF (the local and
 *                     coarse eliminations run without row exchanges in that
 *                     order);
 *   null_value[n]     value (0 or 1) of the field's null-space vector on each
 *                     DOF, or NULL (all 1): 1 for translations and a
 *                     continuous pressure, 1 / 0 on the constant / linear
 *                     functions of a discontinuous pressure;
 *   n_sub, sub_ptr[n + 1], sub_idx[...]
 *                     the subdomains holding each DOF, sorted: DOF d is held
 *                     by sub_idx[sub_ptr[d] .. sub_ptr[d + 1]) (the closures
 *                     of the non-overlapping subdomains, so an interface DOF
 *                     is held by several).
 * From these: D_i = DOFs held by i; Gamma = DOFs held by two or more;
 * I_i = D_i without Gamma; the overlapping set S_i = D_i grown by
 * dec->overlap layers of the matrix graph; interface entities = classes of
 * Gamma DOFs with the same subdomain set (ordered by their smallest DOF
 * index), one coarse column per (entity, field); a field with DOFs but none
 * on Gamma (a discontinuous pressure) gets one column per subdomain, its
 * null-space values there, and the velocity columns are then extended with
 * the velocity block alone.  Two levels, full GDSW: dec->levels must be 2 and
 * dec->coarse_space 0 (EINVAL otherwise); dec->subdomains and
 * local_algebraic are ignored; the other fields mean what they mean for
 * gdsw_setup.  Every other entry point accepts the context except the learned
 * local solve (EUNSUPPORTED) and gdsw_expand_solution, for which the full
 * vector is the free one.  EINVAL on inconsistent input (the message says
 * which); a matrix entry between DOFs that share no subdomain is refused. */
typedef struct {
  int64_t n;
  const int64_t* row_ptr;
  const int32_t* col;
  const double* val;
  const double* rhs;
  const int32_t* field;
  const double* null_value;
  int32_t n_sub;
  const int64_t* sub_ptr;
  const int32_t* sub_idx;
} gdsw_algebraic_problem;

gdsw_status gdsw_setup_algebraic(const gdsw_algebraic_problem* prob, const gdsw_decomposition* dec, void* stream,
                                 gdsw_ctx** out);

/* As gdsw_setup_algebraic without touching the device (see gdsw_setup_host). */
gdsw_status gdsw_setup_algebraic_host(const gdsw_algebraic_problem* prob, const gdsw_decomposition* dec,
                                      gdsw_ctx** out);

gdsw_status gdsw_get_sizes(const gdsw_ctx* ctx, gdsw_sizes* out);

/* Wall time of the two setup phases, as the paper's tables report them
 * (Tables 1-4): symbolic (host: numbering, assembly, decomposition, overlap
 * and interface entities) and numeric (device: local matrices, inverses or
 * factors, Phi, A_0 and the coarse levels), in seconds. */
gdsw_status gdsw_setup_times(const gdsw_ctx* ctx, double* symbolic_s, double* numeric_s);

/* field[k] in {0,1,2,3} (u_x, u_y, u_z, p) and node_abc[3k..3k+2] the Q2
 * node coordinates (pressure nodes (i,j,k) map to (2i,2j,2k)) of free DOF k.
 * Host arrays of n_free and 3 n_free int32. */
gdsw_status gdsw_dof_map(const gdsw_ctx* ctx, int32_t* field, int32_t* node_abc);

/* Copies the host-assembled free-DOF CSR matrix into caller host arrays of
 * n_free + 1 (int64), nnz (int32) and nnz (double) entries. */
gdsw_status gdsw_host_matrix(const gdsw_ctx* ctx, int64_t* row_ptr, int32_t* col,
                             double* val);
/* Copies the lifted right-hand side (host array of n_free doubles). */
gdsw_status gdsw_host_rhs(const gdsw_ctx* ctx, double* b);

/* Operators --------------------------------------------------------------- */

/* b_dev[n_free] = lifted right-hand side of eq. (2.1) on the free DOFs. */
gdsw_status gdsw_rhs(gdsw_ctx* ctx, double* b_dev, void* stream);

/* y = A x, the free-DOF saddle-point matrix of eq. (2.1).  x and y must not
 * overlap. */
gdsw_status gdsw_spmv(gdsw_ctx* ctx, const double* x_dev, double* y_dev, void* stream);

/* z = M^-1 r for nrhs columns (eq. 2.2, or eq. 2.5 with three levels),
 * column-major with leading dimension ld.  r and z must not overlap.
 * Allocates nothing.  Columns are processed max_rhs at a time when the
 * context was set up for several right-hand sides (see max_rhs), else one
 * by one. */
gdsw_status gdsw_apply_precond(gdsw_ctx* ctx, const double* r_dev, double* z_dev,
                               int32_t nrhs, int64_t ld, void* stream);

/* For callers that cannot allocate device memory at call time (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * z = M^-1 r exactly as gdsw_apply_precond computes it (same kernels and
 * summation orders, so bitwise the same result), column by column, with the
 * partial sums of the inverse products (block mode: of the velocity-block,
 * Schur complement and coarse products) in a static device array that the
 * library holds once per device for the whole process (128 MiB; its device
 * address is looked up in gdsw_setup) instead of the context's buffer.
 * Calls no allocating routine.  Every call on a device shares that array and
 * needs no cleared state in it; calls that overlap on one device (two
 * streams, two threads) race.  EINVAL when the problem's partial sums exceed
 * the array (the message gives the bytes needed), EUNSUPPORTED for
 * GDSW_SOLVE_TRIANGULAR or a learned / disabled interior solver. */
gdsw_status gdsw_apply_precond_noalloc(gdsw_ctx* ctx, const double* r_dev, double* z_dev,
                                       int32_t nrhs, int64_t ld, void* stream);

/* Solves A x = b with right-preconditioned FGMRES for nrhs columns from
 * x = 0: max_rhs columns at a time in lockstep when the context was set up
 * for several right-hand sides (every column keeps its own Krylov space,
 * stopping test and iteration count), else one after another.  Blocks until every column is done (the loop reads the
 * residual estimate back to the host once per iteration).  info[nrhs] may be
 * NULL.  Returns ENOCONV if a column missed rtol within max_it (x then holds
 * its last iterate and info is filled in). */
gdsw_status gdsw_fgmres_solve(gdsw_ctx* ctx, const double* b_dev, double* x_dev,
                              int32_t nrhs, int64_t ld, const gdsw_fgmres_opts* opts,
                              gdsw_fgmres_info* info, void* stream);

/* x_full[n_full] = free values scattered into the full DOF vector (velocity
 * 3*node + component, then pressure) with the Dirichlet data re-inserted. */
gdsw_status gdsw_expand_solution(const gdsw_ctx* ctx, const double* x_free_dev,
                                 double* x_full_dev, void* stream);

/* Setup results for inspection (device -> host copies, blocking) --------- */

/* A_0 = Phi^T A Phi as a dense row-major n_coarse^2 host array. */
gdsw_status gdsw_copy_coarse_matrix(const gdsw_ctx* ctx, double* a0_host);

/* Phi as a dense column-major n_free x n_coarse host array (tests only:
 * small problems). */
gdsw_status gdsw_copy_coarse_basis(const gdsw_ctx* ctx, double* phi_host);

/* Overlapping index set of subdomain i (sorted free DOF numbers), host array
 * of local_size(i) int32; pass NULL to query the size into *size. */
gdsw_status gdsw_local_indices(const gdsw_ctx* ctx, int32_t i, int32_t* idx_host,
                               int32_t* size);

/* Learned local solve ----------------------------------------------------------
 * A 4-layer 3x3x3 convolution network (channels 4-32-32-32-4, ReLU between
 * layers, BF16 weights and activations with FP32 accumulation) may replace
 * A_i^-1 of eq. (2.2) on the interior subdomains (those whose local problem
 * does not touch the cube's boundary); FGMRES admits the variable
 * preconditioner.  The network maps r_i / ||r_i|| on the local node grid
 * (channels u_x, u_y, u_z, p; pressure on the Q1 nodes; velocity divided by
 * mu) to A_i^-1 r_i / ||r_i|| scaled per channel.  The exact local solves
 * are kept: they generate the training pairs and serve as fallback. */
typedef struct {
  int32_t grid;               /* nodes per axis of an interior local problem */
  int32_t subdomains;         /* interior subdomains */
  int64_t n_params;           /* weights + biases (flat: W0 b0 W1 b1 W2 b2 W3 b3,
                                 W_l[c_out][c_in][27]) */
  int32_t samples;            /* training pairs generated so far */
  int32_t reserved;
  float sigma[4];             /* per-channel target scales */
} gdsw_learned_info;

/* Allocates the network on the device, He-normal weights from `seed`.
 * EUNSUPPORTED when the decomposition has no interior subdomains (m < 3). */
gdsw_status gdsw_learned_init(gdsw_ctx* ctx, uint64_t seed, gdsw_learned_info* info, void* stream);

/* Generates training pairs from `solves` LU-preconditioned FGMRES solves (the
 * assembled right-hand side, then seeded random ones): every Krylov vector
 * restricted to every interior subdomain gives (r_i, A_i^-1 r_i) by the LU
 * solve.  Then `steps` Adam steps (lr; beta 0.9/0.999) on random batches of
 * `batch` pairs; loss_history[steps] (host, may be NULL) receives the mean
 * masked squared error per step.  solves = 0 keeps the existing pairs. */
gdsw_status gdsw_learned_train(gdsw_ctx* ctx, int32_t solves, int32_t steps, int32_t batch, double lr, uint64_t seed,
                               double* loss_history, void* stream);

/* Sets the FP32 master weights from set_host (n_params floats, may be NULL),
 * then copies to get_host (may be NULL): which = 0 master weights, 1 the
 * BF16-rounded working weights, 2 the last gradients. */
gdsw_status gdsw_learned_weights(gdsw_ctx* ctx, const float* set_host, float* get_host, int32_t which, void* stream);

/* Loss and gradients for host inputs x and targets t ([batch][4][grid^3]
 * each, batch <= max(interior subdomains, 32)): forward and backward kernels
 * exactly as in training.  For checking the kernels against a reference. */
gdsw_status gdsw_learned_loss_grad(gdsw_ctx* ctx, const float* x_host, const float* t_host, int32_t batch,
                                   double* loss, float* grads_host, void* stream);

/* Local solver of the interior subdomains: 0 LU (default), 1 learned with the
 * LU fallback where ||r_i - A_i y_i|| > tau ||r_i||, 2 none (no local
 * correction there; an ablation).  Mode 1 reads one counter back to the host
 * per apply. */
gdsw_status gdsw_set_local_solver(gdsw_ctx* ctx, int32_t mode, double tau);

/* Copies the trained network of src (weights and per-channel output scales)
 * into dst, so that one training serves several problems whose interior
 * subdomains share the node grid (EINVAL otherwise).  The network works at
 * unit viscosity; each problem scales its velocity right-hand sides by 1/mu
 * and the pressure solution by mu, so the problems may differ in viscosity
 * and inflow.  Both contexts need gdsw_learned_init; src may be a batch member. */
gdsw_status gdsw_learned_copy(gdsw_ctx* dst, const gdsw_ctx* src, void* stream);

/* Interior local solves done by the network and by the LU fallback so far. */
gdsw_status gdsw_learned_stats(const gdsw_ctx* ctx, int64_t* learned_solves, int64_t* fallbacks);

/* Writes the network (FP32 master weights and the per-channel output scales)
 * to the file `path`: "GDSWNET1", int32 grid, int32 0, int64 n_params,
 * float sigma[4], float weights[n_params], little-endian.  Synchronises
 * `stream`.  EINVAL if ctx has no network or the file cannot be written. */
gdsw_status gdsw_learned_save(const gdsw_ctx* ctx, const char* path, void* stream);

/* Reads such a file into ctx's network (after gdsw_learned_init), which then
 * counts as trained.  EINVAL if the file is malformed or was written for
 * another interior node grid. */
gdsw_status gdsw_learned_load(gdsw_ctx* ctx, const char* path, void* stream);

/* gdsw_learned_init (if needed, with `seed`), training pairs from 4 solves
 * (if none were generated yet), `steps` Adam steps (batch 32, lr 2e-3) and,
 * when out_weights is not NULL, gdsw_learned_save to that path. */
gdsw_status gdsw_train_local_net(gdsw_ctx* ctx, const char* out_weights, int32_t steps, uint64_t seed,
                                 void* stream);

/* Tuning --------------------------------------------------------------------- */

/* Re-plans the launch schedule of the blocked triangular solves: the factors
 * are split into `phases` groups (1..64) whose forward/backward sweeps start
 * ceil(tiles / phases) launches apart, which evens out the bytes per launch;
 * `waves` (4 or 8) sets the work-group size of the tile kernel (64 * waves
 * threads; 8 needs tile 128).  Results do not depend on either.
 * Synchronises `stream`; must not overlap other calls on ctx. */
gdsw_status gdsw_set_schedule(gdsw_ctx* ctx, int32_t phases, int32_t waves, void* stream);

/* Diagnostics --------------------------------------------------------------- */

/* One gdsw_apply_precond() with HIP events between its phases, recorded on
 * `stream`; blocks until done.  ms[0] = gathers and coarse restriction,
 * ms[1] = triangular solves of the level-1 factor set (with the coarse factor
 * when it shares the set's precision), ms[2] = triangular solves of the FP64
 * coarse-level set, ms[3] = scatter and prolongation (milliseconds). */
gdsw_status gdsw_profile_apply(gdsw_ctx* ctx, const double* r_dev, double* z_dev, void* stream,
                               double* ms);

/* Launch-shape autotuner of the level-1 product, on this context's own
 * matrices (10 products per candidate after 3 untimed, HIP events on
 * `stream`); keeps the fastest and re-plans.
 *   GDSW_SOLVE_INVERSE: column chunks of 512, 1024 and 2048 columns per work
 *     item; chosen receives the chunk, ms[0..2] the mean time of each.
 *   GDSW_SOLVE_SYMMETRIC and GDSW_SOLVE_BLOCK (the velocity-block tiles):
 *     runs of 2 or 1 stored tiles per work-group, each in the plain and in
 *     the XCD-contiguous work-group order; candidates (2, plain), (2, XCD),
 *     (1, plain), (1, XCD) with times in ms[0..3]; chosen = 10 * run + (1 if
 *     XCD order).
 * The shape sets the grouping of the partial sums, so results can change in
 * the last bits; they are again bitwise reproducible for the chosen shape.
 * chosen and ms may be NULL.  Call before gdsw_learned_init; EUNSUPPORTED
 * otherwise or in triangular mode.  Synchronises `stream`. */
gdsw_status gdsw_autotune(gdsw_ctx* ctx, void* stream, int32_t* chosen, double* ms);

/* Autotuner of the several-column MFMA product of the level-1 inverses
 * (GDSW_SOLVE_INVERSE with max_rhs > 1), timed with max_rhs columns (5
 * products per candidate).  Candidates: FP64 storage 0..2 = the direct
 * kernel with 512 / 1024 / 2048 summation columns per work item, 3..5 = the
 * LDS-staged kernel with 256 / 512 / 1024; FP32 and BF16 storage 0..2 = 512
 * / 1024 / 2048 (one kernel).  chosen receives the index of the fastest,
 * ms[0..5] the times (0 where no candidate).  Results can change in the last
 * bits as above.  EUNSUPPORTED for other contexts.  Synchronises `stream`. */
gdsw_status gdsw_autotune_mfma(gdsw_ctx* ctx, void* stream, int32_t* chosen, double* ms);

/* Event timing of the dominant solve kernel.  While enabled, every launch of
 * the level-1 solve kernel in a full apply (the partial-product kernel of
 * GDSW_SOLVE_INVERSE, single- or multi-column, that of GDSW_SOLVE_SYMMETRIC,
 * or each sweep step of GDSW_SOLVE_TRIANGULAR) is bracketed by two HIP events
 * on the stream it runs on, up to 16384 launches.  gdsw_kernel_timer(ctx, 1)
 * resets the count and starts; (ctx, 0) stops.  gdsw_kernel_timer_read waits
 * for the last recorded event and returns the summed kernel time (ms), the
 * number of timed launches and the mean algorithmic bytes per launch (a
 * product launch reads every level-1 matrix once: sum of n^2 * element size,
 * n (n + 1) / 2 * element size for the symmetric storage; a sweep step is
 * charged that sum divided by the steps of one apply). */
gdsw_status gdsw_kernel_timer(gdsw_ctx* ctx, int32_t enable);
gdsw_status gdsw_kernel_timer_read(gdsw_ctx* ctx, double* total_ms, int64_t* launches, uint64_t* bytes_per_launch);

/* Last error text of ctx, or of the calling thread when ctx is NULL. */
const char* gdsw_last_error(const gdsw_ctx* ctx);

/* Releases every device and host resource of ctx (NULL is allowed). */
void gdsw_destroy(gdsw_ctx* ctx);

/* Batches of independent problems ----------------------------------------
 * count problems (each its own mesh and decomposition, e.g. different n,
 * viscosity and inflow), each with its own context, whose level-1 and
 * coarse-level inverse products run as ONE launch pair per level over the
 * matrices of every member (longest matrix first).  Every member must use
 * the same local_solve, GDSW_SOLVE_INVERSE, GDSW_SOLVE_SYMMETRIC or
 * GDSW_SOLVE_BLOCK (EINVAL otherwise), and the same local_precision; with
 * GDSW_SOLVE_BLOCK the merged launch is the velocity-block product, and
 * each member's B row products, Schur complement product and u = U1 - W p
 * follow on its own stream lane.  A member computes
 * exactly what it computes alone (same kernels and summation orders: the
 * results are bitwise those of the member's own gdsw_apply_precond and
 * gdsw_fgmres_solve). */
typedef struct gdsw_batch gdsw_batch; /* opaque, owned by the library */

/* Sets up every member (as gdsw_setup, each with its own budget check), then
 * the merged launch plans.  On failure nothing is kept; the message names
 * the member. */
gdsw_status gdsw_setup_batch(const gdsw_mesh* meshes, const gdsw_decomposition* decs, int32_t count,
                             void* stream, gdsw_batch** out);

/* The context of member k (owned by the batch: use it for gdsw_rhs,
 * gdsw_get_sizes, gdsw_spmv, gdsw_expand_solution; never destroy it). */
gdsw_status gdsw_batch_member(gdsw_batch* batch, int32_t k, gdsw_ctx** member);

/* z_k = M_k^-1 r_k for every member; r and z are host arrays of count
 * device pointers (member k's vectors, length n_free of member k). */
gdsw_status gdsw_apply_precond_batch(gdsw_batch* batch, const double* const* r_dev, double* const* z_dev,
                                     void* stream);

/* FGMRES on every member in lockstep from x = 0: one iteration advances
 * every member that has not yet met its stopping test; a member that has is
 * masked out of the shared launches.  info[count] may be NULL.  ENOCONV if
 * a member reached max_it first. */
gdsw_status gdsw_fgmres_solve_batch(gdsw_batch* batch, const double* const* b_dev, double* const* x_dev,
                                    const gdsw_fgmres_opts* opts, gdsw_fgmres_info* info, void* stream);

/* As gdsw_kernel_timer / gdsw_kernel_timer_read for the batch's merged
 * level-1 partial-product launches (bytes: the matrices of the members
 * active in each launch). */
gdsw_status gdsw_batch_kernel_timer(gdsw_batch* batch, int32_t enable);
gdsw_status gdsw_batch_kernel_timer_read(gdsw_batch* batch, double* total_ms, int64_t* launches,
                                         uint64_t* bytes_per_launch);

void gdsw_destroy_batch(gdsw_batch* batch);

#ifdef __cplusplus
}
#endif
#endif /* GDSW_H */
