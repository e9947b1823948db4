/*
 * mstab.h -- C ABI of the M(s)stab(l) / IDR(s)stab(l) solver for AMD MI355X
 * (gfx950).
 *
 * The method: Neuenhofen, "M(s)stab(l): A Generalization of IDR(s)stab(l) for
 * Sequences of Linear Systems", arXiv 1604.06043.  The problem is the
 * sequence A x^(i) = b^(i) with one fixed sparse nonsymmetric A and right-hand
 * sides that depend on the previous solution (Section 1, equation of the
 * sequence), solved one after the other.  IDR(s)stab(l) is Algorithm 1;
 * M(s)stab(l) is Algorithm 1 fed with the cut-space P and the matrices U, V
 * that a former solve returned (Section 4.2), fetched at the end of one of its
 * cycles (Section 5, preliminaries).
 *
 * Conventions for every call:
 *   - Return value is an mstab_status; calls never abort and never fail
 *     silently.  mstab_last_error() gives the text of the last failure on a
 *     handle (or, for calls without a handle, of the calling thread).
 *   - "device" pointers are HIP device memory (e.g. torch tensors'
 *     data_ptr()); "host" pointers are ordinary host memory.  All arrays are
 *     dense, contiguous, little-endian; matrices in CSR with int32 indices,
 *     columns sorted within a row; blocks of vectors are column-major.
 *   - hip_stream is a hipStream_t (NULL = the legacy default stream).  Every
 *     call enqueues its work on that stream and returns after synchronizing
 *     with it, unless stated otherwise.
 *   - Arguments are borrowed for the duration of the call, except the matrix
 *     arrays passed to mstab_create, which are borrowed until mstab_destroy.
 *   - One thread at a time per handle; distinct handles are independent.
 */
#ifndef MSTAB_H
#define MSTAB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MSTAB_OK = 0,
    MSTAB_NOT_CONVERGED = 1,   /* max_mv reached or replacements exhausted; x = last iterate */
    MSTAB_E_INVALID = -1,      /* bad argument (null pointer, s or l out of range, n <= s, ...) */
    MSTAB_E_HIP = -2,          /* a HIP runtime call failed */
    MSTAB_E_NOMEM = -3,        /* device or host allocation failed */
    MSTAB_E_BREAKDOWN = -4,    /* a singular small system after the allowed restarts */
    MSTAB_E_NONFINITE = -5     /* NaN or Inf in b or in the iteration */
} mstab_status;

typedef enum {
    MSTAB_METHOD_MSTAB = 0,    /* use recycled P, U, V when the handle holds them (Section 4.2) */
    MSTAB_METHOD_IDRSTAB = 1,  /* Arnoldi U, V of level s for every system (Section 5) */
    MSTAB_METHOD_GMRES = 2     /* restarted GMRES(m), m = gmres_restart, one of Section 5.1's
                                  comparison methods (BiCGStab, the other, is IDRSTAB with
                                  s = l = 1, Section 2.3): Arnoldi with classical Gram-Schmidt
                                  applied twice, Givens rotations, |g_{j+1}| <= tol ||b|| ends a
                                  cycle early, and the true residual that starts every cycle
                                  decides convergence.  s and l are not used (pass 1, 1).  Every
                                  product counts in mv (the true residuals included); cycles
                                  counts Arnoldi steps, restarts the cycles after the first,
                                  relres_recursive the last step's estimate; the residual
                                  history holds the initial residual and every step's estimate.
                                  F64 precision and ENGINE_GRID only; split preconditioning and
                                  reordering apply as for the other methods.  The handle keeps
                                  m + 2 extra vectors. */
} mstab_method;

typedef enum {
    MSTAB_PREC_F64 = 0,        /* every vector operation in FP64 */
    MSTAB_PREC_F32_REFINE = 1, /* FP32 M(s)stab(l) whose residual is replaced after every cycle
                                  by the FP64 true residual b - A x, x accumulated in FP64
                                  (the paper's residual replacement of Section 5.1, in mixed
                                  precision); FP64 small solves */
    MSTAB_PREC_F32_MATRIX = 2  /* FP64 M(s)stab(l) whose products use an FP32 copy of A's values
                                  (FP64 vectors and sums); the initial and true residuals use A
                                  itself, and true-residual replacement (up to
                                  max(max_replacements, 10)) corrects the O(eps32) difference */
} mstab_precision;

typedef enum {
    MSTAB_FETCH_THRESHOLD = 0, /* first cycle end with recursive relres <= fetch_rel (else the last) */
    MSTAB_FETCH_AT_LEVEL = 1,  /* cycle end at which the level of U, V equals fetch_level */
    MSTAB_FETCH_AT_END = 2,    /* last cycle end of the solve */
    MSTAB_FETCH_ONCE = 3,      /* THRESHOLD on the first solve, then keep that data for all */
    MSTAB_FETCH_NEVER = 4,     /* never replace the held data */
    MSTAB_FETCH_ESTIMATE = 5   /* the fetch point "shortly before the residual drops" estimated
                                  from the previous solve (Section 5, how to choose the fetching
                                  point: the first system's convergence estimates the second's):
                                  the cycle before that solve's largest one-cycle reduction of the
                                  residual (at least 1).  The first solve of a sequence (or after
                                  mstab_recycle_reset) fetches nothing and only estimates, so the
                                  second also starts like IDR(s)stab and fetches at the estimate;
                                  from then on each solve fetches at the cycle estimated from the
                                  one before (at its last cycle if it stops earlier). */
} mstab_fetch;

typedef enum {
    MSTAB_PRECOND_NONE = 0,    /* solve A x = b as given */
    MSTAB_PRECOND_JACOBI = 1,  /* split diagonal preconditioning, Section 5.1's split form
                                  L^-1 A R^-1 y = L^-1 b, x = R^-1 y, with L = R = |D|^(1/2)
                                  (D = diag(A)).  The handle iterates on the split system:
                                  tol, relres_recursive, relres_true, the residual history and
                                  the true-residual replacement refer to the preconditioned
                                  residual L^-1 (b - A x), and recycled U, V (recycle_get/set)
                                  live in the split system's space.  Every row needs a stored,
                                  finite, nonzero diagonal entry (else E_INVALID at create). */
    MSTAB_PRECOND_ILU0 = 2     /* the same split form with the incomplete LU factorization without
                                  fill-in that Section 5.1 uses: A' = P A P^T in a greedy
                                  multicolour order of A's symmetrized pattern (no entry couples
                                  two rows of one colour), A' ~ L U with (LU)_ij = a'_ij on A''s
                                  pattern, and the iteration runs on L^-1 A' U^-1 y = L^-1 b',
                                  x' = U^-1 y (one triangular-solve launch per colour, in order
                                  for L, in reverse for U).  Each product with that operator counts
                                  as one MV.  As for JACOBI, tol, the residual history and the
                                  replacements refer to the preconditioned residual, and recycled
                                  U, V and mstab_permutation refer to the ordered, split system.
                                  F64 precision and REORDER_NONE only; a missing diagonal entry or
                                  a zero pivot is E_INVALID at create. */
} mstab_precond;

typedef enum {
    MSTAB_REORDER_NONE = 0,    /* iterate in the caller's row order */
    MSTAB_REORDER_RCM = 1      /* iterate on P A P^T with P the reverse Cuthill-McKee order of A's
                                  symmetrized pattern (mstab_rcm_order, computed on the host at
                                  create): neighbouring unknowns get nearby indices, so the
                                  product's gathers of x stay in cache.  b and x keep the caller's
                                  order; the cut-space basis, the residual history and recycled
                                  U, V (recycle_get/set) refer to the reordered rows
                                  (mstab_permutation gives the order).  Applied before
                                  PRECOND_JACOBI. */
} mstab_reorder;

typedef enum {
    MSTAB_FORMAT_AUTO = 0,     /* the device copy of A the products read: a matrix whose entries lie on
                                  at most 16 diagonals (column - row) with under 25% padding is kept
                                  in diagonal storage (64-row slices of nd values, a 16-bit presence
                                  mask per row), and if every diagonal then holds one value wherever
                                  it is present (a constant-coefficient stencil, compared bit for
                                  bit) only those nd values and the mask are kept; any other matrix
                                  in sliced ELLPACK (64-row slices).  Every format gives the same
                                  product bit for bit. */
    MSTAB_FORMAT_DIAGONAL = 1, /* as AUTO without the constant-diagonal form (values streamed) */
    MSTAB_FORMAT_SLICED = 2    /* always sliced ELLPACK */
} mstab_format;

typedef enum {
    MSTAB_ENGINE_GRID = 0,     /* each step of a cycle is one or more grid-wide kernels (all CUs work
                                  on one system); the host reads the status after every cycle */
    MSTAB_ENGINE_WORKGROUP = 1 /* one workgroup runs a whole solve (Algorithm 1 with the same
                                  readings: initial residual, Arnoldi or recycled start, cycles,
                                  replacements, fetch, stopping test) in one kernel, with
                                  workgroup barriers between its steps and the small solves in
                                  LDS; mstab_solve_batch then advances its handles with one
                                  launch, one workgroup each.  For many small systems (a 64 x 64
                                  grid has 4096 rows), which one at a time use a few of the
                                  chip's 256 CUs.  Products read the handle's device copy of
                                  A (matrix_format applies).
                                  Requires n <= 2^20, F64 precision, PRECOND_NONE, REORDER_NONE
                                  and orthonormalize_recycle = 0 (E_INVALID at create otherwise).
                                  The residual history keeps the first 256 entries of a solve
                                  (the estimate of FETCH_ESTIMATE uses all of them);
                                  mstab_kernel_stats does not cover its kernel. */
} mstab_engine;

/* CSR matrix; all arrays are device pointers, n rows, nnz entries. */
typedef struct {
    int64_t n;
    int64_t nnz;
    const int32_t *row_ptr;    /* n+1 */
    const int32_t *col_idx;    /* nnz, sorted within each row */
    const double *val;         /* nnz */
} mstab_csr;

typedef struct {
    int32_t struct_size;       /* sizeof(mstab_options) */
    double tol;                /* relative residual target ||b - A x|| <= tol ||b||; default 1e-8 */
    int64_t max_mv;            /* budget of products with A per system; default 100000 */
    int32_t method;            /* mstab_method; default MSTAB */
    int32_t precision;         /* mstab_precision; default F64 */
    int32_t fetch;             /* mstab_fetch; default THRESHOLD */
    double fetch_rel;          /* THRESHOLD/ONCE level; default sqrt(tol) */
    int64_t fetch_level;       /* AT_LEVEL: level j of the fetched U, V */
    uint64_t p_seed;           /* seed of the cut-space basis P (counter-based uniform entries) */
    int32_t max_replacements;  /* true-residual replacements at the end of a solve; default 3 */
    int32_t max_refinements;   /* F32_REFINE: outer correction steps; default 20 */
    int32_t precond;           /* mstab_precond; default NONE */
    int32_t replace_every;     /* F64, F32_MATRIX: k > 0 replaces the recursive residual by the
                                  true one after every k-th cycle while it is above tol (one
                                  check MV each; the ocean run of Section 5.1 uses k = 1); these
                                  do not count against max_replacements.  Default 0 (only the
                                  final replacements).  F32_REFINE replaces after every cycle
                                  by construction and ignores it. */
    int32_t reorder;           /* mstab_reorder; default NONE */
    int32_t matrix_format;     /* mstab_format; default AUTO */
    int32_t orthonormalize_recycle; /* 1: orthonormalize the U, V a solve fetches (not in the
                                  paper, which keeps them as the cycle leaves them): CholQR
                                  in FP64, G = U^T U = R^T R, U := U R^-1, V := V R^-1 (so
                                  V = A U and span U are kept and the projection of the next
                                  right-hand side, Section 4.2, is unchanged in exact
                                  arithmetic), with P^T V recomputed; F32_REFINE
                                  orthonormalizes its FP32 U in FP64, then recomputes
                                  V = A U.  If U^T U is not numerically positive definite
                                  the data stay as fetched.  Default 0. */
    int32_t engine;            /* mstab_engine; default GRID */
    int32_t gmres_restart;     /* METHOD_GMRES: the restart length m, 1..1024; default 30 */
    const double *p_host;      /* NULL (default): the cut-space basis P is the counter-based one of
                                  p_seed, regenerated inside the kernels.  Else a host array of
                                  n x s doubles, column q at p_host + q n, all finite: the P
                                  that every projection of the handle uses (Section 2.4 leaves P
                                  arbitrary; Section 4.2 keeps it for the whole sequence).
                                  Rows are in the caller's order: with a reordering (RCM, or
                                  the ILU(0) colour order) the library permutes them with A's;
                                  with a splitting, P acts on the split system's residuals.
                                  mstab_create copies it to the device (the caller may free it
                                  afterwards); products then read P (8 s bytes per row) instead
                                  of regenerating it.  A non-finite entry: E_INVALID.  Recycle
                                  blobs carry a digest of it and are refused by a handle whose
                                  P differs. */
} mstab_options;

typedef struct {
    int32_t status;            /* the mstab_status of the solve */
    int32_t converged;         /* true relative residual <= tol */
    int32_t recycled;          /* the solve started from recycled U, V */
    int32_t restarts;          /* breakdown restarts (fresh Arnoldi basis); F32_REFINE: also FP32
                                  processes abandoned for loss of accuracy */
    int32_t replacements;      /* true-residual replacements */
    int32_t refinements;       /* F32_REFINE: FP32 processes started (1 unless one was abandoned) */
    int32_t guess_accepted;    /* mstab_solve_next_guess: the guess passed the residual gate */
    int32_t f64_fallback;      /* F32_REFINE: the FP32 processes stalled and FP64 iterations finished */
    int64_t mv;                /* products with A in the iteration (initial residual, Arnoldi, cycles) */
    int64_t mv_check;          /* products with A for true-residual checks and guess gates */
    int64_t mv_f64;            /* F32_REFINE, F32_MATRIX: products with the FP64 matrix (all in mv/mv_check) */
    int64_t cycles;            /* cycles of Algorithm 1 */
    int64_t level;             /* level j of the final U, V */
    int64_t fetched_level;     /* level of the data fetched by this solve, -1 if none */
    double relres_recursive;   /* ||r|| / ||b|| of the recursive residual at exit */
    double relres_true;        /* ||b - A x|| / ||b|| at exit */
    double seconds;            /* wall time of the call */
} mstab_info;

typedef struct mstab_solver mstab_solver;

#define MSTAB_MAX_BATCH 4096  /* handles per mstab_solve_batch call */

/* Fill o with defaults.  Errors: E_INVALID if o is NULL. */
mstab_status mstab_options_default(mstab_options *o);

/*
 * Create a solver for A with s shadow vectors and degree l (Algorithm 1's s
 * and l; 1 <= s <= 8, 1 <= l <= 8, n > s).  Allocates the workspace of
 * (s+1)(l+2) vectors (Table 1) plus the recycle store, on the current HIP
 * device.  o may be NULL (defaults).  The handle keeps the matrix pointers.
 * A's structure is checked first (as mstab_csr_check does; no product runs
 * on a malformed matrix).
 * Errors: E_INVALID, E_NOMEM, E_HIP; *out is NULL on failure.
 */
mstab_status mstab_create(const mstab_csr *A, int32_t s, int32_t ell, const mstab_options *o,
                          void *hip_stream, mstab_solver **out);

/*
 * Solve the next system of the sequence: A x = b (b, x: device, n doubles).
 * x holds the initial guess on entry (normally the previous solution) and the
 * solution on return.  With method MSTAB and held recycle data the solve starts
 * from it; the fetch policy may replace the held data.  info may be NULL.
 * On failure x holds the last consistent iterate.  With MSTAB_PRECOND_JACOBI,
 * b and x stay in the original system's terms: the call forms L^-1 b and
 * y0 = R x0, iterates on the split system and returns x = R^-1 y.
 */
mstab_status mstab_solve_next(mstab_solver *h, const double *b, double *x, mstab_info *info);

/*
 * mstab_solve_next on count independent handles at once (count <=
 * MSTAB_MAX_BATCH).  Handles of ENGINE_GRID: up to 16 host threads take the
 * handles in turn, each enqueueing on its handle's stream, so that the small
 * kernels of several latency-bound sequences share the GPU (handles on
 * distinct streams run concurrently, handles on one stream in turn).
 * Handles of ENGINE_WORKGROUP: one kernel launch per distinct s on h[0]'s
 * stream (after every handle's stream has drained), one workgroup per
 * handle; all handles must then be of that engine and on one device.  Either
 * way each handle's result equals that of mstab_solve_next on it alone.
 * h, b, x: host arrays of count entries (b[i], x[i]: device, n_i doubles
 * each, as for mstab_solve_next); info: NULL or count entries.  Handles must
 * be distinct.  Returns the first negative status of any handle
 * (mstab_last_error(NULL) names it), else NOT_CONVERGED if any did not
 * converge, else OK; each handle's own status is in info[i].status and its
 * error text in mstab_last_error(h[i]).
 */
mstab_status mstab_solve_batch(mstab_solver *const *h, int32_t count, const double *const *b,
                               double *const *x, mstab_info *info);

/*
 * As mstab_solve_next with an external initial guess: x_guess is used as x0
 * only if ||b - A x_guess|| < ||b - A x_prev|| (two counted check MVs),
 * otherwise x_prev is.  (b, x_prev, x_guess, x: device, n doubles; x may alias
 * x_prev or x_guess.)  info->guess_accepted reports the decision.
 * E_INVALID on a handle created with a preconditioner or a reordering.
 */
mstab_status mstab_solve_next_guess(mstab_solver *h, const double *b, const double *x_prev,
                                    const double *x_guess, double *x, mstab_info *info);

/*
 * r = b - A x with the handle's matrix and product kernel (device, n doubles
 * each; r must not alias b or x); norm2 (host, may be NULL) receives ||r||^2.
 * One product with A, counted in the handle's total (mstab_mv_count) but not
 * in any solve's info.  E_INVALID on a handle created with a preconditioner or a
 * reordering.
 */
mstab_status mstab_residual(mstab_solver *h, const double *b, const double *x, double *r,
                            double *norm2);

/* Products with A (Table 1's #MV, counted as Table 1 does, plus the
 * true-residual checks): over the handle's lifetime and in the last solve. */
mstab_status mstab_mv_count(const mstab_solver *h, int64_t *total, int64_t *last_system);

/*
 * Residual history of one solve on the handle: pairs (products with A so far,
 * recursive relative residual) after the initial residual and after every
 * cycle (the points of the paper's convergence graphs, Section 5.1 and 5.2).
 * system: 0-based index of the solve among all solves on the handle (in call
 * order, mstab_solve_count of them), or -1 for the last.  Host arrays of
 * capacity cap; *len gets the full length (entries beyond cap are dropped).
 * The handle keeps every solve's history until it is destroyed (about 16 bytes
 * per cycle).  Errors: E_INVALID (no such solve, NULL with cap > 0).
 */
mstab_status mstab_residual_history(const mstab_solver *h, int64_t system, int64_t *mv,
                                    double *relres, int64_t cap, int64_t *len);

/* Number of solves made on the handle (each mstab_solve_next, _guess or batch entry). */
mstab_status mstab_solve_count(const mstab_solver *h, int64_t *count);

/* Drop the held recycle data (the next MSTAB solve starts like IDR(s)stab) and
 * FETCH_ESTIMATE's estimate. */
mstab_status mstab_recycle_reset(mstab_solver *h);

/*
 * Copy the held recycle data out (F64 precision only): U, V device, n x s
 * column-major doubles each; level and have on host.  With have == 0 U, V are
 * left untouched.
 */
mstab_status mstab_recycle_get(const mstab_solver *h, double *U, double *V, int64_t *level,
                               int32_t *have);

/*
 * Install recycle data (F64 precision only): U, V device, n x s column-major,
 * with V = A U expected (Algorithm 1's prior requirement); level is recorded.
 */
mstab_status mstab_recycle_set(mstab_solver *h, const double *U, const double *V, int64_t level);

/*
 * Checkpoint and resume of the recycle state, the data a fetch writes out
 * (Section 5, preliminaries): a self-describing host byte blob holding the
 * level, the P^T V cache, U, V and FETCH_ESTIMATE's estimate (with the s, n, cut-space seed,
 * preconditioner and order they belong to).  export: dst (host, cap bytes)
 * receives the blob and *len its size; dst NULL only sets *len.  import:
 * installs a blob exported from a handle of the same problem (same s, n,
 * p_seed, precond and reorder), so that the next solve starts as the
 * exporting handle's would, bit for bit.  F64 and F32_MATRIX precision only.
 * Errors: E_INVALID (NULL, cap too small, foreign or truncated blob), E_HIP.
 */
mstab_status mstab_recycle_export(const mstab_solver *h, void *dst, size_t cap, size_t *len);
mstab_status mstab_recycle_import(mstab_solver *h, const void *src, size_t len);

/* Free the handle and its device memory.  NULL is accepted. */
mstab_status mstab_destroy(mstab_solver *h);

const char *mstab_status_str(mstab_status s);
const char *mstab_last_error(const mstab_solver *h);

/*
 * Kernel timing of the iteration (for roofline measurement): with enable = N
 * > 0, the first of every N launches of each kernel class below is bracketed
 * by HIP events on the handle's stream (N = 1: every launch; a larger N keeps
 * the events' own cost out of the timed work); enable = 0 stops.
 * mstab_kernel_stats returns, for a class since the last enable, the number of
 * timed launches, their summed duration in ms and their summed algorithmic
 * bytes (reads + writes the kernel must make).
 */
typedef enum {
    MSTAB_K_SPMV = 0,          /* y = A x with the P-projection epilogue */
    MSTAB_K_GAMMA = 1,         /* r^(i) -= V^(i) gamma, x += U gamma */
    MSTAB_K_ETA = 2,           /* v_q^(i) := r^(i+1) - [..] eta_q (the lower levels fused with
                                  the next level's gamma step) */
    MSTAB_K_GRAM = 3,          /* Z^T Z, Z^T r^(0) (fused with the last level's lower eta steps
                                  for l <= 4) */
    MSTAB_K_POLY = 4,          /* degree-l update of x, r, U, V with projections */
    MSTAB_K_COUNT = 5
} mstab_kernel_class;
mstab_status mstab_set_profiling(mstab_solver *h, int32_t enable);
mstab_status mstab_kernel_stats(const mstab_solver *h, int32_t kclass, int64_t *launches,
                                double *ms, double *bytes);

/*
 * Assemble the upwind finite-difference matrix of
 *   A = inv_dt I - div(kappa grad .) + beta . grad
 * on the n^dim interior nodes of the unit square (dim 2) or cube (dim 3),
 * x index fastest, homogeneous Dirichlet boundary, h = 1/(n+1).  Row entries in
 * column order (-z, -y, -x, diagonal, +x, +y, +z).  kappa (device, n^dim) may be
 * NULL for kappa = 1; face values are harmonic means, a boundary face takes
 * the node's value.  Arithmetic order (no contraction):
 *   diag = inv_dt + kf h^-2 over faces (-x,+x,-y,+y,-z,+z) + |beta_d| h^-1 over d
 *   lower neighbour: -(kf h^-2) - max(beta_d,0) h^-1
 *   upper neighbour: -(kf h^-2) + min(beta_d,0) h^-1
 * beta: host, 3 doubles (beta[2] ignored in 2-D).  Output device arrays:
 * row_ptr n^dim+1, col_idx and val with mstab_convdiff_nnz(dim, n) entries.
 */
int64_t mstab_convdiff_nnz(int32_t dim, int64_t n);
mstab_status mstab_assemble_convdiff(int32_t dim, int64_t n, const double *beta, double inv_dt,
                                     const double *kappa, int32_t *row_ptr, int32_t *col_idx,
                                     double *val, void *hip_stream);

/*
 * Structure check of an n-row CSR matrix in host memory (row_ptr n+1 and
 * col_idx nnz int32 entries): row_ptr[0] = 0, row_ptr non-decreasing,
 * row_ptr[n] = nnz, and every row's column indices strictly increasing and
 * inside [0, n).  mstab_create, mstab_spmv and mstab_jacobi_split make the
 * same checks on their device matrices (the row pointer on a host copy, the
 * columns in one kernel that reads only col_idx) before any product gathers
 * through the indices.  Host only.  Errors: E_INVALID naming the first
 * violation.
 */
mstab_status mstab_csr_check(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx);

/*
 * perm (host, n int32) receives the handle's row order: perm[new] = old, the
 * identity without MSTAB_REORDER_RCM.  Errors: E_INVALID, E_HIP.
 */
mstab_status mstab_permutation(const mstab_solver *h, int32_t *perm);

/*
 * Reverse Cuthill-McKee order of the symmetrized pattern (A + A^T, diagonal
 * ignored) of an n-row CSR matrix given in host memory: perm (host, n int32)
 * receives perm[new] = old.  Each connected component (taken in order of its
 * lowest-degree node) is searched breadth-first from a pseudo-peripheral node
 * (a minimum-degree node of the last level of a search from that node), each
 * node's unvisited neighbours appended by increasing degree, then index; the
 * order is then reversed.  Host only (no device work).  Errors: E_INVALID
 * (n out of range, NULL, or a pattern that mstab_csr_check refuses with
 * nnz = row_ptr[n]).
 */
mstab_status mstab_rcm_order(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                             int32_t *perm);

/*
 * The split diagonal preconditioning of MSTAB_PRECOND_JACOBI (Section 5.1's
 * split form, L = R = |D|^(1/2)): e_i = sqrt(|a_ii|), d_i = 1 / e_i and
 * val_out[k] = (val[k] d_i) d_j for entry k = (i, j), i.e. the values of
 * L^-1 A R^-1 in A's sparsity pattern.  val_out (nnz), d and e (n each):
 * device doubles; d or e may be NULL.  E_INVALID if a row has no stored,
 * finite, nonzero diagonal entry.
 */
mstab_status mstab_jacobi_split(const mstab_csr *A, double *val_out, double *d, double *e,
                                void *hip_stream);

/* y = A x (device, FP64), the plain sparse product used by the iteration.
 * A's structure is checked first (E_INVALID as mstab_csr_check). */
mstab_status mstab_spmv(const mstab_csr *A, const double *x, double *y, void *hip_stream);

/*
 * out = P^T y for the cut-space basis of p_seed: y device (n doubles), out host
 * (s doubles).  P entries are regenerated from the counter-based hash.
 */
mstab_status mstab_project(int64_t n, int32_t s, uint64_t p_seed, const double *y, double *out,
                           void *hip_stream);

/*
 * mstab_project without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, result and errors as mstab_project; its
 * control block and workgroup partials live in a fixed device array of
 * ~76 KB that the library holds on each GPU it runs on until the process
 * ends.  n must be below 2^29 (E_INVALID otherwise).  Every call on one GPU
 * shares that array: calls that overlap on one GPU (other streams or host
 * threads) race and must be serialized by the caller.
 */
mstab_status mstab_project_noalloc(int64_t n, int32_t s, uint64_t p_seed, const double *y,
                                   double *out, void *hip_stream);

/* Implicit Euler right-hand side b = x inv_dt + f (device, n doubles, no contraction). */
mstab_status mstab_rhs_step(int64_t n, const double *x, double inv_dt, const double *f, double *b,
                            void *hip_stream);

/* ------------------------------------------------------------------------ */
/*
 * Learned initial guess.  The paper solves each system of the sequence
 * (Section 1) starting from the previous solution; this extension offers a
 * better x0: a convolutional network maps the system (x^(i), b^(i+1)) on an
 * H x W grid to the correction d = x^(i+1) - x^(i).  Its features are the
 * residual r0 = b^(i+1) - A x^(i) (mstab_residual) and x^(i): d solves
 * A d = r0, so the map is linear in r0 and, for a matrix with constant
 * coefficients, translation invariant, which a convolution can approximate
 * locally.  The solver has the last word: mstab_solve_next_guess takes the
 * network's guess only if its true residual is below that of x^(i).
 *
 * Network: 6 layers of 3x3 convolutions with zero padding, channels
 * 2 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, ReLU after each layer but the last,
 * loss = mean squared error, Adam (beta 0.9, 0.999, eps 1e-8) on FP32 master
 * parameters.  Forward and backward run on BF16 weights and activations with
 * FP32 accumulation (MFMA for the 32 -> 32 layers).
 * Per sample, s = max|r0| and sx = max|x^(i)|; input channels (r0 / s,
 * x^(i) / sx); target (x^(i+1) - x^(i)) unit / s; guess x^(i) + (s / unit)
 * output.  unit (fixed per network, e.g. the largest diagonal entry of A)
 * makes the target of order one.  Quotients are divisions rounded to FP32,
 * then to BF16 (nearest even); a zero scale gives a zero channel.
 *
 * Layouts: a grid vector is the solver's vector (x index fastest, n = H W,
 * W a multiple of 32).  A prepared input is H W pixels x 2 channels of BF16
 * (channels fastest, 4 bytes per pixel); a batch stores samples one after the
 * other.  Parameters are mstab_cnn_param_count() floats, layer after layer,
 * each w[c_out][c_in][3][3] followed by b[c_out].
 */
typedef struct mstab_cnn mstab_cnn;

/* Number of FP32 parameters (37 889). */
int64_t mstab_cnn_param_count(void);

/*
 * Create a network for H x W grids and batches of up to max_batch samples
 * (H >= 1, W a positive multiple of 32, H W max_batch < 2^31, unit > 0).
 * dilation (host, 6 values in 1..32, NULL = all 1) spaces the taps of layer
 * l dilation[l] cells apart: y(i, j) takes x(i + (di - 1) d, j + (dj - 1) d).
 * Allocates parameters, Adam moments and the activations of a full batch on
 * the current device; parameters start at zero (call mstab_cnn_set_params).
 * Errors: E_INVALID, E_NOMEM, E_HIP; *out is NULL on failure.
 */
mstab_status mstab_cnn_create(int64_t H, int64_t W, int32_t max_batch, double unit,
                              const int32_t *dilation, void *hip_stream, mstab_cnn **out);
mstab_status mstab_cnn_destroy(mstab_cnn *h);

/* Set the FP32 parameters (host, count floats) and reset the Adam state. */
mstab_status mstab_cnn_set_params(mstab_cnn *h, const float *params_host, int64_t count);

/* Copy parameters and/or the last gradient to host (either may be NULL). */
mstab_status mstab_cnn_get_params(const mstab_cnn *h, float *params_host, float *grads_host,
                                  int64_t count);

/*
 * Prepare one sample: input_bf16 (device, 2 H W BF16) from x_prev and r0, and,
 * if target is not NULL, target (device, H W floats) from x_next.  x_prev, r0,
 * x_next: device, H W doubles.  scale (host, may be NULL) receives s.
 */
mstab_status mstab_cnn_prepare(mstab_cnn *h, const double *x_prev, const double *r0,
                               const double *x_next, void *input_bf16, float *target,
                               double *scale);

/* Forward pass of a batch of prepared inputs; out (device, batch H W floats) may be NULL. */
mstab_status mstab_cnn_forward(mstab_cnn *h, const void *input_bf16, int32_t batch, float *out);

/*
 * Forward and backward pass of a batch: the gradient of the batch mean loss
 * is kept on the device for mstab_cnn_adam_step; loss (host, may be NULL)
 * receives the mean loss.  Weight gradients are summed in a fixed order
 * (deterministic).
 */
mstab_status mstab_cnn_gradient(mstab_cnn *h, const void *input_bf16, const float *target,
                                int32_t batch, double *loss);

/* One Adam update with learning rate lr from the last gradient. */
mstab_status mstab_cnn_adam_step(mstab_cnn *h, double lr);

/*
 * x_guess = x_prev + (s / unit) network(r0 / s, x_prev / sx) for one system
 * (device, H W doubles; x_guess may alias x_prev).
 */
mstab_status mstab_cnn_guess(mstab_cnn *h, const double *x_prev, const double *r0,
                             double *x_guess);

/*
 * Copy an internal tensor of the last pass to dst (device, bytes capacity), for
 * tests: which 0 = input of layer `layer` (0..5; BF16, 2 or 32 channels per
 * pixel), 1 = network output (FP32), 2 = gradient of the loss with respect to
 * layer `layer`'s pre-activation output (0..4; BF16, 32 channels), 3 = gradient
 * with respect to the output (FP32).  Sizes are those of a full batch.
 */
mstab_status mstab_cnn_tensor(const mstab_cnn *h, int32_t which, int32_t layer, void *dst,
                              int64_t bytes);

const char *mstab_cnn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MSTAB_H */
