/*
 * refine.h -- C ABI of the MI355X (gfx950) library for iterative refinement
 * of a subset of eigenvectors of a real symmetric matrix (Terao, Ozaki,
 * Imamura and Ogita, "Iterative Refinement for a Subset of Eigenvectors of
 * Symmetric Matrices via Matrix Multiplications", arXiv 2602.23778).
 *
 * Problem (Sec. 1 and Sec. 3, eqs. HX-and-HAX and update-X): A is n x n real
 * symmetric, X (n x k, k < n) approximates k eigenvectors of A.  One
 * refinement step (Algorithm 4 with Algorithm 1) computes
 *     W = A X,  d_j = x_j^T w_j / x_j^T x_j,  R = W - X diag(d),
 *     the compact WY factors Y = X - I_{n,k}, T = -Y1^{-T},
 *     V = H^T R,  the correction matrix E_L (correction step of Algorithm 4),
 *     X <- X + H E_L,  and normalises the columns of X.
 * The targets are the k eigenvalues of largest |lambda - mu| (eq. condition,
 * Sec. 5.1 for the shifted variants); mu = 0 is the paper's default.
 *
 * Conventions for every entry point:
 *   - All matrix and iterate pointers are DEVICE pointers owned by the caller.
 *   - Dense A is row-major with leading dimension lda >= n (A is symmetric,
 *     so row- and column-major coincide).  CSR A has int32 row_ptr[n+1],
 *     int32 col_idx[nnz] (full symmetric pattern) and double val[nnz].
 *   - X is row-major n x k with leading dimension ldx >= k (the layout of a
 *     contiguous PyTorch tensor of shape (n, k)); it is updated in place.
 *   - Work is issued on the HIP stream given at init (NULL = the null
 *     stream).  Calls on one context must not overlap; contexts are not
 *     thread-safe.  A context owns its workspace, its INT8 slices of A (split
 *     mode) and its HIP graphs; A is borrowed and must stay valid until
 *     refine_destroy (in split mode A is read only during refine_init).
 *   - Return values are the status codes below; no C++ exception crosses
 *     the ABI.  On an error status X holds the last iterate that was
 *     accepted (a step whose correction is rejected does not write X).
 */
#ifndef REFINE_H
#define REFINE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define REFINE_OK 0
#define REFINE_NOT_CONVERGED 1   /* refine_run: max_iters reached before tol */
#define REFINE_EINVAL (-1)       /* bad argument (sizes, pointers, options) */
#define REFINE_ENOMEM (-2)       /* device or host allocation failed */
#define REFINE_EHIP (-3)         /* a HIP runtime call failed */
#define REFINE_EWY_SINGULAR (-4) /* Y1 = X(1:k,:) - I_k singular or cond_1 > 1/(n u)
                                    (Algorithm 1 needs Y1 nonsingular, Sec. 3.1.1);
                                    X is unchanged: refine_sign_flip, then step again */
#define REFINE_EDIVERGED (-5)    /* ||E_L||_F >= 1 (the Neumann expansion of
                                    eq. Neumann needs ||E|| < 1), or ||E_L||_F grew
                                    tenfold over three steps (Sec. 4.3 guidance) */
#define REFINE_ENONFINITE (-6)   /* NaN or Inf in X or in the step's reductions */
#define REFINE_ERANK (-7)        /* refine_rayleigh_ritz: X^T X is not numerically
                                    positive definite (dependent columns) */

typedef struct refine_ctx refine_ctx;
typedef struct refine_batch refine_batch;

typedef enum { REFINE_DENSE = 0, REFINE_CSR = 1 } refine_kind;

/* Arithmetic of the product W = A X (product step of Algorithm 4).
 *   REFINE_FP64: every step in IEEE double (the paper's experiments, Sec. 3.1.3).
 *   REFINE_SPLIT_INT8: A X by error-free splitting of A and X into INT8
 *     slices with exact INT32 accumulation on the matrix cores, recombined
 *     into a double-double W; the residual R = W - X diag(d) is then formed
 *     with an exact product, the rest of the step in double (the
 *     mixed-precision direction of Sec. 3.1.3).  Dense only.
 *   REFINE_SPLIT_FP8: declared and rejected (refine_init returns
 *     REFINE_EINVAL).  On this hardware FP8 and INT8 matrix products run at
 *     the same dense rate, and an FP8 (e4m3) slice holds an exact signed digit
 *     of 4 bits against INT8's 8, so an FP8 split needs about twice the slices
 *     and four times the slice products of the INT8 one for the same W.
 *   REFINE_SPLIT_CRT: A X by the modular route to the same double-double W
 *     (Ozaki scheme II, the integer direction of Sec. 3.1.3): A and X are
 *     scaled by powers of two per row and per column and rounded to integers
 *     A', X' of bA and bX bits; N coprime moduli m_t <= 256 (256, 255, 253,
 *     ...) with bA + bX = L - 3 - ceil(log2 n), L the bit length of their
 *     product M, make A'X' the one integer in [-M/2, M/2) with the residues
 *     of the N INT8 products (A' mod m_t)(X' mod m_t) (exact INT32 sums), and
 *     the Chinese remainder theorem (Garner's mixed radix) recovers it; W is
 *     that integer scaled back, as a double-double pair.  One product per
 *     modulus instead of s(s+1)/2 slice products; A's residues take N n^2
 *     bytes (made at init), which is what a step streams.  Dense, one
 *     problem (refine_batch_init returns REFINE_EINVAL). */
typedef enum {
  REFINE_FP64 = 0,
  REFINE_SPLIT_INT8 = 1,
  REFINE_SPLIT_FP8 = 2,
  REFINE_SPLIT_CRT = 3
} refine_precision;

/* Which eigenpairs are targeted (eq. condition and Sec. 5.1):
 *   LARGEST_ABS: mu = 0, the k eigenvalues of largest |lambda|;
 *   SMALLEST:    mu = max_i (a_ii + sum_{j!=i} |a_ij|) (Gershgorin upper bound);
 *   LARGEST:     mu = min_i (a_ii - sum_{j!=i} |a_ij|) (Gershgorin lower bound);
 *   SHIFT:       mu = options.shift, e.g. (||A||_inf + lambda_{k+1})/2 (Sec. 5.1);
 *   SMALLEST_ABS: the k eigenvalues of smallest |lambda| (Sec. 5.2): the method
 *     runs on B = A^2 - alpha I, the product step of Algorithm 4 as A (A X) by two
 *     products (A^2 is never formed), with alpha = (||A||^2 + lhat^2)/2, lhat =
 *     options.shift the caller's estimate of the (k+1)-th smallest |lambda|
 *     (alpha = ||A||^2 when options.shift <= 0, which separates the targets
 *     too, at a slower rate); ||A|| is options.norm_a, else ||A||_inf.  delta
 *     and the residual statistic then use ||A||^2, a bound of ||B||, and the
 *     Rayleigh quotients are those of A^2 (lambda^2).  FP64 only, dense or
 *     CSR.  The paper prints |lhat| where the separation condition asks for
 *     lhat^2 (alpha must exceed (||A||^2 + lambda_k^2)/2). */
typedef enum {
  REFINE_TARGET_LARGEST_ABS = 0,
  REFINE_TARGET_SMALLEST = 1,
  REFINE_TARGET_LARGEST = 2,
  REFINE_TARGET_SHIFT = 3,
  REFINE_TARGET_SMALLEST_ABS = 4
} refine_target;

/* beta_ij for (near-)equal Rayleigh quotients (correction step of Algorithm 4):
 * -x_i^T x_j / 2, or 0 after Rayleigh-Ritz preprocessing (Sec. 3.4). */
typedef enum { REFINE_BETA_HALF_GRAM = 0, REFINE_BETA_ZERO = 1 } refine_beta;

/* Stopping rules of Sec. 3.1.3: a fixed number of steps, ||E_L||_F <= tol,
 * or ||A X - X D||_F / ||A|| <= tol.  The test is made after each step; the
 * statistics describe the iterate that entered that step. */
typedef enum {
  REFINE_STOP_ITERS = 0,
  REFINE_STOP_CORRECTION = 1,
  REFINE_STOP_RESIDUAL = 2
} refine_stop;

typedef struct {
  refine_kind kind;
  int64_t n;
  const double* a;         /* dense: device pointer, row-major, lda >= n */
  int64_t lda;
  const int32_t* row_ptr;  /* CSR: device pointers */
  const int32_t* col_idx;
  const double* val;
  int64_t nnz;
} refine_matrix;

typedef struct {
  refine_precision precision;
  refine_target target;
  double shift;            /* mu for REFINE_TARGET_SHIFT; the estimate lhat for
                              REFINE_TARGET_SMALLEST_ABS */
  double delta_c;          /* delta = delta_c * ||A|| * 2^-53; the paper uses 10 (Sec. 3.1.3) */
  double norm_a;           /* ||A|| for delta and the residual statistic; <= 0: ||A||_inf */
  refine_beta beta;
  int32_t normalize;       /* 1: normalise columns after each update (Sec. 3.1.3) */
  int32_t slices;          /* REFINE_SPLIT_INT8: INT8 digit slices per operand,
                              7..10; 0 = 9 (45 slice products; W then carries
                              about 2^-60 of the row and column scales, below
                              the rounding of an FP64 product).
                              REFINE_SPLIT_CRT: moduli N, 12..16; 0 = 16
                              (bA, bX = 55, 54 bits at n = 16384) */
} refine_options;

typedef struct {
  double corr_fro;         /* ||E_L||_F of the last step */
  double resid_rel;        /* ||A X - X D||_F / ||A|| of the last step's input */
  int32_t iters;           /* steps applied */
  int32_t status;          /* status code of the last step */
} refine_stats;

/* Fills *opt with the defaults: FP64, LARGEST_ABS, delta_c = 10, norm_a = 0
 * (use ||A||_inf), beta = -x_i^T x_j / 2, normalize = 1, slices = 0. */
void refine_options_default(refine_options* opt);

/* Creates a context for one problem with k target vectors, 1 <= k <= 128,
 * k < n, n < 2^31 (CSR nnz < 2^31; split mode n <= 65536).  Computes ||A||_inf
 * and the Gershgorin bounds on the device, slices A in split mode, allocates
 * the workspace and records the step as a HIP graph.  hip_stream is a
 * hipStream_t (NULL for the null stream).  Synchronises the stream. */
int refine_init(refine_ctx** ctx, const refine_matrix* A, int32_t k,
                const refine_options* opt, void* hip_stream);

/* One refinement step on X (device, n x k row-major, leading dimension ldx),
 * in place.  The divergence test (REFINE_EDIVERGED) compares ||E_L||_F with
 * the steps since the context last saw a different X pointer or ldx, an
 * error status or a refine_run: a caller that restarts from new values in
 * the same buffer calls refine_run (or passes another buffer) to start a
 * new history.  stats == NULL: the step is only enqueued (no host
 * synchronisation).  A step enqueued that way that fails keeps its status in
 * the context and the steps enqueued after it do nothing; the next call that
 * reports (refine_step with stats, refine_run, refine_rayleigh_ritz,
 * refine_sign_flip, refine_time_product, or a step on another X) returns
 * that status first, without doing its own work, and clears it.  Otherwise
 * (stats != NULL) the stream is synchronised and *stats filled. */
int refine_step(refine_ctx* ctx, double* X, int64_t ldx, refine_stats* stats);

/* Up to max_iters steps, stopping early when the rule `stop` meets tol or on
 * an error status.  The stopping test runs on the device; the host checks it
 * once per chunk of steps.  Returns REFINE_OK when the rule was met,
 * REFINE_NOT_CONVERGED when max_iters steps ran without meeting it (always
 * for REFINE_STOP_ITERS, which then returns REFINE_OK), or an error code. */
int refine_run(refine_ctx* ctx, double* X, int64_t ldx, int32_t max_iters,
               refine_stop stop, double tol, refine_stats* stats);

/* Scalars computed at init: mu (the shift in use), ||A||_inf, the norm used
 * for delta and the residual, and delta itself. */
int refine_get_info(const refine_ctx* ctx, double* mu, double* norm_inf,
                    double* norm_used, double* delta);

/* Rayleigh-Ritz preprocessing for clustered targets (Sec. 3.4, handling
 * clustered eigenvalues): solves the k x k symmetric-definite problem
 * (X^T A X) S = (X^T X) S Theta and overwrites X (device, n x k, ld ldx >= k,
 * the caller's) with X S, so that X^T X = I and X^T A X = Theta to rounding.
 * Columns come ordered by |theta - mu| descending (ties in ascending theta),
 * each signed so that X(j, j) <= 0.  The next applied step of this context
 * (refine_step or the first of refine_run) then takes the leading k x k block
 * of E_L as zero, so it forms no d_j - d_i denominator; later steps are
 * plain.  A X is formed by the context's product (FP64, split or CSR), the
 * k x k problem on one workgroup (Cholesky, then cyclic Jacobi).  Returns
 * REFINE_OK, REFINE_ERANK when X^T X is not positive definite (X unchanged),
 * or an argument or HIP error.  Synchronises with the host once. */
int refine_rayleigh_ritz(refine_ctx* ctx, double* X, int64_t ldx);

/* One-time column sign flip X <- X Sigma (Sec. 3.1.1), for an X on which the
 * step reports REFINE_EWY_SINGULAR.  Sigma = diag(sigma) is the sign matrix
 * of the modified LU factorisation of X (Algorithm 2: sigma_j = -sign(q_jj)
 * of the diagonal entry at elimination step j, sign(0) = +1), which depends
 * on the leading k x k block of X alone; after the flip, X Sigma - I_{n,k} =
 * Y U Sigma with Y unit lower trapezoidal and |u_jj| >= 1 (Algorithm 3), so
 * the leading block of the compact WY factor is nonsingular and the steps of
 * Algorithm 1 apply.  The flip spans the same space and keeps a Rayleigh-Ritz
 * basis one (the zero leading block of E_L stays armed).
 * X: device, n x k row-major, leading dimension ldx, updated in place.
 * sigma: HOST array of k entries receiving +1 or -1, or NULL.
 * Returns REFINE_OK, REFINE_ENONFINITE for a NaN or Inf in the leading block
 * or a pivot (X unchanged), or an argument or HIP error.  Synchronises with
 * the host once. */
int refine_sign_flip(refine_ctx* ctx, double* X, int64_t ldx, int32_t* sigma);

int refine_destroy(refine_ctx* ctx);

/* Measurement hook for the roofline figures: enqueues `reps` launches of the
 * product W = A X alone (product step of Algorithm 4; its cost is the O(nnz(A) k)
 * row of Table 1; in split mode the slicing of X, the INT8 products and the
 * K-split sum), in the context's precision and launch configuration, on
 * the context's stream between two HIP events, waits for them and stores the
 * mean time of one launch in *ms.  X is only read; the context's workspace
 * copy of W is overwritten, so call it between steps, not inside one. */
int refine_time_product(refine_ctx* ctx, double* X, int64_t ldx, int32_t reps, float* ms);

/* Measurement hook, per kernel: as refine_time_product, but the kernels of
 * the product are timed one by one (HIP events on the context's stream
 * between consecutive launches), after one untimed launch of the whole
 * product.  ms[i] receives the mean time of the product's i-th kernel over
 * `reps` launches (1 <= reps <= 64), in launch order:
 *   FP64 dense: the GEMM (refine_time_product leaves the K-split sum out
 *     alike);
 *   REFINE_SPLIT_INT8: column maxima of |X|, slicing of X, the slice
 *     products, and the K-split sum when there is one;
 *   REFINE_SPLIT_CRT: column maxima of |X|, residues of X, the residue
 *     products, the reconstruction of W;
 *   CSR: the SpMM.
 * *nparts receives the number of kernels (at most max_parts are stored).
 * X is only read; call it between steps. */
int refine_time_product_parts(refine_ctx* ctx, double* X, int64_t ldx, int32_t reps, float* ms,
                              int32_t max_parts, int32_t* nparts);

/* One refinement step that allocates nothing, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the step of refine_step for a dense FP64
 * problem, with every buffer it needs beyond A and X (descriptor, work items,
 * W, the update, the block partials, the k x k area, the control word) in a
 * static 64 MiB array the library keeps on each GPU until the process ends.
 * No context: each call starts from scratch (a first step; no divergence
 * history, no warm start of the k x k solve) and uses a fixed launch
 * configuration.  A, X (device, X updated in place, ld ldx >= k), k and the
 * options as for refine_init and refine_step, except: precision FP64 only;
 * target LARGEST_ABS or SHIFT (mu = options.shift); options.norm_a must be
 * given (> 0), since ||A||_inf would need a host round trip.  The whole
 * workspace must fit the array: about 16 n k + 8 (2k^2 + k) min(n, 64 row
 * blocks) bytes plus small tables (n k up to about 2^21 at k = 128); a larger
 * problem returns REFINE_EINVAL.  Work is enqueued on hip_stream.  stats ==
 * NULL: no host synchronisation, and a failed step is not reported (X is
 * left unchanged by a rejected correction); otherwise the stream is
 * synchronised, *stats filled and the step's status returned.  Calls that
 * overlap on one GPU share the array and race. */
int refine_step_static(const refine_matrix* A, int32_t k, const refine_options* opt, double* X,
                       int64_t ldx, void* hip_stream, refine_stats* stats);

/* Batched problems (independent dense A_p, n_p x n_p, with k_p targets):
 * every step of every problem runs in one grouped launch per kernel, over
 * (problem, tile) work items, and the whole step is one HIP graph.  Options
 * apply to all problems; As[p], ks[p] as in refine_init.  X pointers are
 * given per call.  In REFINE_SPLIT_INT8 mode every A is sliced at init and
 * the products of all problems share one launch. */
int refine_batch_init(refine_batch** b, int32_t count, const refine_matrix* As,
                      const int32_t* ks, const refine_options* opt,
                      void* hip_stream);

/* iters steps on all problems (Xs[p]: device n_p x k_p row-major, ld ldxs[p]).
 * per_problem (count entries) may be NULL: no host synchronisation; a failure
 * of such a run is returned (first failing problem's status) by the next
 * batch call that reports, before it does its own work, as for refine_step. */
int refine_batch_run(refine_batch* b, double* const* Xs, const int64_t* ldxs,
                     int32_t iters, refine_stats* per_problem);

/* Rayleigh-Ritz preprocessing of every problem of a batch, as
 * refine_rayleigh_ritz (Sec. 3.4, clustered eigenvalues): Xs[p] (device,
 * n_p x k_p, ld ldxs[p], NULL ldxs meaning ld = k_p) is overwritten with its
 * Ritz basis and the next applied step of that problem takes the leading
 * block of E_L as zero.  status (count entries) may be NULL; it receives each
 * problem's result (REFINE_OK or REFINE_ERANK, whose X is left unchanged).
 * Returns REFINE_OK, the first failing problem's status, or an argument or
 * HIP error.  Synchronises with the host once. */
int refine_batch_rayleigh_ritz(refine_batch* b, double* const* Xs, const int64_t* ldxs,
                               int32_t* status);

/* The sign flip of refine_sign_flip on every problem of a batch, in one
 * grouped launch (one workgroup per problem for the k_p x k_p elimination,
 * then (problem, row block) items for the column scaling).  status (count
 * entries) may be NULL; it receives each problem's result (REFINE_OK or
 * REFINE_ENONFINITE, whose X is left unchanged).  Returns REFINE_OK, the
 * first failing problem's status, or an argument or HIP error.  Synchronises
 * with the host once. */
int refine_batch_sign_flip(refine_batch* b, double* const* Xs, const int64_t* ldxs,
                           int32_t* status);

int refine_batch_destroy(refine_batch* b);

/* Measurement hook, as refine_time_product for a batch: `reps` launches of
 * the grouped product of all problems (with the X pointers of the last
 * refine_batch_run; in split mode with the slicing of every X), mean time of
 * one launch in *ms.  Call it between runs. */
int refine_batch_time_product(refine_batch* b, int32_t reps, float* ms);

/* Static string for a status code. */
const char* refine_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* REFINE_H */
