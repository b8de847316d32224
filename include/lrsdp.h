/*
 * lrsdp.h -- C ABI of the MI355X (gfx950) solver for the interior-point Hessian
 * equation of a large-and-sparse low-rank SDP.
 *
 * Paper: R. Y. Zhang and J. Lavaei, "Modified Interior-Point Method for
 * Large-and-Sparse Low-Rank Semidefinite Programs" (arXiv 1703.10973).
 *
 * The operation is Algorithm 1 of Section 3.3: given the SDP data A_1..A_m
 * (eqs SDP/SDD), a scaling matrix W (positive definite, Section 2.2), a rank k
 * and a right-hand side r, return y with ||H y - r|| <= eps ||r||, where
 * H = A^T (W kron W) A (eqs hesseqn2 and hesseqn1).  H is applied matrix-free;
 * PCG is preconditioned by H~ = tau^2 A^T A + bold U bold U^T (eq AtIUUtAt)
 * through the Sherman-Morrison-Woodbury form (eq SMW2).
 *
 * Step labels used here and in the sources:
 *   A0 the data A_i as sparse triplets, checked and laid out (Ass. 2, Section 1.1);
 *   A1 the eigen step: tau and the k largest eigenpairs of W (Algorithm 1 step 1a);
 *   A2 U, W0 = W - U U^T and Z = chol(2 W0 + U U^T) with Z^{-1} (step 1b);
 *   A3 formation of bold S = tau^2 I + bold U^T (A^T A)^{-1} bold U (step 2, eq SMW2);
 *   A4 deflation and the Cholesky factor of bold S with its inverse (step 2);
 *   A5 the product H v (eq hesseqn2);
 *   A6 the preconditioner H~^{-1} v (eqs SMW2, Umv; step 3);
 *   A7 H v in the split form of eq hessExp1, the W0 part in lower precision;
 *   A8 PCG, and refinement with double-double residuals (step 3).
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers on the context's device unless the
 *     comment says "host".  The library copies what it keeps; no caller pointer
 *     is retained after a call returns.  The caller owns every array it passes.
 *   - Matrices are dense, row-major, with leading dimension equal to the number
 *     of columns (W, Z, W0 are symmetric or lower triangular n x n).
 *   - Work is enqueued on the context's stream; every call that returns a status
 *     synchronizes that stream before returning, so outputs are ready on return.
 *   - Input ordering: a call reads its device inputs when its work reaches the context's
 *     stream.  A context created with stream == NULL runs on a stream of its own that is
 *     blocking, i.e. ordered after all earlier work on the legacy default stream (stream 0),
 *     so inputs written there (for example by torch on its default stream) need no extra
 *     synchronization.  Inputs written on any other stream must be complete before the call,
 *     or the context must be created on that stream.
 *   - Return value: LRSDP_OK (0), a positive warning, or a negative error.  After
 *     an error every handle stays valid and may be reused or destroyed.
 *   - A handle must not be used by two host threads at once.
 *   - Handles may be destroyed in any order: destroying a context that still has live
 *     problems, or a problem that still has live factors, only marks it, and it is released
 *     together with its last child.  A marked handle must not be used again.
 */
#ifndef LRSDP_H
#define LRSDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Only the functions below are exported from the shared library. */
#if defined(__GNUC__) || defined(__clang__)
#define LRSDP_API __attribute__((visibility("default")))
#else
#define LRSDP_API
#endif

/* ------------------------------------------------------------------ status */
#define LRSDP_OK                      0
#define LRSDP_NOT_CONVERGED           1   /* warning: y holds the last iterate, info filled   */
#define LRSDP_ERR_INVALID_ARG        -1   /* n <= 0, k not in [1, n-1], index out of range,   */
                                          /* row > col, null pointer, bad option value        */
#define LRSDP_ERR_DUPLICATE_PAIR     -2   /* two constraints with the same entry (a, b)      */
#define LRSDP_ERR_UNSUPPORTED        -3   /* a constraint with more than one triplet, i.e.    */
                                          /* A^T A not diagonal (Assumption 2 then needs a     */
                                          /* sparse Cholesky of A^T A, which is not built)     */
#define LRSDP_ERR_NOT_PD_W           -4   /* lambda_min(W) <= 0 or W not finite                */
#define LRSDP_ERR_CHOL_Z             -5   /* Cholesky of 2 W0 + U U^T broke down               */
#define LRSDP_ERR_CHOL_S             -6   /* Cholesky of bold S broke down                     */
#define LRSDP_ERR_OUT_OF_BUDGET      -7   /* the context's HBM budget would be exceeded         */
#define LRSDP_ERR_STAGNATED          -8   /* refinement stopped reducing the true residual     */
#define LRSDP_ERR_INDEFINITE_PRECOND -9   /* PCG met r^T z <= 0 or p^T H p <= 0                */
#define LRSDP_ERR_DEVICE            -10   /* a HIP runtime call failed                          */
#define LRSDP_ERR_EIG               -11   /* the symmetric eigensolver did not converge         */
#define LRSDP_ERR_SCRATCH           -12   /* the call needs more than the library's fixed       */
                                          /* scratch array holds (allocation-free entry point) */
#define LRSDP_ERR_IPM               -13   /* lrsdp_ipm_solve: an iterate X or S lost positive   */
                                          /* definiteness, or the square root of the scaling  */
                                          /* did not converge                                  */
#define LRSDP_PENDING                 2   /* lrsdp_server_poll: the request has not finished   */

/* ------------------------------------------------------------------ handles */
typedef struct lrsdp_ctx lrsdp_ctx;          /* device, stream, HBM budget                     */
typedef struct lrsdp_problem lrsdp_problem;  /* the data A_1..A_m on the device (step A0)      */
typedef struct lrsdp_factor lrsdp_factor;    /* W and the preconditioner factors (Alg. 1 1-2) */

/* ------------------------------------------------------------------ options */
#define LRSDP_PREC_FP64   0   /* H v with W in FP64                                            */
#define LRSDP_PREC_FP32   1   /* split H v: W0 part in FP32 (FP32 accumulation), rest FP64/dd  */
#define LRSDP_PREC_BF16   2   /* split H v: W0 part with BF16 operands, FP32 accumulation      */
#define LRSDP_PREC_AUTO   3   /* FP32 split when the solve refines in double-double anyway     */
                              /* (mu small, see dd_mode), else plain FP64 PCG                   */

#define LRSDP_DD_OFF      0   /* plain PCG in FP64, answer in y only                            */
#define LRSDP_DD_ON       1   /* outer refinement with double-double residual, answer y + y_lo  */
#define LRSDP_DD_AUTO     2   /* ON when lambda_{n-k}(W) / lambda_{n-k+1}(W) < dd_auto_ratio     */

typedef struct lrsdp_opts {
  double eps;            /* target relative residual ||r - H y|| / ||r|| (default 1e-8)     */
  int max_iter;          /* PCG iterations per inner solve (default 200)                    */
  int precision;         /* LRSDP_PREC_* (default FP64)                                     */
  int dd_mode;           /* LRSDP_DD_* (default AUTO)                                       */
  int deflate;           /* 1: deflate the k(k-1)/2 null directions of bold S (default 1)   */
  int max_outer;         /* outer refinement steps (default 8)                              */
  double inner_eps;      /* inner PCG tolerance in refinement mode; 0 (default): 1e-2 with  */
                         /* BF16 W0 products, else 1e-3                                     */
  double dd_auto_ratio;  /* spectral-gap threshold for LRSDP_DD_AUTO (default 2e-5)         */
  int dd_precond;        /* SMW pieces in double-double: 0 off, 1 on, 2 auto (default 2:    */
                         /* on when tau < 1e-7 lambda_max(W))                                */
  int tau_rule;          /* LRSDP_TAU_* (default MEAN)                                      */
  int precond;           /* LRSDP_PRECOND_* (default SMW)                                   */
} lrsdp_opts;

/* The preconditioner of the PCG (a factor is built for one of them).
 *   SMW: H~ = tau^2 A^T A + bold U bold U^T (eq AtIUUtAt), applied by eq SMW2 (Algorithm 1):
 *        Z = chol(2 W0 + U U^T), bold S = tau^2 I + bold U^T (A^T A)^{-1} bold U; its FP64
 *        form loses definiteness as mu -> 0 and is then carried in double-double (dd_precond).
 *   AUG: H^ = A^T (tau^2 I + 2 tau (U U^T kron I)) A (eq sparse_prec, Section 4.2), applied
 *        through the augmented system of eq aug_prec: x is eliminated first (1 x 1 pivots
 *        tau^2 (A^T A)_ii, no fill outside the pattern) and the trailing nk x nk block
 *        tau/2 I + B^T (A^T A)^{-1} B, B = A^T (U kron I), is factored densely (Cholesky and
 *        inverse, FP64 MFMA).  No Z, no bold S formation GEMMs, no double-double pieces: the
 *        condition number of eq aug_prec is Theta(1/sqrt(mu)).  PCG needs about
 *        k^2 + O(log 1/(eps mu)) iterations (Lemma aug_prec).  dd_precond and deflate are
 *        ignored. */
#define LRSDP_PRECOND_SMW 0
#define LRSDP_PRECOND_AUG 1

/* The shift tau of the split W = W0 + U U^T (eq Wsplit2).  Algorithm 1 step 1a takes
 * tau = lambda_min(W); Section 3.1 allows any tau in [lambda_min(Lambda_s), lambda_max(Lambda_s)),
 * and Lemmas kappaW and Htilde hold for every such tau with the same kappa(W0). */
#define LRSDP_TAU_MIN     0   /* lambda_min(W) (Householder tridiagonalization + bisection)     */
#define LRSDP_TAU_MEAN    1   /* mean of the n-k smallest eigenvalues = (tr W - sum Lambda_l) /   */
                              /* (n - k); the k largest pairs come from subspace iteration with   */
                              /* Rayleigh-Ritz, falling back to the Householder path when W has  */
                              /* no usable spectral gap                                          */

typedef struct lrsdp_info {
  int status;            /* same as the return value                                        */
  int iters;             /* PCG iterations, summed over inner solves                        */
  int outer_iters;       /* refinement steps (0 when dd_mode resolved to OFF)               */
  int dd_used;           /* 1 if the answer is the pair y + y_lo                            */
  double relres;         /* final relative residual: recursive (OFF) or double-double true  */
  double tau;            /* the shift tau of the factor (see LRSDP_TAU_*)                  */
  double setup_ms;       /* time of the factor this solve used (Alg. 1 steps 1-2)           */
  double solve_ms;       /* wall time of this call                                          */
  int eig_sweeps;        /* subspace-iteration sweeps of the factor (0: Householder path)   */
  double phase_ms[4];    /* the factor's setup by phase, device time between events on its  */
                         /* stream: [0] eigen step (step 1a), [1] U, W0 and Z with Z^{-1}    */
                         /* (step 1b), [2] bold S formation and deflation (step 2), [3] the  */
                         /* Cholesky factor of bold S and its inverse (step 2)                */
  int lockstep;          /* lrsdp_solve_batch: 1 when the solve advanced together with the   */
                         /* batch's other solves of its step sequence (one launch per step  */
                         /* for all of them), 0 when it ran alone                             */
} lrsdp_info;

/* Fills *o with the defaults listed above.  o: host. */
LRSDP_API void lrsdp_opts_default(lrsdp_opts* o);

/* Human-readable name of a status code (static storage). */
LRSDP_API const char* lrsdp_status_string(int status);

/* ------------------------------------------------------------------ context */
/* Creates a context on HIP device `device`.  `stream` is a hipStream_t to run on (NULL:
 * the library creates its own default-priority blocking stream, see "Input ordering").  `hbm_budget_bytes` caps the
 * device memory all handles of this context may hold (0: no cap).  out: host. */
LRSDP_API int lrsdp_ctx_create(int device, void* stream, size_t hbm_budget_bytes, lrsdp_ctx** out);
LRSDP_API void lrsdp_ctx_destroy(lrsdp_ctx* ctx);
/* Device bytes currently held by handles of this context.  out: host. */
LRSDP_API int lrsdp_ctx_memory(const lrsdp_ctx* ctx, size_t* in_use, size_t* budget);

/* Kernel timing: with profiling on, selected kernels are bracketed by HIP events on the
 * context's stream and their count, total time and algorithmic bytes / flops accumulate per
 * class.  `enable` is a bit mask of classes (bit LRSDP_K_*; -1 all, 0 off); every call resets
 * the counters.  Used by benchmarks to compute roofline fractions. */
#define LRSDP_K_HV      0   /* fused scatter -> SpMM -> sampled-gather H v kernel (A5/A7)     */
#define LRSDP_K_GEMM    1   /* FP64 MFMA GEMM of the method: bold S formation, the Cholesky's */
                            /* panel solves and trailing updates, deflation (flops counted    */
                            /* on the structurally nonzero operand entries only)              */
#define LRSDP_K_TRI     2   /* Householder tridiagonalization step (A1)                       */
#define LRSDP_K_GEMV    3   /* bold S^{-1} w = L^{-T} (L^{-1} w), two triangular GEMVs (A6)    */
#define LRSDP_K_BZ      4   /* sparse B_JL Z pass of bold S formation (A3)                    */
#define LRSDP_K_RESDD   5   /* double-double residual r - H y (A8)                            */
#define LRSDP_K_LEAF    6   /* 64 x 64 Cholesky and inverse of a diagonal block (A2/A4)       */
#define LRSDP_K_TILE    7   /* 64 x 64 MFMA block steps of the right-looking factorization    */
                            /* (flops: the Cholesky's own, not the L^{-1} products or the     */
                            /* recomputed panel blocks the steps also execute)                */
#define LRSDP_K_GEMMINV 8   /* FP64 MFMA GEMMs that form the explicit inverse factor L^{-1}   */
#define LRSDP_K_COUNT   9
LRSDP_API int lrsdp_ctx_profile(lrsdp_ctx* ctx, int enable);
/* Time only one launch in `every` (>= 1) of each enabled class, so that a timed run is not
 * slowed by the events; counts restart.  Default 1. */
LRSDP_API int lrsdp_ctx_profile_sample(lrsdp_ctx* ctx, int every);
/* Counters of one kernel class; every output is host and may be NULL. */
LRSDP_API int lrsdp_ctx_profile_read(const lrsdp_ctx* ctx, int kernel_class, int64_t* launches,
                                     double* total_ms, double* bytes, double* flops);

/* ------------------------------------------------------------------ A0: data */
/* The constraint matrices as triplets (eqs SDP/SDD; Assumption 2).  Entry t says
 * (A_con[t])_{row[t], col[t]} = (A_con[t])_{col[t], row[t]} = val[t], row[t] <= col[t],
 * 0-based.  Each constraint must own exactly one triplet and the pairs (row, col) must be
 * distinct, so the supports are disjoint and A^T A is diagonal with entries val^2 (row ==
 * col) or 2 val^2.  con, row, col: int32 device arrays of length nnz; val: double device
 * array.  Errors: INVALID_ARG, DUPLICATE_PAIR, UNSUPPORTED (nnz != m or a constraint
 * without / with several triplets), OUT_OF_BUDGET.  Builds the symmetric sparsity pattern of
 * mat(A v) (CSR, sorted columns) used by every product with A and A^T. */
LRSDP_API int lrsdp_problem_create(lrsdp_ctx* ctx, int64_t n, int64_t m, int64_t nnz,
                         const int32_t* con, const int32_t* row, const int32_t* col,
                         const double* val, lrsdp_problem** out);
LRSDP_API void lrsdp_problem_destroy(lrsdp_problem* p);
/* n, m and the number of stored entries of the symmetric pattern.  Outputs: host. */
LRSDP_API int lrsdp_problem_info(const lrsdp_problem* p, int64_t* n, int64_t* m, int64_t* nnz_pattern);

/* ------------------------------------------------------------------ A5: H v */
/* Hv = H v = [A_i . (W mat(A v) W)]_i in FP64 (eq hesseqn2), W an n x n symmetric device
 * array (not retained), v and Hv length-m device arrays.  Parity hook for step A5. */
LRSDP_API int lrsdp_hessian_apply(lrsdp_problem* p, const double* W, const double* v, double* Hv);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lrsdp_hessian_apply without any allocation.
 * Same arguments, layout and result (bitwise) as lrsdp_hessian_apply; the values of mat(A v)
 * go to a fixed scratch array that every GPU the library runs on holds for the life of the
 * process (16 MiB: patterns of up to 2^21 stored entries; problems with n >= 2048, whose
 * H v keeps rows of T in global scratch, are refused too).  Errors: INVALID_ARG, SCRATCH
 * (too large), DEVICE.  The array is shared by every call on a GPU and keeps the last call's
 * contents: two calls that overlap on one GPU (different host threads, or streams of
 * different contexts on one device) race and must be serialized by the caller. */
LRSDP_API int lrsdp_hessian_apply_noalloc(lrsdp_problem* p, const double* W, const double* v,
                                          double* Hv);

/* ------------------------------------------------------------------ A1-A4: setup */
/* Algorithm 1 steps 1-2 for scaling matrix W (n x n symmetric positive definite, device,
 * copied) and rank k (1 <= k <= 16, k < n, n <= 4096 on the Householder path): the k largest
 * eigenpairs of W and tau (opts->tau_rule), U = V_l (Lambda_l - tau)^{1/2}, W0 = W - U U^T, Z = chol(2 W0
 * + U U^T) (eqs Wsplit1, Wsplit2, hessExp2), bold S = tau^2 I + bold U^T (A^T A)^{-1} bold U
 * (eq SMW2), its deflation (opts->deflate) and Cholesky factor L, kept as the explicit
 * inverse bold S^{-1} = L^{-T} L^{-1}.  opts may be NULL (defaults).  Errors: INVALID_ARG,
 * NOT_PD_W, EIG, CHOL_Z, CHOL_S, OUT_OF_BUDGET, DEVICE. */
LRSDP_API int lrsdp_factor_create(lrsdp_problem* p, const double* W, int32_t k, const lrsdp_opts* opts,
                        lrsdp_factor** out);
LRSDP_API void lrsdp_factor_destroy(lrsdp_factor* f);
/* Sizes of a factor: n, the problem's m, and k.  Every output is host and may be NULL. */
LRSDP_API int lrsdp_factor_info(const lrsdp_factor* f, int64_t* n, int64_t* m, int32_t* k);

/* Export of the setup results for parity checks.  Host outputs: tau, shift (the deflation
 * shift, 0 if none), lam[k + 1] = {tau, then the k largest eigenvalues ascending},
 * setup_ms.  Device outputs (each may be NULL): U (n x k), W0 (n x n), Z (n x n, lower, zero
 * above the diagonal; INVALID_ARG for an LRSDP_PRECOND_AUG factor, which has none), Sinv
 * (nk x nk, full symmetric, nk index p + n j: bold S^{-1}, or for LRSDP_PRECOND_AUG the
 * inverse of tau/2 I + B^T (A^T A)^{-1} B). */
LRSDP_API int lrsdp_factor_export(const lrsdp_factor* f, double* tau, double* shift, double* lam,
                        double* setup_ms, double* U, double* W0, double* Z, double* Sinv);

/* Step A7 parity hook: H v in the split form of eq hessExp1 with the W0 part computed in
 * `precision` (LRSDP_PREC_*) and the rank-k part in FP64 with M U in double-double. */
LRSDP_API int lrsdp_hessian_apply_split(lrsdp_factor* f, const double* v, double* Hv, int precision);

/* Step A6 parity hook: z = H~^{-1} v by eq SMW2.  dd = 0: FP64 with the explicit bold S^{-1};
 * dd = 1: w = bold U^T G^{-1} v and t = bold S^{-1} w carried in double-double (t refined
 * against the matrix-free bold S); dd = 2: FP64 with one refinement step of t.  v, z:
 * length-m device arrays.  For an LRSDP_PRECOND_AUG factor: z = H^{-1} v (eq aug_prec) in
 * FP64, dd must be 0. */
LRSDP_API int lrsdp_precond_apply(lrsdp_factor* f, const double* v, double* z, int dd);

/* The true relative residual ||r - H (y + y_lo)|| / ||r|| with every product in
 * double-double (step A8's outer residual).  y_lo may be NULL.  res (device, length m, may be
 * NULL) receives r - H y rounded to FP64; relres: host. */
LRSDP_API int lrsdp_residual_dd(lrsdp_factor* f, const double* r, const double* y, const double* y_lo,
                      double* res, double* relres);

/* ------------------------------------------------------------------ A8: solve */
/* Algorithm 1 step 3: PCG on H y = r (r, y: length-m device arrays) with the factor's
 * preconditioner, to ||H y - r|| <= eps ||r||.  With refinement (dd_mode) the answer is the
 * double-double pair y + y_lo (y_lo: length-m device array; required when dd_mode != OFF,
 * zero-filled when the pair is not needed).  info: host, may be NULL.  Returns OK,
 * NOT_CONVERGED, STAGNATED, INDEFINITE_PRECOND, INVALID_ARG or DEVICE.  With NOT_CONVERGED,
 * STAGNATED and INDEFINITE_PRECOND y (+ y_lo) holds the last iterate before the stop (zero
 * when PCG broke down at its first step), info->relres its relative residual. */
LRSDP_API int lrsdp_solve(lrsdp_factor* f, const double* r, double* y, double* y_lo,
                const lrsdp_opts* opts, lrsdp_info* info);

/* ------------------------------------------------------------------ many instances */
/* One Hessian-equation instance: the constraint triplets (as for lrsdp_problem_create), the
 * scaling matrix W (n x n), k, the right-hand side r (m) and the outputs y, y_lo (m; y_lo may
 * be NULL when the options never ask for the double-double pair).  Every pointer is a device
 * pointer owned by the caller; inputs must be complete before submission and stay unchanged,
 * and outputs untouched, until the instance has finished. */
typedef struct lrsdp_instance {
  int64_t n, m;
  int32_t k;
  const int32_t* con;
  const int32_t* row;
  const int32_t* col;
  const double* val;
  const double* W;
  const double* r;
  double* y;
  double* y_lo;
} lrsdp_instance;

/* Independent instances (a batch of interior-point solves, or one per outer iteration of
 * several SDPs): each is A0 + Algorithm 1 steps 1-3.  `workers` host threads, each with its
 * own stream on ctx's device, set the instances up (A0, steps 1-2); the solves (step 3) of
 * instances that take the same step sequence then advance in lock-step, one launch per step for
 * all of them (info->lockstep = 1), the first half of the batch while the workers set up the
 * second; each of the others is solved alone by the worker that set it up, right after its
 * setup.  Results are bitwise the same as those of
 * lrsdp_problem_create + lrsdp_factor_create + lrsdp_solve on one instance alone.  The worker
 * and solver contexts stay with ctx, their memory pools holding the batch's memory for the next
 * call, until ctx is destroyed; calls on one ctx must not overlap.  status and info (host
 * arrays of length count; info may be NULL) receive each instance's outcome.  Returns OK once
 * every instance has finished (whatever its status), INVALID_ARG or DEVICE. */
LRSDP_API int lrsdp_solve_batch(lrsdp_ctx* ctx, int count, const lrsdp_instance* inst,
                                const lrsdp_opts* opts, int workers, int* status,
                                lrsdp_info* info);

/* Serving: requests are queued and taken by `workers` host threads (own streams) as they
 * arrive, each while the estimated device memory of the instances in flight stays within
 * hbm_budget_bytes (0: no cap; a request larger than the cap runs alone).  submit copies the
 * instance descriptor and options and returns a ticket (host); poll reports LRSDP_PENDING
 * until the request has finished, then OK with its status and info (host, may be NULL).
 * With wait != 0 poll blocks until the request finishes.  A ticket is released by the poll
 * that returns OK.  destroy waits for every submitted request. */
typedef struct lrsdp_server lrsdp_server;
LRSDP_API int lrsdp_server_create(lrsdp_ctx* ctx, int workers, size_t hbm_budget_bytes,
                                  lrsdp_server** out);
LRSDP_API int lrsdp_server_submit(lrsdp_server* srv, const lrsdp_instance* inst,
                                  const lrsdp_opts* opts, uint64_t* ticket);
LRSDP_API int lrsdp_server_poll(lrsdp_server* srv, uint64_t ticket, int wait, int* status,
                                lrsdp_info* info);
/* Sessions: one SDP's data and its current factor resident on the device between requests,
 * as an interior-point method uses them (Section 2: a new scaling matrix W at every step,
 * one or a few right-hand sides per W, eqs hesseqn2 and Newt).  open queues the ingest of the
 * triplets (as lrsdp_problem_create; the arrays must stay valid until that request finishes)
 * and returns the session id and the request's ticket.  A factor request builds the factor of
 * W (n x n, valid until it finishes) with rank k (Algorithm 1 steps 1-2), replacing the
 * previous one; a solve request runs step 3 against the current factor (r, y, y_lo as for
 * lrsdp_solve, valid until it finishes; INVALID_ARG without a factor); close releases the
 * session after its earlier requests.  A session has a device stream of its own; its requests
 * run one at a time in submission order, on whichever worker is free, beside other sessions
 * and instances.
 * Results are bitwise those of lrsdp_problem_create / lrsdp_factor_create / lrsdp_solve alone.
 * Memory: a session holds its problem's bytes from open to close and its largest factor's
 * estimated peak bytes (lrsdp_instance_bytes less the problem's share) from its first factor
 * request to close, against the server's budget.  Every call returns a ticket for
 * lrsdp_server_poll; requests on an unknown or closing session return INVALID_ARG. */
LRSDP_API int lrsdp_server_session_open(lrsdp_server* srv, int64_t n, int64_t m,
                                        const int32_t* con, const int32_t* row,
                                        const int32_t* col, const double* val,
                                        uint64_t* session, uint64_t* ticket);
LRSDP_API int lrsdp_server_submit_factor(lrsdp_server* srv, uint64_t session, const double* W,
                                         int32_t k, const lrsdp_opts* opts, uint64_t* ticket);
LRSDP_API int lrsdp_server_submit_solve(lrsdp_server* srv, uint64_t session, const double* r,
                                        double* y, double* y_lo, const lrsdp_opts* opts,
                                        uint64_t* ticket);
LRSDP_API int lrsdp_server_session_close(lrsdp_server* srv, uint64_t session, uint64_t* ticket);
/* Requests queued, running and finished-but-unpolled, and the estimated bytes in flight;
 * every output is host and may be NULL. */
LRSDP_API int lrsdp_server_stats(lrsdp_server* srv, int* queued, int* running, int* done,
                                 size_t* bytes_in_flight);
LRSDP_API void lrsdp_server_destroy(lrsdp_server* srv);
/* Device bytes one instance is estimated to hold at its peak (setup). */
LRSDP_API size_t lrsdp_instance_bytes(int64_t n, int64_t m, int32_t k);

/* ------------------------------------------------------------------ the outer method */
/* The interior-point method the Hessian equation comes from (Section 2), run on the device:
 * infeasible primal-dual path following on  min C . X  s.t.  A_i . X = b_i, X PSD  (eq SDP)
 * and its dual (eq SDD) with the Nesterov-Todd scaling W (W S W = X, Section 2.2).  Each
 * iteration solves H dy = b - sigma mu A(S^{-1}) + A(W R_d W), R_d = C - S - sum y_i A_i
 * (eqs hesseqn1, hesseqn2), with Algorithm 1 (lrsdp_factor_create with rank k, then
 * lrsdp_solve); then dS = R_d - sum dy_i A_i, dX = sigma mu S^{-1} - X - W dS W, and X and
 * (y, S) each take `frac` of the step to the boundary of the cone (capped at 1).  Start:
 * X = xi I, S = eta I, y = 0 with xi = max(10, sqrt n, n max_i (1 + |b_i|) / (1 + sqrt((A^T A)_ii)))
 * and eta = max(10, sqrt n, 1 + ||C||_F).  Stops when max(pinf, dinf, gap) <= tol with
 * pinf = ||b - A(X)|| / (1 + ||b||), dinf = ||R_d||_F / (1 + ||C||_F) and
 * gap = X . S / (1 + |C . X| + |b^T y|). */
typedef struct lrsdp_ipm_opts {
  double tol;            /* stopping threshold (default 1e-9)                               */
  int max_iter;          /* iterations (default 60)                                          */
  double sigma;          /* centering parameter, or its floor with predictor (default 0.1)  */
  int predictor;         /* 1: per step, the affine direction (sigma = 0) is solved first    */
                         /* and the step uses min(1, max(sigma, (mu_aff / mu)^3)), mu_aff the */
                         /* duality measure that direction reaches with its full steps to the */
                         /* boundary (Mehrotra's rule, no second-order corrector; the two     */
                         /* Hessian solves share one factor); 0: sigma every step (default 1) */
  int warm_start;        /* 1: start from the X, y, S passed in (X and S symmetric positive   */
                         /* definite, else LRSDP_ERR_IPM at the first step); 0: the standard */
                         /* start X = xi I, S = eta I, y = 0 (default 0)                      */
  int stall_iters;       /* > 0: stop when max(pinf, dinf, gap) has not fallen below 0.9 of   */
                         /* its best value for this many steps (the accuracy FP64 allows is  */
                         /* reached); 0: run to max_iter (default 5)                          */
  double frac;           /* fraction of the step to the boundary (default 0.9)             */
  int32_t k;             /* rank of the preconditioner's split of W (default 2); its upper  */
                         /* bound k_max when rank_eta > 0                                   */
  double rank_eta;       /* > 0: estimate the rank per step (Section 5) as the largest       */
                         /* i <= k with lambda_i(W) >= rank_eta lambda_{i+1}(W), at least 1  */
                         /* (default 0: k fixed)                                             */
  double pcg_eps;        /* tolerance of each Hessian solve (default 1e-9)                  */
  double pcg_eps_mu;     /* > 0: tolerance min(1e-3, max(pcg_eps, pcg_eps_mu mu / mu_0)),   */
                         /* mu_0 the starting mu, keeping eps / mu about constant (default 0) */
  int max_ns_iter;       /* Newton-Schulz steps for the scaling's square root (default 100) */
  int householder_eig;   /* 1: the steps to the boundary and the rank estimate from the       */
                         /* Householder eigen step only (default 0: Lanczos, Householder where */
                         /* Lanczos stops short)                                              */
  double ns_tol;         /* ||I - Z Y||_F at which that iteration stops (default 1e-10)     */
  lrsdp_opts solve;      /* options of the factor and the solves (eps is pcg_eps)           */
} lrsdp_ipm_opts;

typedef struct lrsdp_ipm_info {
  int status;            /* same as the return value                                         */
  int iters;             /* Newton steps taken                                              */
  int records;           /* entries written to recs                                         */
  int pcg_iters_total;   /* PCG iterations over all Hessian solves                          */
  double mu, pinf, dinf, gap;      /* at the iterate returned                                */
  double primal_obj, dual_obj;     /* C . X and b^T y at the iterate returned                */
  double ms;             /* wall time of the call                                           */
  int best_iter;         /* the step whose iterate is returned (the best one seen)           */
  int stalled;           /* 1: stopped by stall_iters; 2: stopped by a numerical breakdown of  */
                         /* a step after the first (last_error)                              */
  int last_error;        /* with stalled = 2: the breakdown (IPM, CHOL_Z, CHOL_S, NOT_PD_W,   */
                         /* EIG or INDEFINITE_PRECOND); 0 otherwise                          */
  int fail_stage;        /* with LRSDP_ERR_IPM: 1 the start X or S does not factor, 2 the    */
                         /* scaling's square root did not reach ns_tol in max_ns_iter steps, */
                         /* 3 the new iterate did not factor after 10 shortened steps        */
  double ns_resid;       /* with fail_stage 2: the last ||I - Z Y||_F                        */
} lrsdp_ipm_info;

/* One Newton step: the measures of the iterate it started from, the Hessian solve and the
 * step lengths. */
typedef struct lrsdp_ipm_record {
  double mu, pinf, dinf, gap;
  double alpha_p, alpha_d;         /* step lengths of X and of (y, S)                        */
  int pcg_iters, outer_iters;      /* of the Hessian solve                                    */
  int ns_iters;                    /* Newton-Schulz steps of the scaling                     */
  int k;                           /* rank of the split used                                 */
  int solve_status;                /* the Hessian solve's status (NOT_CONVERGED and          */
                                   /* STAGNATED still give the step their best iterate)      */
  double eps;                      /* the Hessian solve's tolerance                          */
  double relres;                   /* the Hessian solve's final relative residual            */
  double factor_ms, solve_ms, ms;  /* its setup, its solve, the whole step                   */
  double scaling_ms;               /* W and S^{-1} (Newton-Schulz and products)              */
  double rank_ms;                  /* the rank estimate (0 when k is fixed)                  */
  double steps_ms;                 /* the two steps to the boundary and the update (Cholesky */
                                   /* factors of the new X and S)                            */
  double sigma;                    /* the centering parameter the step used                  */
  int pred_pcg_iters;              /* the predictor's Hessian solve (0 without predictor)    */
  double pred_ms;                  /* the predictor: its solve, direction and two steps      */
  int backtracks;                  /* times the step was shortened by 0.8 because the new X  */
                                   /* or S did not factor (FP64 end-game; 0 before it)       */
} lrsdp_ipm_record;

/* Fills *o with the defaults listed above.  o: host. */
LRSDP_API void lrsdp_ipm_opts_default(lrsdp_ipm_opts* o);
/* Runs the method on problem p (its constraints A_i) with right-hand side b (device, m) and
 * cost C (device, n x n symmetric; NULL: the identity).  X, S (device, n x n) and y (device, m)
 * receive the iterate that met tol, or else the best one seen (smallest max(pinf, dinf, gap)).
 * info (host, may be NULL); recs (host, may be NULL) receives up to max_recs per-step records.
 * A Hessian solve that stops short of its tolerance (NOT_CONVERGED, STAGNATED, or a PCG
 * breakdown, INDEFINITE_PRECOND, from rounding once W is ill-conditioned) gives the step its
 * last iterate as an inexact Newton direction.  Returns OK, NOT_CONVERGED (max_iter reached,
 * stalled, or a numerical breakdown after the first step: info->stalled, info->last_error), or
 * the error that ended the call (the start does not factor, INVALID_ARG, DEVICE,
 * OUT_OF_BUDGET): X, y, S then hold the best iterate.  Requires 3 <= n <= 4096 and
 * 1 <= k <= 16, k < n. */
LRSDP_API int lrsdp_ipm_solve(lrsdp_problem* p, const double* b, const double* C,
                              const lrsdp_ipm_opts* opts, double* X, double* y, double* S,
                              lrsdp_ipm_info* info, lrsdp_ipm_record* recs, int max_recs);

/* Section 4.1, eq aug_ex: x = W~^{-1} b for W~ = tau I + U U^T (eq tIUUt) through the symmetric
 * indefinite augmented system [[tau I, sqrt(tau) U], [sqrt(tau) U^T, -tau I]] [x; y] = [b; 0],
 * solved by LU with partial pivoting (backward stable: ||b - W~ x|| stays at the rounding level
 * of ||W~|| ||x|| as tau -> 0, where the Sherman-Morrison-Woodbury route of eq wsmf loses
 * u kappa(W~)).  Ut: U^T, k x n row-major (the factor's U layout); b, x: length-n; all device
 * arrays, b and x may not overlap.  Dense: (n + k)^2 doubles of device memory from ctx's pool
 * and O((n + k)^3) work, for n + k <= 16384.  Synchronous on ctx's stream.  Errors:
 * INVALID_ARG (sizes, tau <= 0 or not finite, or a zero or non-finite pivot: U or b not
 * finite), OUT_OF_BUDGET, DEVICE. */
LRSDP_API int lrsdp_aug_wtilde_solve(lrsdp_ctx* ctx, int32_t n, int32_t k, double tau,
                                     const double* Ut, const double* b, double* x);

#ifdef __cplusplus
}
#endif
#endif /* LRSDP_H */
