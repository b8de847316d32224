// Handles and kernel launchers of the Hessian-equation solver (internal).
#pragma once

#include <unordered_map>
#include <vector>

#include "common.h"

namespace lrsdp {

// Per-context kernel timing (HIP events on the context's stream around selected launches).
struct ProfStat {
  int64_t launches = 0;
  double ms = 0.0, bytes = 0.0, flops = 0.0;
};
struct Profiler {
  bool enabled = false;
  unsigned mask = 0;  // bit i: time kernel class i
  int every = 1;      // time one launch in `every` of each class
  int64_t seen[LRSDP_K_COUNT] = {};
  ProfStat stat[LRSDP_K_COUNT];
  struct Pending {
    int kid;
    hipEvent_t a, b;
    double bytes, flops;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
};

}  // namespace lrsdp

struct lrsdp_ctx {
  lrsdp::Profiler prof;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0;   // 0: unlimited
  size_t in_use = 0;
  std::unordered_map<size_t, std::vector<void*>> pool;  // cached device blocks by size
  size_t pooled = 0;                       // bytes in the cache
  size_t pool_cap = (size_t)16 << 30;      // the cache is trimmed beyond this
  hipStream_t side = nullptr;   // second stream of the factorization (created on first use)
  hipEvent_t side_ev[48] = {};  // its join events, two per recursion depth
  double* h_pinned = nullptr;   // small pinned host staging area (scalars)
  hipEvent_t phase_ev[5] = {};  // boundaries of the setup phases of a factor
  hipEvent_t scal_ev[2] = {};   // PCG: the host copies of two iterations' scalars are done
  int* d_flag = nullptr;        // device error/status words: [0] general and bold S, [1] Z,
                                // [2] scratch for factorizations whose failure is not an error
  int children = 0;             // live problems created under this context
  bool closing = false;         // destroyed while children were alive: released with the last
  std::unordered_map<uint64_t, int> tuned;  // autotuned launch shapes of lock-step batches
  std::vector<lrsdp_ctx*> batch_workers;  // lrsdp_solve_batch's worker contexts, kept with their
                                          // memory pools for the next batch until this one
                                          // is released
};

// From this n on, the H v kernels keep their rows of T in global scratch (L2-resident) and
// only rows of W in LDS, so each workgroup covers more rows of W per pass over the pattern.
constexpr int kTGlobalMinN = 2048;

struct lrsdp_problem {
  lrsdp_ctx* ctx = nullptr;
  int n = 0, m = 0, nnz = 0;        // nnz: entries of the symmetric pattern of mat(A v)
  int32_t* a = nullptr;             // m, row of the entry of A_i (a <= b)
  int32_t* b = nullptr;             // m, column
  double* val = nullptr;            // m, (A_i)_ab
  double* coef = nullptr;           // m, A_i . X = coef_i X_ab for symmetric X
  double* ginv = nullptr;           // m, 1 / (A^T A)_ii
  int32_t* rowptr = nullptr;        // n + 1, CSR of the symmetric pattern, sorted columns
  int32_t* colidx = nullptr;        // nnz
  int32_t* src = nullptr;           // nnz, constraint supplying each pattern entry
  int32_t* own_ptr = nullptr;       // n + 1, constraints grouped by the index that computes them
  int32_t* own_con = nullptr;       // m, constraint id
  int32_t* own_oth = nullptr;       // m, the other index of the pair
  int32_t* pat = nullptr;           // 2 m, pattern entries (a,b) and (b,a) of each constraint
  double* mval = nullptr;           // nnz scratch: values of mat(A v) in pattern order
  double* vec_scratch = nullptr;    // 4 m scratch for parity hooks
  double* tscr = nullptr;           // 2 n^2 (n >= kTGlobalMinN only): rows of T = W mat(A v)
                                    // for the H v kernels once T no longer fits in LDS
  size_t bytes = 0;
  int children = 0;                 // live factors created on this problem
  bool closing = false;             // destroyed while factors were alive: released with the last
};

namespace lrsdp {

// ---------------------------------------------------------------- profiling
// The API entry points bind the context's profiler to the calling thread (ProfScope);
// launch sites bracket the kernels they want timed with prof_begin / prof_end.
extern thread_local Profiler* tls_prof;
struct ProfMark {
  int kid = -1;
  hipEvent_t a = nullptr;
};
ProfMark prof_begin(int kid, hipStream_t s);
void prof_end(const ProfMark& mk, hipStream_t s, double bytes, double flops);
inline bool prof_on() { return tls_prof && tls_prof->enabled; }
void prof_flush(Profiler* p);  // after the stream is synchronized
struct ProfScope {
  Profiler* prev;
  Profiler* mine;
  explicit ProfScope(lrsdp_ctx* c) : prev(tls_prof), mine(&c->prof) { tls_prof = mine; }
  ~ProfScope() {
    prof_flush(mine);
    tls_prof = prev;
  }
};

// ---------------------------------------------------------------- contexts
// blocking: the context's own stream (stream == NULL) is ordered after the legacy default
// stream; the server's worker contexts are created non-blocking.
int ctx_create(int device, void* stream, size_t budget, bool blocking, lrsdp_ctx** out);

// ---------------------------------------------------------------- memory
bool opts_ok(const lrsdp_opts& o);  // the option checks of the entry points
// x = (tau I + U U^T)^{-1} b through the augmented system of eq aug_ex (augsys.hip)
int aug_wtilde_solve(lrsdp_ctx* ctx, int n, int k, double tau, const double* Ut, const double* b,
                     double* x);
int dev_alloc(lrsdp_ctx* ctx, void** p, size_t bytes);
void dev_free(lrsdp_ctx* ctx, void* p, size_t bytes);

template <typename T>
int dev_alloc_n(lrsdp_ctx* ctx, T** p, size_t count) {
  return dev_alloc(ctx, reinterpret_cast<void**>(p), count * sizeof(T));
}

// ---------------------------------------------------------------- A0 ingest (ingest.hip)
int ingest(lrsdp_ctx* ctx, lrsdp_problem* P, const int32_t* con, const int32_t* row,
           const int32_t* col, const double* val, int64_t nnz_triplets);

// ---------------------------------------------------------------- A5 / A7 H v (hv.hip)
// Hv = coef * (W mat(A v) W)_{ab}; W given in FP64, FP32 or BF16 (uint16 bits).
int hv_apply_f64(const lrsdp_problem* P, const double* W, const double* v, double* Hv,
                 hipStream_t s);
int hv_apply_f32(const lrsdp_problem* P, const float* W, const double* v, double* Hv,
                 hipStream_t s);
int hv_apply_bf16(const lrsdp_problem* P, const uint16_t* W, const double* v, double* Hv,
                  hipStream_t s);
// The allocation-free H v: mat(A v) in the library's fixed per-device scratch array, whose
// device address noalloc_scratch_setup looks up once per device (with that device current).
// Problems whose pattern has more entries than the array holds, or that keep rows of T in
// global scratch (n >= kTGlobalMinN), are refused with LRSDP_ERR_SCRATCH.
int noalloc_scratch_setup(int device);
size_t noalloc_scratch_doubles();
int hv_apply_f64_noalloc(const lrsdp_problem* P, const double* W, const double* v, double* Hv,
                         int device, hipStream_t s);
// Double-double H (y + ylo); writes res = r - H y (rounded) and per-block partial sums of
// res^2 and r^2 into part (2 * gridDim doubles); returns nothing on host.
int hv_residual_dd(const lrsdp_problem* P, const double* W, const double* r, const double* y,
                   const double* ylo, double* res, double* res_lo, hipStream_t s);

}  // namespace lrsdp

// ------------------------------------------------------------------ the factor (Alg. 1 1-2)
struct lrsdp_factor {
  lrsdp_problem* P = nullptr;
  int n = 0, k = 0, nk = 0, r = 0;   // r = k(k-1)/2 deflation directions kept
  double tau = 0.0, tau2 = 0.0, shift = 0.0, setup_ms = 0.0;
  double phase_ms[4] = {0.0, 0.0, 0.0, 0.0};  // setup phases (see lrsdp_info)
  int eig_sweeps = 0;                // subspace-iteration sweeps (0: Householder path)
  int precond = LRSDP_PRECOND_SMW;   // LRSDP_PRECOND_*: AUG has no Z (Z, Zt null) and keeps the
                                     // inverse of tau/2 I + B^T G^{-1} B in Sinv
  std::vector<double> lam;           // host copy: tau, then the k largest ascending
  double* lam_dev = nullptr;         // k + 1
  double* W = nullptr;               // n x n, copy of the caller's W
  double* W0 = nullptr;              // n x n, W - U U^T rounded once from double-double
  float* W0f = nullptr;              // n x n, FP32 copy of W0 (lazy)
  uint16_t* W0b = nullptr;           // n x n, BF16 copy of W0 (lazy)
  double* U = nullptr;               // k x n (n x k column-major)
  double* Z = nullptr;               // n x n lower, Z Z^T = 2 W0 + U U^T
  double* Zt = nullptr;              // n x n, Z^T
  double* Sinv = nullptr;            // nk x nk: L^{-1} (lower) and L^{-T} (upper), bold S = L L^T,
                                     // block-explicit above the right-looking size (sinv_split)
  int sinv_split = 0;                // 0: Sinv holds L^{-1}; else N1 of potrf_binv's blocks
  double* QN = nullptr;              // nk x r orthonormal deflation basis
  // per-solve work vectors (allocated with the factor)
  double* work = nullptr;            // see factor.hip for the carve-up
  size_t work_doubles = 0;
  double* sc = nullptr;              // device scalars
  size_t bytes = 0;
};

namespace lrsdp {

int factor_setup(lrsdp_factor* f, const double* W, const lrsdp_opts& o);
void factor_release(lrsdp_factor* f);
int ensure_lowprec(lrsdp_factor* f, int precision, hipStream_t s);
// bold S^{-1} = L^{-T} L^{-1} as a full symmetric nk x nk matrix (parity export)
int export_sinv(const lrsdp_factor* f, double* out, hipStream_t s);

// Work-vector views (each m or nk long) inside f->work.
struct Work {
  // m-vectors
  double *x, *r, *z, *p, *q, *t0, *t1, *t2, *t3, *ylo, *dd0, *dd1;
  // nk-vectors / k x n blocks
  double *w, *wl, *t, *tl, *s, *sl, *y, *yl, *g0, *g1, *h, *h2, *h3;  // h, h2, h3 contiguous
  // small
  double *kk;     // k x k
  double *part;   // reduction partials
};
Work work_view(const lrsdp_factor* f);
size_t work_doubles(int n, int m, int k);

// ---------------------------------------------------------------- apply.hip
// out[j][p] = sum_{q in range(p)} A[p][q] X[j][q], X and out k x n (k <= 16);
// range 0 full, 1 q <= p (lower), 2 q >= p (upper).  One wavefront per row of A.
int rows_k(int n, int k, const double* A, int range, const double* X, double* out,
           hipStream_t s);
int precond_apply_f64(const lrsdp_factor* f, const double* v, double* z, hipStream_t s,
                      int refine);
int precond_apply_dd(const lrsdp_factor* f, const double* v, double* z, hipStream_t s,
                     int nref);
int split_apply(lrsdp_factor* f, const double* v, double* Hv, int precision, hipStream_t s);

// ---------------------------------------------------------------- pcg.hip
// How a factor's solve runs under options o (step A8): double-double refinement (use_dd),
// the inner H v precision, refinement at all, the SMW pieces in double-double, one FP64
// refinement step of bold S^{-1} w (ref64), and the double-double steps of that refinement.
struct SolveMode {
  bool use_dd = false, refine = false, dd_prec = false;
  int prec = LRSDP_PREC_FP64, ref64 = 0, dd_steps = 1;
};
SolveMode solve_mode(const lrsdp_factor* f, const lrsdp_opts& o);
// The inner PCG tolerance of the refinement: inner_eps when given, else 1e-2 with BF16 W0
// products (whose operator is off by ~2^-8, so converging further buys nothing the outer
// double-double step keeps) and 1e-3 otherwise.
inline double inner_tol(const lrsdp_opts& o, const SolveMode& md) {
  if (o.inner_eps > 0.0) return o.inner_eps;
  return md.prec == LRSDP_PREC_BF16 ? 1e-2 : 1e-3;
}
// The step sequence of a factor's solve as one number: solves with equal keys can advance in
// lock-step (solve_lockstep); -1 when the solve takes a step that is not batched (the
// double-double SMW pieces, the augmented preconditioner, the block-explicit inverse, k > 4,
// or the global H v scratch of n >= 2048).
int64_t lockstep_key(const lrsdp_factor* f, const lrsdp_opts& o);
// Solves of factors with one lockstep_key, advancing together on ctx's stream: per instance
// the same steps, shapes and results as lrsdp_solve (r, y, ylo as there; st and info: host,
// count entries).
int solve_lockstep(lrsdp_ctx* ctx, int count, lrsdp_factor* const* F, const double* const* r,
                   double* const* y, double* const* ylo, const lrsdp_opts& o, int* st,
                   lrsdp_info* info);
int solve_run(lrsdp_factor* f, const double* r, double* y, double* ylo, const lrsdp_opts& o,
              lrsdp_info* info);
int residual_dd(lrsdp_factor* f, const double* r, const double* y, const double* ylo,
                double* res, double* res_lo, double* relres);

// ---------------------------------------------------------------- lock-step batches
// Many instances' solves advance together: each launch of a batched kernel covers one step for
// every active instance (grid.y = instance), and each instance runs the grid it would use
// alone (workgroups past it return), so every sum has the order it has alone and the results
// are those of the instance alone, bit for bit.
enum BRole : int {
  kVx, kVr, kVz, kVp, kVq,                // PCG vectors (m)
  kVrhs, kVy, kVyl, kVdd0, kVdd1,         // the solve's right-hand side, answer, residual pair
  kVwy, kVww, kVwt, kVws, kVwh, kVwh2, kVwg0, kVwg1, kVwt0,  // nk / k x n work
  kVRoles
};
struct BInst {
  int n = 0, m = 0, k = 0, nk = 0, nnz = 0, r = 0;
  // problem
  const int32_t *a = nullptr, *b = nullptr, *src = nullptr, *rowptr = nullptr,
                *colidx = nullptr, *own_ptr = nullptr, *own_con = nullptr, *own_oth = nullptr;
  const double *val = nullptr, *coef = nullptr, *ginv = nullptr;
  double *mval = nullptr, *mlo = nullptr;
  // factor
  const double *W = nullptr, *W0 = nullptr, *U = nullptr, *Z = nullptr, *Zt = nullptr,
               *Sinv = nullptr, *QN = nullptr;
  const float* W0f = nullptr;
  const uint16_t* W0b = nullptr;
  double tau2 = 0.0, inv_tau2 = 0.0, shift = 0.0;
  double* kk = nullptr;
  double* v[kVRoles] = {};
  double *sc = nullptr, *part = nullptr;
  int* counter = nullptr;
  // the grids the instance's launches use alone
  int g_vec = 1, g_red = 1, g_m256 = 1, g_nk256 = 1, g_nnz256 = 1, g_rowsU = 1, g_rows = 1,
      g_gemv = 1;
};
// A lock-step launch packs the instances' grids into one: workgroup g of kind K belongs to
// the instance z with off[K][z] <= g < off[K][z + 1] (prefix sums of the instances' own grids),
// so no workgroup is launched for nothing.
// (kKhv1 .. kKhv8: H v with 1, 2, 4, 8 rows of W per workgroup; kKres1 .. kKres4: the
// double-double residual with 1, 2, 4)
enum BKind : int {
  kKvec, kKred, kKm256, kKnk256, kKnnz256, kKrowsU, kKrows, kKgemv, kKhv1, kKhv2, kKhv4, kKhv8,
  kKres1, kKres2, kKres4, kKkk, kKr, kBKinds
};
// the kind of an H v (residual) launch with cb rows of W per workgroup
__host__ __device__ inline int hv_kind(int cb) {
  return cb == 1 ? kKhv1 : cb == 2 ? kKhv2 : cb == 4 ? kKhv4 : kKhv8;
}
__host__ __device__ inline int res_kind(int cb) { return cb == 1 ? kKres1 : cb == 2 ? kKres2 : kKres4; }
struct BL {                 // what the batched kernels take (by value)
  const BInst* I = nullptr;   // count descriptors
  const int* act = nullptr;   // count flags: the instances taking this step
  const int* off = nullptr;   // kBKinds x (count + 1) prefix sums
  int count = 0;
};
// The instance of packed workgroup g of kind K, and (bx) its workgroup within that instance's
// own grid; instances with an empty grid of that kind own no workgroup.
__device__ __forceinline__ int bl_find(const BL& b, int kind, int g, int* bx) {
  const int* o = b.off + (size_t)kind * (b.count + 1);
  int lo = 0, hi = b.count;  // o[lo] <= g < o[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (o[mid] <= g) lo = mid;
    else hi = mid;
  }
  *bx = g - o[lo];
  return lo;
}
struct BLaunch {            // the host side: the packed grid sizes and the batch's largest shapes
  BL b;
  int tot[kBKinds] = {};
  int nmax = 0, kmax = 0, rmax = 0;
};
// apply.hip / hv.hip / dense.hip: the solve's products, as in the single-instance calls
// (cb: the rows of W per H v workgroup, the same for every instance of the batch)
int bl_hv(const BLaunch& L, int precision, int cb, bool whole_w, int vrole, int orole,
          hipStream_t s);
int bl_split_apply(const BLaunch& L, int precision, int cb, int vrole, int orole, hipStream_t s);
int bl_precond_f64(const BLaunch& L, int refine, int vrole, int zrole, hipStream_t s);
int bl_residual_dd(const BLaunch& L, int cb, hipStream_t s);
int bl_gemv_pair(const BLaunch& L, int xrole, int xsub_role, int tmp_role, int yrole,
                 bool accumulate, hipStream_t s);

// ---------------------------------------------------------------- ipm.hip
int ipm_run(lrsdp_problem* P, const double* bvec, const double* C, const lrsdp_ipm_opts& o,
            double* X, double* y, double* S, lrsdp_ipm_info* info, lrsdp_ipm_record* recs,
            int max_recs);

}  // namespace lrsdp
