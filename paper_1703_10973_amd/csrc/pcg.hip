// Step A8: PCG on H y = r (Algorithm 1 step 3) and the outer refinement loop.
//
// PCG follows the preconditioned conjugate gradient of the Barrett et al. templates (the
// text the paper defers to in Section 2.1) from y0 = 0.  Inner products are FP64 with a
// fixed two-level reduction order (per-block partials, then one block), so results do not
// depend on scheduling.  The scalars alpha, beta live on the device; the host reads one
// residual norm per iteration to decide convergence.
//
// Refinement (double-double mode): y <- y + PCG(H_split, r - H y) with y kept as a
// double-double pair and r - H y evaluated in double-double from the plain definition of
// H; the inner H v is the split form with the W0 part in FP64, FP32 or BF16.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "dense.h"

namespace lrsdp {
namespace {

constexpr int kT = 256;
constexpr int kG = 256;  // partial sums per reduction

// scalar slots
enum : int { kRho0 = 0, kRho1 = 1, kPQ = 2, kRR = 3, kRR0 = 4, kMisc = 8, kCounter = 32 };

// True in every thread of the workgroup that finishes last.  Each workgroup's partial is
// written before its arrival is counted (release); the last one then reads all partials
// (acquire) and sums them in index order, so the result does not depend on scheduling.
// (gx: the number of workgroups of the reduction, gridDim.x or an instance's own grid in a
// lock-step batch)
__device__ __forceinline__ bool arrive_last(int* counter, int gx) {
  __shared__ int last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(counter, 1) == gx - 1;
    if (last) __threadfence();
  }
  __syncthreads();
  return last != 0;
}

// *out = sum of part[0..gx) (called by the last workgroup), counter reset for the next use
__device__ __forceinline__ void finish_sum(const double* part, int* counter, double* out,
                                           double* red, int gx) {
  const volatile double* vp = part;
  double s = ((int)threadIdx.x < gx) ? vp[threadIdx.x] : 0.0;
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    *out = s;
    *counter = 0;
  }
}

// *out = a . b in one launch: per-workgroup partials, summed by the last workgroup
__device__ __forceinline__ void dot_body(int bx, int gx, int m, const double* a, const double* b,
                                         double* part, int* counter, double* out) {
  __shared__ double red[kT / kWave];
  double s = 0.0;
  for (int i = bx * kT + threadIdx.x; i < m; i += gx * kT) s = fma(a[i], b[i], s);
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[bx] = s;
  if (arrive_last(counter, gx)) finish_sum(part, counter, out, red, gx);
}
__global__ __launch_bounds__(kT) void k_dot(int m, const double* a, const double* b,
                                            double* part, int* counter, double* out) {
  dot_body(blockIdx.x, gridDim.x, m, a, b, part, counter, out);
}

// alpha = rho / pq;  y += alpha p;  r -= alpha q;  sc[kRR] = r.r.  A breakdown (pq <= 0 or
// rho <= 0, from rounding or an indefinite preconditioner) leaves y and r as they are, so the
// caller, which stops there, keeps the last iterate
__device__ __forceinline__ void update_xr_body(int bx, int gx, int m, double* sc, int rho_slot,
                                               double* x, double* r, const double* p,
                                               const double* q, double* part, int* counter) {
  __shared__ double red[kT / kWave];
  const double rho = sc[rho_slot], pq = sc[kPQ];
  const double alpha = (pq > 0.0 && rho > 0.0) ? rho / pq : 0.0;
  double s = 0.0;
  for (int i = bx * kT + threadIdx.x; i < m; i += gx * kT) {
    x[i] = fma(alpha, p[i], x[i]);
    const double ri = fma(-alpha, q[i], r[i]);
    r[i] = ri;
    s = fma(ri, ri, s);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[bx] = s;
  if (arrive_last(counter, gx)) finish_sum(part, counter, sc + kRR, red, gx);
}
__global__ __launch_bounds__(kT) void k_update_xr(int m, double* sc, int rho_slot, double* x,
                                                  double* r, const double* p, const double* q,
                                                  double* part, int* counter) {
  update_xr_body(blockIdx.x, gridDim.x, m, sc, rho_slot, x, r, p, q, part, counter);
}

// The element-wise steps (grid-stride over the workgroups bx of gx, kT threads each)
// p = z + (rho_new / rho_old) p
__device__ __forceinline__ void update_p_body(int bx, int gx, int m, const double* sc,
                                              int rho_new, int rho_old, const double* z,
                                              double* p) {
  const double beta = sc[rho_new] / sc[rho_old];
  for (int i = bx * kT + threadIdx.x; i < m; i += gx * kT) p[i] = fma(beta, p[i], z[i]);
}
__device__ __forceinline__ void copy_body(int bx, int gx, int m, const double* a, double* b) {
  for (int i = bx * kT + threadIdx.x; i < m; i += gx * kT) b[i] = a[i];
}
__device__ __forceinline__ void zero_body(int bx, int gx, int m, double* a) {
  for (int i = bx * kT + threadIdx.x; i < m; i += gx * kT) a[i] = 0.0;
}
// (yh, yl) += d
__device__ __forceinline__ void dd_add_vec_body(int bx, int gx, int m, double* yh, double* yl,
                                                const double* d) {
  for (int i = bx * kT + threadIdx.x; i < m; i += gx * kT) {
    dd u = dd_add_d({yh[i], yl[i]}, d[i]);
    yh[i] = u.hi;
    yl[i] = u.lo;
  }
}
__device__ __forceinline__ void round_pair_body(int bx, int gx, int m, double* yh,
                                                const double* yl) {
  for (int i = bx * kT + threadIdx.x; i < m; i += gx * kT) yh[i] = yh[i] + yl[i];
}
__global__ __launch_bounds__(kT) void k_update_p(int m, const double* sc, int rho_new,
                                                 int rho_old, const double* z, double* p) {
  update_p_body(blockIdx.x, gridDim.x, m, sc, rho_new, rho_old, z, p);
}
__global__ __launch_bounds__(kT) void k_copy(int m, const double* a, double* b) {
  copy_body(blockIdx.x, gridDim.x, m, a, b);
}
__global__ __launch_bounds__(kT) void k_zero(int m, double* a) {
  zero_body(blockIdx.x, gridDim.x, m, a);
}
__global__ __launch_bounds__(kT) void k_dd_add_vec(int m, double* yh, double* yl,
                                                   const double* d) {
  dd_add_vec_body(blockIdx.x, gridDim.x, m, yh, yl, d);
}
__global__ __launch_bounds__(kT) void k_round_pair(int m, double* yh, const double* yl) {
  round_pair_body(blockIdx.x, gridDim.x, m, yh, yl);
}

// Lock-step batches on a packed grid (bl_find): each instance runs its own grid.
#define LRSDP_B_HEAD(KIND)                         \
  int bx;                                          \
  const int z = bl_find(b, KIND, blockIdx.x, &bx); \
  if (!b.act[z]) return;                           \
  const BInst& d = b.I[z];
__global__ __launch_bounds__(kT) void k_zero_b(const BL b, int role) {
  LRSDP_B_HEAD(kKvec)
  zero_body(bx, d.g_vec, d.m, d.v[role]);
}
__global__ __launch_bounds__(kT) void k_copy_b(const BL b, int from, int to) {
  LRSDP_B_HEAD(kKvec)
  copy_body(bx, d.g_vec, d.m, d.v[from], d.v[to]);
}
__global__ __launch_bounds__(kT) void k_dot_b(const BL b, int ra, int rb, int slot) {
  LRSDP_B_HEAD(kKred)
  dot_body(bx, d.g_red, d.m, d.v[ra], d.v[rb], d.part, d.counter, d.sc + slot);
}
__global__ __launch_bounds__(kT) void k_update_xr_b(const BL b, int rho_slot) {
  LRSDP_B_HEAD(kKred)
  update_xr_body(bx, d.g_red, d.m, d.sc, rho_slot, d.v[kVx], d.v[kVr], d.v[kVp], d.v[kVq],
                 d.part, d.counter);
}
__global__ __launch_bounds__(kT) void k_update_p_b(const BL b, int rho_new, int rho_old) {
  LRSDP_B_HEAD(kKvec)
  update_p_body(bx, d.g_vec, d.m, d.sc, rho_new, rho_old, d.v[kVz], d.v[kVp]);
}
__global__ __launch_bounds__(kT) void k_dd_add_vec_b(const BL b) {
  LRSDP_B_HEAD(kKvec)
  dd_add_vec_body(bx, d.g_vec, d.m, d.v[kVy], d.v[kVyl], d.v[kVx]);
}
__global__ __launch_bounds__(kT) void k_round_pair_b(const BL b) {
  LRSDP_B_HEAD(kKvec)
  round_pair_body(bx, d.g_vec, d.m, d.v[kVy], d.v[kVyl]);
}
#undef LRSDP_B_HEAD
// out[z * ns + j] = I[z].sc[slot0 + j]: the instances' scalars in one array for one copy
__global__ void k_gather_sc_b(const BInst* __restrict__ I, int count, int slot0, int ns,
                              double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count * ns) return;
  const int z = t / ns, j = t - z * ns;
  out[t] = I[z].sc[slot0 + j];
}

// The reduction counter lives in the factor's scalar block (zeroed at setup, reset by every
// reduction's last workgroup).
int* red_counter(const lrsdp_factor* f) { return reinterpret_cast<int*>(f->sc + kCounter); }

// workgroups of a one-launch reduction over m values: one per kT values, at most kG (the
// partials then stay few, and the grid depends only on m, so the sum order does too)
int red_grid(int m) { return std::max(1, std::min(kG, (m + kT - 1) / kT)); }

int dot(const lrsdp_factor* f, int m, const double* a, const double* b, double* part,
        double* out, hipStream_t s) {
  k_dot<<<red_grid(m), kT, 0, s>>>(m, a, b, part, red_counter(f), out);
  return LRSDP_OK;
}

struct PcgOut {
  int iters = 0;
  double relres = 1.0;
  int status = LRSDP_OK;
};

// PCG from 0 on H x = b.  Hmul(v, out), Pinv(v, out).  x, r, z, p, q: Work vectors.
template <typename HM, typename PM>
int pcg(lrsdp_factor* f, const double* b, double eps, int max_iter, HM Hmul, PM Pinv,
        PcgOut* out) {
  lrsdp_ctx* ctx = f->P->ctx;
  hipStream_t s = ctx->stream;
  const Work w = work_view(f);
  const int m = f->P->m;
  double* sc = f->sc;
  const int vg = grid_for(m, kT, 1024);
  k_zero<<<vg, kT, 0, s>>>(m, w.x);
  k_copy<<<vg, kT, 0, s>>>(m, b, w.r);
  LRSDP_TRY(dot(f, m, w.r, w.r, w.part, sc + kRR0, s));
  LRSDP_TRY(Pinv(w.r, w.z));
  LRSDP_TRY(dot(f, m, w.r, w.z, w.part, sc + kRho0, s));
  k_copy<<<vg, kT, 0, s>>>(m, w.z, w.p);
  // The starting scalars (r.r, r.z) are read together with the first iteration's: a zero
  // right-hand side or an indefinite preconditioner is then caught one iteration late, and
  // the first iteration's (meaningless) update of x is undone.
  // Each iteration's scalars go to a host slot of their own behind an event.  While the host
  // waits for them, the iteration's preconditioner step (z, r.z and p, which touch neither
  // x nor r) is already queued when the residual history says that the iteration will not be
  // the last one, so the device does not idle through the host's check.  A wrong guess costs
  // that step's work once; x and r are those of the stopping iteration either way, and every
  // kernel runs on the same data as without the look-ahead.
  double rr0 = 0.0, rel1 = 1.0, rel2 = 1.0;  // relative residuals of iterations it-1, it-2
  out->iters = 0;
  out->relres = 1.0;
  out->status = LRSDP_NOT_CONVERGED;
  int cur = kRho0, nxt = kRho1;
  auto precond_step = [&]() -> int {
    LRSDP_TRY(Pinv(w.r, w.z));
    LRSDP_TRY(dot(f, m, w.r, w.z, w.part, sc + nxt, s));
    k_update_p<<<vg, kT, 0, s>>>(m, sc, nxt, cur, w.z, w.p);
    return LRSDP_OK;
  };
  for (int it = 1; it <= max_iter; ++it) {
    LRSDP_TRY(Hmul(w.p, w.q));
    LRSDP_TRY(dot(f, m, w.p, w.q, w.part, sc + kPQ, s));
    k_update_xr<<<red_grid(m), kT, 0, s>>>(m, sc, cur, w.x, w.r, w.p, w.q, w.part,
                                          red_counter(f));
    double* slot = ctx->h_pinned + 16 + 8 * (it & 1);
    hipEvent_t ev = ctx->scal_ev[it & 1];
    LRSDP_HIP(hipMemcpyAsync(slot, sc, 8 * sizeof(double), hipMemcpyDeviceToHost, s));
    LRSDP_HIP(hipEventRecord(ev, s));
    // guess: the residual keeps shrinking at the last rate, squared (CG tends to speed up)
    const double q = it >= 2 ? rel1 / rel2 : 1.0;
    const bool ahead = it < max_iter && rel1 * q * q > eps;
    if (ahead) LRSDP_TRY(precond_step());
    LRSDP_HIP(hipEventSynchronize(ev));
    double h[8];
    for (int i = 0; i < 8; ++i) h[i] = slot[i];
    if (it == 1) {
      rr0 = h[kRR0];
      if (rr0 == 0.0 || !(h[kRho0] > 0.0)) {
        k_zero<<<vg, kT, 0, s>>>(m, w.x);
        out->relres = rr0 == 0.0 ? 0.0 : 1.0;
        out->status = rr0 == 0.0 ? LRSDP_OK : LRSDP_ERR_INDEFINITE_PRECOND;
        return LRSDP_OK;
      }
    }
    out->iters = it;
    const double rel = std::sqrt(std::fmax(h[kRR], 0.0) / rr0);
    out->relres = rel;
    if (!std::isfinite(rel) || !(h[kPQ] > 0.0)) {
      out->status = std::isfinite(rel) ? LRSDP_ERR_INDEFINITE_PRECOND : LRSDP_ERR_DEVICE;
      return LRSDP_OK;
    }
    if (rel <= eps) {
      out->status = LRSDP_OK;
      return LRSDP_OK;
    }
    if (!ahead) LRSDP_TRY(precond_step());
    rel2 = rel1;
    rel1 = rel;
    std::swap(cur, nxt);
  }
  return LRSDP_OK;
}

}  // namespace

int residual_dd(lrsdp_factor* f, const double* r, const double* y, const double* ylo,
                double* res, double* res_lo, double* relres) {
  lrsdp_ctx* ctx = f->P->ctx;
  hipStream_t s = ctx->stream;
  const Work w = work_view(f);
  const int m = f->P->m;
  LRSDP_TRY(hv_residual_dd(f->P, f->W, r, y, ylo, res, res_lo, s));
  LRSDP_TRY(dot(f, m, res, res, w.part, f->sc + kMisc, s));
  LRSDP_TRY(dot(f, m, r, r, w.part, f->sc + kMisc + 1, s));
  double h[2];
  LRSDP_HIP(hipMemcpyAsync(ctx->h_pinned, f->sc + kMisc, 2 * sizeof(double),
                           hipMemcpyDeviceToHost, s));
  LRSDP_HIP(hipStreamSynchronize(s));
  h[0] = ctx->h_pinned[0];
  h[1] = ctx->h_pinned[1];
  *relres = (h[1] > 0.0) ? std::sqrt(h[0] / h[1]) : 0.0;
  return LRSDP_OK;
}

SolveMode solve_mode(const lrsdp_factor* f, const lrsdp_opts& o) {
  SolveMode md;
  if (o.dd_mode == LRSDP_DD_ON) md.use_dd = true;
  else if (o.dd_mode == LRSDP_DD_OFF) md.use_dd = false;
  else md.use_dd = f->tau < o.dd_auto_ratio * f->lam[1];
  // AUTO: the low-precision W0 product pays only inside refinement, which the solve needs
  // anyway once the answer is a double-double pair; otherwise plain FP64 PCG is cheaper
  md.prec = o.precision == LRSDP_PREC_AUTO ? (md.use_dd ? LRSDP_PREC_FP32 : LRSDP_PREC_FP64)
                                           : o.precision;
  md.refine = md.use_dd || md.prec != LRSDP_PREC_FP64;
  // SMW pieces: double-double when tau^2 is within a few units of u ||bold S|| (dd_precond on
  // or auto with tau < 1e-7 lambda_max), else FP64 with one refinement step of bold S^{-1} w
  // once tau / lambda_max < 1e-3 (where the explicit inverse alone loses definiteness).
  const double ratio = f->tau / f->lam[f->k];
  if (o.dd_precond == 1) md.dd_prec = true;
  else if (o.dd_precond == 0) md.dd_prec = false;
  else md.dd_prec = ratio < 1e-7;
  md.ref64 = ratio < 1e-3 ? 1 : 0;
  // Double-double refinement steps of bold S t = w inside the preconditioner.  kappa(bold S)
  // grows like 1 / ratio, so the FP64 inverse leaves a relative error of about u / ratio in t
  // and one step squares it; the SMW subtraction then magnifies what is left by about
  // 1 / ratio.  One step keeps the preconditioner within 1e-5 of exact down to
  // ratio = 1e-9, far inside the inner tolerance; below that a second step is taken.
  md.dd_steps = ratio >= 1e-9 ? 1 : 2;
  if (f->precond == LRSDP_PRECOND_AUG) {  // FP64 only (eq aug_prec is Theta(1/sqrt(mu)))
    md.dd_prec = false;
    md.ref64 = 0;
  }
  return md;
}

int solve_run(lrsdp_factor* f, const double* r, double* y, double* ylo, const lrsdp_opts& o,
              lrsdp_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  lrsdp_ctx* ctx = f->P->ctx;
  hipStream_t s = ctx->stream;
  const Work w = work_view(f);
  const int m = f->P->m;
  const int vg = grid_for(m, kT, 1024);
  lrsdp_info inf{};
  inf.tau = f->tau;
  inf.setup_ms = f->setup_ms;
  inf.eig_sweeps = f->eig_sweeps;
  for (int i = 0; i < 4; ++i) inf.phase_ms[i] = f->phase_ms[i];

  const SolveMode md = solve_mode(f, o);
  const bool use_dd = md.use_dd, refine = md.refine, dd_prec = md.dd_prec;
  const int prec = md.prec, ref64 = md.ref64, dd_steps = md.dd_steps;

  auto Pinv = [&](const double* v, double* z) -> int {
    return dd_prec ? precond_apply_dd(f, v, z, s, dd_steps)
                   : precond_apply_f64(f, v, z, s, ref64);
  };
  int status = LRSDP_OK;
  if (!refine) {
    auto Hm = [&](const double* v, double* out) -> int { return hv_apply_f64(f->P, f->W, v, out, s); };
    PcgOut po;
    LRSDP_TRY(pcg(f, r, o.eps, o.max_iter, Hm, Pinv, &po));
    k_copy<<<vg, kT, 0, s>>>(m, w.x, y);
    if (ylo) k_zero<<<vg, kT, 0, s>>>(m, ylo);
    inf.iters = po.iters;
    inf.relres = po.relres;
    status = po.status;
  } else {
    // y as a double-double pair; the low part lives in the caller's buffer or in w.ylo
    double* yl = ylo ? ylo : w.ylo;
    k_zero<<<vg, kT, 0, s>>>(m, y);
    k_zero<<<vg, kT, 0, s>>>(m, yl);
    auto Hm = [&](const double* v, double* out) -> int {
      return split_apply(f, v, out, prec, s);
    };
    double best = 1e300;
    int stall = 0;
    status = LRSDP_NOT_CONVERGED;
    for (int outer = 0; outer <= o.max_outer; ++outer) {
      double rel = 1.0;
      if (outer == 0) {  // y = 0: the residual is r itself (relative size 1; r = 0 is caught
                         // by the inner solve, whose answer then leaves y = 0)
        k_copy<<<vg, kT, 0, s>>>(m, r, w.dd0);
      } else {
        LRSDP_TRY(residual_dd(f, r, y, yl, w.dd0, w.dd1, &rel));
      }
      inf.relres = rel;
      if (!std::isfinite(rel)) {
        status = LRSDP_ERR_DEVICE;
        break;
      }
      if (rel <= o.eps) {
        status = LRSDP_OK;
        break;
      }
      if (outer == o.max_outer) break;
      if (rel < 0.5 * best) {
        best = rel;
        stall = 0;
      } else if (++stall >= 2) {
        status = LRSDP_ERR_STAGNATED;
        break;
      }
      PcgOut po;
      LRSDP_TRY(pcg(f, w.dd0, inner_tol(o, md), o.max_iter, Hm, Pinv, &po));
      inf.iters += po.iters;
      inf.outer_iters = outer + 1;
      if (po.status < 0) {
        status = po.status;
        break;
      }
      k_dd_add_vec<<<vg, kT, 0, s>>>(m, y, yl, w.x);
    }
    if (!ylo) k_round_pair<<<vg, kT, 0, s>>>(m, y, yl);
    inf.dd_used = ylo ? 1 : 0;
  }
  LRSDP_HIP(hipStreamSynchronize(s));
  auto t1 = std::chrono::steady_clock::now();
  inf.solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  inf.status = status;
  if (info) *info = inf;
  return status;
}

// ---------------------------------------------------------------- lock-step batches
namespace {

// Bytes of one value of the W operand in the solve's H v (plain FP64 PCG multiplies by W)
int hv_bytes_of(const SolveMode& md) {
  return (md.refine && md.prec != LRSDP_PREC_FP64) ? 4 : 8;
}
// Rows of W per H v (or double-double residual) workgroup in a lock-step batch.  A product's
// arithmetic does not depend on them (fixed lane-to-entry maps and reduction trees), so every
// choice gives the instance's results alone; which is fastest depends on the batch (few rows:
// more workgroups, each streaming the whole pattern; many rows: fewer passes, fewer
// workgroups).  The largest that the LDS holds for two workgroups per CU (80 KB) bounds them.
int batch_rows_max(int nmax, size_t bytes_per_row, int cap) {
  int cb = cap;
  while (cb > 1 && (size_t)cb * bytes_per_row * nmax > 80 * 1024) cb >>= 1;
  return cb;
}
// The autotuner: the first lock-step batch of a shape class on a context times each choice
// of rows per workgroup on its own data (results identical, so nothing else changes) and
// keeps the fastest for the class: kind (1 H v, 2 residual), value bytes, the batch's
// largest n and its size, each rounded up to a power of two.
uint64_t tune_key(int kind, int bytes, int whole, int nmax, int count) {
  auto p2 = [](int v) { int q = 1; while (q < v) q <<= 1; return q; };
  return ((uint64_t)kind << 56) | ((uint64_t)bytes << 48) | ((uint64_t)whole << 44) |
         ((uint64_t)p2(nmax) << 20) | (uint64_t)p2(count);
}

}  // namespace

int64_t lockstep_key(const lrsdp_factor* f, const lrsdp_opts& o) {
  if (f->precond != LRSDP_PRECOND_SMW || f->sinv_split != 0 || f->k < 1 || f->k > 4 ||
      f->P->tscr != nullptr)
    return -1;
  const SolveMode md = solve_mode(f, o);
  if (md.dd_prec) return -1;
  // one row of W and of T (and of the residual's pair) in LDS at the least
  if ((size_t)2 * hv_bytes_of(md) * f->n > 80 * 1024 || (size_t)3 * 8 * f->n > 80 * 1024)
    return -1;
  int64_t key = md.refine ? 1 : 0;
  key |= (int64_t)md.prec << 1;
  key |= (int64_t)md.ref64 << 3;
  key |= (int64_t)(f->k <= 2 ? 0 : 1) << 4;
  return key;
}

int solve_lockstep(lrsdp_ctx* ctx, int count, lrsdp_factor* const* F, const double* const* r,
                   double* const* y, double* const* ylo, const lrsdp_opts& o, int* st,
                   lrsdp_info* info) {
  if (count <= 0) return LRSDP_OK;
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = ctx->stream;
  const SolveMode md = solve_mode(F[0], o);
  int nmax = 0;
  for (int z = 0; z < count; ++z) nmax = std::max(nmax, F[z]->n);
  const int hv_cap = batch_rows_max(nmax, 2 * (size_t)hv_bytes_of(md), 8);
  const int res_cap = batch_rows_max(nmax, 3 * sizeof(double), 4);
  int hv_cb = hv_cap, res_cb = res_cap;  // until tuned
  // descriptors, and the packed grids (prefix sums of the instances' own grids per kind)
  std::vector<BInst> h(count);
  BLaunch L;
  std::vector<int> off((size_t)kBKinds * (count + 1), 0);
  for (int z = 0; z < count; ++z) {
    const lrsdp_factor* f = F[z];
    const lrsdp_problem* P = f->P;
    const Work w = work_view(f);
    BInst& d = h[z];
    d.n = P->n; d.m = P->m; d.k = f->k; d.nk = f->nk; d.nnz = P->nnz; d.r = f->r;
    d.a = P->a; d.b = P->b; d.src = P->src; d.rowptr = P->rowptr; d.colidx = P->colidx;
    d.own_ptr = P->own_ptr; d.own_con = P->own_con; d.own_oth = P->own_oth;
    d.val = P->val; d.coef = P->coef; d.ginv = P->ginv;
    d.mval = P->mval; d.mlo = P->vec_scratch;
    d.W = f->W; d.W0 = f->W0; d.U = f->U; d.Z = f->Z; d.Zt = f->Zt; d.Sinv = f->Sinv;
    d.QN = f->QN; d.W0f = f->W0f; d.W0b = f->W0b;
    d.tau2 = f->tau2; d.inv_tau2 = 1.0 / f->tau2; d.shift = f->shift;
    d.kk = w.kk;
    d.v[kVx] = w.x; d.v[kVr] = w.r; d.v[kVz] = w.z; d.v[kVp] = w.p; d.v[kVq] = w.q;
    d.v[kVrhs] = const_cast<double*>(r[z]); d.v[kVy] = y[z];
    d.v[kVyl] = ylo[z] ? ylo[z] : w.ylo;
    d.v[kVdd0] = w.dd0; d.v[kVdd1] = w.dd1;
    d.v[kVwy] = w.y; d.v[kVww] = w.w; d.v[kVwt] = w.t; d.v[kVws] = w.s; d.v[kVwh] = w.h;
    d.v[kVwh2] = w.h2;
    d.v[kVwg0] = w.g0; d.v[kVwg1] = w.g1; d.v[kVwt0] = w.t0;
    d.sc = f->sc; d.part = w.part; d.counter = red_counter(f);
    d.g_vec = grid_for(d.m, kT, 1024);
    d.g_red = red_grid(d.m);
    d.g_m256 = grid_for(d.m, 256);
    d.g_nk256 = grid_for(d.nk, 256);
    d.g_nnz256 = grid_for(d.nnz, 256);
    d.g_rowsU = (d.n + 15) / 16;
    d.g_rows = (d.n + 3) / 4;
    d.g_gemv = (d.nk + 3) / 4;
    const int g[kBKinds] = {d.g_vec, d.g_red, d.g_m256, d.g_nk256, d.g_nnz256, d.g_rowsU,
                            d.g_rows, d.g_gemv, d.n, (d.n + 1) / 2, (d.n + 3) / 4,
                            (d.n + 7) / 8, d.n, (d.n + 1) / 2, (d.n + 3) / 4, d.k * d.k, d.r};
    for (int kd = 0; kd < kBKinds; ++kd)
      off[(size_t)kd * (count + 1) + z + 1] = off[(size_t)kd * (count + 1) + z] + g[kd];
    L.nmax = std::max(L.nmax, d.n);
    L.kmax = std::max(L.kmax, d.k);
    L.rmax = std::max(L.rmax, d.r);
    lrsdp_info& inf = info[z];
    inf = lrsdp_info{};
    inf.tau = f->tau;
    inf.setup_ms = f->setup_ms;
    inf.eig_sweeps = f->eig_sweeps;
    for (int i = 0; i < 4; ++i) inf.phase_ms[i] = f->phase_ms[i];
    st[z] = LRSDP_NOT_CONVERGED;
  }
  for (int kd = 0; kd < kBKinds; ++kd) L.tot[kd] = off[(size_t)kd * (count + 1) + count];
  // device copies; pinned host staging for the activity flags and the scalars
  constexpr int kNs = 5;  // scalar slots read per PCG iteration: kRho0 .. kRR0
  BInst* dI = nullptr;
  int* dact = nullptr;
  int* doff = nullptr;
  double* dsc = nullptr;
  void* hpin = nullptr;
  const size_t ib = (size_t)count * sizeof(BInst), ab = (size_t)count * sizeof(int),
               ob = off.size() * sizeof(int), sb = (size_t)count * kNs * sizeof(double);
  int rc = dev_alloc(ctx, reinterpret_cast<void**>(&dI), ib);
  if (rc == LRSDP_OK) rc = dev_alloc(ctx, reinterpret_cast<void**>(&dact), ab);
  if (rc == LRSDP_OK) rc = dev_alloc(ctx, reinterpret_cast<void**>(&doff), ob);
  if (rc == LRSDP_OK) rc = dev_alloc(ctx, reinterpret_cast<void**>(&dsc), sb);
  if (rc == LRSDP_OK &&
      hipHostMalloc(&hpin, ib + ob + ab + sb, hipHostMallocDefault) != hipSuccess) {
    hpin = nullptr;
    rc = LRSDP_ERR_DEVICE;
  }
  L.b.I = dI;
  L.b.act = dact;
  L.b.off = doff;
  L.b.count = count;
  auto body = [&]() -> int {
    LRSDP_TRY(rc);
    BInst* hI = static_cast<BInst*>(hpin);
    int* hoff = reinterpret_cast<int*>(static_cast<char*>(hpin) + ib);
    int* hact = reinterpret_cast<int*>(static_cast<char*>(hpin) + ib + ob);
    double* hsc = reinterpret_cast<double*>(static_cast<char*>(hpin) + ib + ob + ab);
    std::copy(h.begin(), h.end(), hI);
    std::copy(off.begin(), off.end(), hoff);
    LRSDP_HIP(hipMemcpyAsync(dI, hI, ib, hipMemcpyHostToDevice, s));
    LRSDP_HIP(hipMemcpyAsync(doff, hoff, ob, hipMemcpyHostToDevice, s));
    std::vector<char> on(count, 1);
    auto upload = [&](const std::vector<char>& flags) -> int {
      // the previous upload must have been read before hact is rewritten: every caller
      // synchronizes the stream between uploads (the scalar reads), except the first
      LRSDP_HIP(hipStreamSynchronize(s));
      for (int z = 0; z < count; ++z) hact[z] = flags[z] ? 1 : 0;
      LRSDP_HIP(hipMemcpyAsync(dact, hact, ab, hipMemcpyHostToDevice, s));
      return LRSDP_OK;
    };
    auto read_sc = [&](int slot0, int ns) -> int {
      k_gather_sc_b<<<grid_for((int64_t)count * ns, 256), 256, 0, s>>>(dI, count, slot0, ns, dsc);
      LRSDP_HIP(hipMemcpyAsync(hsc, dsc, (size_t)count * ns * sizeof(double),
                               hipMemcpyDeviceToHost, s));
      LRSDP_HIP(hipStreamSynchronize(s));
      return LRSDP_OK;
    };
    const int gv = L.tot[kKvec], gr = L.tot[kKred];
    // autotune the rows per workgroup of H v and of the residual (first batch of a class)
    auto tune = [&](int kind, int cap, int* best) -> int {
      const int whole = md.refine ? 0 : 1;
      const int bytes = kind == 1 ? hv_bytes_of(md) : 8;
      const uint64_t key = tune_key(kind, bytes + (md.prec == LRSDP_PREC_BF16 ? 1 : 0), whole,
                                    L.nmax, count);
      auto it = ctx->tuned.find(key);
      if (it != ctx->tuned.end() && it->second <= cap) {
        *best = it->second;
        return LRSDP_OK;
      }
      hipEvent_t e0 = nullptr, e1 = nullptr;
      LRSDP_HIP(hipEventCreate(&e0));
      LRSDP_HIP(hipEventCreate(&e1));
      std::vector<char> all(count, 1);
      int rc2 = upload(all);
      float best_ms = 1e30f;
      for (int cb = 1; cb <= cap && rc2 == LRSDP_OK; cb <<= 1) {
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && rc2 == LRSDP_OK; ++rep) {  // the second run is timed
          if (hipEventRecord(e0, s) != hipSuccess) rc2 = LRSDP_ERR_DEVICE;
          if (rc2 == LRSDP_OK)
            rc2 = kind == 1 ? bl_hv(L, md.refine ? md.prec : LRSDP_PREC_FP64, cb, whole != 0,
                                    kVrhs, kVq, s)
                            : bl_residual_dd(L, cb, s);
          if (rc2 == LRSDP_OK && hipEventRecord(e1, s) != hipSuccess) rc2 = LRSDP_ERR_DEVICE;
          if (rc2 == LRSDP_OK && hipEventSynchronize(e1) != hipSuccess) rc2 = LRSDP_ERR_DEVICE;
          if (rc2 == LRSDP_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            rc2 = LRSDP_ERR_DEVICE;
        }
        if (rc2 == LRSDP_OK && ms < best_ms) {
          best_ms = ms;
          *best = cb;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (rc2 == LRSDP_OK) ctx->tuned[key] = *best;
      return rc2;
    };
    LRSDP_TRY(tune(1, hv_cap, &hv_cb));
    auto Pinv = [&](int vrole, int zrole) {
      return bl_precond_f64(L, md.ref64, vrole, zrole, s);
    };
    auto Hmul = [&](int vrole, int orole) {
      return md.refine ? bl_split_apply(L, md.prec, hv_cb, vrole, orole, s)
                       : bl_hv(L, LRSDP_PREC_FP64, hv_cb, true, vrole, orole, s);
    };
    // PCG from 0 on H x = b (b = v[brole]) for the instances in sel, as pcg() takes it
    std::vector<PcgOut> po(count);
    // One PCG iteration of the class is a fixed launch sequence, captured as two graphs per
    // parity of the scalar slots (rho of the iteration in cur, the next in nxt): part A is
    // q = H p, p.q, the x and r updates and the copy of the scalars to the host; part B, after
    // the host's checks, is z = M^{-1} r, r.z and p.  They are instantiated once per call and
    // replayed every iteration of every refinement step; the activity flags they read are
    // rewritten between replays.
    hipGraphExec_t gA[2] = {nullptr, nullptr}, gB[2] = {nullptr, nullptr};
    std::vector<hipGraph_t> graphs;
    struct GraphsGuard {  // released on every way out of the body (after the stream is idle)
      hipStream_t s;
      hipGraphExec_t* ex[4];
      std::vector<hipGraph_t>* g;
      ~GraphsGuard() {
        (void)hipStreamSynchronize(s);
        for (hipGraphExec_t* e : ex)
          if (*e) (void)hipGraphExecDestroy(*e);
        for (hipGraph_t x : *g) (void)hipGraphDestroy(x);
      }
    } graphs_guard{s, {&gA[0], &gA[1], &gB[0], &gB[1]}, &graphs};
    auto capture = [&](auto&& fn, hipGraphExec_t* ex) -> int {
      LRSDP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
      const int frc = fn();
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(s, &g);
      if (g) graphs.push_back(g);
      if (frc != LRSDP_OK) return frc;
      if (e != hipSuccess || !g) return LRSDP_ERR_DEVICE;
      LRSDP_HIP(hipGraphInstantiate(ex, g, nullptr, nullptr, 0));
      return LRSDP_OK;
    };
    auto part_a = [&](int cur) -> int {
      LRSDP_TRY(Hmul(kVp, kVq));
      k_dot_b<<<gr, kT, 0, s>>>(L.b, kVp, kVq, kPQ);
      k_update_xr_b<<<gr, kT, 0, s>>>(L.b, cur);
      k_gather_sc_b<<<grid_for((int64_t)count * kNs, 256), 256, 0, s>>>(dI, count, 0, kNs, dsc);
      LRSDP_HIP(hipMemcpyAsync(hsc, dsc, (size_t)count * kNs * sizeof(double),
                               hipMemcpyDeviceToHost, s));
      return LRSDP_OK;
    };
    auto part_b = [&](int cur, int nxt) -> int {
      LRSDP_TRY(Pinv(kVr, kVz));
      k_dot_b<<<gr, kT, 0, s>>>(L.b, kVr, kVz, nxt);
      k_update_p_b<<<gv, kT, 0, s>>>(L.b, nxt, cur);
      LRSDP_HIP(hipGetLastError());
      return LRSDP_OK;
    };
    auto pcg_ls = [&](const std::vector<char>& sel, int brole, double eps, int max_iter) -> int {
      std::vector<char> a = sel;
      std::vector<double> rr0(count, 0.0);
      for (int z = 0; z < count; ++z) po[z] = PcgOut{0, 1.0, LRSDP_NOT_CONVERGED};
      LRSDP_TRY(upload(a));
      k_zero_b<<<gv, kT, 0, s>>>(L.b, kVx);
      k_copy_b<<<gv, kT, 0, s>>>(L.b, brole, kVr);
      k_dot_b<<<gr, kT, 0, s>>>(L.b, kVr, kVr, kRR0);
      LRSDP_TRY(Pinv(kVr, kVz));
      k_dot_b<<<gr, kT, 0, s>>>(L.b, kVr, kVz, kRho0);
      k_copy_b<<<gv, kT, 0, s>>>(L.b, kVz, kVp);
      LRSDP_HIP(hipGetLastError());
      int cur = kRho0, nxt = kRho1;
      for (int it = 1; it <= max_iter; ++it) {
        const int par = cur == kRho0 ? 0 : 1;
        if (!gA[par]) LRSDP_TRY(capture([&] { return part_a(cur); }, &gA[par]));
        LRSDP_HIP(hipGraphLaunch(gA[par], s));
        LRSDP_HIP(hipStreamSynchronize(s));
        bool changed = false, any = false;
        for (int z = 0; z < count; ++z) {
          if (!a[z]) continue;
          const double* hz = hsc + (size_t)z * kNs;
          PcgOut& out = po[z];
          if (it == 1) {
            rr0[z] = hz[kRR0];
            if (rr0[z] == 0.0 || !(hz[kRho0] > 0.0)) {
              const int vg = grid_for(h[z].m, kT, 1024);
              k_zero<<<vg, kT, 0, s>>>(h[z].m, h[z].v[kVx]);
              out.relres = rr0[z] == 0.0 ? 0.0 : 1.0;
              out.status = rr0[z] == 0.0 ? LRSDP_OK : LRSDP_ERR_INDEFINITE_PRECOND;
              a[z] = 0;
              changed = true;
              continue;
            }
          }
          out.iters = it;
          const double rel = std::sqrt(std::fmax(hz[kRR], 0.0) / rr0[z]);
          out.relres = rel;
          if (!std::isfinite(rel) || !(hz[kPQ] > 0.0)) {
            out.status = std::isfinite(rel) ? LRSDP_ERR_INDEFINITE_PRECOND : LRSDP_ERR_DEVICE;
            a[z] = 0;
            changed = true;
            continue;
          }
          if (rel <= eps) {
            out.status = LRSDP_OK;
            a[z] = 0;
            changed = true;
            continue;
          }
          any = true;
        }
        if (!any) break;
        if (changed) LRSDP_TRY(upload(a));
        if (!gB[par]) LRSDP_TRY(capture([&] { return part_b(cur, nxt); }, &gB[par]));
        LRSDP_HIP(hipGraphLaunch(gB[par], s));
        std::swap(cur, nxt);
      }
      return LRSDP_OK;
    };
    if (!md.refine) {
      LRSDP_TRY(pcg_ls(on, kVrhs, o.eps, o.max_iter));
      LRSDP_TRY(upload(on));
      k_copy_b<<<gv, kT, 0, s>>>(L.b, kVx, kVy);
      std::vector<char> with_lo(count);
      for (int z = 0; z < count; ++z) with_lo[z] = ylo[z] != nullptr;
      LRSDP_TRY(upload(with_lo));
      k_zero_b<<<gv, kT, 0, s>>>(L.b, kVyl);
      LRSDP_HIP(hipGetLastError());
      for (int z = 0; z < count; ++z) {
        info[z].iters = po[z].iters;
        info[z].relres = po[z].relres;
        st[z] = po[z].status;
      }
    } else {
      // y as a double-double pair, refined against the double-double residual (solve_run)
      LRSDP_TRY(upload(on));
      k_zero_b<<<gv, kT, 0, s>>>(L.b, kVy);
      k_zero_b<<<gv, kT, 0, s>>>(L.b, kVyl);
      LRSDP_HIP(hipGetLastError());
      LRSDP_TRY(tune(2, res_cap, &res_cb));  // (on y = 0: writes only dd0 and dd1)
      std::vector<double> best(count, 1e300);
      std::vector<int> stall(count, 0);
      std::vector<char> live = on;
      for (int outer = 0; outer <= o.max_outer; ++outer) {
        LRSDP_TRY(upload(live));
        if (outer == 0) {
          k_copy_b<<<gv, kT, 0, s>>>(L.b, kVrhs, kVdd0);
          LRSDP_HIP(hipGetLastError());
        } else {
          LRSDP_TRY(bl_residual_dd(L, res_cb, s));
          k_dot_b<<<gr, kT, 0, s>>>(L.b, kVdd0, kVdd0, kMisc);
          k_dot_b<<<gr, kT, 0, s>>>(L.b, kVrhs, kVrhs, kMisc + 1);
          LRSDP_HIP(hipGetLastError());
          LRSDP_TRY(read_sc(kMisc, 2));
        }
        bool any = false;
        for (int z = 0; z < count; ++z) {
          if (!live[z]) continue;
          double rel = 1.0;
          if (outer > 0) {
            const double h0 = hsc[2 * z], h1 = hsc[2 * z + 1];
            rel = (h1 > 0.0) ? std::sqrt(h0 / h1) : 0.0;
          }
          info[z].relres = rel;
          if (!std::isfinite(rel)) {
            st[z] = LRSDP_ERR_DEVICE;
            live[z] = 0;
            continue;
          }
          if (rel <= o.eps) {
            st[z] = LRSDP_OK;
            live[z] = 0;
            continue;
          }
          if (outer == o.max_outer) {
            live[z] = 0;
            continue;
          }
          if (rel < 0.5 * best[z]) {
            best[z] = rel;
            stall[z] = 0;
          } else if (++stall[z] >= 2) {
            st[z] = LRSDP_ERR_STAGNATED;
            live[z] = 0;
            continue;
          }
          any = true;
        }
        if (!any) break;
        LRSDP_TRY(pcg_ls(live, kVdd0, inner_tol(o, md), o.max_iter));
        for (int z = 0; z < count; ++z) {
          if (!live[z]) continue;
          info[z].iters += po[z].iters;
          info[z].outer_iters = outer + 1;
          if (po[z].status < 0) {
            st[z] = po[z].status;
            live[z] = 0;
          }
        }
        LRSDP_TRY(upload(live));
        k_dd_add_vec_b<<<gv, kT, 0, s>>>(L.b);
        LRSDP_HIP(hipGetLastError());
      }
      std::vector<char> no_lo(count);
      for (int z = 0; z < count; ++z) {
        no_lo[z] = ylo[z] == nullptr;
        info[z].dd_used = ylo[z] ? 1 : 0;
      }
      LRSDP_TRY(upload(no_lo));
      k_round_pair_b<<<gv, kT, 0, s>>>(L.b);
      LRSDP_HIP(hipGetLastError());
    }
    LRSDP_HIP(hipStreamSynchronize(s));
    return LRSDP_OK;
  };
  const int brc = body();
  (void)hipStreamSynchronize(s);
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int z = 0; z < count; ++z) {
    info[z].solve_ms = ms;
    info[z].lockstep = 1;
    if (brc < 0) st[z] = brc;
    info[z].status = st[z];
  }
  if (hpin) (void)hipHostFree(hpin);
  if (dsc) dev_free(ctx, dsc, sb);
  if (doff) dev_free(ctx, doff, ob);
  if (dact) dev_free(ctx, dact, ab);
  if (dI) dev_free(ctx, dI, ib);
  return brc;
}

}  // namespace lrsdp
