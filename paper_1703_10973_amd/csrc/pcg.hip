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
__device__ __forceinline__ bool arrive_last(int* counter) {
  __shared__ int last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(counter, 1) == (int)gridDim.x - 1;
    if (last) __threadfence();
  }
  __syncthreads();
  return last != 0;
}

// *out = sum of part[0..gridDim.x) (called by the last workgroup), counter reset for the next
// use
__device__ __forceinline__ void finish_sum(const double* part, int* counter, double* out,
                                           double* red) {
  const volatile double* vp = part;
  double s = (threadIdx.x < gridDim.x) ? vp[threadIdx.x] : 0.0;
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    *out = s;
    *counter = 0;
  }
}

// *out = a . b in one launch: per-workgroup partials, summed by the last workgroup
__global__ __launch_bounds__(kT) void k_dot(int m, const double* a, const double* b,
                                            double* part, int* counter, double* out) {
  __shared__ double red[kT / kWave];
  double s = 0.0;
  for (int i = blockIdx.x * kT + threadIdx.x; i < m; i += gridDim.x * kT) s = fma(a[i], b[i], s);
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
  if (arrive_last(counter)) finish_sum(part, counter, out, red);
}

// alpha = rho / pq;  y += alpha p;  r -= alpha q;  sc[kRR] = r.r.  A breakdown (pq <= 0 or
// rho <= 0, from rounding or an indefinite preconditioner) leaves y and r as they are, so the
// caller, which stops there, keeps the last iterate
__global__ __launch_bounds__(kT) void k_update_xr(int m, double* sc, int rho_slot, double* x,
                                                  double* r, const double* p, const double* q,
                                                  double* part, int* counter) {
  __shared__ double red[kT / kWave];
  const double rho = sc[rho_slot], pq = sc[kPQ];
  const double alpha = (pq > 0.0 && rho > 0.0) ? rho / pq : 0.0;
  double s = 0.0;
  for (int i = blockIdx.x * kT + threadIdx.x; i < m; i += gridDim.x * kT) {
    x[i] = fma(alpha, p[i], x[i]);
    const double ri = fma(-alpha, q[i], r[i]);
    r[i] = ri;
    s = fma(ri, ri, s);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
  if (arrive_last(counter)) finish_sum(part, counter, sc + kRR, red);
}

// p = z + (rho_new / rho_old) p
__global__ void k_update_p(int m, const double* sc, int rho_new, int rho_old, const double* z,
                           double* p) {
  const double beta = sc[rho_new] / sc[rho_old];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    p[i] = fma(beta, p[i], z[i]);
}

__global__ void k_copy(int m, const double* a, double* b) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    b[i] = a[i];
}

__global__ void k_zero(int m, double* a) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    a[i] = 0.0;
}

// (yh, yl) += d
__global__ void k_dd_add_vec(int m, double* yh, double* yl, const double* d) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    dd u = dd_add_d({yh[i], yl[i]}, d[i]);
    yh[i] = u.hi;
    yl[i] = u.lo;
  }
}

__global__ void k_round_pair(int m, double* yh, const double* yl) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    yh[i] = yh[i] + yl[i];
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

  bool use_dd;
  if (o.dd_mode == LRSDP_DD_ON) use_dd = true;
  else if (o.dd_mode == LRSDP_DD_OFF) use_dd = false;
  else use_dd = f->tau < o.dd_auto_ratio * f->lam[1];
  // AUTO: the low-precision W0 product pays only inside refinement, which the solve needs
  // anyway once the answer is a double-double pair; otherwise plain FP64 PCG is cheaper
  const int prec = o.precision == LRSDP_PREC_AUTO ? (use_dd ? LRSDP_PREC_FP32 : LRSDP_PREC_FP64)
                                                  : o.precision;
  const bool refine = use_dd || prec != LRSDP_PREC_FP64;
  // SMW pieces: double-double when tau^2 is within a few units of u ||bold S|| (dd_precond on
  // or auto with tau < 1e-7 lambda_max), else FP64 with one refinement step of bold S^{-1} w
  // once tau / lambda_max < 1e-3 (where the explicit inverse alone loses definiteness).
  const double ratio = f->tau / f->lam[f->k];
  bool dd_prec;
  if (o.dd_precond == 1) dd_prec = true;
  else if (o.dd_precond == 0) dd_prec = false;
  else dd_prec = ratio < 1e-7;
  int ref64 = ratio < 1e-3 ? 1 : 0;
  // Double-double refinement steps of bold S t = w inside the preconditioner.  kappa(bold S)
  // grows like 1 / ratio, so the FP64 inverse leaves a relative error of about u / ratio in t
  // and one step squares it; the SMW subtraction then magnifies what is left by about
  // 1 / ratio.  One step keeps the preconditioner within 1e-5 of exact down to
  // ratio = 1e-9, far inside the inner tolerance; below that a second step is taken.
  const int dd_steps = ratio >= 1e-9 ? 1 : 2;
  if (f->precond == LRSDP_PRECOND_AUG) {  // FP64 only (eq aug_prec is Theta(1/sqrt(mu)))
    dd_prec = false;
    ref64 = 0;
  }

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
      LRSDP_TRY(pcg(f, w.dd0, o.inner_eps, o.max_iter, Hm, Pinv, &po));
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

}  // namespace lrsdp
