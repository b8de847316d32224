// The C ABI declared in include/lrsdp.h: handles, validation, budget accounting.
#include <chrono>
#include <iterator>
#include <cstring>
#include <new>

#include "dense.h"

namespace lrsdp {

// Device memory is cached per context: a freed block returns to a free list keyed by its
// rounded size and is handed out again by a later request of that size.  hipFree (which
// waits for the whole device) then runs only when the cache outgrows its cap or the context
// ends, so concurrent contexts do not stall each other, and stream order on the context's one
// stream makes reuse safe.  The budget counts the bytes held by live handles.
static size_t pool_size_class(size_t bytes) {
  const size_t q = bytes >= ((size_t)1 << 20) ? ((size_t)1 << 20) : 4096;
  return (bytes + q - 1) / q * q;
}

static void pool_trim(lrsdp_ctx* ctx, size_t keep) {
  for (auto it = ctx->pool.begin(); it != ctx->pool.end() && ctx->pooled > keep;) {
    while (!it->second.empty() && ctx->pooled > keep) {
      (void)hipFree(it->second.back());
      it->second.pop_back();
      ctx->pooled -= it->first;
    }
    it = it->second.empty() ? ctx->pool.erase(it) : std::next(it);
  }
}

int dev_alloc(lrsdp_ctx* ctx, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return LRSDP_OK;
  const size_t sz = pool_size_class(bytes);
  if (ctx->budget && ctx->in_use + sz > ctx->budget) return LRSDP_ERR_OUT_OF_BUDGET;
  auto it = ctx->pool.find(sz);
  if (it != ctx->pool.end() && !it->second.empty()) {
    *p = it->second.back();
    it->second.pop_back();
    ctx->pooled -= sz;
    ctx->in_use += sz;
    return LRSDP_OK;
  }
  if (hipMalloc(p, sz) != hipSuccess) {
    (void)hipGetLastError();
    pool_trim(ctx, 0);  // give the cache back and try once more
    if (hipMalloc(p, sz) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return LRSDP_ERR_OUT_OF_BUDGET;
    }
  }
  ctx->in_use += sz;
  return LRSDP_OK;
}

void dev_free(lrsdp_ctx* ctx, void* p, size_t bytes) {
  if (!p) return;
  const size_t sz = pool_size_class(bytes);
  ctx->pool[sz].push_back(p);
  ctx->pooled += sz;
  ctx->in_use -= sz;
  if (ctx->pooled > ctx->pool_cap) pool_trim(ctx, ctx->pool_cap / 2);
}

int ctx_side(lrsdp_ctx* ctx, SideStream* out) {
  if (!ctx->side) {
    if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess) {
      ctx->side = nullptr;
      return LRSDP_ERR_DEVICE;
    }
    for (hipEvent_t& e : ctx->side_ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return LRSDP_ERR_DEVICE;
  }
  out->stream = ctx->side;
  out->ev = ctx->side_ev;
  out->depths = (int)(sizeof(ctx->side_ev) / sizeof(ctx->side_ev[0])) / 2;
  return LRSDP_OK;
}

thread_local Profiler* tls_prof = nullptr;

static hipEvent_t prof_event(Profiler* p) {
  if (!p->pool.empty()) {
    hipEvent_t e = p->pool.back();
    p->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfMark prof_begin(int kid, hipStream_t s) {
  ProfMark mk;
  if (!prof_on() || !(tls_prof->mask & (1u << kid))) return mk;
  if (tls_prof->seen[kid]++ % tls_prof->every != 0) return mk;
  mk.a = prof_event(tls_prof);
  if (!mk.a || hipEventRecord(mk.a, s) != hipSuccess) {
    mk.a = nullptr;
    return mk;
  }
  mk.kid = kid;
  return mk;
}

void prof_end(const ProfMark& mk, hipStream_t s, double bytes, double flops) {
  if (mk.kid < 0 || !prof_on()) return;
  hipEvent_t b = prof_event(tls_prof);
  if (!b || hipEventRecord(b, s) != hipSuccess) return;
  tls_prof->pending.push_back({mk.kid, mk.a, b, bytes, flops});
}

void prof_flush(Profiler* p) {
  if (p->pending.empty()) return;
  for (auto& q : p->pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(q.b) == hipSuccess && hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
      ProfStat& st = p->stat[q.kid];
      st.launches += 1;
      st.ms += ms;
      st.bytes += q.bytes;
      st.flops += q.flops;
    }
    p->pool.push_back(q.a);
    p->pool.push_back(q.b);
  }
  p->pending.clear();
}

}  // namespace lrsdp

using namespace lrsdp;

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

bool opts_valid(const lrsdp_opts& o) {
  return o.eps > 0.0 && o.max_iter >= 1 && o.precision >= 0 && o.precision <= 3 &&
         o.dd_mode >= 0 && o.dd_mode <= 2 && o.max_outer >= 0 && o.inner_eps >= 0.0 &&
         o.inner_eps < 1.0 && o.dd_precond >= 0 && o.dd_precond <= 2 && o.tau_rule >= 0 &&
         o.tau_rule <= 1 && (o.precond == LRSDP_PRECOND_SMW || o.precond == LRSDP_PRECOND_AUG);
}

}  // namespace

namespace lrsdp {
bool opts_ok(const lrsdp_opts& o) { return opts_valid(o); }
}  // namespace lrsdp

extern "C" {

void lrsdp_opts_default(lrsdp_opts* o) {
  if (!o) return;
  o->eps = 1e-8;
  o->max_iter = 200;
  o->precision = LRSDP_PREC_FP64;
  o->dd_mode = LRSDP_DD_AUTO;
  o->deflate = 1;
  o->max_outer = 8;
  o->inner_eps = 0.0;  // by precision (inner_tol)
  o->dd_auto_ratio = 2e-5;
  o->dd_precond = 2;
  o->tau_rule = LRSDP_TAU_MEAN;
  o->precond = LRSDP_PRECOND_SMW;
}

const char* lrsdp_status_string(int s) {
  switch (s) {
    case LRSDP_OK: return "OK";
    case LRSDP_NOT_CONVERGED: return "NOT_CONVERGED";
    case LRSDP_ERR_INVALID_ARG: return "INVALID_ARG";
    case LRSDP_ERR_DUPLICATE_PAIR: return "DUPLICATE_PAIR";
    case LRSDP_ERR_UNSUPPORTED: return "UNSUPPORTED";
    case LRSDP_ERR_NOT_PD_W: return "NOT_PD_W";
    case LRSDP_ERR_CHOL_Z: return "CHOL_Z";
    case LRSDP_ERR_CHOL_S: return "CHOL_S";
    case LRSDP_ERR_OUT_OF_BUDGET: return "OUT_OF_BUDGET";
    case LRSDP_ERR_STAGNATED: return "STAGNATED";
    case LRSDP_ERR_INDEFINITE_PRECOND: return "INDEFINITE_PRECOND";
    case LRSDP_ERR_DEVICE: return "DEVICE_ERROR";
    case LRSDP_ERR_EIG: return "EIG_FAILED";
    case LRSDP_ERR_SCRATCH: return "SCRATCH_TOO_SMALL";
    case LRSDP_ERR_IPM: return "IPM_FAILED";
    default: return "UNKNOWN";
  }
}

}  // extern "C"

namespace lrsdp {

// A context on `device`.  With stream == NULL the context makes its own stream: blocking
// (ordered after work on the legacy default stream, where callers such as torch produce their
// inputs) for the public entry point, non-blocking for the server's workers, whose requests
// are complete before submission and which must not serialize with each other through it.
int ctx_create(int device, void* stream, size_t budget, bool blocking, lrsdp_ctx** out) {
  if (!out) return LRSDP_ERR_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return LRSDP_ERR_INVALID_ARG;
  DeviceGuard g(device);
  lrsdp_ctx* c = new (std::nothrow) lrsdp_ctx();
  if (!c) return LRSDP_ERR_OUT_OF_BUDGET;
  c->device = device;
  c->budget = budget;
  if (stream) {
    c->stream = static_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, blocking ? hipStreamDefault : hipStreamNonBlocking) !=
        hipSuccess) {
      delete c;
      return LRSDP_ERR_DEVICE;
    }
    c->own_stream = true;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_pinned), 64 * sizeof(double),
                    hipHostMallocDefault) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&c->d_flag), 4 * sizeof(int)) != hipSuccess) {
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return LRSDP_ERR_DEVICE;
  }
  // the allocation-free entry point's fixed scratch: its address on this device, once
  if (noalloc_scratch_setup(device) != LRSDP_OK) {
    lrsdp_ctx_destroy(c);
    return LRSDP_ERR_DEVICE;
  }
  for (hipEvent_t& e : c->phase_ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      lrsdp_ctx_destroy(c);
      return LRSDP_ERR_DEVICE;
    }
  }
  for (hipEvent_t& e : c->scal_ev) {
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      e = nullptr;
      lrsdp_ctx_destroy(c);
      return LRSDP_ERR_DEVICE;
    }
  }
  *out = c;
  return LRSDP_OK;
}

}  // namespace lrsdp

extern "C" {

int lrsdp_ctx_create(int device, void* stream, size_t budget, lrsdp_ctx** out) {
  return ctx_create(device, stream, budget, true, out);
}

}  // extern "C"

namespace {

void ctx_release(lrsdp_ctx* c) {
  for (lrsdp_ctx* w : c->batch_workers) ctx_release(w);
  c->batch_workers.clear();
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  prof_flush(&c->prof);
  for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    for (hipEvent_t e : c->side_ev)
      if (e) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(c->side);
  }
  pool_trim(c, 0);
  for (hipEvent_t e : c->phase_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->scal_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->h_pinned) (void)hipHostFree(c->h_pinned);
  if (c->d_flag) (void)hipFree(c->d_flag);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

// Releases a problem's device memory and the handle; then its context, if that was destroyed
// while this was its last live problem.
void problem_release(lrsdp_problem* p) {
  lrsdp_ctx* c = p->ctx;
  {
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    const size_t m = p->m, n = p->n, nnz = p->nnz;
    dev_free(c, p->a, m * 4);
    dev_free(c, p->b, m * 4);
    dev_free(c, p->val, m * 8);
    dev_free(c, p->coef, m * 8);
    dev_free(c, p->ginv, m * 8);
    dev_free(c, p->rowptr, (n + 1) * 4);
    dev_free(c, p->own_ptr, (n + 1) * 4);
    dev_free(c, p->own_con, m * 4);
    dev_free(c, p->own_oth, m * 4);
    dev_free(c, p->pat, 2 * m * 4);
    dev_free(c, p->colidx, nnz * 4);
    dev_free(c, p->src, nnz * 4);
    dev_free(c, p->mval, nnz * 8);
    dev_free(c, p->vec_scratch, 4 * m * 8);
    dev_free(c, p->tscr, 2 * n * n * 8);
  }
  delete p;
  if (--c->children == 0 && c->closing) ctx_release(c);
}

}  // namespace

extern "C" {

// Destroying a handle that still has live children (problems of a context, factors of a
// problem) only marks it: it is released together with its last child, so handles may be
// destroyed in any order (for example by a garbage collector).
void lrsdp_ctx_destroy(lrsdp_ctx* c) {
  if (!c) return;
  if (c->children > 0) {
    c->closing = true;
    return;
  }
  ctx_release(c);
}

int lrsdp_ctx_profile(lrsdp_ctx* c, int enable) {
  if (!c) return LRSDP_ERR_INVALID_ARG;
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  prof_flush(&c->prof);
  for (auto& st : c->prof.stat) st = ProfStat();
  c->prof.enabled = enable != 0;
  c->prof.mask = static_cast<unsigned>(enable);
  for (auto& v : c->prof.seen) v = 0;
  return LRSDP_OK;
}

int lrsdp_ctx_profile_sample(lrsdp_ctx* c, int every) {
  if (!c || every < 1) return LRSDP_ERR_INVALID_ARG;
  c->prof.every = every;
  for (auto& v : c->prof.seen) v = 0;
  return LRSDP_OK;
}

int lrsdp_ctx_profile_read(const lrsdp_ctx* c, int kid, int64_t* launches, double* ms,
                           double* bytes, double* flops) {
  if (!c || kid < 0 || kid >= LRSDP_K_COUNT) return LRSDP_ERR_INVALID_ARG;
  const ProfStat& st = c->prof.stat[kid];
  if (launches) *launches = st.launches;
  if (ms) *ms = st.ms;
  if (bytes) *bytes = st.bytes;
  if (flops) *flops = st.flops;
  return LRSDP_OK;
}

int lrsdp_ctx_memory(const lrsdp_ctx* c, size_t* in_use, size_t* budget) {
  if (!c) return LRSDP_ERR_INVALID_ARG;
  if (in_use) *in_use = c->in_use;
  if (budget) *budget = c->budget;
  return LRSDP_OK;
}

void lrsdp_problem_destroy(lrsdp_problem* p) {
  if (!p) return;
  if (p->children > 0) {
    p->closing = true;
    return;
  }
  problem_release(p);
}

int lrsdp_problem_create(lrsdp_ctx* c, int64_t n, int64_t m, int64_t nnz, const int32_t* con,
                         const int32_t* row, const int32_t* col, const double* val,
                         lrsdp_problem** out) {
  if (!c || !out) return LRSDP_ERR_INVALID_ARG;
  *out = nullptr;
  if (n < 2 || m < 1 || nnz < 1 || n > (1 << 20) || m > (1LL << 30) || nnz > (1LL << 30) ||
      !con || !row || !col || !val)
    return LRSDP_ERR_INVALID_ARG;
  if (nnz != m) return LRSDP_ERR_UNSUPPORTED;
  DeviceGuard g(c->device);
  lrsdp_problem* p = new (std::nothrow) lrsdp_problem();
  if (!p) return LRSDP_ERR_OUT_OF_BUDGET;
  p->ctx = c;
  p->n = (int)n;
  p->m = (int)m;
  ++c->children;  // released (and counted down) by problem_release, also on failure
  int rc = LRSDP_OK;
  do {
    if ((rc = dev_alloc_n(c, &p->a, (size_t)m))) break;
    if ((rc = dev_alloc_n(c, &p->b, (size_t)m))) break;
    if ((rc = dev_alloc_n(c, &p->val, (size_t)m))) break;
    if ((rc = dev_alloc_n(c, &p->coef, (size_t)m))) break;
    if ((rc = dev_alloc_n(c, &p->ginv, (size_t)m))) break;
    if ((rc = dev_alloc_n(c, &p->rowptr, (size_t)n + 1))) break;
    if ((rc = dev_alloc_n(c, &p->own_ptr, (size_t)n + 1))) break;
    if ((rc = dev_alloc_n(c, &p->own_con, (size_t)m))) break;
    if ((rc = dev_alloc_n(c, &p->own_oth, (size_t)m))) break;
    if ((rc = dev_alloc_n(c, &p->pat, 2 * (size_t)m))) break;
    if ((rc = dev_alloc_n(c, &p->vec_scratch, 4 * (size_t)m))) break;
    if (n >= kTGlobalMinN && (rc = dev_alloc_n(c, &p->tscr, 2 * (size_t)n * n))) break;
    ProfScope ps(c);
    rc = ingest(c, p, con, row, col, val, nnz);
  } while (0);
  if (rc != LRSDP_OK) {
    problem_release(p);
    return rc;
  }
  p->bytes = c->in_use;
  *out = p;
  return LRSDP_OK;
}

int lrsdp_problem_info(const lrsdp_problem* p, int64_t* n, int64_t* m, int64_t* nnz) {
  if (!p) return LRSDP_ERR_INVALID_ARG;
  if (n) *n = p->n;
  if (m) *m = p->m;
  if (nnz) *nnz = p->nnz;
  return LRSDP_OK;
}

int lrsdp_hessian_apply(lrsdp_problem* p, const double* W, const double* v, double* Hv) {
  if (!p || !W || !v || !Hv) return LRSDP_ERR_INVALID_ARG;
  DeviceGuard g(p->ctx->device);
  ProfScope ps(p->ctx);
  LRSDP_TRY(hv_apply_f64(p, W, v, Hv, p->ctx->stream));
  LRSDP_HIP(hipStreamSynchronize(p->ctx->stream));
  return LRSDP_OK;
}

int lrsdp_aug_wtilde_solve(lrsdp_ctx* ctx, int32_t n, int32_t k, double tau, const double* Ut,
                           const double* b, double* x) {
  if (!ctx) return LRSDP_ERR_INVALID_ARG;
  DeviceGuard g(ctx->device);
  return aug_wtilde_solve(ctx, n, k, tau, Ut, b, x);
}

int lrsdp_hessian_apply_noalloc(lrsdp_problem* p, const double* W, const double* v, double* Hv) {
  if (!p || !W || !v || !Hv) return LRSDP_ERR_INVALID_ARG;
  DeviceGuard g(p->ctx->device);
  LRSDP_TRY(hv_apply_f64_noalloc(p, W, v, Hv, p->ctx->device, p->ctx->stream));
  LRSDP_HIP(hipStreamSynchronize(p->ctx->stream));
  return LRSDP_OK;
}

int lrsdp_factor_create(lrsdp_problem* p, const double* W, int32_t k, const lrsdp_opts* opts,
                        lrsdp_factor** out) {
  if (!p || !W || !out) return LRSDP_ERR_INVALID_ARG;
  *out = nullptr;
  lrsdp_opts o;
  lrsdp_opts_default(&o);
  if (opts) o = *opts;
  if (!opts_valid(o)) return LRSDP_ERR_INVALID_ARG;
  if (k < 1 || k >= p->n || k > 16) return LRSDP_ERR_INVALID_ARG;
  DeviceGuard g(p->ctx->device);
  ProfScope ps(p->ctx);
  lrsdp_factor* f = new (std::nothrow) lrsdp_factor();
  if (!f) return LRSDP_ERR_OUT_OF_BUDGET;
  f->P = p;
  f->n = p->n;
  f->k = k;
  f->nk = p->n * k;
  int rc = factor_setup(f, W, o);
  if (rc != LRSDP_OK) {
    (void)hipStreamSynchronize(p->ctx->stream);
    if (p->ctx->side) (void)hipStreamSynchronize(p->ctx->side);
    factor_release(f);
    delete f;
    return rc;
  }
  ++p->children;
  *out = f;
  return LRSDP_OK;
}

int lrsdp_factor_info(const lrsdp_factor* f, int64_t* n, int64_t* m, int32_t* k) {
  if (!f) return LRSDP_ERR_INVALID_ARG;
  if (n) *n = f->n;
  if (m) *m = f->P->m;
  if (k) *k = f->k;
  return LRSDP_OK;
}

void lrsdp_factor_destroy(lrsdp_factor* f) {
  if (!f) return;
  lrsdp_problem* p = f->P;
  {
    DeviceGuard g(p->ctx->device);
    (void)hipStreamSynchronize(p->ctx->stream);
    factor_release(f);
  }
  delete f;
  if (--p->children == 0 && p->closing) problem_release(p);
}

int lrsdp_factor_export(const lrsdp_factor* f, double* tau, double* shift, double* lam,
                        double* setup_ms, double* U, double* W0, double* Z, double* Sinv) {
  if (!f) return LRSDP_ERR_INVALID_ARG;
  DeviceGuard g(f->P->ctx->device);
  hipStream_t s = f->P->ctx->stream;
  const size_t nn = (size_t)f->n * f->n, nk = f->nk;
  if (tau) *tau = f->tau;
  if (shift) *shift = f->shift;
  if (setup_ms) *setup_ms = f->setup_ms;
  if (lam) std::memcpy(lam, f->lam.data(), f->lam.size() * sizeof(double));
  if (U) LRSDP_HIP(hipMemcpyAsync(U, f->U, nk * 8, hipMemcpyDeviceToDevice, s));
  if (W0) LRSDP_HIP(hipMemcpyAsync(W0, f->W0, nn * 8, hipMemcpyDeviceToDevice, s));
  if (Z && !f->Z) return LRSDP_ERR_INVALID_ARG;  // the augmented preconditioner has no Z
  if (Z) LRSDP_HIP(hipMemcpyAsync(Z, f->Z, nn * 8, hipMemcpyDeviceToDevice, s));
  if (Sinv) LRSDP_TRY(export_sinv(f, Sinv, s));
  LRSDP_HIP(hipStreamSynchronize(s));
  return LRSDP_OK;
}

int lrsdp_hessian_apply_split(lrsdp_factor* f, const double* v, double* Hv, int precision) {
  if (!f || !v || !Hv || precision < 0 || precision > 2) return LRSDP_ERR_INVALID_ARG;
  DeviceGuard g(f->P->ctx->device);
  ProfScope ps(f->P->ctx);
  LRSDP_TRY(split_apply(f, v, Hv, precision, f->P->ctx->stream));
  LRSDP_HIP(hipStreamSynchronize(f->P->ctx->stream));
  return LRSDP_OK;
}

int lrsdp_precond_apply(lrsdp_factor* f, const double* v, double* z, int ddm) {
  if (!f || !v || !z) return LRSDP_ERR_INVALID_ARG;
  DeviceGuard g(f->P->ctx->device);
  ProfScope ps(f->P->ctx);
  hipStream_t s = f->P->ctx->stream;
  if (f->precond == LRSDP_PRECOND_AUG && ddm != 0) return LRSDP_ERR_INVALID_ARG;
  if (ddm == 1) LRSDP_TRY(precond_apply_dd(f, v, z, s, 2));
  else LRSDP_TRY(precond_apply_f64(f, v, z, s, ddm == 2));
  LRSDP_HIP(hipStreamSynchronize(s));
  return LRSDP_OK;
}

int lrsdp_residual_dd(lrsdp_factor* f, const double* r, const double* y, const double* ylo,
                      double* res, double* relres) {
  if (!f || !r || !y || !relres) return LRSDP_ERR_INVALID_ARG;
  DeviceGuard g(f->P->ctx->device);
  ProfScope ps(f->P->ctx);
  const Work w = work_view(f);
  double rel = 0.0;
  LRSDP_TRY(residual_dd(f, r, y, ylo, res ? res : w.dd0, w.dd1, &rel));
  *relres = rel;
  return LRSDP_OK;
}

int lrsdp_solve(lrsdp_factor* f, const double* r, double* y, double* ylo, const lrsdp_opts* opts,
                lrsdp_info* info) {
  if (!f || !r || !y) return LRSDP_ERR_INVALID_ARG;
  lrsdp_opts o;
  lrsdp_opts_default(&o);
  if (opts) o = *opts;
  if (!opts_valid(o)) return LRSDP_ERR_INVALID_ARG;
  DeviceGuard g(f->P->ctx->device);
  ProfScope ps(f->P->ctx);
  return solve_run(f, r, y, ylo, o, info);
}

void lrsdp_ipm_opts_default(lrsdp_ipm_opts* o) {
  if (!o) return;
  o->tol = 1e-9;
  o->max_iter = 60;
  o->sigma = 0.1;
  o->predictor = 1;
  o->warm_start = 0;
  o->stall_iters = 5;
  o->frac = 0.9;
  o->k = 2;
  o->rank_eta = 0.0;
  o->pcg_eps = 1e-9;
  o->pcg_eps_mu = 0.0;
  o->max_ns_iter = 100;
  o->householder_eig = 0;
  o->ns_tol = 1e-10;
  lrsdp_opts_default(&o->solve);
  o->solve.precision = LRSDP_PREC_AUTO;
  o->solve.dd_mode = LRSDP_DD_AUTO;
}

int lrsdp_ipm_solve(lrsdp_problem* p, const double* b, const double* C,
                    const lrsdp_ipm_opts* opts, double* X, double* y, double* S,
                    lrsdp_ipm_info* info, lrsdp_ipm_record* recs, int max_recs) {
  if (!p || !b || !X || !y || !S || max_recs < 0) return LRSDP_ERR_INVALID_ARG;
  lrsdp_ipm_opts o;
  lrsdp_ipm_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.tol > 0.0) || o.max_iter < 0 || !(o.sigma >= 0.0 && o.sigma < 1.0) ||
      !(o.frac > 0.0 && o.frac < 1.0) || o.k < 1 || o.k > 16 || o.k >= p->n ||
      !(o.pcg_eps > 0.0 && o.pcg_eps < 1.0) || !(o.pcg_eps_mu >= 0.0) || !(o.rank_eta >= 0.0) ||
      o.max_ns_iter < 1 || !(o.ns_tol > 0.0) || (o.householder_eig != 0 && o.householder_eig != 1) ||
      (o.predictor != 0 && o.predictor != 1) || (o.warm_start != 0 && o.warm_start != 1) ||
      o.stall_iters < 0 || (o.rank_eta > 0.0 && o.k + 1 >= p->n) ||
      !opts_valid(o.solve) || p->n < 3 || p->n > 4096)
    return LRSDP_ERR_INVALID_ARG;
  DeviceGuard g(p->ctx->device);
  ProfScope ps(p->ctx);
  return ipm_run(p, b, C, o, X, y, S, info, recs, max_recs);
}

}  // extern "C"
