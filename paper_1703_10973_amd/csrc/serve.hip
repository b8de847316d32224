// Many independent instances: a batch call and a request server.
//
// Each worker is a host thread with a context of its own (its own stream, pinned staging and
// status word on the same device), so instances run concurrently and never share scratch.
// An instance is the whole hot path: A0 (problem), Algorithm 1 steps 1-2 (factor) and
// step 3 (solve), then its handles are released.  The kernels and their launch shapes do not
// depend on what else runs, so a result is bitwise the one the instance gets alone.
//
// Admission: the server starts a queued request only while the estimated device memory of
// the requests in flight, plus its own, stays within the budget (a request larger than the
// whole budget runs alone).  Requests start in submission order.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace {

struct Job {
  uint64_t ticket = 0;
  lrsdp_instance inst{};
  lrsdp_opts opts{};
  size_t bytes = 0;
  int status = LRSDP_PENDING;
  lrsdp_info info{};
  bool done = false;
};

int run_instance(lrsdp_ctx* ctx, const lrsdp_instance& in, const lrsdp_opts& o,
                 lrsdp_info* info) {
  lrsdp_problem* P = nullptr;
  int rc = lrsdp_problem_create(ctx, in.n, in.m, in.m, in.con, in.row, in.col, in.val, &P);
  if (rc != LRSDP_OK) return rc;
  lrsdp_factor* F = nullptr;
  rc = lrsdp_factor_create(P, in.W, in.k, &o, &F);
  if (rc == LRSDP_OK) {
    rc = lrsdp_solve(F, in.r, in.y, in.y_lo, &o, info);
    lrsdp_factor_destroy(F);
  }
  lrsdp_problem_destroy(P);
  return rc;
}

}  // namespace

struct lrsdp_server {
  int device = 0;
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_work;  // workers: a request may be startable
  std::condition_variable cv_done;  // pollers: a request finished
  std::deque<Job*> queue;
  std::unordered_map<uint64_t, Job*> jobs;  // every ticket not yet released
  uint64_t next_ticket = 1;
  size_t in_flight = 0;
  int running = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<lrsdp_ctx*> ctxs;

  // the front request may start now
  bool startable() const {
    if (queue.empty()) return false;
    const size_t b = queue.front()->bytes;
    return budget == 0 || running == 0 || in_flight + b <= budget;
  }

  void work(lrsdp_ctx* ctx) {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_work.wait(lk, [&] { return stop || startable(); });
      if (!startable()) {
        if (stop && queue.empty()) return;
        continue;
      }
      Job* j = queue.front();
      queue.pop_front();
      in_flight += j->bytes;
      ++running;
      lk.unlock();
      lrsdp_info info{};
      const int st = run_instance(ctx, j->inst, j->opts, &info);
      lk.lock();
      j->status = st;
      j->info = info;
      j->done = true;
      in_flight -= j->bytes;
      --running;
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

extern "C" {

size_t lrsdp_instance_bytes(int64_t n, int64_t m, int32_t k) {
  const double nn = (double)n * n, nk = (double)n * k;
  const double pairs = (double)k * (k + 1) / 2;
  const double pair_cap = std::max(1.0, std::min(pairs, (double)(1u << 28) / nn));
  const double r = (double)k * (k - 1) / 2;
  // persistent factor (W, W0, its low-precision copy, Z, Z^T, L^{-1}, Q_N, work) plus the
  // setup temporaries (bold S, the Cholesky scratch, Z^{-1}, P_J, the R_JL blocks, the eigen
  // workspace) plus the problem (pairs, pattern, owner lists, scratch)
  const double doubles = 6.0 * nn + 2.25 * nk * nk + nk * r + 12.0 * m + 11.0 * nk +
                         (2.0 + k + pair_cap) * nn + pairs * n + nk * r + 8192.0;
  const double problem = 112.0 * m + 16.0 * n + 65536.0 +
                         (n >= kTGlobalMinN ? 16.0 * (double)n * n : 0.0);
  return (size_t)(8.0 * doubles + problem);
}

int lrsdp_server_create(lrsdp_ctx* ctx, int workers, size_t hbm_budget_bytes,
                        lrsdp_server** out) {
  if (!ctx || !out || workers < 1 || workers > 64) return LRSDP_ERR_INVALID_ARG;
  *out = nullptr;
  lrsdp_server* s = new (std::nothrow) lrsdp_server();
  if (!s) return LRSDP_ERR_OUT_OF_BUDGET;
  s->device = ctx->device;
  s->budget = hbm_budget_bytes;
  for (int w = 0; w < workers; ++w) {
    lrsdp_ctx* c = nullptr;
    const int rc = lrsdp::ctx_create(ctx->device, nullptr, 0, false, &c);
    if (rc != LRSDP_OK) {
      for (lrsdp_ctx* x : s->ctxs) lrsdp_ctx_destroy(x);
      delete s;
      return rc;
    }
    s->ctxs.push_back(c);
  }
  for (lrsdp_ctx* c : s->ctxs)
    s->workers.emplace_back([s, c] {
      (void)hipSetDevice(c->device);
      s->work(c);
    });
  *out = s;
  return LRSDP_OK;
}

int lrsdp_server_submit(lrsdp_server* s, const lrsdp_instance* inst, const lrsdp_opts* opts,
                        uint64_t* ticket) {
  if (!s || !inst || !ticket) return LRSDP_ERR_INVALID_ARG;
  Job* j = new (std::nothrow) Job();
  if (!j) return LRSDP_ERR_OUT_OF_BUDGET;
  j->inst = *inst;
  lrsdp_opts_default(&j->opts);
  if (opts) j->opts = *opts;
  j->bytes = lrsdp_instance_bytes(inst->n, inst->m, inst->k);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete j;
      return LRSDP_ERR_INVALID_ARG;
    }
    j->ticket = s->next_ticket++;
    s->jobs[j->ticket] = j;
    s->queue.push_back(j);
  }
  *ticket = j->ticket;
  s->cv_work.notify_all();
  return LRSDP_OK;
}

int lrsdp_server_poll(lrsdp_server* s, uint64_t ticket, int wait, int* status,
                      lrsdp_info* info) {
  if (!s) return LRSDP_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return LRSDP_ERR_INVALID_ARG;
  Job* j = it->second;
  if (wait) s->cv_done.wait(lk, [&] { return j->done; });
  if (!j->done) return LRSDP_PENDING;
  if (status) *status = j->status;
  if (info) *info = j->info;
  s->jobs.erase(it);
  delete j;
  return LRSDP_OK;
}

int lrsdp_server_stats(lrsdp_server* s, int* queued, int* running, int* done,
                       size_t* bytes_in_flight) {
  if (!s) return LRSDP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  int d = 0;
  for (const auto& kv : s->jobs) d += kv.second->done ? 1 : 0;
  if (queued) *queued = (int)s->queue.size();
  if (running) *running = s->running;
  if (done) *done = d;
  if (bytes_in_flight) *bytes_in_flight = s->in_flight;
  return LRSDP_OK;
}

void lrsdp_server_destroy(lrsdp_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (lrsdp_ctx* c : s->ctxs) lrsdp_ctx_destroy(c);
  for (auto& kv : s->jobs) delete kv.second;
  delete s;
}

int lrsdp_solve_batch(lrsdp_ctx* ctx, int count, const lrsdp_instance* inst,
                      const lrsdp_opts* opts, int workers, int* status, lrsdp_info* info) {
  if (!ctx || count < 0 || (count > 0 && (!inst || !status)) || workers < 1)
    return LRSDP_ERR_INVALID_ARG;
  if (count == 0) return LRSDP_OK;
  lrsdp_server* s = nullptr;
  LRSDP_TRY(lrsdp_server_create(ctx, std::min(workers, count), ctx->budget, &s));
  std::vector<uint64_t> t(count);
  int rc = LRSDP_OK;
  for (int i = 0; i < count && rc == LRSDP_OK; ++i) rc = lrsdp_server_submit(s, &inst[i], opts, &t[i]);
  for (int i = 0; i < count; ++i) {
    if (rc != LRSDP_OK) {
      status[i] = rc;
      continue;
    }
    lrsdp_info inf{};
    const int prc = lrsdp_server_poll(s, t[i], 1, &status[i], &inf);
    if (prc != LRSDP_OK) status[i] = prc;
    if (info) info[i] = inf;
  }
  lrsdp_server_destroy(s);
  return rc;
}

}  // extern "C"
