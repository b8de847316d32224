// Many Hessian-equation solves on one device: a batch call and a request server.
//
// Each worker is a host thread with a context of its own (its own stream, pinned staging and
// status word on the same device), so requests run concurrently and never share scratch.
// The kernels and their launch shapes depend only on their own instance, so a result is
// bitwise the one the instance gets alone.
//
// The batch call sets its instances up on the workers and solves them in lock-step: the solves
// that take one step sequence advance together, one launch per step for all of them
// (solve_lockstep), the first half of the batch while the workers set up the second.
//
// Requests are of two sorts.
//   * Instances: the whole hot path, A0 (problem), Algorithm 1 steps 1-2 (factor) and step 3
//     (solve), after which the handles are released.
//   * Requests on a session: a session keeps one SDP's data (the problem) and its current
//     factor resident on the device between requests, the way an interior-point method uses
//     them (Section 2: one scaling matrix W per step, one or a few right-hand sides per W).
//     A factor request builds the factor of a new W (steps 1-2); a solve request runs step 3
//     against the resident factor.  A session has a context of its own (stream and memory
//     pool), so whichever worker is free runs its next request; its requests run one at a
//     time, in submission order, and overlap with those of other sessions and instances.
//
// Admission by device memory: an instance holds its estimated peak bytes while it runs; a
// session holds its problem's bytes from open to close and its factor's estimated peak bytes
// from its first factor request to close.  A request starts only while the bytes held, plus
// what it adds, fit the budget (a request that alone exceeds the budget runs when nothing
// else is running).  Requests that need memory are admitted in submission order; a request
// waiting for its session's previous request does not hold up others.
#include <algorithm>
#include <atomic>
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

enum JobKind : int { kInstance = 0, kOpen = 1, kFactor = 2, kSolve = 3, kClose = 4 };

struct Session {
  uint64_t id = 0;
  lrsdp_ctx* ctx = nullptr;      // its own context (created by the open request)
  bool busy = false;             // one of its requests is running
  bool closing = false;          // close submitted: no further requests are accepted
  int pending = 0;               // submitted requests not finished
  int64_t n = 0, m = 0;
  lrsdp_problem* P = nullptr;
  lrsdp_factor* F = nullptr;
  size_t problem_bytes = 0;      // held from open to close
  size_t factor_bytes = 0;       // held from the first factor request to close
};

struct Job {
  uint64_t ticket = 0;
  int kind = kInstance;
  lrsdp_instance inst{};  // instance: everything; open: n, m and the triplets; factor: W, k;
                          // solve: r, y, y_lo
  lrsdp_opts opts{};
  size_t bytes = 0;       // instance: held while it runs; open / factor: the session's share
  Session* sess = nullptr;
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

void session_release(Session* S) {
  if (S->F) lrsdp_factor_destroy(S->F);
  if (S->P) lrsdp_problem_destroy(S->P);
  if (S->ctx) lrsdp_ctx_destroy(S->ctx);
  S->F = nullptr;
  S->P = nullptr;
  S->ctx = nullptr;
}

// A session request, on the session's own context, from the worker thread that runs it (one
// at a time per session).
int run_session_job(int device, Job* j, lrsdp_info* info) {
  Session* S = j->sess;
  const lrsdp_instance& in = j->inst;
  switch (j->kind) {
    case kOpen: {
      const int rc = lrsdp::ctx_create(device, nullptr, 0, false, &S->ctx);
      if (rc != LRSDP_OK) return rc;
      return lrsdp_problem_create(S->ctx, in.n, in.m, in.m, in.con, in.row, in.col, in.val,
                                  &S->P);
    }
    case kFactor: {
      if (!S->P) return LRSDP_ERR_INVALID_ARG;
      if (S->F) {  // the previous W's factor goes first (its memory is reused)
        lrsdp_factor_destroy(S->F);
        S->F = nullptr;
      }
      const int rc = lrsdp_factor_create(S->P, in.W, in.k, &j->opts, &S->F);
      if (rc == LRSDP_OK) {
        info->setup_ms = S->F->setup_ms;
        info->tau = S->F->tau;
        info->eig_sweeps = S->F->eig_sweeps;
        for (int i = 0; i < 4; ++i) info->phase_ms[i] = S->F->phase_ms[i];
      }
      info->status = rc;
      return rc;
    }
    case kSolve:
      if (!S->F) return LRSDP_ERR_INVALID_ARG;
      return lrsdp_solve(S->F, in.r, in.y, in.y_lo, &j->opts, info);
    case kClose:
      session_release(S);
      return LRSDP_OK;
  }
  return LRSDP_ERR_INVALID_ARG;
}

size_t problem_bytes_estimate(int64_t n, int64_t m) {
  return (size_t)(112.0 * m + 16.0 * n + 65536.0 +
                  (n >= kTGlobalMinN ? 16.0 * (double)n * n : 0.0));
}

}  // namespace

struct lrsdp_server {
  int device = 0;
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_work;  // workers: a request may be startable
  std::condition_variable cv_done;  // pollers: a request finished
  std::deque<Job*> queue;
  std::unordered_map<uint64_t, Job*> jobs;          // every ticket not yet released
  std::unordered_map<uint64_t, Session*> sessions;  // sessions not yet fully closed
  uint64_t next_ticket = 1, next_session = 1;
  size_t in_flight = 0;   // bytes held by running instances and by open sessions
  int running = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<lrsdp_ctx*> ctxs;

  // Bytes a job adds to in_flight when it starts.
  static size_t need(const Job* j) {
    if (j->kind == kInstance || j->kind == kOpen) return j->bytes;
    if (j->kind == kFactor && j->bytes > j->sess->factor_bytes)
      return j->bytes - j->sess->factor_bytes;
    return 0;
  }

  // The first queued job that may start now, or the end of the queue.  A job waiting for its
  // session's previous request is passed over; one that needs memory the budget cannot give
  // yet stops the search, so memory is granted in submission order.
  std::deque<Job*>::iterator pick() {
    for (auto it = queue.begin(); it != queue.end(); ++it) {
      Job* j = *it;
      if (j->sess && j->sess->busy) continue;
      const size_t b = need(j);
      if (b == 0 || budget == 0 || running == 0 || in_flight + b <= budget) return it;
      return queue.end();
    }
    return queue.end();
  }

  void finish(Job* j, int st, const lrsdp_info& info, size_t held) {
    j->status = st;
    j->info = info;
    j->done = true;
    in_flight -= held;
    if (Session* S = j->sess) {
      S->busy = false;
      --S->pending;
      if (j->kind == kClose) {
        in_flight -= S->problem_bytes + S->factor_bytes;
        S->problem_bytes = S->factor_bytes = 0;
        sessions.erase(S->id);
        delete S;
        j->sess = nullptr;
      }
    }
    --running;
    cv_done.notify_all();
    cv_work.notify_all();
  }

  void work(lrsdp_ctx* ctx) {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      auto it = queue.end();
      cv_work.wait(lk, [&] { return (it = pick()) != queue.end() || (stop && queue.empty()); });
      if (it == queue.end()) return;  // stopping, nothing left
      Job* j = *it;
      queue.erase(it);
      size_t held = 0;  // released when the job finishes (instances only)
      const size_t add = need(j);
      in_flight += add;
      if (j->kind == kInstance) held = add;
      if (Session* S = j->sess) {
        S->busy = true;
        if (j->kind == kOpen) {
          S->problem_bytes = add;
        } else if (j->kind == kFactor) {
          S->factor_bytes += add;
        }
      }
      ++running;
      lk.unlock();
      lrsdp_info info{};
      const int st = j->sess ? run_session_job(ctx->device, j, &info)
                             : run_instance(ctx, j->inst, j->opts, &info);
      lk.lock();
      finish(j, st, info, held);
    }
  }

  // Queues a job (the lock is held); returns its ticket.
  uint64_t enqueue(Job* j) {
    j->ticket = next_ticket++;
    jobs[j->ticket] = j;
    queue.push_back(j);
    if (j->sess) ++j->sess->pending;
    return j->ticket;
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
  const double doubles = 6.0 * nn + 2.25 * nk * nk + nk * r + 12.0 * m + 13.0 * nk +
                         (2.0 + k + pair_cap) * nn + pairs * n + nk * r + 8192.0;
  return (size_t)(8.0 * doubles) + problem_bytes_estimate(n, m);
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
  for (int w = 0; w < workers; ++w)
    s->workers.emplace_back([s, w] {
      lrsdp_ctx* c = s->ctxs[w];
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
    *ticket = s->enqueue(j);
  }
  s->cv_work.notify_all();
  return LRSDP_OK;
}

int lrsdp_server_session_open(lrsdp_server* s, int64_t n, int64_t m, const int32_t* con,
                              const int32_t* row, const int32_t* col, const double* val,
                              uint64_t* session, uint64_t* ticket) {
  if (!s || !session || !ticket || n < 2 || m < 1 || !con || !row || !col || !val)
    return LRSDP_ERR_INVALID_ARG;
  Session* S = new (std::nothrow) Session();
  Job* j = new (std::nothrow) Job();
  if (!S || !j) {
    delete S;
    delete j;
    return LRSDP_ERR_OUT_OF_BUDGET;
  }
  S->n = n;
  S->m = m;
  j->kind = kOpen;
  j->sess = S;
  j->inst.n = n;
  j->inst.m = m;
  j->inst.con = con;
  j->inst.row = row;
  j->inst.col = col;
  j->inst.val = val;
  lrsdp_opts_default(&j->opts);
  j->bytes = problem_bytes_estimate(n, m);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete S;
      delete j;
      return LRSDP_ERR_INVALID_ARG;
    }
    S->id = s->next_session++;
    s->sessions[S->id] = S;
    *session = S->id;
    *ticket = s->enqueue(j);
  }
  s->cv_work.notify_all();
  return LRSDP_OK;
}

namespace {

// Queues a factor, solve or close request on an open session.
int submit_on_session(lrsdp_server* s, uint64_t session, Job* j, uint64_t* ticket) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->sessions.find(session);
    if (s->stop || it == s->sessions.end() || it->second->closing) {
      delete j;
      return LRSDP_ERR_INVALID_ARG;
    }
    j->sess = it->second;
    if (j->kind == kFactor)
      j->bytes = lrsdp_instance_bytes(j->sess->n, j->sess->m, j->inst.k) -
                 problem_bytes_estimate(j->sess->n, j->sess->m);
    if (j->kind == kClose) j->sess->closing = true;
    *ticket = s->enqueue(j);
  }
  s->cv_work.notify_all();
  return LRSDP_OK;
}

}  // namespace

int lrsdp_server_submit_factor(lrsdp_server* s, uint64_t session, const double* W, int32_t k,
                               const lrsdp_opts* opts, uint64_t* ticket) {
  if (!s || !W || !ticket) return LRSDP_ERR_INVALID_ARG;
  Job* j = new (std::nothrow) Job();
  if (!j) return LRSDP_ERR_OUT_OF_BUDGET;
  j->kind = kFactor;
  j->inst.W = W;
  j->inst.k = k;
  lrsdp_opts_default(&j->opts);
  if (opts) j->opts = *opts;
  return submit_on_session(s, session, j, ticket);
}

int lrsdp_server_submit_solve(lrsdp_server* s, uint64_t session, const double* r, double* y,
                              double* y_lo, const lrsdp_opts* opts, uint64_t* ticket) {
  if (!s || !r || !y || !ticket) return LRSDP_ERR_INVALID_ARG;
  Job* j = new (std::nothrow) Job();
  if (!j) return LRSDP_ERR_OUT_OF_BUDGET;
  j->kind = kSolve;
  j->inst.r = r;
  j->inst.y = y;
  j->inst.y_lo = y_lo;
  lrsdp_opts_default(&j->opts);
  if (opts) j->opts = *opts;
  return submit_on_session(s, session, j, ticket);
}

int lrsdp_server_session_close(lrsdp_server* s, uint64_t session, uint64_t* ticket) {
  if (!s || !ticket) return LRSDP_ERR_INVALID_ARG;
  Job* j = new (std::nothrow) Job();
  if (!j) return LRSDP_ERR_OUT_OF_BUDGET;
  j->kind = kClose;
  return submit_on_session(s, session, j, ticket);
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
  // sessions left open: release their handles (the workers have finished)
  for (auto& kv : s->sessions) {
    session_release(kv.second);
    delete kv.second;
  }
  for (lrsdp_ctx* c : s->ctxs) lrsdp_ctx_destroy(c);
  for (auto& kv : s->jobs) delete kv.second;
  delete s;
}

int lrsdp_solve_batch(lrsdp_ctx* ctx, int count, const lrsdp_instance* inst,
                      const lrsdp_opts* opts, int workers, int* status, lrsdp_info* info) {
  if (!ctx || count < 0 || (count > 0 && (!inst || !status)) || workers < 1)
    return LRSDP_ERR_INVALID_ARG;
  if (count == 0) return LRSDP_OK;
  lrsdp_opts o;
  lrsdp_opts_default(&o);
  if (opts) o = *opts;
  if (!lrsdp::opts_ok(o)) return LRSDP_ERR_INVALID_ARG;
  int prev_dev = -1;
  if (hipGetDevice(&prev_dev) != hipSuccess) prev_dev = -1;
  (void)hipSetDevice(ctx->device);
  // Contexts kept with ctx between calls (their memory pools then serve the next batch, and
  // freeing thousands of blocks is not paid per call): the workers that set the instances up,
  // and two that run the lock-step solves while the workers go on with the next wave.
  constexpr int kSolvers = 2;
  const int nw = std::min(workers, count);
  int rc = LRSDP_OK;
  while ((int)ctx->batch_workers.size() < nw + kSolvers && rc == LRSDP_OK) {
    lrsdp_ctx* c = nullptr;
    rc = lrsdp::ctx_create(ctx->device, nullptr, 0, false, &c);
    if (rc == LRSDP_OK) ctx->batch_workers.push_back(c);
  }
  std::vector<lrsdp_problem*> P(count, nullptr);
  std::vector<lrsdp_factor*> F(count, nullptr);
  std::vector<int> src(count, LRSDP_OK);
  std::vector<int64_t> key(count, -1);
  std::vector<lrsdp_info> inf(count);
  std::vector<int> asrc(count, LRSDP_OK);  // results of the solves outside lock-step
  if (rc == LRSDP_OK) {
    std::vector<lrsdp_ctx*> solver(ctx->batch_workers.begin(),
                                   ctx->batch_workers.begin() + kSolvers);
    std::vector<lrsdp_ctx*> wctx(ctx->batch_workers.begin() + kSolvers,
                                 ctx->batch_workers.begin() + kSolvers + nw);
    // 1. A0 and Algorithm 1 steps 1-2 on the worker threads, in index order; an instance is
    //    ready once its factor (and low-precision copy of W0) is complete on the device.  An
    //    instance outside every lock-step sequence is then solved alone by the worker that set
    //    it up, on that worker's context (no other thread uses it), into asrc and inf.
    std::mutex mu;
    std::condition_variable cv;
    std::vector<char> ready(count, 0);
    std::atomic<int> next{0};
    std::vector<std::thread> th;
    for (int w = 0; w < nw; ++w)
      th.emplace_back([&, w] {
        (void)hipSetDevice(ctx->device);
        for (;;) {
          const int i = next.fetch_add(1);
          if (i >= count) break;
          const lrsdp_instance& in = inst[i];
          int r = lrsdp_problem_create(wctx[w], in.n, in.m, in.m, in.con, in.row, in.col, in.val,
                                       &P[i]);
          if (r == LRSDP_OK) r = lrsdp_factor_create(P[i], in.W, in.k, &o, &F[i]);
          if (r == LRSDP_OK) {
            key[i] = lrsdp::lockstep_key(F[i], o);
            const lrsdp::SolveMode md = lrsdp::solve_mode(F[i], o);
            if (key[i] >= 0 && md.refine && md.prec != LRSDP_PREC_FP64)
              r = lrsdp::ensure_lowprec(F[i], md.prec, wctx[w]->stream);
          }
          if (hipStreamSynchronize(wctx[w]->stream) != hipSuccess && r == LRSDP_OK)
            r = LRSDP_ERR_DEVICE;
          src[i] = r;
          {
            std::lock_guard<std::mutex> lk(mu);
            ready[i] = 1;
          }
          cv.notify_all();
          if (r == LRSDP_OK && key[i] < 0)
            asrc[i] = lrsdp_solve(F[i], in.r, in.y, in.y_lo, &o, &inf[i]);
        }
      });
    // 2. step 3 in two waves: the first half's solves run (lock-step, one launch per step for
    //    all solves of a step sequence, the sequences side by side on the solver contexts)
    //    while the workers set up the second half
    auto solve_wave = [&](int lo, int hi) {
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] {
          for (int i = lo; i < hi; ++i)
            if (!ready[i]) return false;
          return true;
        });
      }
      std::unordered_map<int64_t, std::vector<int>> groups;
      for (int i = lo; i < hi; ++i) {
        if (src[i] == LRSDP_OK && key[i] >= 0) groups[key[i]].push_back(i);
      }
      std::vector<const std::vector<int>*> glist;
      for (auto& kv : groups) glist.push_back(&kv.second);
      std::atomic<int> gnext{0};
      auto run_groups = [&](lrsdp_ctx* sc) {
        (void)hipSetDevice(ctx->device);
        for (;;) {
          const int g = gnext.fetch_add(1);
          if (g >= (int)glist.size()) break;
          const std::vector<int>& ids = *glist[g];
          const int c = (int)ids.size();
          std::vector<lrsdp_factor*> gf(c);
          std::vector<const double*> gr(c);
          std::vector<double*> gy(c), gl(c);
          std::vector<int> gs(c);
          std::vector<lrsdp_info> gi(c);
          for (int j = 0; j < c; ++j) {
            gf[j] = F[ids[j]];
            gr[j] = inst[ids[j]].r;
            gy[j] = inst[ids[j]].y;
            gl[j] = inst[ids[j]].y_lo;
          }
          const int lrc = lrsdp::solve_lockstep(sc, c, gf.data(), gr.data(), gy.data(),
                                                gl.data(), o, gs.data(), gi.data());
          for (int j = 0; j < c; ++j) {
            src[ids[j]] = lrc < 0 ? lrc : gs[j];
            inf[ids[j]] = gi[j];
          }
        }
      };
      const int nt = std::min<int>((int)glist.size(), kSolvers);
      std::vector<std::thread> gt;
      for (int t = 0; t < nt; ++t) gt.emplace_back(run_groups, solver[t]);
      for (auto& t : gt) t.join();
    };
    const int half = count >= 32 ? count / 2 : count;
    solve_wave(0, half);
    if (half < count) solve_wave(half, count);
    for (auto& t : th) t.join();
    for (int i = 0; i < count; ++i)
      if (src[i] == LRSDP_OK && key[i] < 0) src[i] = asrc[i];
    for (lrsdp_ctx* c : solver) (void)hipStreamSynchronize(c->stream);
    (void)hipStreamSynchronize(ctx->stream);
    for (int i = 0; i < count; ++i) {
      status[i] = src[i];
      if (info) {
        info[i] = inf[i];
        info[i].status = src[i];
      }
    }
  } else {
    for (int i = 0; i < count; ++i) status[i] = rc;
  }
  // 3. release (factors and problems go back to the workers' memory pools)
  for (int i = 0; i < count; ++i) {
    if (F[i]) lrsdp_factor_destroy(F[i]);
    if (P[i]) lrsdp_problem_destroy(P[i]);
  }
  if (prev_dev >= 0) (void)hipSetDevice(prev_dev);
  return rc == LRSDP_OK ? LRSDP_OK : rc;
}

}  // extern "C"
