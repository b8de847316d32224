"""MI355X (gfx950) solver for the interior-point Hessian equation of low-rank SDPs.

Hot path of Zhang and Lavaei's modified interior-point method (arXiv 1703.10973,
Algorithm 1): PCG on H y = r with H = A^T (W kron W) A applied matrix-free and the
low-rank-correcting preconditioner built from a partial eigendecomposition of W.
All computation runs in the HIP library liblrsdp.so (include/lrsdp.h); this package is
its thin Python binding.  The C functions are re-exported under their own names, and
Context / Problem / Factor wrap the handles.
"""

from __future__ import annotations

import atexit
import weakref

import torch

from ._lib import (  # noqa: F401
    LRSDP_DD_AUTO, LRSDP_DD_OFF, LRSDP_DD_ON, LRSDP_PREC_BF16, LRSDP_PREC_FP32, LRSDP_TAU_MEAN,
    LRSDP_PREC_AUTO,
    LRSDP_TAU_MIN, LRSDP_PRECOND_SMW, LRSDP_PRECOND_AUG,
    LRSDP_PREC_FP64, LrsdpError, header_symbols, lib, lrsdp_ctx_create, lrsdp_ctx_destroy,
    lrsdp_ctx_memory, lrsdp_ctx_profile, lrsdp_ctx_profile_read, lrsdp_ctx_profile_sample,
    LRSDP_K_NAMES,
    lrsdp_factor_create, lrsdp_factor_destroy, lrsdp_factor_export, lrsdp_factor_info,
    lrsdp_hessian_apply, lrsdp_hessian_apply_noalloc, lrsdp_hessian_apply_split, lrsdp_info,
    lrsdp_aug_wtilde_solve,
    lrsdp_opts,
    lrsdp_opts_default, lrsdp_precond_apply, lrsdp_problem_create, lrsdp_problem_destroy,
    lrsdp_problem_info, lrsdp_residual_dd, lrsdp_solve, status_string, lrsdp_instance,
    make_instance, lrsdp_solve_batch, lrsdp_server_create, lrsdp_server_submit,
    lrsdp_server_poll, lrsdp_server_stats, lrsdp_server_destroy, lrsdp_instance_bytes,
    lrsdp_server_session_open, lrsdp_server_submit_factor, lrsdp_server_submit_solve,
    lrsdp_server_session_close,
    LRSDP_PENDING, LRSDP_ERR_IPM, lrsdp_ipm_opts, lrsdp_ipm_opts_default, lrsdp_ipm_solve)


def opts(**kw):
    """lrsdp_opts with the library defaults, overridden by keyword."""
    o = lrsdp_opts_default()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def ipm_opts(**kw):
    """lrsdp_ipm_opts with the library defaults, overridden by keyword (solve=... takes an
    lrsdp_opts)."""
    o = lrsdp_ipm_opts_default()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


# Live contexts, closed (children first) by an exit hook while the interpreter and the HIP
# runtime are still whole, rather than by finalizers late in interpreter shutdown.
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    for c in list(_LIVE):
        try:
            c.close()
        except Exception:
            pass


class Context:
    """A device, stream and HBM budget.  Closing it first closes every problem, factor and
    server created under it that is still alive.  The library defers releasing a parent
    handle destroyed before its children until the last child is destroyed, so the order in
    which garbage collection finalizes these objects does not matter."""

    def __init__(self, device=0, stream=None, hbm_budget_bytes=0):
        """stream: a hipStream_t handle to run on.  None: torch's current stream on `device`
        when that is a stream of its own; when it is the default stream, the library's own
        blocking stream, which is ordered after work on the default stream.  Either way the
        library reads tensors that torch wrote before the call in order."""
        self.device = device
        self.handle = None
        self._children = weakref.WeakSet()
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream or None
        self.handle = lrsdp_ctx_create(device, stream, hbm_budget_bytes)
        _LIVE.add(self)

    def memory(self):
        return lrsdp_ctx_memory(self.handle)

    def profile(self, enable=True, every=1):
        """Time kernel classes (bit mask) with HIP events, one launch in `every`."""
        lrsdp_ctx_profile_sample(self.handle, every)
        lrsdp_ctx_profile(self.handle, enable)

    def aug_wtilde_solve(self, Ut, tau, b, out=None):
        """x = (tau I + U U^T)^{-1} b through the augmented system of Section 4.1 (eq aug_ex),
        by LU with partial pivoting on the device; Ut is U^T (k x n)."""
        x = torch.empty_like(b) if out is None else out
        _caller_work_done(self)
        lrsdp_aug_wtilde_solve(self.handle, Ut, tau, b, x)
        return x

    def profile_read(self):
        return {name: lrsdp_ctx_profile_read(self.handle, i) for i, name in enumerate(LRSDP_K_NAMES)}

    def close(self):
        if self.handle:
            for ch in list(self._children):
                ch.close()
            lrsdp_ctx_destroy(self.handle)
            self.handle = None
        _LIVE.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """Constraint data A_1..A_m as device triplets (step A0)."""

    def __init__(self, ctx: Context, n, m, con, row, col, val):
        self.ctx = ctx
        self.n, self.m = int(n), int(m)
        self.handle = None
        self._children = weakref.WeakSet()
        self.handle = lrsdp_problem_create(ctx.handle, n, m, con, row, col, val)
        ctx._children.add(self)

    def hessian_apply(self, W, v, out=None):
        out = torch.empty_like(v) if out is None else out
        lrsdp_hessian_apply(self.handle, W, v, out)
        return out

    def info(self):
        return lrsdp_problem_info(self.handle)

    def ipm_solve(self, b, C=None, options=None, max_recs=200, start=None, **kw):
        """The interior-point method on this problem (lrsdp_ipm_solve): right-hand side b
        (device, m), cost C (device n x n, None: the identity).  options: an lrsdp_ipm_opts,
        or keywords of it (k=..., tol=...).  start: (X, y, S) to start from (copied; sets
        warm_start).  Returns (X, y, S, status, info, records)."""
        o = options if options is not None else ipm_opts(**kw)
        if start is not None:
            X, y, S = (t.detach().to(device=b.device, dtype=torch.float64).contiguous().clone()
                       for t in start)
            if X.shape != (self.n, self.n) or S.shape != (self.n, self.n) or y.shape != (self.m,):
                raise ValueError("start: X and S must be n x n and y of length m")
            o.warm_start = 1
        else:
            X = torch.empty(self.n, self.n, dtype=torch.float64, device=b.device)
            S = torch.empty_like(X)
            y = torch.empty(self.m, dtype=torch.float64, device=b.device)
        st, info, recs = lrsdp_ipm_solve(self.handle, b, C, o, X, y, S, max_recs)
        return X, y, S, st, info, recs

    def close(self):
        if self.handle:
            for ch in list(self._children):
                ch.close()
            lrsdp_problem_destroy(self.handle)
            self.handle = None
        self.ctx._children.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Factor:
    """W and the preconditioner of Algorithm 1 steps 1-2."""

    def __init__(self, problem: Problem, W, k, options=None):
        self.problem = problem
        self.k = int(k)
        self.handle = None
        self.handle = lrsdp_factor_create(problem.handle, W, k, options)
        problem._children.add(self)

    def export(self, U=False, W0=False, Z=False, Sinv=False):
        n, k = self.problem.n, self.k
        dev = torch.device("cuda", self.problem.ctx.device)
        mk = lambda flag, shape: torch.empty(shape, dtype=torch.float64, device=dev) if flag else None  # noqa: E731
        tU, tW0, tZ, tS = mk(U, (k, n)), mk(W0, (n, n)), mk(Z, (n, n)), mk(Sinv, (n * k, n * k))
        out = lrsdp_factor_export(self.handle, k, tU, tW0, tZ, tS)
        out.update(U=tU, W0=tW0, Z=tZ, Sinv=tS)
        return out

    def hessian_apply_split(self, v, precision=LRSDP_PREC_FP64, out=None):
        out = torch.empty_like(v) if out is None else out
        lrsdp_hessian_apply_split(self.handle, v, out, precision)
        return out

    def precond_apply(self, v, dd=False, out=None, mode=None):
        """z = H~^{-1} v.  mode 0: FP64; 1: double-double w and t; 2: FP64 with one
        refinement step of t (default: 1 if dd else 0)."""
        out = torch.empty_like(v) if out is None else out
        lrsdp_precond_apply(self.handle, v, out, (1 if dd else 0) if mode is None else int(mode))
        return out

    def residual_dd(self, r, y, y_lo=None):
        return lrsdp_residual_dd(self.handle, r, y, y_lo)

    def solve(self, r, options=None, want_lo=True):
        y = torch.empty_like(r)
        ylo = torch.empty_like(r) if want_lo else None
        st, info = lrsdp_solve(self.handle, r, y, ylo, options)
        return y, ylo, st, info

    def close(self):
        if self.handle:
            lrsdp_factor_destroy(self.handle)
            self.handle = None
        self.problem._children.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _caller_work_done(ctx: "Context"):
    """The server's and the batch's workers run on streams of their own, which are not ordered
    after the caller's: finish what the caller's current stream still has to write into the
    request's tensors (inputs, and outputs such as a freshly zeroed y) before handing them over."""
    torch.cuda.current_stream(ctx.device).synchronize()


class Server:
    """Request server over the C ABI: submit instances, poll their results.  Each request
    keeps references to its tensors until its result has been polled.  Submissions first wait
    for the caller's current stream, so tensors it is still writing are complete."""

    def __init__(self, ctx: "Context", workers=8, hbm_budget_bytes=0):
        self.ctx = ctx
        self.handle = None
        self.handle = lrsdp_server_create(ctx.handle, workers, hbm_budget_bytes)
        self._keep = {}
        self._sessions = {}
        ctx._children.add(self)

    def submit(self, n, k, con, row, col, val, W, r, y, y_lo=None, options=None):
        _caller_work_done(self.ctx)
        inst = make_instance(n, k, con, row, col, val, W, r, y, y_lo)
        t = lrsdp_server_submit(self.handle, inst, options)
        self._keep[t] = (con, row, col, val, W, r, y, y_lo)
        return t

    def open_session(self, n, m, con, row, col, val):
        """A resident session for one SDP's data; returns (session, ticket)."""
        _caller_work_done(self.ctx)
        sid, t = lrsdp_server_session_open(self.handle, n, m, con, row, col, val)
        self._keep[t] = (con, row, col, val)
        self._sessions[sid] = (int(n), int(m))
        return sid, t

    def submit_factor(self, session, W, k, options=None):
        n, _ = self._sessions[session]
        _caller_work_done(self.ctx)
        t = lrsdp_server_submit_factor(self.handle, session, n, W, k, options)
        self._keep[t] = (W,)
        return t

    def submit_solve(self, session, r, y, y_lo=None, options=None):
        _, m = self._sessions[session]
        _caller_work_done(self.ctx)
        t = lrsdp_server_submit_solve(self.handle, session, m, r, y, y_lo, options)
        self._keep[t] = (r, y, y_lo)
        return t

    def close_session(self, session):
        return lrsdp_server_session_close(self.handle, session)

    def poll(self, ticket, wait=False):
        out = lrsdp_server_poll(self.handle, ticket, wait)
        if out is not None:
            self._keep.pop(ticket, None)
        return out

    def stats(self):
        return lrsdp_server_stats(self.handle)

    def close(self):
        if self.handle:
            lrsdp_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()
        self.ctx._children.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(ctx: "Context", instances, options=None, workers=8):
    """instances: list of dicts with n, k, con, row, col, val, W, r, y and optionally y_lo
    (torch device tensors).  Returns (statuses, infos)."""
    _caller_work_done(ctx)
    insts = [make_instance(d["n"], d["k"], d["con"], d["row"], d["col"], d["val"], d["W"],
                           d["r"], d["y"], d.get("y_lo")) for d in instances]
    return lrsdp_solve_batch(ctx.handle, insts, options, workers)
