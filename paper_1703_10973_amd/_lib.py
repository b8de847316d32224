"""ctypes binding of liblrsdp.so: the C ABI of include/lrsdp.h, same names, marshalling only.

Every array argument is a torch tensor on the GPU (its device pointer is passed); scalars
and the options / info structs are host values.  Nothing here computes: each call goes
straight to the HIP library, and importing fails loudly when the library is not built.
"""

from __future__ import annotations

import ctypes as C
import os
import re

import torch  # noqa: F401  (loads torch's HIP runtime first so the library binds to it)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblrsdp.so")

LRSDP_OK = 0
LRSDP_NOT_CONVERGED = 1
LRSDP_ERR_INVALID_ARG = -1
LRSDP_ERR_DUPLICATE_PAIR = -2
LRSDP_ERR_UNSUPPORTED = -3
LRSDP_ERR_NOT_PD_W = -4
LRSDP_ERR_CHOL_Z = -5
LRSDP_ERR_CHOL_S = -6
LRSDP_ERR_OUT_OF_BUDGET = -7
LRSDP_ERR_STAGNATED = -8
LRSDP_ERR_INDEFINITE_PRECOND = -9
LRSDP_ERR_DEVICE = -10
LRSDP_ERR_EIG = -11
LRSDP_ERR_SCRATCH = -12
LRSDP_ERR_IPM = -13
LRSDP_PENDING = 2

LRSDP_PREC_FP64, LRSDP_PREC_FP32, LRSDP_PREC_BF16, LRSDP_PREC_AUTO = 0, 1, 2, 3
LRSDP_DD_OFF, LRSDP_DD_ON, LRSDP_DD_AUTO = 0, 1, 2
LRSDP_TAU_MIN, LRSDP_TAU_MEAN = 0, 1
LRSDP_PRECOND_SMW, LRSDP_PRECOND_AUG = 0, 1


class lrsdp_opts(C.Structure):
    _fields_ = [("eps", C.c_double), ("max_iter", C.c_int), ("precision", C.c_int),
                ("dd_mode", C.c_int), ("deflate", C.c_int), ("max_outer", C.c_int),
                ("inner_eps", C.c_double), ("dd_auto_ratio", C.c_double),
                ("dd_precond", C.c_int), ("tau_rule", C.c_int), ("precond", C.c_int)]


class lrsdp_info(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("outer_iters", C.c_int),
                ("dd_used", C.c_int), ("relres", C.c_double), ("tau", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("eig_sweeps", C.c_int),
                ("phase_ms", C.c_double * 4), ("lockstep", C.c_int)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["phase_ms"] = list(d["phase_ms"])
        return d


class lrsdp_ipm_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("sigma", C.c_double),
                ("predictor", C.c_int), ("warm_start", C.c_int), ("stall_iters", C.c_int),
                ("frac", C.c_double), ("k", C.c_int32), ("rank_eta", C.c_double),
                ("pcg_eps", C.c_double), ("pcg_eps_mu", C.c_double),
                ("max_ns_iter", C.c_int), ("householder_eig", C.c_int), ("ns_tol", C.c_double),
                ("solve", lrsdp_opts)]


class lrsdp_ipm_info(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("records", C.c_int),
                ("pcg_iters_total", C.c_int), ("mu", C.c_double), ("pinf", C.c_double),
                ("dinf", C.c_double), ("gap", C.c_double), ("primal_obj", C.c_double),
                ("dual_obj", C.c_double), ("ms", C.c_double), ("best_iter", C.c_int),
                ("stalled", C.c_int), ("last_error", C.c_int), ("fail_stage", C.c_int),
                ("ns_resid", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lrsdp_ipm_record(C.Structure):
    _fields_ = [("mu", C.c_double), ("pinf", C.c_double), ("dinf", C.c_double),
                ("gap", C.c_double), ("alpha_p", C.c_double), ("alpha_d", C.c_double),
                ("pcg_iters", C.c_int), ("outer_iters", C.c_int), ("ns_iters", C.c_int),
                ("k", C.c_int), ("solve_status", C.c_int), ("eps", C.c_double),
                ("relres", C.c_double), ("factor_ms", C.c_double), ("solve_ms", C.c_double),
                ("ms", C.c_double), ("scaling_ms", C.c_double), ("rank_ms", C.c_double),
                ("steps_ms", C.c_double), ("sigma", C.c_double), ("pred_pcg_iters", C.c_int),
                ("pred_ms", C.c_double), ("backtracks", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lrsdp_instance(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("k", C.c_int32), ("con", C.c_void_p),
                ("row", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p),
                ("W", C.c_void_p), ("r", C.c_void_p), ("y", C.c_void_p), ("y_lo", C.c_void_p)]


class LrsdpError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


_lib = None

_P = C.c_void_p
_SIGS = {
    "lrsdp_opts_default": (None, [C.POINTER(lrsdp_opts)]),
    "lrsdp_status_string": (C.c_char_p, [C.c_int]),
    "lrsdp_ctx_create": (C.c_int, [C.c_int, _P, C.c_size_t, C.POINTER(_P)]),
    "lrsdp_ctx_destroy": (None, [_P]),
    "lrsdp_ctx_memory": (C.c_int, [_P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "lrsdp_ctx_profile": (C.c_int, [_P, C.c_int]),
    "lrsdp_ctx_profile_sample": (C.c_int, [_P, C.c_int]),
    "lrsdp_ctx_profile_read": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                         C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "lrsdp_problem_create": (C.c_int, [_P, C.c_int64, C.c_int64, C.c_int64, _P, _P, _P, _P,
                                       C.POINTER(_P)]),
    "lrsdp_problem_destroy": (None, [_P]),
    "lrsdp_problem_info": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64)]),
    "lrsdp_hessian_apply": (C.c_int, [_P, _P, _P, _P]),
    "lrsdp_hessian_apply_noalloc": (C.c_int, [_P, _P, _P, _P]),
    "lrsdp_aug_wtilde_solve": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_double, _P, _P, _P]),
    "lrsdp_factor_create": (C.c_int, [_P, _P, C.c_int32, C.POINTER(lrsdp_opts), C.POINTER(_P)]),
    "lrsdp_factor_destroy": (None, [_P]),
    "lrsdp_factor_info": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int32)]),
    "lrsdp_factor_export": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.POINTER(C.c_double), _P, _P, _P,
                                      _P]),
    "lrsdp_hessian_apply_split": (C.c_int, [_P, _P, _P, C.c_int]),
    "lrsdp_precond_apply": (C.c_int, [_P, _P, _P, C.c_int]),
    "lrsdp_residual_dd": (C.c_int, [_P, _P, _P, _P, _P, C.POINTER(C.c_double)]),
    "lrsdp_solve": (C.c_int, [_P, _P, _P, _P, C.POINTER(lrsdp_opts), C.POINTER(lrsdp_info)]),
    "lrsdp_solve_batch": (C.c_int, [_P, C.c_int, C.POINTER(lrsdp_instance), C.POINTER(lrsdp_opts),
                                    C.c_int, C.POINTER(C.c_int), C.POINTER(lrsdp_info)]),
    "lrsdp_server_create": (C.c_int, [_P, C.c_int, C.c_size_t, C.POINTER(_P)]),
    "lrsdp_server_submit": (C.c_int, [_P, C.POINTER(lrsdp_instance), C.POINTER(lrsdp_opts),
                                      C.POINTER(C.c_uint64)]),
    "lrsdp_server_poll": (C.c_int, [_P, C.c_uint64, C.c_int, C.POINTER(C.c_int),
                                    C.POINTER(lrsdp_info)]),
    "lrsdp_server_session_open": (C.c_int, [_P, C.c_int64, C.c_int64, _P, _P, _P, _P,
                                            C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "lrsdp_server_submit_factor": (C.c_int, [_P, C.c_uint64, _P, C.c_int32,
                                             C.POINTER(lrsdp_opts), C.POINTER(C.c_uint64)]),
    "lrsdp_server_submit_solve": (C.c_int, [_P, C.c_uint64, _P, _P, _P, C.POINTER(lrsdp_opts),
                                            C.POINTER(C.c_uint64)]),
    "lrsdp_server_session_close": (C.c_int, [_P, C.c_uint64, C.POINTER(C.c_uint64)]),
    "lrsdp_server_stats": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                     C.POINTER(C.c_int), C.POINTER(C.c_size_t)]),
    "lrsdp_server_destroy": (None, [_P]),
    "lrsdp_instance_bytes": (C.c_size_t, [C.c_int64, C.c_int64, C.c_int32]),
    "lrsdp_ipm_opts_default": (None, [C.POINTER(lrsdp_ipm_opts)]),
    "lrsdp_ipm_solve": (C.c_int, [_P, _P, _P, C.POINTER(lrsdp_ipm_opts), _P, _P, _P,
                                  C.POINTER(lrsdp_ipm_info), C.POINTER(lrsdp_ipm_record),
                                  C.c_int]),
}


def header_symbols():
    """Function names declared in include/lrsdp.h (parsed from the header text)."""
    hdr = os.path.join(os.path.dirname(HERE), "include", "lrsdp.h")
    with open(hdr) as f:
        text = f.read()
    return sorted(set(re.findall(r"LRSDP_API\s+[\w\s\*]*?\b(lrsdp_\w+)\s*\(", text)))


def _check_single_hip_runtime():
    """Refuse to run with two HIP runtimes mapped (torch's and another one)."""
    try:
        with open("/proc/self/maps") as f:
            paths = {ln.split()[-1] for ln in f if "libamdhip64" in ln}
    except OSError:
        return
    real = {os.path.realpath(p) for p in paths}
    if len(real) > 1:
        raise RuntimeError(f"two HIP runtimes are loaded: {sorted(real)}")


def lib():
    """The loaded library (loaded on first use)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1703_10973_amd.build`")
        h = C.CDLL(LIB_PATH, mode=C.RTLD_LOCAL)
        for name, (res, args) in _SIGS.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _check_single_hip_runtime()
        _lib = h
    return _lib


def status_string(s):
    return lib().lrsdp_status_string(int(s)).decode()


def _ptr(t, dtype=None, numel=None, name="array"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    return C.c_void_p(t.data_ptr())


def _ok(st, where, allow_warn=False):
    if st < 0 or (st > 0 and not allow_warn):
        raise LrsdpError(st, where)
    return st


# ----------------------------------------------------------------- C ABI, same names

def lrsdp_opts_default():
    o = lrsdp_opts()
    lib().lrsdp_opts_default(C.byref(o))
    return o


def lrsdp_ctx_create(device=0, stream=None, hbm_budget_bytes=0):
    out = C.c_void_p()
    sp = C.c_void_p(stream) if stream else None
    _ok(lib().lrsdp_ctx_create(int(device), sp, C.c_size_t(hbm_budget_bytes), C.byref(out)),
        "lrsdp_ctx_create")
    return out


def lrsdp_ctx_destroy(ctx):
    lib().lrsdp_ctx_destroy(ctx)


def lrsdp_ctx_memory(ctx):
    a, b = C.c_size_t(), C.c_size_t()
    _ok(lib().lrsdp_ctx_memory(ctx, C.byref(a), C.byref(b)), "lrsdp_ctx_memory")
    return a.value, b.value


LRSDP_K_NAMES = ["hv", "gemm", "tri", "gemv", "bz", "resdd", "leaf", "tile", "gemm_inv"]


def lrsdp_ctx_profile(ctx, enable):
    _ok(lib().lrsdp_ctx_profile(ctx, int(enable)), "lrsdp_ctx_profile")


def lrsdp_ctx_profile_sample(ctx, every):
    _ok(lib().lrsdp_ctx_profile_sample(ctx, int(every)), "lrsdp_ctx_profile_sample")


def lrsdp_ctx_profile_read(ctx, kernel_class):
    n, ms, by, fl = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
    _ok(lib().lrsdp_ctx_profile_read(ctx, int(kernel_class), C.byref(n), C.byref(ms), C.byref(by),
                                     C.byref(fl)), "lrsdp_ctx_profile_read")
    return dict(launches=n.value, ms=ms.value, bytes=by.value, flops=fl.value)


def lrsdp_problem_create(ctx, n, m, con, row, col, val):
    nnz = con.numel()
    out = C.c_void_p()
    st = lib().lrsdp_problem_create(
        ctx, int(n), int(m), int(nnz), _ptr(con, torch.int32, nnz, "con"),
        _ptr(row, torch.int32, nnz, "row"), _ptr(col, torch.int32, nnz, "col"),
        _ptr(val, torch.float64, nnz, "val"), C.byref(out))
    _ok(st, "lrsdp_problem_create")
    return out


def lrsdp_problem_destroy(p):
    lib().lrsdp_problem_destroy(p)


def lrsdp_problem_info(p):
    n, m, z = C.c_int64(), C.c_int64(), C.c_int64()
    _ok(lib().lrsdp_problem_info(p, C.byref(n), C.byref(m), C.byref(z)), "lrsdp_problem_info")
    return n.value, m.value, z.value


def lrsdp_hessian_apply(p, W, v, Hv):
    n, m, _ = lrsdp_problem_info(p)
    _ok(lib().lrsdp_hessian_apply(p, _ptr(W, torch.float64, n * n, "W"),
                                  _ptr(v, torch.float64, m, "v"),
                                  _ptr(Hv, torch.float64, m, "Hv")),
        "lrsdp_hessian_apply")


def lrsdp_hessian_apply_noalloc(p, W, v, Hv):
    """lrsdp_hessian_apply with its scratch in the library's fixed per-device array."""
    n, m, _ = lrsdp_problem_info(p)
    _ok(lib().lrsdp_hessian_apply_noalloc(p, _ptr(W, torch.float64, n * n, "W"),
                                          _ptr(v, torch.float64, m, "v"),
                                          _ptr(Hv, torch.float64, m, "Hv")),
        "lrsdp_hessian_apply_noalloc")


def lrsdp_aug_wtilde_solve(ctx, Ut, tau, b, x):
    """x = (tau I + U U^T)^{-1} b through the augmented system of Section 4.1 (eq aug_ex);
    Ut is U^T (k x n)."""
    k, n = int(Ut.shape[0]), int(Ut.shape[1])
    _ok(lib().lrsdp_aug_wtilde_solve(ctx, n, k, float(tau), _ptr(Ut, torch.float64, n * k, "Ut"),
                                     _ptr(b, torch.float64, n, "b"),
                                     _ptr(x, torch.float64, n, "x")),
        "lrsdp_aug_wtilde_solve")


def lrsdp_factor_create(p, W, k, opts=None):
    n, _, _ = lrsdp_problem_info(p)
    out = C.c_void_p()
    st = lib().lrsdp_factor_create(p, _ptr(W, torch.float64, n * n, "W"), int(k),
                                   C.byref(opts) if opts is not None else None, C.byref(out))
    _ok(st, "lrsdp_factor_create")
    return out


def lrsdp_factor_info(f):
    """(n, m, k) of a factor."""
    n, m, k = C.c_int64(), C.c_int64(), C.c_int32()
    _ok(lib().lrsdp_factor_info(f, C.byref(n), C.byref(m), C.byref(k)), "lrsdp_factor_info")
    return n.value, m.value, k.value


def lrsdp_factor_destroy(f):
    lib().lrsdp_factor_destroy(f)


def lrsdp_factor_export(f, k, U=None, W0=None, Z=None, Sinv=None):
    n, _, fk = lrsdp_factor_info(f)
    if int(k) != fk:
        raise ValueError(f"k = {k} does not match the factor's k = {fk}")
    tau, shift, ms = C.c_double(), C.c_double(), C.c_double()
    lam = (C.c_double * (k + 1))()
    st = lib().lrsdp_factor_export(f, C.byref(tau), C.byref(shift), lam, C.byref(ms),
                                   _ptr(U, torch.float64, n * k, "U"),
                                   _ptr(W0, torch.float64, n * n, "W0"),
                                   _ptr(Z, torch.float64, n * n, "Z"),
                                   _ptr(Sinv, torch.float64, (n * k) ** 2, "Sinv"))
    _ok(st, "lrsdp_factor_export")
    return dict(tau=tau.value, shift=shift.value, lam=list(lam), setup_ms=ms.value)


def lrsdp_hessian_apply_split(f, v, Hv, precision):
    m = lrsdp_factor_info(f)[1]
    _ok(lib().lrsdp_hessian_apply_split(f, _ptr(v, torch.float64, m, "v"),
                                        _ptr(Hv, torch.float64, m, "Hv"),
                                        int(precision)), "lrsdp_hessian_apply_split")


def lrsdp_precond_apply(f, v, z, dd=0):
    m = lrsdp_factor_info(f)[1]
    _ok(lib().lrsdp_precond_apply(f, _ptr(v, torch.float64, m, "v"),
                                  _ptr(z, torch.float64, m, "z"), int(dd)),
        "lrsdp_precond_apply")


def lrsdp_residual_dd(f, r, y, y_lo=None, res=None):
    m = lrsdp_factor_info(f)[1]
    rel = C.c_double()
    _ok(lib().lrsdp_residual_dd(f, _ptr(r, torch.float64, m, "r"),
                                _ptr(y, torch.float64, m, "y"),
                                _ptr(y_lo, torch.float64, m, "y_lo"),
                                _ptr(res, torch.float64, m, "res"), C.byref(rel)),
        "lrsdp_residual_dd")
    return rel.value


def lrsdp_solve(f, r, y, y_lo=None, opts=None):
    m = lrsdp_factor_info(f)[1]
    info = lrsdp_info()
    st = lib().lrsdp_solve(f, _ptr(r, torch.float64, m, "r"),
                           _ptr(y, torch.float64, m, "y"),
                           _ptr(y_lo, torch.float64, m, "y_lo"),
                           C.byref(opts) if opts is not None else None, C.byref(info))
    if st < 0 and st != LRSDP_ERR_STAGNATED:
        raise LrsdpError(st, "lrsdp_solve")
    return st, info.as_dict()


# ----------------------------------------------------------------- many instances

def make_instance(n, k, con, row, col, val, W, r, y, y_lo=None):
    """An lrsdp_instance over torch device tensors (the caller keeps them alive)."""
    m = r.numel()
    return lrsdp_instance(int(n), int(m), int(k), _ptr(con, torch.int32, m, "con"),
                          _ptr(row, torch.int32, m, "row"), _ptr(col, torch.int32, m, "col"),
                          _ptr(val, torch.float64, m, "val"),
                          _ptr(W, torch.float64, int(n) * int(n), "W"),
                          _ptr(r, torch.float64, m, "r"), _ptr(y, torch.float64, m, "y"),
                          _ptr(y_lo, torch.float64, m, "y_lo"))


def lrsdp_solve_batch(ctx, instances, opts=None, workers=8):
    """Solve every instance; returns (statuses, infos)."""
    cnt = len(instances)
    arr = (lrsdp_instance * max(cnt, 1))(*instances)
    st = (C.c_int * max(cnt, 1))()
    inf = (lrsdp_info * max(cnt, 1))()
    _ok(lib().lrsdp_solve_batch(ctx, cnt, arr, C.byref(opts) if opts is not None else None,
                                int(workers), st, inf), "lrsdp_solve_batch")
    return [st[i] for i in range(cnt)], [inf[i].as_dict() for i in range(cnt)]


def lrsdp_server_create(ctx, workers=8, hbm_budget_bytes=0):
    out = _P()
    _ok(lib().lrsdp_server_create(ctx, int(workers), int(hbm_budget_bytes), C.byref(out)),
        "lrsdp_server_create")
    return out


def lrsdp_server_submit(srv, inst, opts=None):
    t = C.c_uint64()
    _ok(lib().lrsdp_server_submit(srv, C.byref(inst), C.byref(opts) if opts is not None else None,
                                  C.byref(t)), "lrsdp_server_submit")
    return t.value


def lrsdp_server_poll(srv, ticket, wait=False):
    """None while pending, else (status, info)."""
    st = C.c_int()
    inf = lrsdp_info()
    rc = lib().lrsdp_server_poll(srv, C.c_uint64(ticket), int(bool(wait)), C.byref(st), C.byref(inf))
    if rc == LRSDP_PENDING:
        return None
    _ok(rc, "lrsdp_server_poll")
    return st.value, inf.as_dict()


def lrsdp_server_session_open(srv, n, m, con, row, col, val):
    """Returns (session, ticket)."""
    s, t = C.c_uint64(), C.c_uint64()
    _ok(lib().lrsdp_server_session_open(srv, int(n), int(m), _ptr(con, torch.int32, m, "con"),
                                        _ptr(row, torch.int32, m, "row"),
                                        _ptr(col, torch.int32, m, "col"),
                                        _ptr(val, torch.float64, m, "val"), C.byref(s), C.byref(t)),
        "lrsdp_server_session_open")
    return s.value, t.value


def lrsdp_server_submit_factor(srv, session, n, W, k, opts=None):
    t = C.c_uint64()
    _ok(lib().lrsdp_server_submit_factor(srv, C.c_uint64(session),
                                         _ptr(W, torch.float64, int(n) * int(n), "W"), int(k),
                                         C.byref(opts) if opts is not None else None, C.byref(t)),
        "lrsdp_server_submit_factor")
    return t.value


def lrsdp_server_submit_solve(srv, session, m, r, y, y_lo=None, opts=None):
    t = C.c_uint64()
    _ok(lib().lrsdp_server_submit_solve(srv, C.c_uint64(session), _ptr(r, torch.float64, m, "r"),
                                        _ptr(y, torch.float64, m, "y"),
                                        _ptr(y_lo, torch.float64, m, "y_lo"),
                                        C.byref(opts) if opts is not None else None, C.byref(t)),
        "lrsdp_server_submit_solve")
    return t.value


def lrsdp_server_session_close(srv, session):
    t = C.c_uint64()
    _ok(lib().lrsdp_server_session_close(srv, C.c_uint64(session), C.byref(t)),
        "lrsdp_server_session_close")
    return t.value


def lrsdp_server_stats(srv):
    q, r, d, b = C.c_int(), C.c_int(), C.c_int(), C.c_size_t()
    _ok(lib().lrsdp_server_stats(srv, C.byref(q), C.byref(r), C.byref(d), C.byref(b)),
        "lrsdp_server_stats")
    return dict(queued=q.value, running=r.value, done=d.value, bytes_in_flight=b.value)


def lrsdp_server_destroy(srv):
    if srv:
        lib().lrsdp_server_destroy(srv)


def lrsdp_instance_bytes(n, m, k):
    return int(lib().lrsdp_instance_bytes(int(n), int(m), int(k)))


# ----------------------------------------------------------------- the outer method

def lrsdp_ipm_opts_default():
    o = lrsdp_ipm_opts()
    lib().lrsdp_ipm_opts_default(C.byref(o))
    return o


def lrsdp_ipm_solve(p, b, C_, opts, X, y, S, max_recs=200):
    n, m, _ = lrsdp_problem_info(p)
    info = lrsdp_ipm_info()
    recs = (lrsdp_ipm_record * max_recs)()
    st = lib().lrsdp_ipm_solve(p, _ptr(b, torch.float64, m, "b"),
                               _ptr(C_, torch.float64, n * n, "C"),
                               C.byref(opts) if opts is not None else None,
                               _ptr(X, torch.float64, n * n, "X"),
                               _ptr(y, torch.float64, m, "y"),
                               _ptr(S, torch.float64, n * n, "S"),
                               C.byref(info), recs, int(max_recs))
    out = [recs[i].as_dict() for i in range(min(info.records, max_recs))]
    if st < 0:
        e = LrsdpError(st, "lrsdp_ipm_solve")
        e.info, e.records = info.as_dict(), out  # the steps taken before the failure
        raise e
    return st, info.as_dict(), out
