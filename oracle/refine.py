"""Extended-precision pieces of Algorithm 1 for small duality-gap parameters mu.

Test infrastructure (see oracle/__init__.py).

Why they are needed (readings of the paper, not printed in it):
  * kappa(H) = O(1/mu^2) (Section 2.1).  For a generic right-hand side the solution
    has ||y|| ~ ||r|| / mu^2, so an FP64 y, or H y evaluated in FP64, cannot certify a
    relative residual of 1e-8 once mu is below about 1e-5.  The answer is then a
    double-double pair and the outer residual is evaluated in double-double (dd.py).
  * Iterative refinement: y <- y + PCG(r - H y), with the inner H v taken in the
    split form of eq "hessExp1": H v = A^T vec(W0 M W0) + A^T vec(U P^T W0 + W0 P U^T
    + U K U^T), P = M U, K = U^T P, M = mat(A v).  W0 = W - U U^T is evaluated in
    double-double and rounded once, and P and K are carried in double-double, so that
    the mu^2-sized part of H v keeps its relative accuracy.
  * Section 4 notes that the Sherman-Morrison-Woodbury form is numerically unstable as
    mu -> 0.  At mu ~ 1e-8 the FP64 H~^{-1} is indefinite; carrying w = bold U^T G^{-1} v
    (its sparse product M U) and t = bold S^{-1} w (FP64 Cholesky plus residual
    refinement with bold S applied matrix-free in double-double) restores it.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import dd as ddm
from .alg1 import Constraints, Factor, pcg


# --------------------------------------------------------------------------- dd sparse helpers

def _sym_entries(C: Constraints, vh, vl):
    """Entries of mat(A v) on the symmetric pattern (row, col, hi, lo), row-sorted."""
    mh, ml = ddm.two_prod(C.val, vh)
    ml = ml + C.val * vl
    mh, ml = ddm.quick_two_sum(mh, ml)
    return ddm._csr_symmetric(C.n, C.a, C.b, mh, ml)


def dd_spmm(n, rows, cols, h, l, B):
    """(M B) in double-double for a sparse M given by row-sorted entries and FP64 B."""
    r = B.shape[1]
    Oh = np.zeros((n, r))
    Ol = np.zeros((n, r))
    counts = np.bincount(rows, minlength=n)
    start = np.concatenate([[0], np.cumsum(counts)[:-1]])
    for slot in range(int(counts.max(initial=0))):
        live = np.nonzero(counts > slot)[0]
        e = start[live] + slot
        q = cols[e]
        ph, pl = ddm.two_prod(h[e][:, None], B[q, :])
        pl = pl + l[e][:, None] * B[q, :]
        Oh[live], Ol[live] = ddm.dd_add(Oh[live], Ol[live], ph, pl)
    return Oh, Ol


def dd_sampled(C: Constraints, Ph, Pl, Q):
    """[A_i . (P Q^T)]_i in double-double, P a dd n x r matrix, Q FP64 n x r."""
    a, b = C.a, C.b
    xh, xl = ddm.dd_dot_rows(Q[b], Ph[a], Pl[a])      # (P Q^T)_ab
    yh, yl = ddm.dd_dot_rows(Q[a], Ph[b], Pl[b])      # (P Q^T)_ba
    sh, sl = ddm.dd_add(xh, xl, yh, yl)
    diag = a == b
    sh = np.where(diag, xh, sh)
    sl = np.where(diag, xl, sl)
    return ddm.dd_mul_d(sh, sl, C.val)


def dd_W0(W, U):
    """W0 = W - U U^T evaluated in double-double and rounded once to FP64."""
    n, k = U.shape
    h = W.copy()
    l = np.zeros_like(W)
    for j in range(k):
        ph, pl = ddm.two_prod(U[:, j:j + 1], U[:, j][None, :])
        h, l = ddm.dd_add(h, l, -ph, -pl)
    return h + l


# --------------------------------------------------------------------------- split H v

@dataclass
class SplitOperator:
    C: Constraints
    W0: np.ndarray         # FP64 (rounded once from double-double)
    U: np.ndarray

    def __call__(self, v):
        C, U, W0 = self.C, self.U, self.W0
        T = C.mat(v) @ W0
        h0 = C.At(W0 @ T)
        rows, cols, h, l = _sym_entries(C, v, np.zeros_like(v))
        Ph, Pl = dd_spmm(C.n, rows, cols, h, l, U)
        Q = W0 @ Ph
        Kh, Kl = ddm.dd_matmul(U.T, Ph, Pl)
        K = Kh + Kl
        low = C.sampled_dot(U, Q) + C.sampled_dot(Q, U) + C.sampled_dot(U @ K, U)
        return h0 + low


# --------------------------------------------------------------------------- dd preconditioner

def _dd_Umul(F: Factor, th, tl):
    """bold U t in double-double: [A_i . ((Z T) U^T)]_i, T = reshape(t, n, k)."""
    n, k = F.split.U.shape
    Th = th.reshape(k, n).T
    Tl = tl.reshape(k, n).T
    Yh, Yl = ddm.dd_matmul(F.split.Z, np.ascontiguousarray(Th), np.ascontiguousarray(Tl))
    return dd_sampled(F.C, Yh, Yl, F.split.U)


def _dd_Utmul(F: Factor, vh, vl):
    """bold U^T v in double-double: vec(Z^T mat(A v) U)."""
    C = F.C
    rows, cols, h, l = _sym_entries(C, vh, vl)
    Ph, Pl = dd_spmm(C.n, rows, cols, h, l, F.split.U)
    Oh, Ol = ddm.dd_matmul(F.split.Z.T, Ph, Pl)
    return Oh.T.reshape(-1), Ol.T.reshape(-1)


def dd_schur_apply(F: Factor, th, tl):
    """bold S t (deflated as factored) in double-double, matrix-free."""
    g = F.C.g
    yh, yl = _dd_Umul(F, th, tl)
    yh, yl = ddm.dd_mul_d(yh, yl, 1.0 / g)
    sh, sl = _dd_Utmul(F, yh, yl)
    tau2 = F.tau * F.tau
    ah, al = ddm.dd_mul_d(th, tl, tau2)
    sh, sl = ddm.dd_add(sh, sl, ah, al)
    if F.QN.shape[1]:
        ch, cl = ddm.dd_matmul(F.QN.T, th[:, None], tl[:, None])
        qh, ql = ddm.dd_matmul(F.QN, ch, cl)
        qh, ql = ddm.dd_mul_d(qh[:, 0], ql[:, 0], F.shift)
        sh, sl = ddm.dd_add(sh, sl, qh, ql)
    return sh, sl


def dd_schur_solve(F: Factor, wh, wl, nref=2):
    """t = bold S^{-1} w: FP64 Cholesky solve plus residual refinement in double-double."""
    def chol(x):
        y = sla.solve_triangular(F.L, x, lower=True)
        return sla.solve_triangular(F.L, y, lower=True, trans="T")
    th = chol(wh + wl)
    tl = np.zeros_like(th)
    for _ in range(nref):
        sh, sl = dd_schur_apply(F, th, tl)
        rh, rl = ddm.dd_add(wh, wl, -sh, -sl)
        d = chol(rh + rl)
        th, tl = ddm.dd_add(th, tl, d, np.zeros_like(d))
    return th, tl


def dd_precond_apply(F: Factor, v, nref=2):
    """H~^{-1} v with w and t carried in double-double."""
    g = F.C.g
    uh, ul = ddm.dd_mul_d(v, np.zeros_like(v), 1.0 / g)
    wh, wl = _dd_Utmul(F, uh, ul)
    th, tl = dd_schur_solve(F, wh, wl, nref=nref)
    xh, xl = _dd_Umul(F, th, tl)
    zh, zl = ddm.dd_add(v, np.zeros_like(v), -xh, -xl)
    return (zh + zl) / (F.tau * F.tau * g)


# --------------------------------------------------------------------------- refinement

@dataclass
class RefineResult:
    yh: np.ndarray
    yl: np.ndarray
    outer: int
    inner: list
    relres: float           # true relative residual (double-double evaluation)
    history: list


def refine(F: Factor, r, eps=1e-8, inner_eps=1e-3, max_outer=12, max_inner=200,
           dd_precond=None, precond=None):
    """Outer iterative refinement y <- y + PCG(H_split, r - H y) with y a double-double
    pair and r - H y evaluated in double-double from the plain definition of H.  F: an
    Algorithm 1 factor (its U is the split's; its preconditioner H~ is used unless `precond`
    gives another, e.g. the augmented preconditioner of oracle.aug)."""
    C = F.C
    U = F.U if precond is not None else F.split.U
    W0 = dd_W0(F.W, U)
    Hs = SplitOperator(C, W0, U)
    if precond is not None:
        Pinv = precond
    else:
        if dd_precond is None:
            dd_precond = F.tau < 1e-7 * float(F.split.lam[-1])
        Pinv = (lambda v: dd_precond_apply(F, v)) if dd_precond else None
    if Pinv is None:
        from .alg1 import precond_apply
        Pinv = lambda v: precond_apply(F, v)  # noqa: E731
    yh = np.zeros(C.m)
    yl = np.zeros(C.m)
    inner = []
    hist = []
    rel = 1.0
    for outer in range(max_outer + 1):
        rel, res = ddm.true_relative_residual(F.W, C.a, C.b, C.val, r, yh, yl)
        hist.append(rel)
        if rel <= eps or outer == max_outer:
            break
        out = pcg(Hs, Pinv, res, eps=inner_eps, max_iter=max_inner)
        inner.append(out.iters)
        yh, yl = ddm.dd_add(yh, yl, out.y, np.zeros_like(out.y))
    return RefineResult(yh=yh, yl=yl, outer=len(inner), inner=inner, relres=rel, history=hist)
