"""Algorithm 1 of the paper (formation, factorization, PCG) in plain numpy FP64.

Test infrastructure (see oracle/__init__.py).

Steps, in the paper's order and notation (Section 3.3, Algorithm 1):
  1a  W = V Lambda V^T, tau = lambda_min(W)                      eq "Wsplit1"
  1b  U = V_l (Lambda_l - tau I)^{1/2}, W0 = W - U U^T,          eq "Wsplit2"
      Z Z^T = 2 W0 + U U^T (lower Cholesky)                      eq "hessExp2"
  2   bold S = tau^2 I + bold U^T (A^T A)^{-1} bold U,           eq "SMW2"
      bold U = A^T (U kron Z);  bold S = L L^T
  3   PCG on H y = r with preconditioner H~ = tau^2 A^T A + bold U bold U^T
      (eq "AtIUUtAt"), applied by Sherman-Morrison-Woodbury (eq "SMW2") with
      bold S^{-1} = L^{-T} L^{-1}.

Readings of the paper taken here (each is listed with its reason in the design notes):
  * bold S uses tau^2 (eq "SMW2"); the tau printed in Algorithm 1 step 2 is read as tau^2.
  * vec is column-major, so (U kron Z) vec X = vec(Z X U^T) for X in R^{n x k}
    and the nk index of (p, j) is p + n j (eq "Umv").
  * For k >= 2 bold S has k(k-1)/2 eigenvalues equal to tau^2 whose eigenvectors
    vec(Z^{-1} U K), K skew, are annihilated by bold U.  They are deflated by adding
    shift * Q_N Q_N^T (Q_N an orthonormal basis of them, shift = max diag(bold S)),
    which leaves bold U bold S^{-1} bold U^T, hence H~^{-1}, unchanged.
  * PCG is the preconditioned CG of Barrett et al., Templates (1994), from y0 = 0,
    stopping on the recursive residual ||r_i|| <= eps ||r||.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import dd as ddm
from .hessian import half_scale, normal_diag


# --------------------------------------------------------------------------- formation

@dataclass
class Split:
    tau: float
    lam: np.ndarray        # all eigenvalues of W, ascending
    V_l: np.ndarray        # n x k eigenvectors of the k largest eigenvalues
    U: np.ndarray          # n x k
    W0: np.ndarray         # n x n
    Z: np.ndarray          # n x n lower triangular, Z Z^T = 2 W0 + U U^T


def formation(W, k, tau_rule="min"):
    """Algorithm 1 step 1 (eqs Wsplit1, Wsplit2, hessExp2).

    tau_rule "min": tau = lambda_min(W), as Algorithm 1 step 1a prints it.
    tau_rule "mean": tau = the mean of the n - k smallest eigenvalues, i.e.
    (tr W - sum of the k largest) / (n - k); Section 3.1 allows any tau with
    lambda_min(Lambda_s) <= tau < lambda_max(Lambda_s), and the mean lies in that range."""
    n = W.shape[0]
    lam, V = np.linalg.eigh(W)
    if tau_rule == "min":
        tau = float(lam[0])
    elif tau_rule == "mean":
        tau = float((np.trace(W) - lam[n - k:].sum()) / (n - k))
    else:
        raise ValueError(tau_rule)
    V_l = V[:, n - k:]
    lam_l = lam[n - k:]
    U = V_l * np.sqrt(lam_l - tau)[None, :]
    W0 = W - U @ U.T
    Z = np.linalg.cholesky(2.0 * W0 + U @ U.T)
    return Split(tau=tau, lam=lam, V_l=V_l, U=U, W0=W0, Z=Z)


# --------------------------------------------------------------------------- products with A

class Constraints:
    """The data matrices A_i as triplets, with the products of Assumption 2."""

    def __init__(self, n, a, b, val):
        self.n = int(n)
        self.a = np.asarray(a, dtype=np.int64)
        self.b = np.asarray(b, dtype=np.int64)
        self.val = np.asarray(val, dtype=np.float64)
        self.m = len(self.a)
        self.s = half_scale(self.a, self.b, self.val)
        self.g = normal_diag(self.a, self.b, self.val)
        off = self.a != self.b
        self._rows = np.concatenate([self.a, self.b[off]])
        self._cols = np.concatenate([self.b, self.a[off]])
        self._src = np.concatenate([np.arange(self.m), np.nonzero(off)[0]])
        # 0/1 pattern Omega-bar of the sampled entries (symmetric)
        self.pattern = sp.csr_matrix((np.ones(len(self._rows)), (self._rows, self._cols)),
                                     shape=(self.n, self.n))

    def mat(self, v):
        """mat(A v) = sum_i v_i A_i as a sparse matrix."""
        w = (self.val * v)[self._src]
        return sp.csr_matrix((w, (self._rows, self._cols)), shape=(self.n, self.n))

    def At(self, X):
        """[A_i . X]_i for dense X."""
        a, b = self.a, self.b
        return np.where(a == b, self.val * X[a, b], self.val * (X[a, b] + X[b, a]))

    def sampled_dot(self, P, Q):
        """[A_i . (P Q^T)]_i for n x r factors P, Q, without forming P Q^T."""
        a, b = self.a, self.b
        xab = np.einsum("ij,ij->i", P[a], Q[b])
        xba = np.einsum("ij,ij->i", P[b], Q[a])
        return np.where(a == b, self.val * xab, self.val * (xab + xba))


def hessian_apply_mf(C: Constraints, W, v, chunk=8192):
    """Matrix-free H v (eq hesseqn2): M = mat(A v); T = M W; (H v)_i = A_i . (W T)."""
    T = C.mat(v) @ W                  # dense n x n
    Tt = np.ascontiguousarray(T.T)
    out = np.empty(C.m)
    for s0 in range(0, C.m, chunk):
        s1 = min(C.m, s0 + chunk)
        a, b = C.a[s0:s1], C.b[s0:s1]
        xab = np.einsum("ij,ij->i", W[a], Tt[b])        # (W M W)_ab
        out[s0:s1] = np.where(a == b, C.val[s0:s1] * xab, 2.0 * C.val[s0:s1] * xab)
    return out


# --------------------------------------------------------------------------- bold U, bold S

def bold_U_explicit(C: Constraints, Z, U):
    """bold U = A^T (U kron Z), m x nk; entry (i, p + n j) = u_j^T A_i z_p (eq hessExp2)."""
    n, k = U.shape
    a, b, s = C.a, C.b, C.s
    blocks = []
    for j in range(k):
        blocks.append(s[:, None] * (U[a, j][:, None] * Z[b, :] + U[b, j][:, None] * Z[a, :]))
    return np.concatenate(blocks, axis=1)


def bold_U_apply(C: Constraints, Z, U, x):
    """bold U vec X = [tr A_i (Z X) U^T]_i  (eq Umv, first line), X = reshape(x, n, k) column-major."""
    n, k = U.shape
    X = x.reshape(k, n).T
    return C.sampled_dot(Z @ X, U)


def bold_Ut_apply(C: Constraints, Z, U, y):
    """bold U^T y = vec(Z^T (sum_i y_i A_i) U)  (eq Umv, second line)."""
    P = C.mat(y) @ U
    return (Z.T @ P).T.reshape(-1)


def schur_explicit(bU, g, tau):
    """bold S = tau^2 I + bold U^T (A^T A)^{-1} bold U from an explicit bold U."""
    S = bU.T @ (bU / g[:, None])
    S[np.diag_indices_from(S)] += tau * tau
    return S


def schur_blocks(C: Constraints, Z, U, tau):
    """bold S from its block structure: block (j, l) equals
    tau^2 delta_jl I + 1/2 Z^T [diag(Obar (u_j o u_l)) + D_{u_l} Obar D_{u_j}] Z,
    obtained by writing (A^T A)^{-1} through the orthogonal projector onto span{A_i},
    which samples the symmetric part of a matrix on the pattern Obar."""
    n, k = U.shape
    S = np.empty((n * k, n * k))
    Ob = C.pattern
    for j in range(k):
        for l in range(j, k):
            d = Ob @ (U[:, j] * U[:, l])
            B = sp.diags(U[:, l]) @ Ob @ sp.diags(U[:, j]) + sp.diags(d)
            blk = 0.5 * (Z.T @ (B @ Z))
            if j == l:
                blk[np.diag_indices(n)] += tau * tau
            S[n * j:n * (j + 1), n * l:n * (l + 1)] = blk
            if l != j:
                S[n * l:n * (l + 1), n * j:n * (j + 1)] = blk.T
    return S


def null_basis(Z, U):
    """Columns vec(Z^{-1} U K_ij), K_ij = e_i e_j^T - e_j e_i^T, i < j: a basis of the
    part of null(bold U) that makes bold S singular up to tau^2."""
    n, k = U.shape
    Y = sla.solve_triangular(Z, U, lower=True)
    cols = []
    for i in range(k):
        for j in range(i + 1, k):
            v = np.zeros((n, k))
            v[:, j] = Y[:, i]
            v[:, i] = -Y[:, j]
            cols.append(v.T.reshape(-1))
    if not cols:
        return np.zeros((n * k, 0))
    return np.stack(cols, axis=1)


# --------------------------------------------------------------------------- the factor

@dataclass
class Factor:
    C: Constraints
    W: np.ndarray
    k: int
    split: Split
    S: np.ndarray          # bold S as factored (deflated when k >= 2 and deflate=True)
    L: np.ndarray          # lower Cholesky factor of S
    QN: np.ndarray         # orthonormal deflation basis (nk x k(k-1)/2), may be empty
    shift: float
    bU: np.ndarray = None  # explicit bold U when requested

    @property
    def tau(self):
        return self.split.tau


def factor(C: Constraints, W, k, deflate=True, explicit=None, tau_rule="min"):
    """Algorithm 1 steps 1 and 2."""
    spl = formation(W, k, tau_rule=tau_rule)
    if explicit is None:
        explicit = C.m * C.n * k <= 4_000_000
    bU = None
    if explicit:
        bU = bold_U_explicit(C, spl.Z, spl.U)
        S = schur_explicit(bU, C.g, spl.tau)
    else:
        S = schur_blocks(C, spl.Z, spl.U, spl.tau)
    QN = np.zeros((S.shape[0], 0))
    shift = 0.0
    if deflate and k >= 2:
        QN, _ = np.linalg.qr(null_basis(spl.Z, spl.U))
        shift = float(np.max(np.diag(S)))
        S = S + shift * (QN @ QN.T)
    L = np.linalg.cholesky(S)
    return Factor(C=C, W=W, k=k, split=spl, S=S, L=L, QN=QN, shift=shift, bU=bU)


def _Umul(F: Factor, x):
    if F.bU is not None:
        return F.bU @ x
    return bold_U_apply(F.C, F.split.Z, F.split.U, x)


def _Utmul(F: Factor, y):
    if F.bU is not None:
        return F.bU.T @ y
    return bold_Ut_apply(F.C, F.split.Z, F.split.U, y)


def schur_solve(F: Factor, w):
    """t = bold S^{-1} w = L^{-T} L^{-1} w (Algorithm 1 step 3b)."""
    t = sla.solve_triangular(F.L, w, lower=True)
    return sla.solve_triangular(F.L, t, lower=True, trans="T")


def precond_apply(F: Factor, v):
    """z = H~^{-1} v = (tau^2 A^T A)^{-1} (v - bold U bold S^{-1} bold U^T (A^T A)^{-1} v)."""
    g = F.C.g
    w = _Utmul(F, v / g)
    t = schur_solve(F, w)
    return (v - _Umul(F, t)) / (F.tau ** 2 * g)


def precond_dense(F: Factor):
    """H~ = tau^2 A^T A + bold U bold U^T as a dense matrix (small sizes only)."""
    bU = F.bU if F.bU is not None else bold_U_explicit(F.C, F.split.Z, F.split.U)
    Ht = bU @ bU.T
    Ht[np.diag_indices_from(Ht)] += F.tau ** 2 * F.C.g
    return Ht


# --------------------------------------------------------------------------- PCG

@dataclass
class PCGResult:
    y: np.ndarray
    iters: int
    relres: float          # recursive residual at exit
    converged: bool
    history: list


def pcg(Hmul, Pinv, r, eps=1e-8, max_iter=200):
    """Preconditioned CG (Barrett et al. Templates, Fig. 2.5) from y0 = 0.
    Returns after the first iteration whose recursive residual meets eps."""
    y = np.zeros_like(r)
    res = r.copy()
    nr0 = float(np.linalg.norm(r))
    hist = [1.0]
    if nr0 == 0.0:
        return PCGResult(y, 0, 0.0, True, hist)
    z = Pinv(res)
    p = z.copy()
    rho = float(res @ z)
    it = 0
    conv = False
    while it < max_iter:
        it += 1
        q = Hmul(p)
        pq = float(p @ q)
        alpha = rho / pq
        y += alpha * p
        res -= alpha * q
        rel = float(np.linalg.norm(res)) / nr0
        hist.append(rel)
        if rel <= eps:
            conv = True
            break
        z = Pinv(res)
        rho_new = float(res @ z)
        beta = rho_new / rho
        p = z + beta * p
        rho = rho_new
    return PCGResult(y, it, hist[-1], conv, hist)


def solve(F: Factor, r, eps=1e-8, max_iter=200, Hmul=None):
    """Algorithm 1 step 3 in FP64."""
    if Hmul is None:
        Hmul = lambda v: hessian_apply_mf(F.C, F.W, v)  # noqa: E731
    return pcg(Hmul, lambda v: precond_apply(F, v), r, eps=eps, max_iter=max_iter)
