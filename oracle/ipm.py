"""A tiny primal-dual interior-point method around the Hessian equation (test infrastructure).

Used to check, on a real interior-point path, that the Hessian equation the GPU
library solves is the one an interior-point method needs (Section 2), that the
iterates become ill-conditioned as the paper describes (Proposition "Weig"), and
that PCG with the paper's preconditioner needs a flat, small number of
iterations as mu -> 0 (Section 3, Lemma "Htilde").

Problem: the bipartite matrix-completion SDP (eq matcomp_sdp), n = p + q,
A_i = 1/2 [[0, E^T], [E, 0]] for each observed (i, j), C = I.

Method: infeasible path-following with the Nesterov-Todd scaling (Section 2.2,
third bullet): W is the positive definite matrix with X = W S W.  With
R_d = C - S - sum y_i A_i, the NT Newton system reduces to the Hessian equation
(eq hesseqn1)  H dy = b - sigma mu A(S^{-1}) + A(W R_d W),
then dS = R_d - sum dy_i A_i and dX = sigma mu S^{-1} - X - W dS W
(Todd, Toh and Tutuncu, SIAM J. Optim. 1998).  Steps go 0.9 of the way to the
boundary of the cone.  The centering parameter is either fixed (sigma = 0.1) or,
by default, set per step by Mehrotra's predictor rule with that value as its floor:
the affine direction (sigma = 0) is taken first, its full steps to the boundary (at
most 1) give the duality measure mu_aff it would reach, and the step uses
min(1, max(sigma, (mu_aff / mu)^3)), solving the Hessian equation again (no
second-order corrector).  With a fixed sigma the iterates drift from the central
path on sparsely sampled instances and the steps shrink to a few percent; the rule
raises the centering exactly there and otherwise keeps the fixed value.  The paper's own outer solver is SeDuMi's, which is not
reproduced: parity with it is unpinned.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import alg1
from .hessian import hessian_dense


def matcomp_instance(p, q, k, m, seed):
    rng = np.random.default_rng(seed)
    G1 = rng.standard_normal((p, k))
    G2 = rng.standard_normal((q, k))
    Mtrue = G1 @ G2.T
    t = np.sort(rng.choice(p * q, size=m, replace=False))
    ii, jj = t // q, t % q
    a = ii.astype(np.int64)
    b = (p + jj).astype(np.int64)
    val = np.full(m, 0.5)
    bvec = Mtrue[ii, jj]
    return dict(n=p + q, p=p, q=q, k=k, a=a, b=b, val=val, bvec=bvec, Mtrue=Mtrue)


def _sqrtm_psd(X):
    lam, V = np.linalg.eigh(X)
    return (V * np.sqrt(np.maximum(lam, 0.0))) @ V.T


def nt_scaling(X, S):
    """W = S^{-1/2} (S^{1/2} X S^{1/2})^{1/2} S^{-1/2}; satisfies W S W = X."""
    lam, V = np.linalg.eigh(S)
    Sh = (V * np.sqrt(lam)) @ V.T
    Sih = (V / np.sqrt(lam)) @ V.T
    W = Sih @ _sqrtm_psd(Sh @ X @ Sh) @ Sih
    return 0.5 * (W + W.T)


def _max_step(X, dX):
    L = np.linalg.cholesky(X)
    Li = np.linalg.inv(L)
    lam = np.linalg.eigvalsh(Li @ dX @ Li.T)
    lo = lam[0]
    return np.inf if lo >= 0 else -1.0 / lo


@dataclass
class IPMRecord:
    mu: float
    pinf: float
    dinf: float
    gap: float
    pcg_iters: int
    dy_rel_diff: float     # ||dy_pcg - dy_dense|| / ||dy_dense||
    w_gap: float           # lambda_k(W) / lambda_{k+1}(W)
    alpha_p: float = 0.0   # step lengths of X and of (y, S)
    alpha_d: float = 0.0
    sigma: float = 0.0     # the centering parameter the step used


@dataclass
class IPMResult:
    X: np.ndarray
    y: np.ndarray
    S: np.ndarray
    iters: int
    converged: bool
    records: list = field(default_factory=list)


def run(inst, tol=1e-9, max_iter=60, sigma=0.1, frac=0.9, pcg_k=None, pcg_eps=1e-10, C=None,
        predictor=True):
    """C: the cost matrix of eq SDP (n x n symmetric; None: the identity of eq matcomp_sdp).
    predictor: the centering by Mehrotra's rule from the affine direction, at least sigma;
    False: sigma every step."""
    n, a, b, val, bvec = inst["n"], inst["a"], inst["b"], inst["val"], inst["bvec"]
    m = len(a)
    Cst = alg1.Constraints(n, a, b, val)
    Cmat = np.eye(n) if C is None else np.asarray(C, dtype=np.float64)
    xi = max(10.0, np.sqrt(n), n * float(np.max((1 + np.abs(bvec)) / (1 + np.sqrt(Cst.g)))))
    eta = max(10.0, np.sqrt(n), 1.0 + np.linalg.norm(Cmat))
    X = xi * np.eye(n)
    S = eta * np.eye(n)
    y = np.zeros(m)
    k = pcg_k if pcg_k is not None else inst["k"]
    recs = []
    conv = False
    it = 0
    for it in range(max_iter):
        mu = float(np.sum(X * S)) / n
        Ay = Cst.mat(y).toarray()
        Rd = Cmat - S - Ay
        Rp = bvec - Cst.At(X)
        pinf = np.linalg.norm(Rp) / (1 + np.linalg.norm(bvec))
        dinf = np.linalg.norm(Rd) / (1 + np.linalg.norm(Cmat))
        gap = float(np.sum(X * S)) / (1 + abs(float(np.sum(Cmat * X))) + abs(bvec @ y))
        if max(pinf, dinf, gap) <= tol:
            conv = True
            break
        W = nt_scaling(X, S)
        Si = np.linalg.inv(S)
        H = hessian_dense(W, a, b, val)
        sg = sigma
        if predictor:
            # the affine direction: the Newton system with sigma = 0
            dy_a = np.linalg.solve(H, bvec + Cst.At(W @ Rd @ W))
            dS_a = Rd - Cst.mat(dy_a).toarray()
            dX_a = -X - W @ dS_a @ W
            dX_a = 0.5 * (dX_a + dX_a.T)
            ap_a = min(1.0, _max_step(X, dX_a))
            ad_a = min(1.0, _max_step(S, dS_a))
            mu_a = float(np.sum((X + ap_a * dX_a) * (S + ad_a * dS_a))) / n
            sg = min(1.0, max(sigma, (mu_a / mu) ** 3))
        rhs = bvec - sg * mu * Cst.At(Si) + Cst.At(W @ Rd @ W)
        dy = np.linalg.solve(H, rhs)
        # the same Newton system solved by Algorithm 1 (PCG, true rank k)
        lamW = np.linalg.eigvalsh(W)
        F = alg1.factor(Cst, W, k)
        res = alg1.solve(F, rhs, eps=pcg_eps, max_iter=500,
                         Hmul=lambda v: H @ v)
        diff = float(np.linalg.norm(res.y - dy) / max(np.linalg.norm(dy), 1e-300))
        dS = Rd - Cst.mat(dy).toarray()
        dX = sg * mu * Si - X - W @ dS @ W
        dX = 0.5 * (dX + dX.T)
        ap = min(1.0, frac * _max_step(X, dX))
        ad = min(1.0, frac * _max_step(S, dS))
        recs.append(IPMRecord(mu=mu, pinf=pinf, dinf=dinf, gap=gap, pcg_iters=res.iters,
                              dy_rel_diff=diff, w_gap=float(lamW[n - k] / lamW[n - k - 1]),
                              alpha_p=ap, alpha_d=ad, sigma=sg))
        X = X + ap * dX
        X = 0.5 * (X + X.T)
        y = y + ad * dy
        S = S + ad * dS
        S = 0.5 * (S + S.T)
    return IPMResult(X=X, y=y, S=S, iters=it, converged=conv, records=recs)
