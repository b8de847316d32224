"""The augmented system of Section 4.1 (eq aug_ex) for the n-sized preconditioner equation, beside
the Sherman-Morrison-Woodbury route of eq wsmf; plain numpy.

Test infrastructure (see oracle/__init__.py).

Section 3.1 approximates W by the low-rank perturbation of the identity

    W~ = tau I + U U^T,  U in R^{n x k}                                   (eq tIUUt)

and applies W~^{-1} by eq wsmf, W~^{-1} = (I - U S^{-1} U^T) / tau with the k x k Schur
complement S = tau I + U^T U.  kappa(W~) = (tau + ||U||^2) / tau grows like 1/mu as tau does
not, and eq wsmf then loses digits.  Section 4.1 solves instead the symmetric indefinite system

    [ tau I        sqrt(tau) U ] [x]   [b]
    [ sqrt(tau) U^T   -tau I   ] [y] = [0]                                (eq aug_ex)

whose second row gives y = U^T x / sqrt(tau) and whose first then reads W~ x = b.  Eliminating x
first without pivoting (pivots tau) leaves the Schur complement -S for y and back-substitution
gives eq wsmf term by term.  The matrix has condition number sqrt(1 + ||U||^2 / tau): on each
singular pair (sigma, p, q) of U it acts on span{(p, 0), (0, q)} as [[tau, sqrt(tau) sigma],
[sqrt(tau) sigma, -tau]] with eigenvalues +-sqrt(tau (tau + sigma^2)), and as tau on the rest of
the x-space.  A stable method (the paper names LDL^T with threshold pivoting) therefore loses
about half as many digits as eq wsmf.  The oracle solves it with LAPACK's LU with partial
pivoting, a backward-stable method.

U is passed as k x n (row j is the j-th column of U), the library's layout.
"""

from __future__ import annotations

import numpy as np


def wtilde(Ut, tau):
    """W~ = tau I + U U^T (eq tIUUt); Ut is U^T (k x n)."""
    U = np.asarray(Ut, dtype=np.float64).T
    return tau * np.eye(U.shape[0]) + U @ U.T


def smw_solve(Ut, tau, b):
    """x = W~^{-1} b by eq wsmf: (b - U S^{-1} U^T b) / tau, S = tau I + U^T U."""
    U = np.asarray(Ut, dtype=np.float64).T
    k = U.shape[1]
    S = tau * np.eye(k) + U.T @ U
    return (b - U @ np.linalg.solve(S, U.T @ b)) / tau


def aug_matrix(Ut, tau):
    """The (n + k) x (n + k) matrix of eq aug_ex."""
    U = np.asarray(Ut, dtype=np.float64).T
    n, k = U.shape
    st = np.sqrt(tau)
    K = np.zeros((n + k, n + k))
    K[:n, :n] = tau * np.eye(n)
    K[:n, n:] = st * U
    K[n:, :n] = st * U.T
    K[n:, n:] = -tau * np.eye(k)
    return K


def aug_solve(Ut, tau, b):
    """x of eq aug_ex with right-hand side (b, 0), by LU with partial pivoting."""
    n = np.asarray(Ut).shape[1]
    K = aug_matrix(Ut, tau)
    rhs = np.concatenate([np.asarray(b, dtype=np.float64), np.zeros(K.shape[0] - n)])
    return np.linalg.solve(K, rhs)[:n]


def aug_solve_unpivoted(Ut, tau, b):
    """x of eq aug_ex by Gaussian elimination in the natural order without pivoting (the x block
    first), written out as plain elimination on the assembled matrix: the steps of eq wsmf."""
    n = np.asarray(Ut).shape[1]
    K = aug_matrix(Ut, tau)
    N = K.shape[0]
    r = np.concatenate([np.asarray(b, dtype=np.float64), np.zeros(N - n)])
    for j in range(N):
        for i in range(j + 1, N):
            if K[i, j] != 0.0:
                l = K[i, j] / K[j, j]
                K[i, j:] -= l * K[j, j:]
                r[i] -= l * r[j]
    z = np.zeros(N)
    for j in range(N - 1, -1, -1):
        z[j] = (r[j] - K[j, j + 1:] @ z[j + 1:]) / K[j, j]
    return z[:n]


def aug_cond(Ut, tau):
    """The 2-norm condition number of the matrix of eq aug_ex, sqrt(1 + ||U||^2 / tau)."""
    s = np.linalg.norm(np.asarray(Ut, dtype=np.float64), 2)
    return float(np.sqrt(1.0 + s * s / tau))


def wtilde_cond(Ut, tau):
    """kappa(W~) = (tau + ||U||^2) / tau (k < n, so tau is an eigenvalue)."""
    s = np.linalg.norm(np.asarray(Ut, dtype=np.float64), 2)
    return float((tau + s * s) / tau)


def exact_solve(Ut, tau, b, digits=50):
    """x = W~^{-1} b to `digits` digits (mpmath): eq wsmf in extended precision, where its
    cancellation costs nothing; O(n k^2) extended-precision operations."""
    import mpmath as mp
    mp.mp.dps = digits
    Ut = np.asarray(Ut, dtype=np.float64)
    k, n = Ut.shape
    t = mp.mpf(tau)
    U = [[mp.mpf(float(Ut[j, i])) for i in range(n)] for j in range(k)]
    bb = [mp.mpf(float(v)) for v in b]
    S = mp.matrix(k, k)
    for a in range(k):
        for c in range(k):
            S[a, c] = mp.fsum(U[a][i] * U[c][i] for i in range(n)) + (t if a == c else 0)
    g = mp.matrix([mp.fsum(U[a][i] * bb[i] for i in range(n)) for a in range(k)])
    h = mp.lu_solve(S, g)
    return np.array([float((bb[i] - mp.fsum(U[a][i] * h[a] for a in range(k))) / t)
                     for i in range(n)])
