"""Exact solves of tiny Hessian equations with mpmath (test infrastructure).

H is formed from its definition, eq hesseqn2: H_ij = A_i . (W A_j W) = tr(A_i W A_j W),
with every A_i built as a dense n x n matrix from its triplet and every product and trace
taken entry by entry in 50-digit arithmetic, starting from the exact FP64 bits of W.  No
closed form of the entries is used, so this reference is independent of the sampled
formula the other oracle modules and the GPU path use.  H y = r is then solved by LU in
the same precision.  This is the brute-force reference for the double-double refinement
and for the FP64 floor at small mu.  Cost: O(m n^3 + m^2 n^2), so tiny sizes only.
"""

from __future__ import annotations

import mpmath
import numpy as np


def _dense_constraint(n, a, b, v):
    """A_i as a dense mpmath matrix: (A_i)_ab = (A_i)_ba = v."""
    A = mpmath.zeros(n, n)
    A[a, b] = v
    A[b, a] = v
    return A


def exact_hessian(W, a, b, val, dps=50):
    """H_ij = tr(A_i W A_j W) with dense A_i (eq hesseqn2), in `dps` digits."""
    mpmath.mp.dps = dps
    n = W.shape[0]
    m = len(a)
    Wm = mpmath.matrix(n, n)
    for i in range(n):
        for j in range(n):
            Wm[i, j] = mpmath.mpf(float(W[i, j]))
    As = [_dense_constraint(n, int(a[i]), int(b[i]), mpmath.mpf(float(val[i]))) for i in range(m)]
    H = mpmath.matrix(m, m)
    for j in range(m):
        X = Wm * As[j] * Wm                       # W A_j W, dense
        for i in range(m):
            Ai = As[i]
            t = mpmath.mpf(0)
            for p in range(n):                    # tr(A_i X) = sum_pq (A_i)_pq X_qp
                for q in range(n):
                    if Ai[p, q] != 0:
                        t += Ai[p, q] * X[q, p]
            H[i, j] = t
    return H


def exact_solve(W, a, b, val, r, dps=50):
    H = exact_hessian(W, a, b, val, dps=dps)
    rv = mpmath.matrix([mpmath.mpf(float(x)) for x in r])
    y = mpmath.lu_solve(H, rv)
    return H, y


def to_dd(y):
    """Split an mpmath vector into a double-double pair (hi, lo)."""
    hi = np.array([float(v) for v in y])
    lo = np.array([float(v - mpmath.mpf(h)) for v, h in zip(y, hi)])
    return hi, lo


def relative_residual(H, y_hi, y_lo, r):
    """||r - H (y_hi + y_lo)|| / ||r|| in mpmath."""
    yv = mpmath.matrix([mpmath.mpf(float(h)) + mpmath.mpf(float(l)) for h, l in zip(y_hi, y_lo)])
    rv = mpmath.matrix([mpmath.mpf(float(x)) for x in r])
    res = rv - H * yv
    return float(mpmath.norm(res) / mpmath.norm(rv))
