"""Exact solves of tiny Hessian equations with mpmath (test infrastructure).

H is formed entry by entry from the trace definition H_ij = tr(A_i W A_j W)
(eq hesseqn2) in 50-digit arithmetic, starting from the exact FP64 bits of W,
and H y = r is solved by LU in the same precision.  This is the brute-force
reference for the double-double refinement and for the FP64 floor at small mu.
"""

from __future__ import annotations

import mpmath
import numpy as np


def exact_solve(W, a, b, val, r, dps=50):
    mpmath.mp.dps = dps
    n = W.shape[0]
    m = len(a)
    Wm = mpmath.matrix(n, n)
    for i in range(n):
        for j in range(n):
            Wm[i, j] = mpmath.mpf(float(W[i, j]))
    s = [mpmath.mpf(float(v)) / (2 if ai == bi else 1) for v, ai, bi in zip(val, a, b)]
    H = mpmath.matrix(m, m)
    for i in range(m):
        ai, bi = int(a[i]), int(b[i])
        for j in range(m):
            c, d = int(a[j]), int(b[j])
            H[i, j] = 2 * s[i] * s[j] * (Wm[ai, c] * Wm[bi, d] + Wm[ai, d] * Wm[bi, c])
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
    m = len(r)
    yv = mpmath.matrix([mpmath.mpf(float(h)) + mpmath.mpf(float(l)) for h, l in zip(y_hi, y_lo)])
    rv = mpmath.matrix([mpmath.mpf(float(x)) for x in r])
    res = rv - H * yv
    return float(mpmath.norm(res) / mpmath.norm(rv))
