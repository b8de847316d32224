"""Double-double (FP64 pair) arithmetic and the true residual of the Hessian equation.

Test infrastructure (see oracle/__init__.py).

A value is the unevaluated sum hi + lo of two FP64 numbers.  The error-free
transformations are Knuth's TwoSum and Dekker's TwoProduct with Veltkamp
splitting (numpy has no fused multiply-add), as in Dekker, "A floating-point
technique for extending the available precision" (1971).

The true relative residual ||r - H y|| / ||r|| of an answer y (FP64 or a
double-double pair) is evaluated from the plain definition of H
(equation "hesseqn2": M = mat(A y), then W M W sampled at the constraints)
with every product and sum carried in double-double.  With W given as exact
FP64 bits, M = mat(A y) is exact, and the result is accurate to about
u^2 * kappa, far below the 1e-8 threshold at every mu used here.
"""

from __future__ import annotations

import numpy as np

_SPLIT = 134217729.0  # 2^27 + 1


def two_sum(a, b):
    s = a + b
    bb = s - a
    e = (a - (s - bb)) + (b - bb)
    return s, e


def quick_two_sum(a, b):
    s = a + b
    e = b - (s - a)
    return s, e


def split(a):
    t = _SPLIT * a
    hi = t - (t - a)
    lo = a - hi
    return hi, lo


def two_prod(a, b):
    p = a * b
    ah, al = split(a)
    bh, bl = split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def dd_add(ah, al, bh, bl):
    s, e = two_sum(ah, bh)
    t, f = two_sum(al, bl)
    e = e + t
    s, e = quick_two_sum(s, e)
    e = e + f
    return quick_two_sum(s, e)


def dd_add_d(ah, al, b):
    s, e = two_sum(ah, b)
    e = e + al
    return quick_two_sum(s, e)


def dd_mul_d(ah, al, b):
    p, e = two_prod(ah, b)
    e = e + al * b
    return quick_two_sum(p, e)


def dd_mul(ah, al, bh, bl):
    p, e = two_prod(ah, bh)
    e = e + (ah * bl + al * bh)
    return quick_two_sum(p, e)


def dd_neg(h, l):
    return -h, -l


def dd_sum_axis1(h, l):
    """Pairwise double-double sum of the rows of (rows x cols) arrays."""
    h = np.array(h, dtype=np.float64, copy=True)
    l = np.array(l, dtype=np.float64, copy=True)
    while h.shape[1] > 1:
        c = h.shape[1]
        if c % 2:
            h = np.concatenate([h, np.zeros((h.shape[0], 1))], axis=1)
            l = np.concatenate([l, np.zeros((l.shape[0], 1))], axis=1)
            c += 1
        h, l = dd_add(h[:, 0::2], l[:, 0::2], h[:, 1::2], l[:, 1::2])
    return h[:, 0], l[:, 0]


def dd_dot_rows(X, Yh, Yl=None):
    """Row-wise dot products sum_p X[i,p] * Y[i,p] in double-double, X in FP64."""
    ph, pl = two_prod(X, Yh)
    if Yl is not None:
        pl = pl + X * Yl
    return dd_sum_axis1(ph, pl)


def dd_matmul(A, Bh, Bl=None):
    """C = A @ B with A in FP64 and B a double-double matrix, accumulated in double-double."""
    n_in = A.shape[1]
    Ch = np.zeros((A.shape[0], Bh.shape[1]))
    Cl = np.zeros_like(Ch)
    for p in range(n_in):
        ph, pl = two_prod(A[:, p:p + 1], Bh[p:p + 1, :])
        if Bl is not None:
            pl = pl + A[:, p:p + 1] * Bl[p:p + 1, :]
        Ch, Cl = dd_add(Ch, Cl, ph, pl)
    return Ch, Cl


def _csr_symmetric(n, a, b, vh, vl):
    """Symmetric pattern of mat(A y): entries (a,b) and (b,a) with dd values."""
    off = a != b
    rows = np.concatenate([a, b[off]])
    cols = np.concatenate([b, a[off]])
    h = np.concatenate([vh, vh[off]])
    l = np.concatenate([vl, vl[off]])
    order = np.lexsort((cols, rows))
    return rows[order], cols[order], h[order], l[order]


def dd_hessian_apply(W, a, b, val, yh, yl=None, chunk=4096):
    """H (y_hi + y_lo) in double-double from equation hesseqn2; returns (hi, lo)."""
    n = W.shape[0]
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    if yl is None:
        yl = np.zeros_like(yh)
    # M = mat(A y): the entry val_i * y_i, exact as a double-double
    mh, ml = two_prod(val, yh)
    ml = ml + val * yl
    mh, ml = quick_two_sum(mh, ml)
    rows, cols, h, l = _csr_symmetric(n, a, b, mh, ml)
    # T = M W, row p of T = sum_q M_pq W[q, :]; loop over the k-th nonzero of every row
    Th = np.zeros((n, n))
    Tl = np.zeros((n, n))
    counts = np.bincount(rows, minlength=n)
    start = np.concatenate([[0], np.cumsum(counts)[:-1]])
    for slot in range(int(counts.max(initial=0))):
        live = np.nonzero(counts > slot)[0]
        e = start[live] + slot
        q = cols[e]
        ph, pl = two_prod(h[e][:, None], W[q, :])
        pl = pl + l[e][:, None] * W[q, :]
        Th[live], Tl[live] = dd_add(Th[live], Tl[live], ph, pl)
    # X_ab = sum_p W[a,p] T[p,b]  (W M W is symmetric, so X_ab = X_ba)
    m = len(a)
    outh = np.empty(m)
    outl = np.empty(m)
    TtH = np.ascontiguousarray(Th.T)
    TtL = np.ascontiguousarray(Tl.T)
    for s0 in range(0, m, chunk):
        s1 = min(m, s0 + chunk)
        xh, xl = dd_dot_rows(W[a[s0:s1], :], TtH[b[s0:s1], :], TtL[b[s0:s1], :])
        outh[s0:s1], outl[s0:s1] = xh, xl
    coef = np.where(a == b, val, 2.0 * val)
    return dd_mul_d(outh, outl, coef)


def true_relative_residual(W, a, b, val, r, yh, yl=None):
    """||r - H y||_2 / ||r||_2 with H y and the subtraction in double-double."""
    hh, hl = dd_hessian_apply(W, a, b, val, yh, yl)
    rh, rl = dd_add(r, np.zeros_like(r), -hh, -hl)
    res = rh + rl
    return float(np.linalg.norm(res) / np.linalg.norm(r)), res
