"""Plain definitions of the interior-point Hessian H = A^T (W kron W) A.

Test infrastructure (see oracle/__init__.py): nothing in the product may use it.

Constraint i is given by one triplet (a_i, b_i, val_i), a_i <= b_i, meaning
(A_i)_{ab} = (A_i)_{ba} = val_i.  Writing A_i = s_i (e_a e_b^T + e_b e_a^T) with
s_i = val_i (a != b) or val_i / 2 (a == b) covers both cases with one formula.

Paper: Section 2, equations "hesseqn2" and "hesseqn1": the Hessian equation is
A_i . [W (sum_j y_j A_j) W] = r_i, i.e. (A^T D A) y = r with D = W kron W.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def half_scale(a, b, val):
    """s_i with A_i = s_i (e_a e_b^T + e_b e_a^T)."""
    a = np.asarray(a)
    b = np.asarray(b)
    val = np.asarray(val, dtype=np.float64)
    return np.where(a == b, 0.5 * val, val)


def dense_constraints(n, a, b, val):
    """The m dense matrices A_i (tiny sizes only)."""
    m = len(a)
    A = np.zeros((m, n, n))
    idx = np.arange(m)
    A[idx, a, b] = val
    A[idx, b, a] = val
    return A


def normal_diag(a, b, val):
    """g = diag(A^T A), g_i = ||A_i||_F^2 (A^T A is diagonal when supports are disjoint;
    Assumption 2, Section 1.1)."""
    val = np.asarray(val, dtype=np.float64)
    return np.where(np.asarray(a) == np.asarray(b), val * val, 2.0 * val * val)


def hessian_trace_form(W, Adense):
    """H_ij = tr(A_i W A_j W) straight from the definition (tiny sizes only)."""
    m = Adense.shape[0]
    WA = np.einsum("pq,iqr->ipr", W, Adense)          # W A_i
    H = np.empty((m, m))
    for i in range(m):
        for j in range(m):
            H[i, j] = np.trace(WA[i] @ WA[j])        # tr(A_i W A_j W) = tr(W A_i W A_j)
    return H


def hessian_dense(W, a, b, val):
    """Explicit H from its closed form.  For A_i = s_i(E_ab + E_ba), A_j = s_j(E_cd + E_dc):
    tr(A_i W A_j W) = 2 s_i s_j (W_ac W_bd + W_ad W_bc)."""
    s = half_scale(a, b, val)
    a = np.asarray(a)
    b = np.asarray(b)
    H = W[np.ix_(a, a)] * W[np.ix_(b, b)]
    H += W[np.ix_(a, b)] * W[np.ix_(b, a)]
    H *= 2.0 * s[:, None] * s[None, :]
    return H


def mat_Av(n, a, b, val, v):
    """mat(A v) = sum_i v_i A_i as a dense n x n matrix."""
    M = np.zeros((n, n))
    np.add.at(M, (a, b), val * v)
    off = a != b
    np.add.at(M, (b[off], a[off]), (val * v)[off])
    return M


def At_vec(X, a, b, val):
    """[A_i . X]_i for a dense (not necessarily symmetric) X."""
    return np.where(a == b, val * X[a, b], val * (X[a, b] + X[b, a]))


def hessian_apply(W, a, b, val, v):
    """(H v)_i = A_i . (W M W) with M = mat(A v): equation hesseqn2 evaluated densely."""
    n = W.shape[0]
    M = mat_Av(n, a, b, val, v)
    X = W @ M @ W
    return At_vec(X, a, b, val)


def check_spd(H):
    """Symmetry (exact by construction) and positive definiteness of H."""
    sym = float(np.max(np.abs(H - H.T)))
    try:
        sla.cholesky(H, lower=True, check_finite=False)
        pd = True
    except np.linalg.LinAlgError:
        pd = False
    return sym == 0.0, pd


def solve_dense(H, r):
    """y = H^{-1} r by dense Cholesky: the standard approach the paper improves on
    (Section 2.1, first paragraph)."""
    c = sla.cho_factor(H, lower=True, check_finite=False)
    return sla.cho_solve(c, r, check_finite=False)


def hessian_storage_bytes(m, packed=True):
    """FP64 bytes to hold H explicitly (packed symmetric storage by default)."""
    return 8 * (m * (m + 1) // 2 if packed else m * m)
