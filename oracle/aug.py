"""The augmented preconditioner of Section 4.2 (eqs sparse_prec, aug_prec), plain numpy/scipy.

Test infrastructure (see oracle/__init__.py).

Section 4.2 replaces the dense 2 W0 + U U^T = Z Z^T inside H~ by the scaled identity 2 tau I:

    H^ = A^T (tau^2 I + 2 tau (U U^T kron I)) A                      (eq sparse_prec)

and applies H^{-1} by solving the sparse symmetric indefinite augmented system

    [ tau^2 A^T A               tau^{3/2} A^T (U kron I) ] [x]   [b]
    [ tau^{3/2} (U kron I)^T A  -tau^2/2 I_nk            ] [y] = [0]  (eq aug_prec)

whose x-block is H^{-1} b (eliminate y).  The oracle forms that matrix as written and solves
it with a general sparse LU with partial pivoting (a stable method, as the paper asks for;
the paper used an LDL^T with threshold pivoting).  Lemma aug_prec: with
lambda_min(W0) <= tau <= lambda_max(W0), every eigenvalue of H^{-1} H beyond the k^2 largest
lies within a factor kappa^2(W0) of the smallest, so PCG needs about k^2 + O(log 1/(eps mu))
iterations, and the augmented matrix has condition number Theta(1/sqrt(mu)).

vec is column-major: (U kron I) vec X = vec(X U^T) for X in R^{n x k}, nk index p + n j.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .alg1 import Constraints, formation


def bold_B(C: Constraints, U):
    """B = A^T (U kron I) as a sparse m x nk matrix: row i is vec(A_i U)^T, i.e. entries
    s_i U[a_i, j] at column b_i + n j and s_i U[b_i, j] at a_i + n j (A_i = s_i (E_ab + E_ba))."""
    n, k = U.shape
    a, b, s = C.a, C.b, C.s
    rows, cols, vals = [], [], []
    for j in range(k):
        rows += [np.arange(C.m), np.arange(C.m)]
        cols += [b + n * j, a + n * j]
        vals += [s * U[a, j], s * U[b, j]]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(C.m, n * k))


def hat_H_definition(Adense_vec, U, tau):
    """H^ from eq sparse_prec with explicit vec(A_i) columns and numpy's Kronecker product
    (tiny sizes only).  Adense_vec: n^2 x m, column-major vec of each A_i."""
    n, k = U.shape
    D = tau * tau * np.eye(n * n) + 2.0 * tau * np.kron(U @ U.T, np.eye(n))
    return Adense_vec.T @ D @ Adense_vec


def augmented_matrix(C: Constraints, U, tau):
    """The (m + nk) x (m + nk) matrix of eq aug_prec (sparse)."""
    n, k = U.shape
    B = bold_B(C, U)
    G = sp.diags(C.g)                              # A^T A (diagonal for disjoint supports)
    return sp.bmat([[tau * tau * G, tau ** 1.5 * B],
                    [tau ** 1.5 * B.T, -(tau * tau / 2.0) * sp.eye(n * k)]]).tocsc()


@dataclass
class AugFactor:
    C: Constraints
    W: np.ndarray
    k: int
    tau: float
    U: np.ndarray
    W0: np.ndarray
    K: object              # the augmented matrix
    lu: object             # its sparse LU with partial pivoting

    def apply(self, b):
        """H^{-1} b: the x-block of the solution of eq aug_prec with right-hand side [b; 0]."""
        rhs = np.concatenate([b, np.zeros(self.K.shape[0] - self.C.m)])
        return self.lu.solve(rhs)[: self.C.m]


def aug_factor(C: Constraints, W, k, tau_rule="mean"):
    """The split of Algorithm 1 step 1 (U, tau) and the factorization of eq aug_prec."""
    spl = formation(W, k, tau_rule=tau_rule)
    K = augmented_matrix(C, spl.U, spl.tau)
    lu = spla.splu(K, permc_spec="COLAMD")
    return AugFactor(C=C, W=W, k=k, tau=spl.tau, U=spl.U, W0=spl.W0, K=K, lu=lu)


def trailing_schur(C: Constraints, U, tau):
    """The nk x nk block left after eliminating x from eq aug_prec, divided by -tau:
    (tau/2) I + B^T (A^T A)^{-1} B (symmetric positive definite; dense, small sizes)."""
    B = bold_B(C, U)
    n, k = U.shape
    return (tau / 2.0) * np.eye(n * k) + (B.T @ sp.diags(1.0 / C.g) @ B).toarray()
