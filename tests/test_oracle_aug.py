"""Pins for the augmented preconditioner oracle (Section 4.2, eqs sparse_prec and aug_prec)."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import alg1, aug, dd as ddo, hessian as hs, mp, refine
from synth import make_instance


def vec_cols(n, a, b, val):
    A = hs.dense_constraints(n, a, b, val)
    return np.stack([A[i].reshape(-1, order="F") for i in range(len(a))], axis=1)


@pytest.mark.parametrize("mu", [1e-2, 1e-6])
def test_augmented_solve_is_the_inverse_of_the_definition(mu):
    """The x-block of eq aug_prec solved with [b; 0] equals H^{-1} b for H^ built from eq
    sparse_prec with explicit vec(A_i) and Kronecker products."""
    inst = make_instance(12, 2, 40, mu, seed=3)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    F = aug.aug_factor(C, inst.W, inst.k)
    Hh = aug.hat_H_definition(vec_cols(inst.n, inst.a, inst.b, inst.val), F.U, F.tau)
    b = np.random.default_rng(1).standard_normal(inst.m)
    x = F.apply(b)
    ref = np.linalg.solve(Hh, b)
    # both are backward-stable solves: forward errors of order u kappa(H^)
    tol = 100 * np.finfo(float).eps * np.linalg.cond(Hh)
    assert np.linalg.norm(x - ref) <= tol * np.linalg.norm(ref)
    # and B^T (A^T A)^{-1} B written as a sum over constraints equals the sparse product
    S = aug.trailing_schur(C, F.U, F.tau)
    n, k = F.U.shape
    Bd = np.zeros((inst.m, n * k))
    for i in range(inst.m):
        Ai = hs.dense_constraints(n, inst.a[i:i + 1], inst.b[i:i + 1], inst.val[i:i + 1])[0]
        Bd[i] = (Ai @ F.U).reshape(-1, order="F")          # vec(A_i U), column-major
    S2 = (F.tau / 2) * np.eye(n * k) + Bd.T @ (Bd / C.g[:, None])
    assert np.max(np.abs(S - S2)) <= 1e-13 * np.max(np.abs(S2))


def test_augmented_condition_number_grows_like_inverse_sqrt_mu():
    """Section 4.2: the matrix of eq aug_prec has condition number Theta(1/sqrt(mu))."""
    conds = []
    for mu in (1e-2, 1e-4, 1e-6):
        inst = make_instance(30, 2, 200, mu, seed=5)
        C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
        spl = alg1.formation(inst.W, inst.k, tau_rule="mean")
        K = aug.augmented_matrix(C, spl.U, spl.tau).toarray()
        conds.append(np.linalg.cond(K))
    r1, r2 = conds[1] / conds[0], conds[2] / conds[1]
    assert 5.0 < r1 < 20.0 and 5.0 < r2 < 20.0, conds      # about 10 per factor 100 in mu


@pytest.mark.parametrize("k,mu", [(2, 1e-4), (3, 1e-6)])
def test_lemma_aug_prec_eigenvalue_bound(k, mu):
    """Lemma aug_prec: lambda_j(H^{-1} H) / lambda_min(H^{-1} H) <= kappa(W0)^2 for j > k^2."""
    inst = make_instance(30, k, 250, mu, seed=7)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    F = aug.aug_factor(C, inst.W, k)
    Hh = aug.hat_H_definition(vec_cols(inst.n, inst.a, inst.b, inst.val), F.U, F.tau)
    H = hs.hessian_dense(inst.W, inst.a, inst.b, inst.val)
    L = np.linalg.cholesky(Hh)
    Li = np.linalg.inv(L)
    ev = np.linalg.eigvalsh(Li @ H @ Li.T)               # eigenvalues of H^{-1} H, ascending
    w0 = np.linalg.eigvalsh(F.W0)
    kap = w0[-1] / w0[0]
    assert ev[-k * k - 1] / ev[0] <= kap * kap * (1 + 1e-8)
    assert ev[-1] / ev[0] > 10 * kap * kap                 # the k^2 outliers are real


def test_rank_k2_difference_gives_k2_plus_one_iterations():
    """With W0 = tau I exactly (every small eigenvalue equal), H - H^ = A^T (U U^T kron U U^T) A
    (Lemma sym_kron), a PSD matrix of rank <= k^2, so PCG with H^ converges in at most
    k^2 + 1 iterations in exact arithmetic."""
    inst = make_instance(40, 2, 300, 1e-2, seed=9)
    rng = np.random.default_rng(10)
    q, r = np.linalg.qr(rng.standard_normal((40, 40)))
    q = q * np.sign(np.diag(r))[None, :]
    lam = np.concatenate([np.full(38, 0.03), [1.2, 1.7]])
    inst.W = np.ascontiguousarray(0.5 * ((q * lam) @ q.T + ((q * lam) @ q.T).T))
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    F = aug.aug_factor(C, inst.W, 2)
    assert abs(F.tau - 0.03) <= 1e-12
    out = alg1.pcg(lambda v: alg1.hessian_apply_mf(C, inst.W, v), F.apply, inst.r, eps=1e-10)
    assert out.converged and out.iters <= 2 * 2 + 1 + 1, out.iters


@pytest.mark.parametrize("mu", [1e-6, 1e-8])
def test_refinement_with_aug_matches_exact(mu):
    """Double-double refinement with H^ as the inner preconditioner (no double-double SMW
    pieces) reaches the exact (50-digit) solution of a tiny instance."""
    inst = make_instance(12, 2, 40, mu, seed=31)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    F = aug.aug_factor(C, inst.W, inst.k)
    out = refine.refine(F, inst.r, eps=1e-10, precond=F.apply)
    assert out.relres <= 1e-10
    Hx, y = mp.exact_solve(inst.W, inst.a, inst.b, inst.val, inst.r)
    eh, el = mp.to_dd(y)
    err = np.linalg.norm((out.yh - eh) + (out.yl - el)) / np.linalg.norm(eh)
    assert err <= 1e-8


def test_trailing_block_fills_in():
    """Why the nk x nk trailing block of eq aug_prec is factored as a dense matrix: on a
    matrix-completion pattern (random Omega, ~39 entries per row) its Cholesky factor is
    nearly full even under a fill-reducing (reverse Cuthill-McKee) ordering."""
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    inst = make_instance(300, 2, 6000, 1e-2, seed=13)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    spl = alg1.formation(inst.W, 2, tau_rule="mean")
    S = sp.csr_matrix(aug.trailing_schur(C, spl.U, spl.tau))
    p = reverse_cuthill_mckee(S, symmetric_mode=True)
    L = np.linalg.cholesky(S[p][:, p].toarray())
    nk = S.shape[0]
    frac = np.count_nonzero(np.abs(L) > 1e-300) / (nk * (nk + 1) / 2)
    assert S.nnz / nk ** 2 < 0.2 and frac > 0.5, (S.nnz / nk ** 2, frac)
