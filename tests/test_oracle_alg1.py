"""Pins for the oracle's Algorithm 1 (Section 3): split, bold U, bold S, SMW, PCG."""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import alg1, dd, hessian as hs
from synth import make_instance
from test_oracle_hessian import tiny_general, vec_cols


def setup(n=40, k=2, m=300, mu=1e-3, seed=5):
    inst = make_instance(n, k, m, mu, seed=seed)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    return inst, C


@pytest.mark.parametrize("mu", [1e-2, 1e-4, 1e-8])
def test_split_identities(mu):
    """W = W0 + U U^T, Z Z^T = 2 W0 + U U^T, spectrum of W0 = {Lambda_s, tau} (eq Wsplit2)."""
    inst, C = setup(mu=mu, k=3)
    s = alg1.formation(inst.W, inst.k)
    nW = np.linalg.norm(inst.W, 2)
    assert np.linalg.norm(s.W0 + s.U @ s.U.T - inst.W, 2) <= 1e-14 * nW * 10
    assert np.linalg.norm(s.Z @ s.Z.T - (2 * s.W0 + s.U @ s.U.T), 2) <= 1e-14 * nW * 10
    np.testing.assert_allclose(s.lam, inst.lam, rtol=1e-9, atol=1e-14 * nW * 10)
    assert s.tau == s.lam[0]
    lam0 = np.linalg.eigvalsh(s.W0)
    expect = np.sort(np.concatenate([s.lam[: inst.n - inst.k], [s.tau] * inst.k]))
    np.testing.assert_allclose(lam0, expect, rtol=1e-6, atol=1e-14 * nW * 10)
    # the synthetic spectrum has kappa(W0) <= 2 (small eigenvalues mu U[1,2))
    assert lam0[-1] / lam0[0] <= 2.0 + 1e-6


def test_hessian_splits_exactly():
    """H = H0 + bold U bold U^T with H0 = A^T (W0 kron W0) A (eq hessExp2)."""
    inst, C = setup(mu=1e-3)
    s = alg1.formation(inst.W, inst.k)
    H = hs.hessian_dense(inst.W, inst.a, inst.b, inst.val)
    H0 = hs.hessian_dense(s.W0, inst.a, inst.b, inst.val)
    bU = alg1.bold_U_explicit(C, s.Z, s.U)
    assert np.max(np.abs(H - H0 - bU @ bU.T)) <= 1e-13 * np.max(np.abs(H))


def test_bold_U_against_kronecker(rng):
    """bold U = A^T (U kron Z) from numpy's Kronecker product; products eq Umv (a), (b)."""
    W, a, b, val = tiny_general(rng, n=6, m=12)
    n, k = 6, 2
    C = alg1.Constraints(n, a, b, val)
    U = rng.standard_normal((n, k))
    Z = np.tril(rng.standard_normal((n, n)))
    A = vec_cols(hs.dense_constraints(n, a, b, val))
    bU = A.T @ np.kron(U, Z)
    np.testing.assert_allclose(alg1.bold_U_explicit(C, Z, U), bU, atol=1e-14)
    x = rng.standard_normal(n * k)
    y = rng.standard_normal(len(a))
    np.testing.assert_allclose(alg1.bold_U_apply(C, Z, U, x), bU @ x, atol=1e-13)
    np.testing.assert_allclose(alg1.bold_Ut_apply(C, Z, U, y), bU.T @ y, atol=1e-13)


def test_schur_block_formula_matches_explicit():
    inst, C = setup(k=3, mu=1e-3)
    s = alg1.formation(inst.W, inst.k)
    S1 = alg1.schur_explicit(alg1.bold_U_explicit(C, s.Z, s.U), C.g, s.tau)
    S2 = alg1.schur_blocks(C, s.Z, s.U, s.tau)
    assert np.max(np.abs(S1 - S2)) <= 1e-13 * np.max(np.abs(S1))


@pytest.mark.parametrize("k", [2, 3])
def test_null_space_of_bold_U(k):
    """bold U vec(Z^{-1} U K) = 0 for skew K, so bold S has k(k-1)/2 eigenvalues tau^2."""
    inst, C = setup(k=k, mu=1e-3)
    s = alg1.formation(inst.W, inst.k)
    bU = alg1.bold_U_explicit(C, s.Z, s.U)
    N = alg1.null_basis(s.Z, s.U)
    assert N.shape[1] == k * (k - 1) // 2
    assert np.linalg.norm(bU @ N) <= 1e-13 * np.linalg.norm(bU, 2) * np.linalg.norm(N)
    S = alg1.schur_explicit(bU, C.g, s.tau)
    lam = np.linalg.eigvalsh(S)
    np.testing.assert_allclose(lam[: N.shape[1]], s.tau ** 2, rtol=1e-6)


def test_deflation_leaves_preconditioner_unchanged():
    inst, C = setup(k=3, mu=1e-2)
    F1 = alg1.factor(C, inst.W, inst.k, deflate=False)
    F2 = alg1.factor(C, inst.W, inst.k, deflate=True)
    assert np.linalg.cond(F2.S) < np.linalg.cond(F1.S)
    v = np.random.default_rng(2).standard_normal(inst.m)
    z1 = alg1.precond_apply(F1, v)
    z2 = alg1.precond_apply(F2, v)
    assert np.linalg.norm(z1 - z2) <= 1e-9 * np.linalg.norm(z1)


@pytest.mark.parametrize("mu", [1e-2, 1e-4])
def test_smw_equals_dense_solve(mu):
    """H~^{-1} v by eq SMW2 equals a dense solve with tau^2 A^T A + bold U bold U^T."""
    inst, C = setup(mu=mu)
    F = alg1.factor(C, inst.W, inst.k)
    Ht = alg1.precond_dense(F)
    v = np.random.default_rng(3).standard_normal(inst.m)
    z = alg1.precond_apply(F, v)
    zd = sla.solve(Ht, v, assume_a="pos")
    assert np.linalg.norm(z - zd) <= 1e-8 * np.linalg.norm(zd)


def test_lemma_kappaW():
    """kappa(W, W~) = kappa(W0) with W~ = tau I + U U^T (Lemma kappaW)."""
    inst, C = setup(k=3, mu=1e-3)
    s = alg1.formation(inst.W, inst.k)
    Wt = s.tau * np.eye(inst.n) + s.U @ s.U.T
    lam = sla.eigh(inst.W, Wt, eigvals_only=True)
    l0 = np.linalg.eigvalsh(s.W0)
    np.testing.assert_allclose(lam[-1] / lam[0], l0[-1] / l0[0], rtol=1e-8)


@pytest.mark.parametrize("mu", [1e-2, 1e-3])
def test_lemma_Htilde(mu):
    """kappa(H, H~) <= kappa(W0)^2 (Lemma Htilde)."""
    inst, C = setup(k=2, mu=mu)
    F = alg1.factor(C, inst.W, inst.k)
    H = hs.hessian_dense(inst.W, inst.a, inst.b, inst.val)
    lam = sla.eigh(H, alg1.precond_dense(F), eigvals_only=True)
    l0 = np.linalg.eigvalsh(F.split.W0)
    assert lam[-1] / lam[0] <= (l0[-1] / l0[0]) ** 2 * (1 + 1e-8)


def test_equal_small_eigenvalues_give_exact_preconditioner():
    """Lambda_s = tau I  =>  W0 = tau I  =>  H~ = H: PCG converges in one iteration."""
    n, k, m = 40, 2, 300
    inst = make_instance(n, k, m, 1e-3, seed=11)
    lam, V = np.linalg.eigh(inst.W)
    lam[: n - k] = 1e-3
    W = (V * lam) @ V.T
    W = 0.5 * (W + W.T)
    C = alg1.Constraints(n, inst.a, inst.b, inst.val)
    F = alg1.factor(C, W, k)
    H = hs.hessian_dense(W, inst.a, inst.b, inst.val)
    assert np.max(np.abs(alg1.precond_dense(F) - H)) <= 1e-9 * np.max(np.abs(H))
    out = alg1.solve(F, inst.r, eps=1e-8, Hmul=lambda v: H @ v)
    assert out.iters == 1


def test_preconditioner_invariant_to_factor_rotation():
    """H~ depends on U and Z only through U U^T and Z Z^T."""
    inst, C = setup(k=3, mu=1e-3)
    s = alg1.formation(inst.W, inst.k)
    rng = np.random.default_rng(9)
    Ok, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    On, _ = np.linalg.qr(rng.standard_normal((inst.n, inst.n)))
    B1 = alg1.bold_U_explicit(C, s.Z, s.U)
    B2 = alg1.bold_U_explicit(C, s.Z @ On, s.U @ Ok)
    np.testing.assert_allclose(B1 @ B1.T, B2 @ B2.T, atol=1e-12 * np.max(np.abs(B1 @ B1.T)))


def test_pcg_iterations_flat_and_plain_cg_grows():
    """PCG needs a few tens of iterations whatever mu (Section 5.2: 15-25); plain CG
    grows as kappa(H) = O(1/mu^2) (Section 2.1)."""
    pcg_its, cg_its = [], []
    for mu in (1e-2, 1e-4, 1e-6):
        inst = make_instance(100, 2, 1000, mu, seed=1001)
        C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
        F = alg1.factor(C, inst.W, inst.k)
        pcg_its.append(alg1.solve(F, inst.r, eps=1e-8).iters)
        H = lambda v, C=C, W=inst.W: alg1.hessian_apply_mf(C, W, v)  # noqa: E731
        cg_its.append(alg1.pcg(H, lambda v: v, inst.r, eps=1e-8, max_iter=400).iters)
    assert max(pcg_its) <= 25
    assert cg_its[0] < cg_its[1] <= cg_its[2]
    assert cg_its[1] > 4 * max(pcg_its)


@pytest.mark.parametrize("mu", [1e-2, 1e-4])
def test_fp64_solve_matches_dense_cholesky(mu):
    inst = make_instance(100, 2, 1000, mu, seed=1001)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    F = alg1.factor(C, inst.W, inst.k)
    out = alg1.solve(F, inst.r, eps=1e-8)
    H = hs.hessian_dense(inst.W, inst.a, inst.b, inst.val)
    ystar = hs.solve_dense(H, inst.r)
    assert np.linalg.norm(out.y - ystar) <= 1e-6 * np.linalg.norm(ystar)
    rel, _ = dd.true_relative_residual(inst.W, inst.a, inst.b, inst.val, inst.r, out.y)
    assert rel <= 1e-8


@pytest.mark.parametrize("mu", [1e-2, 1e-4])
def test_mean_tau_rule(mu):
    """tau = mean of the n - k smallest eigenvalues lies in the range Section 3.1 allows, gives
    the same kappa(W0) (so Lemma Htilde's bound), keeps H~ SPD, and PCG still converges to the
    same solution (the preconditioner does not change y*)."""
    inst, C = setup(k=3, mu=mu)
    lam = np.linalg.eigvalsh(inst.W)
    n, k = inst.n, inst.k
    s_min = alg1.formation(inst.W, k, "min")
    s_mean = alg1.formation(inst.W, k, "mean")
    assert lam[0] <= s_mean.tau < lam[n - k - 1]
    np.testing.assert_allclose(s_mean.tau, lam[: n - k].mean(), rtol=1e-9)
    l0 = np.linalg.eigvalsh(s_mean.W0)
    l1 = np.linalg.eigvalsh(s_min.W0)
    np.testing.assert_allclose(l0[-1] / l0[0], l1[-1] / l1[0], rtol=1e-6)
    F = alg1.factor(C, inst.W, k, tau_rule="mean")
    H = hs.hessian_dense(inst.W, inst.a, inst.b, inst.val)
    g = sla.eigh(H, alg1.precond_dense(F), eigvals_only=True)
    assert g[0] > 0 and g[-1] / g[0] <= (l0[-1] / l0[0]) ** 2 * (1 + 1e-8)
    out = alg1.solve(F, inst.r, eps=1e-10, Hmul=lambda v: H @ v)
    ref = alg1.solve(alg1.factor(C, inst.W, k), inst.r, eps=1e-10, Hmul=lambda v: H @ v)
    assert np.linalg.norm(out.y - ref.y) <= 1e-6 * np.linalg.norm(ref.y)
