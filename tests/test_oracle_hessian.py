"""Pins for the oracle's plain definitions of H (eqs hesseqn2 / hesseqn1)."""

import json
import os

import numpy as np
import pytest

from oracle import alg1, hessian as hs, mp
from synth import make_instance

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_general(rng, n=6, m=12):
    """Disjoint-support triplets with arbitrary values, diagonals included."""
    pairs = [(i, j) for i in range(n) for j in range(i, n)]
    pick = rng.choice(len(pairs), size=m, replace=False)
    a = np.array([pairs[t][0] for t in pick])
    b = np.array([pairs[t][1] for t in pick])
    val = rng.uniform(0.3, 2.0, size=m)
    G = rng.standard_normal((n, n))
    W = G @ G.T + 0.5 * np.eye(n)
    return W, a, b, val


def vec_cols(Adense):
    """A = [vec A_1, ..., vec A_m] with column-major vec."""
    m, n, _ = Adense.shape
    return np.stack([Adense[i].reshape(-1, order="F") for i in range(m)], axis=1)


def test_closed_form_equals_trace_definition(rng):
    W, a, b, val = tiny_general(rng)
    A = hs.dense_constraints(W.shape[0], a, b, val)
    H1 = hs.hessian_trace_form(W, A)
    H2 = hs.hessian_dense(W, a, b, val)
    assert np.max(np.abs(H1 - H2)) <= 1e-13 * np.max(np.abs(H1))


def test_closed_form_equals_kronecker_definition(rng):
    """H = A^T (W kron W) A with explicit vec and numpy's Kronecker product."""
    W, a, b, val = tiny_general(rng)
    A = vec_cols(hs.dense_constraints(W.shape[0], a, b, val))
    H1 = A.T @ np.kron(W, W) @ A
    H2 = hs.hessian_dense(W, a, b, val)
    assert np.max(np.abs(H1 - H2)) <= 1e-13 * np.max(np.abs(H1))


def test_closed_form_equals_exact_arithmetic(rng):
    W, a, b, val = tiny_general(rng, n=5, m=9)
    Hx, _ = mp.exact_solve(W, a, b, val, np.ones(len(a)))
    H2 = hs.hessian_dense(W, a, b, val)
    Hf = np.array([[float(Hx[i, j]) for j in range(len(a))] for i in range(len(a))])
    assert np.max(np.abs(Hf - H2)) <= 4e-16 * np.max(np.abs(Hf)) * 4


def test_lemma_sym_kron(rng):
    """A^T (X kron Y) A = A^T (Y kron X) A for non-symmetric X, Y (Lemma sym_kron)."""
    W, a, b, val = tiny_general(rng)
    n = W.shape[0]
    A = vec_cols(hs.dense_constraints(n, a, b, val))
    X = rng.standard_normal((n, n))
    Y = rng.standard_normal((n, n))
    L = A.T @ np.kron(X, Y) @ A
    R = A.T @ np.kron(Y, X) @ A
    assert np.max(np.abs(L - R)) <= 1e-12 * np.max(np.abs(L))


@pytest.mark.parametrize("mu", [1e-2, 1e-4])
def test_matrix_free_products_match_dense(mu):
    inst = make_instance(60, 2, 600, mu, seed=7)
    H = hs.hessian_dense(inst.W, inst.a, inst.b, inst.val)
    v = np.random.default_rng(1).standard_normal(inst.m)
    ref = H @ v
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    for got in (hs.hessian_apply(inst.W, inst.a, inst.b, inst.val, v),
                alg1.hessian_apply_mf(C, inst.W, v)):
        assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def test_scaled_identity_gives_diagonal_hessian(rng):
    """W = c I  =>  H = c^2 A^T A, diagonal for disjoint supports; y_i = r_i / (c^2 g_i)."""
    W, a, b, val = tiny_general(rng)
    c = 1.7
    Wc = c * np.eye(W.shape[0])
    H = hs.hessian_dense(Wc, a, b, val)
    g = hs.normal_diag(a, b, val)
    assert np.max(np.abs(H - np.diag(np.diag(H)))) == 0.0
    np.testing.assert_allclose(np.diag(H), c * c * g, rtol=1e-15)
    r = rng.standard_normal(len(a))
    np.testing.assert_allclose(hs.solve_dense(H, r), r / (c * c * g), rtol=1e-14)


def test_normal_matrix_is_diagonal(rng):
    W, a, b, val = tiny_general(rng)
    A = vec_cols(hs.dense_constraints(W.shape[0], a, b, val))
    G = A.T @ A
    np.testing.assert_allclose(G, np.diag(hs.normal_diag(a, b, val)), atol=1e-15)


@pytest.mark.parametrize("mu", [1e-2, 1e-3, 1e-4])
def test_spd_and_conditioning_scales_like_inverse_mu_squared(mu):
    """H is SPD; kappa(H) = O(1/mu^2) (Section 2.1)."""
    inst = make_instance(40, 2, 300, mu, seed=3)
    H = hs.hessian_dense(inst.W, inst.a, inst.b, inst.val)
    sym, pd = hs.check_spd(H)
    assert sym and pd
    lam = np.linalg.eigvalsh(H)
    assert lam[0] > 0
    kappa = lam[-1] / lam[0]
    assert 1e-3 < kappa * mu * mu < 10.0


def test_dense_solve_meets_residual():
    inst = make_instance(100, 2, 1000, 1e-2, seed=1001)
    H = hs.hessian_dense(inst.W, inst.a, inst.b, inst.val)
    y = hs.solve_dense(H, inst.r)
    assert np.linalg.norm(H @ y - inst.r) <= 1e-10 * np.linalg.norm(inst.r)


def test_paper_hessian_storage_figure():
    """The paper's 1,600 GB for an explicit Hessian at m = 6.31e5 (FP64, packed symmetric)."""
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as f:
        g = json.load(f)["largest_instance"]
    gb = hs.hessian_storage_bytes(g["m"]) / 1e9
    assert abs(gb - g["hessian_storage_GB"]) / g["hessian_storage_GB"] < 0.01


def test_check_spd_rejects_indefinite_and_nonsymmetric(rng):
    """check_spd must say no to an indefinite H and to a non-symmetric one."""
    inst = make_instance(30, 2, 120, 1e-2, seed=5)
    H = hs.hessian_dense(inst.W, inst.a, inst.b, inst.val)
    assert hs.check_spd(H) == (True, True)
    lam, V = np.linalg.eigh(H)
    Hneg = H - 2.0 * lam[0] * np.outer(V[:, 0], V[:, 0])   # smallest eigenvalue -> -lam[0]
    Hneg = 0.5 * (Hneg + Hneg.T)
    sym, pd = hs.check_spd(Hneg)
    assert not pd
    Hns = H.copy()
    Hns[0, 1] += 1e-9 * abs(H[0, 1]) + 1e-300
    sym, _ = hs.check_spd(Hns)
    assert not sym
    # a PSD but singular H (a repeated constraint row) is not positive definite
    Hs = H.copy()
    Hs[:, 1] = Hs[:, 0]
    Hs[1, :] = Hs[0, :]
    assert hs.check_spd(Hs)[1] is False


def test_exact_hessian_is_the_trace_of_dense_products(rng):
    """mp.exact_hessian (dense A_i, 50 digits) against the Kronecker definition
    A^T (W kron W) A in FP64, on general disjoint-support data (values other than 1/2)."""
    W, a, b, val = tiny_general(rng, n=6, m=10)
    Hx = mp.exact_hessian(W, a, b, val)
    A = vec_cols(hs.dense_constraints(W.shape[0], a, b, val))
    Hk = A.T @ np.kron(W, W) @ A
    Hf = np.array([[float(Hx[i, j]) for j in range(len(a))] for i in range(len(a))])
    assert np.max(np.abs(Hf - Hk)) <= 1e-13 * np.max(np.abs(Hk))
