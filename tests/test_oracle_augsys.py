"""Pins of oracle/augsys.py (the augmented system of Section 4.1, eq aug_ex, beside eq wsmf)
against what the paper and the algebra fix, independently of the oracle's own formulas."""

import numpy as np
import pytest

from oracle import augsys as A


def _case(n=30, k=3, seed=5, in_range=False):
    rng = np.random.default_rng(seed)
    Ut = rng.standard_normal((k, n)) / np.sqrt(n) * np.linspace(3.0, 1.0, k)[:, None]
    b = Ut.T @ rng.standard_normal(k) if in_range else rng.standard_normal(n)
    return Ut, b


def _dense_exact(Ut, tau, b):
    """W~^{-1} b from the dense W~ = tau I + U U^T by mpmath LU (no use of eq wsmf)."""
    import mpmath as mp
    mp.mp.dps = 50
    k, n = Ut.shape
    W = mp.matrix(n, n)
    for i in range(n):
        for j in range(n):
            W[i, j] = mp.fsum(mp.mpf(float(Ut[a, i])) * mp.mpf(float(Ut[a, j])) for a in range(k))
            if i == j:
                W[i, j] += mp.mpf(tau)
    x = mp.lu_solve(W, mp.matrix([mp.mpf(float(v)) for v in b]))
    return np.array([float(v) for v in x])


@pytest.mark.parametrize("tau", [1e-2, 1e-6])
def test_exact_reference_is_the_dense_solve(tau):
    """exact_solve (eq wsmf in 50 digits) against a 50-digit LU of the dense W~: pins the
    extended-precision reference the other pins use."""
    Ut, b = _case(n=12, k=2, seed=3, in_range=True)
    xe = A.exact_solve(Ut, tau, b)
    xd = _dense_exact(Ut, tau, b)
    assert np.linalg.norm(xe - xd) <= 1e-14 * np.linalg.norm(xd)


def test_augmented_system_solves_wtilde():
    """The x block of eq aug_ex solves W~ x = b and its y block is U^T x / sqrt(tau)."""
    Ut, b = _case()
    tau = 1e-3
    K = A.aug_matrix(Ut, tau)
    n = Ut.shape[1]
    z = np.linalg.solve(K, np.concatenate([b, np.zeros(Ut.shape[0])]))
    x, y = z[:n], z[n:]
    W = tau * np.eye(n) + Ut.T @ Ut
    assert np.linalg.norm(W @ x - b) <= 1e-12 * np.linalg.norm(b)
    # (the y block is a sum with cancellation: measured against ||U|| ||x|| / sqrt(tau))
    assert np.linalg.norm(y - Ut @ x / np.sqrt(tau)) <= \
        1e-13 * np.linalg.norm(Ut, 2) * np.linalg.norm(x) / np.sqrt(tau)
    assert np.allclose(A.aug_solve(Ut, tau, b), x, rtol=0, atol=1e-12 * np.abs(x).max())


@pytest.mark.parametrize("tau", [1e-1, 1e-4, 1e-8])
def test_condition_numbers_closed_form(tau):
    """kappa_2 of the matrix of eq aug_ex is sqrt(1 + ||U||^2 / tau) (Section 4.1), and that of
    W~ is (tau + ||U||^2) / tau: numpy's condition numbers of the assembled matrices agree."""
    Ut, _ = _case()
    assert abs(np.linalg.cond(A.aug_matrix(Ut, tau)) - A.aug_cond(Ut, tau)) <= \
        1e-8 * A.aug_cond(Ut, tau)
    assert abs(np.linalg.cond(A.wtilde(Ut, tau)) - A.wtilde_cond(Ut, tau)) <= \
        1e-6 * A.wtilde_cond(Ut, tau)


def test_unpivoted_elimination_is_the_smw_formula():
    """Gaussian elimination on eq aug_ex without pivoting (x first) takes the steps of eq wsmf
    (Section 4.1): both give the same x to rounding on a generic right-hand side."""
    Ut, b = _case()
    tau = 1e-2
    xs = A.smw_solve(Ut, tau, b)
    xu = A.aug_solve_unpivoted(Ut, tau, b)
    assert np.linalg.norm(xs - xu) <= 1e-13 * np.linalg.norm(xs)


def test_augmented_solve_is_backward_stable_where_smw_is_not():
    """With b in range(U) (where eq wsmf cancels), the pivoted solve of eq aug_ex keeps the
    backward error ||b - W~ x|| / (||W~|| ||x|| + ||b||) at the rounding level for every tau,
    while that of eq wsmf grows like u kappa(W~); both forward errors stay within
    kappa(W~) times a small multiple of u of the exact answer."""
    Ut, b = _case(n=40, k=3, seed=9, in_range=True)
    u = np.finfo(np.float64).eps
    smw_back = []
    for tau in (1e-4, 1e-8, 1e-12):
        W = A.wtilde(Ut, tau)
        xe = A.exact_solve(Ut, tau, b)
        kw = A.wtilde_cond(Ut, tau)
        for name, f in (("smw", A.smw_solve), ("aug", A.aug_solve)):
            x = f(Ut, tau, b)
            back = np.linalg.norm(b - W @ x) / (np.linalg.norm(W, 2) * np.linalg.norm(x) +
                                                np.linalg.norm(b))
            fwd = np.linalg.norm(x - xe) / np.linalg.norm(xe)
            assert fwd <= 100 * kw * u, (name, tau, fwd)
            if name == "aug":
                assert back <= 10 * u, (tau, back)
            else:
                smw_back.append(back)
    # eq wsmf: the backward error grows with kappa(W~) (a factor 1e4 per step of tau here)
    assert smw_back[-1] >= 1e3 * smw_back[0] and smw_back[-1] >= 1e-6, smw_back
