"""Pins for the double-double pieces and the refinement loop (small mu)."""

import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import alg1, dd, mp, refine
from synth import make_instance

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_error_free_transformations_are_exact(rng):
    a = rng.standard_normal(200) * 10.0 ** rng.integers(-8, 8, 200)
    b = rng.standard_normal(200) * 10.0 ** rng.integers(-8, 8, 200)
    s, e = dd.two_sum(a, b)
    p, f = dd.two_prod(a, b)
    for i in range(200):
        assert Fraction(s[i]) + Fraction(e[i]) == Fraction(a[i]) + Fraction(b[i])
        assert Fraction(p[i]) + Fraction(f[i]) == Fraction(a[i]) * Fraction(b[i])


def tiny(mu, n=10, k=2, m=30, seed=21):
    return make_instance(n, k, m, mu, seed=seed)


@pytest.mark.parametrize("mu", [1e-4, 1e-8])
def test_dd_hessian_apply_matches_exact(mu):
    inst = tiny(mu)
    Hx, _ = mp.exact_solve(inst.W, inst.a, inst.b, inst.val, inst.r)
    y = np.random.default_rng(4).standard_normal(inst.m) * 1e6
    yl = y * 1e-17
    hh, hl = dd.dd_hessian_apply(inst.W, inst.a, inst.b, inst.val, y, yl)
    import mpmath
    yv = mpmath.matrix([mpmath.mpf(float(h)) + mpmath.mpf(float(l)) for h, l in zip(y, yl)])
    ex = Hx * yv
    err = max(abs(mpmath.mpf(float(hh[i])) + mpmath.mpf(float(hl[i])) - ex[i]) for i in range(inst.m))
    scale = max(abs(ex[i]) for i in range(inst.m))
    assert float(err / scale) < 1e-28


def test_fp64_floor_and_dd_answer():
    """At small mu the FP64-rounded exact solution misses 1e-8 (the representation floor
    that follows from kappa(H) = O(1/mu^2)), while its double-double pair meets it."""
    inst = tiny(1e-8)
    Hx, y = mp.exact_solve(inst.W, inst.a, inst.b, inst.val, inst.r)
    yh, yl = mp.to_dd(y)
    assert mp.relative_residual(Hx, yh, np.zeros_like(yh), inst.r) > 1e-8
    assert mp.relative_residual(Hx, yh, yl, inst.r) < 1e-14
    rel, _ = dd.true_relative_residual(inst.W, inst.a, inst.b, inst.val, inst.r, yh, yl)
    assert rel < 1e-14


def test_dd_W0_is_accurate():
    inst = make_instance(30, 3, 200, 1e-8, seed=2)
    s = alg1.formation(inst.W, inst.k)
    W0 = refine.dd_W0(inst.W, s.U)
    # W0 + U U^T reproduces W to a rounding of W0 (not of W) when the sum is taken exactly
    import mpmath
    mpmath.mp.dps = 40
    worst = 0.0
    for i in range(0, 30, 7):
        for j in range(0, 30, 5):
            ex = mpmath.mpf(inst.W[i, j]) - sum(mpmath.mpf(s.U[i, t]) * mpmath.mpf(s.U[j, t]) for t in range(3))
            worst = max(worst, float(abs(ex - mpmath.mpf(W0[i, j]))))
    assert worst <= 2.3e-16 * np.max(np.abs(W0))


@pytest.mark.parametrize("mu", [1e-2, 1e-6, 1e-8])
def test_split_operator_matches_exact(mu):
    """The split H v (eq hessExp1) is relatively accurate even where plain FP64 is not."""
    inst = tiny(mu)
    Hx, _ = mp.exact_solve(inst.W, inst.a, inst.b, inst.val, inst.r)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    s = alg1.formation(inst.W, inst.k)
    op = refine.SplitOperator(C, refine.dd_W0(inst.W, s.U), s.U)
    # the eigenvector of H's smallest eigenvalue (the mu^2-sized part of the spectrum)
    import mpmath
    Hf = np.array([[float(Hx[i, j]) for j in range(inst.m)] for i in range(inst.m)])
    lam, V = np.linalg.eigh(Hf)
    v = V[:, 0].copy()
    vm = mpmath.matrix([mpmath.mpf(float(x)) for x in v])
    ex = np.array([float(t) for t in Hx * vm])
    got = op(v)
    assert np.linalg.norm(got - ex) <= 1e-6 * np.linalg.norm(ex)


def test_dd_preconditioner_agrees_with_fp64_at_moderate_mu():
    inst = tiny(1e-4, n=30, m=200)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    F = alg1.factor(C, inst.W, inst.k)
    v = np.random.default_rng(6).standard_normal(inst.m)
    z1 = alg1.precond_apply(F, v)
    z2 = refine.dd_precond_apply(F, v)
    assert np.linalg.norm(z1 - z2) <= 1e-7 * np.linalg.norm(z1)


def test_dd_preconditioner_stays_positive_at_tiny_mu():
    """At mu = 1e-8 the double-double SMW pieces keep v^T H~^{-1} v > 0 (Section 4)."""
    inst = make_instance(100, 2, 1000, 1e-8, seed=1001)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    F = alg1.factor(C, inst.W, inst.k)
    rng = np.random.default_rng(8)
    for _ in range(5):
        v = rng.standard_normal(inst.m)
        assert v @ refine.dd_precond_apply(F, v) > 0


@pytest.mark.parametrize("mu", [1e-6, 1e-8])
def test_refinement_reaches_target_and_matches_exact(mu):
    inst = tiny(mu, n=12, k=2, m=40, seed=31)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    F = alg1.factor(C, inst.W, inst.k)
    out = refine.refine(F, inst.r, eps=1e-8)
    assert out.relres <= 1e-8
    Hx, y = mp.exact_solve(inst.W, inst.a, inst.b, inst.val, inst.r)
    eh, el = mp.to_dd(y)
    err = np.linalg.norm((out.yh - eh) + (out.yl - el)) / np.linalg.norm(eh)
    assert err <= 1e-6
    assert mp.relative_residual(Hx, out.yh, out.yl, inst.r) <= 1e-8


def test_golden_exact_solution():
    """Stored 50-digit solution of a tiny instance (written by tests/golden/make_golden.py)."""
    with open(os.path.join(GOLDEN, "tiny_exact.json")) as f:
        g = json.load(f)
    inst = make_instance(g["n"], g["k"], g["m"], g["mu"], g["seed"])
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    F = alg1.factor(C, inst.W, inst.k)
    out = refine.refine(F, inst.r, eps=1e-10)
    yh = np.array(g["y_hi"])
    yl = np.array(g["y_lo"])
    err = np.linalg.norm((out.yh - yh) + (out.yl - yl)) / np.linalg.norm(yh)
    assert err <= 1e-8


@pytest.mark.parametrize("mu", [1e-6, 1e-8])
def test_refinement_at_c1_shape(mu):
    inst = make_instance(100, 2, 1000, mu, seed=1001)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    F = alg1.factor(C, inst.W, inst.k)
    out = refine.refine(F, inst.r, eps=1e-8)
    assert out.relres <= 1e-8
    assert out.outer <= 4
    assert max(out.inner) <= 25
