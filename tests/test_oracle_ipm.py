"""The tiny interior-point method: feasibility, gap, and flat PCG iteration counts."""

import numpy as np
import pytest

from oracle import ipm


def test_tiny_ipm_converges_and_pcg_stays_flat():
    inst = ipm.matcomp_instance(10, 10, 2, 90, seed=5)
    out = ipm.run(inst, tol=1e-9)
    assert out.converged
    assert out.iters <= 40                     # "tens of iterations" (Section 2)
    X, y, S = out.X, out.y, out.S
    n = inst["n"]
    from oracle.alg1 import Constraints
    C = Constraints(n, inst["a"], inst["b"], inst["val"])
    pinf = np.linalg.norm(C.At(X) - inst["bvec"]) / (1 + np.linalg.norm(inst["bvec"]))
    Rd = np.eye(n) - S - C.mat(y).toarray()
    dinf = np.linalg.norm(Rd) / (1 + np.sqrt(n))
    gap = np.sum(X * S) / (1 + abs(np.trace(X)) + abs(inst["bvec"] @ y))
    assert pinf <= 1e-8 and dinf <= 1e-8 and gap <= 1e-8
    assert np.linalg.eigvalsh(X)[0] > 0 and np.linalg.eigvalsh(S)[0] > 0
    # matrix completion recovers M (Section 5.1)
    p = inst["p"]
    err = np.linalg.norm(X[:p, p:] - inst["Mtrue"]) / np.linalg.norm(inst["Mtrue"])
    assert err <= 1e-6
    # rank(X*) = k: the scaling matrix develops the Theta(1/mu) gap of Proposition Weig
    recs = out.records
    late = [r for r in recs if r.mu < 1e-3]
    assert late and min(r.w_gap for r in late) > 10
    # PCG with the paper's preconditioner needs a flat, small iteration count as mu falls,
    # until mu reaches the FP64 floor of an O(1/mu^2)-conditioned system
    flat = [r for r in recs if 1e-6 <= r.mu <= 1.0]
    assert len(flat) >= 5
    assert max(r.pcg_iters for r in flat) <= 25
    # the PCG direction agrees with the dense-Cholesky one while FP64 still resolves it
    assert all(r.dy_rel_diff <= 1e-5 for r in recs if r.mu >= 1e-4)


def test_first_predictor_step_closed_form():
    """At the start X = xi I, S = eta I, y = 0 of the completion SDP (C = I) everything in
    the affine predictor has a closed form: W = sqrt(xi / eta) I, A(diagonal) = 0, and
    distinct sampled entries make H = (xi / eta) (1/2) I, so dy_a = 2 eta b / xi.  With
    B = sum dy_a,i A_i (a bipartite matrix whose eigenvalues are +- the singular values of
    its off-diagonal block, 1/2 dy_a in the sampled places) the iterates along the
    direction are X + t dX_a = xi ((1 - t / eta) I + (t / eta) B) and
    S + t dS_a = (eta + t (1 - eta)) I - t B, so the steps to the boundary, the duality
    measure they reach and sigma = (mu_aff / mu)^3 follow from ||B||_2 and ||B||_F (the
    rule's floor is set below that value here, so the rule decides)."""
    inst = ipm.matcomp_instance(10, 10, 2, 90, seed=5)
    out = ipm.run(inst, tol=1e-9, max_iter=1, sigma=1e-6)
    r = out.records[0]
    n, p, q = inst["n"], inst["p"], inst["q"]
    from oracle.alg1 import Constraints
    C = Constraints(n, inst["a"], inst["b"], inst["val"])
    bv = inst["bvec"]
    xi = max(10.0, np.sqrt(n), n * float(np.max((1 + np.abs(bv)) / (1 + np.sqrt(C.g)))))
    eta = max(10.0, np.sqrt(n), 1.0 + np.sqrt(n))
    dy = 2.0 * eta * bv / xi
    D = np.zeros((p, q))
    D[inst["a"], inst["b"] - p] = 0.5 * dy
    nrm2 = np.linalg.svd(D, compute_uv=False)[0]
    fro2 = 2.0 * np.sum(D * D)
    tp = min(1.0, eta / (1.0 + nrm2))
    den = eta - 1.0 + nrm2
    td = 1.0 if den <= 0 else min(1.0, eta / den)
    xs = xi * ((1.0 - tp / eta) * (eta + td * (1.0 - eta)) * n - (tp * td / eta) * fro2)
    mu = xi * eta
    sigma = min(1.0, (xs / n / mu) ** 3)
    assert r.mu == pytest.approx(mu, rel=1e-14)
    assert r.sigma == pytest.approx(sigma, rel=1e-9), (r.sigma, sigma)
    assert 1e-6 < r.sigma < 0.1
    # with the default floor of 0.1 the same step takes the floor
    assert ipm.run(inst, tol=1e-9, max_iter=1).records[0].sigma == 0.1


def test_fixed_centering_still_available():
    """The fixed rule (sigma = 0.1 every step) is the predictor rule's floor; it too reaches the
    target on the small instance, with sigma recorded as given, and the predictor rule, never
    below it, takes at most one more step to the same X."""
    inst = ipm.matcomp_instance(10, 10, 2, 90, seed=5)
    out = ipm.run(inst, tol=1e-9, predictor=False)
    assert out.converged and all(r.sigma == 0.1 for r in out.records)
    adaptive = ipm.run(inst, tol=1e-9)
    assert adaptive.converged and adaptive.iters <= out.iters + 1
    assert all(r.sigma >= 0.1 for r in adaptive.records)
    assert np.linalg.norm(adaptive.X - out.X) <= 1e-6 * np.linalg.norm(out.X)
