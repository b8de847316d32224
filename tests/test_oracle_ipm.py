"""The tiny interior-point method: feasibility, gap, and flat PCG iteration counts."""

import numpy as np

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
