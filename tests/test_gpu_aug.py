"""The augmented preconditioner H^ of Section 4.2 (eqs sparse_prec, aug_prec) on the GPU,
through the C ABI, against the oracle (oracle/aug.py: eq aug_prec formed as written and solved
by a sparse LU with partial pivoting).  No double-double SMW pieces are used on this path."""

import numpy as np
import pytest
import torch

from oracle import alg1, aug, dd as ddo, hessian as hs, refine
from synth import make_instance

pytestmark = pytest.mark.gpu

pk = pytest.importorskip("paper_1703_10973_amd")
from gpu_util import host, problem_from, rel, to_dev  # noqa: E402

AUG = dict(precond=1)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pk.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("k,mu", [(2, 1e-4), (3, 1e-8), (1, 1e-2)])
def test_aug_factor_matches_oracle(ctx, k, mu):
    inst = make_instance(90, k, 900, mu, seed=70 + k)
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), k, pk.opts(**AUG))
    ex = F.export(U=True, Sinv=True)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    Fo = aug.aug_factor(C, inst.W, k)
    # tau = (tr W - sum of the k largest) / (n - k) cancels by about lambda_max n / (tau n)
    assert abs(ex["tau"] - Fo.tau) <= 1e-12 * Fo.tau + 1e-15 * np.max(np.abs(inst.W)) * inst.n
    U = host(ex["U"]).T
    np.testing.assert_allclose(U @ U.T, Fo.U @ Fo.U.T, atol=1e-10 * np.max(inst.W))
    # the inverse of tau/2 I + B^T (A^T A)^{-1} B built from the GPU's own U (signs free)
    Sh = aug.trailing_schur(C, U, ex["tau"])
    Sinv = host(ex["Sinv"])
    kap = np.linalg.cond(Sh)
    assert np.linalg.norm(Sinv @ Sh - np.eye(inst.n * k), 2) <= 1e-12 * kap
    with pytest.raises(pk.LrsdpError):          # no Z on this path
        F.export(Z=True)
    with pytest.raises(pk.LrsdpError):          # and no double-double preconditioner
        F.precond_apply(to_dev(inst.r), mode=1)
    F.close()
    P.close()


@pytest.mark.parametrize("mu,tol", [(1e-2, 1e-11), (1e-4, 1e-9), (1e-8, 1e-6)])
def test_aug_precond_matches_oracle(ctx, mu, tol):
    """H^{-1} v (FP64, explicit inverse of the trailing block) against the oracle's pivoted
    sparse LU of eq aug_prec, for a random v and for v in range(B) (where the elimination of
    x cancels most): the error is O(u / mu) for the SMW-form elimination (Section 4.2's
    condition number Theta(1/sqrt(mu)), squared), far from the O(u / mu^2) of eq SMW2."""
    inst = make_instance(100, 2, 1000, mu, seed=1001)
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), inst.k, pk.opts(**AUG))
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    Fo = aug.aug_factor(C, inst.W, inst.k)
    rng = np.random.default_rng(3)
    B = aug.bold_B(C, Fo.U)
    for v in (rng.standard_normal(inst.m), B @ rng.standard_normal(inst.n * inst.k)):
        z = host(F.precond_apply(to_dev(v)))
        zo = Fo.apply(v)
        assert rel(z, zo) <= tol, rel(z, zo)
        assert v @ z > 0
    F.close()
    P.close()


_REFS = {}


@pytest.mark.parametrize("mu", [1e-2, 1e-4, 1e-6, 1e-8])
def test_aug_solve_c1_every_mu(ctx, mu):
    """n = 100, k = 2, m = 1000: the solve with H^ reaches the target true residual (oracle,
    double-double) and the oracle's answer at every mu, with no double-double preconditioner
    pieces; the PCG iteration counts are reported (Lemma aug_prec: about k^2 + O(log))."""
    inst = make_instance(100, 2, 1000, mu, seed=1001)
    P = problem_from(ctx, inst)
    o = pk.opts(precision=pk.LRSDP_PREC_AUTO, **AUG)
    F = pk.Factor(P, to_dev(inst.W), inst.k, o)
    y, ylo, st, info = F.solve(to_dev(inst.r), o)
    assert st == 0, info
    yh, yl = host(y), host(ylo)
    r_true, _ = ddo.true_relative_residual(inst.W, inst.a, inst.b, inst.val, inst.r, yh, yl)
    assert r_true <= 1e-8
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    if mu >= 1e-4:
        ref = hs.solve_dense(hs.hessian_dense(inst.W, inst.a, inst.b, inst.val), inst.r)
    else:
        Fo = aug.aug_factor(C, inst.W, inst.k)
        out = refine.refine(Fo, inst.r, eps=1e-10, precond=Fo.apply)
        ref = out.yh + out.yl
    assert rel(yh + yl, ref) <= 1e-6
    print(f"aug mu={mu:g}: iters={info['iters']} outer={info['outer_iters']} "
          f"true relres={r_true:.2e}", flush=True)
    assert info["iters"] <= (inst.k ** 2 + 40) * max(1, info["outer_iters"])
    F.close()
    P.close()


@pytest.mark.parametrize("k", [1, 3, 7, 12])
def test_aug_every_width(ctx, k):
    """Every column-count width of the reduction kernels (k <= 2, 4, 8, 16) at mu = 1e-6."""
    inst = make_instance(60, k, 600, 1e-6, seed=50 + k)
    P = problem_from(ctx, inst)
    o = pk.opts(**AUG)
    F = pk.Factor(P, to_dev(inst.W), k, o)
    y, ylo, st, info = F.solve(to_dev(inst.r), o)
    assert st == 0, info
    r_true, _ = ddo.true_relative_residual(inst.W, inst.a, inst.b, inst.val, inst.r, host(y),
                                           host(ylo))
    assert r_true <= 1e-8
    F.close()
    P.close()


def test_aug_batch_matches_alone(ctx):
    from synth import batch_instances
    insts = batch_instances(6, base_seed=3100)
    o = pk.opts(precision=pk.LRSDP_PREC_AUTO, **AUG)
    devs = []
    for inst in insts:
        con, row, col, val = inst.triplets()
        d = dict(n=inst.n, k=inst.k, con=to_dev(con, torch.int32), row=to_dev(row, torch.int32),
                 col=to_dev(col, torch.int32), val=to_dev(val), W=to_dev(inst.W), r=to_dev(inst.r),
                 y=torch.zeros(inst.m, dtype=torch.float64, device="cuda"),
                 y_lo=torch.zeros(inst.m, dtype=torch.float64, device="cuda"))
        devs.append(d)
    torch.cuda.synchronize()
    st, info = pk.solve_batch(ctx, devs, o, workers=3)
    assert all(x == 0 for x in st), st
    for inst, d in zip(insts, devs):
        P = problem_from(ctx, inst)
        F = pk.Factor(P, d["W"], inst.k, o)
        y, ylo, s2, _ = F.solve(d["r"], o)
        assert s2 == 0
        assert np.array_equal(host(y), host(d["y"])) and np.array_equal(host(ylo), host(d["y_lo"]))
        F.close()
        P.close()
