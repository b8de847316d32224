"""Edge cases and special cases of the hot path through the C ABI.

* Lambda_s = tau I (every small eigenvalue equal): then W0 = tau I exactly, the preconditioner
  equals H (Section 3.2, eq hessExp2 with W0 = tau I), and PCG needs a single iteration.
* The preconditioner against the dense solve of (tau^2 A^T A + bold U bold U^T) z = v
  (eq AtIUUtAt / SMW2) at mu = 1e-4.
* k = 1 (no null space to deflate), k = 16 (the largest k), only diagonal constraints
  (m = n), sizes that are not multiples of the 64-wide tiles, and the error paths.
"""

import numpy as np
import pytest
import torch

from oracle import alg1, dd as ddo, hessian as hs
from synth import make_instance

pytestmark = pytest.mark.gpu

pk = pytest.importorskip("paper_1703_10973_amd")
from gpu_util import host, problem_from, rel, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pk.Context(0)
    yield c
    c.close()


def _with_spectrum(inst, lam, seed):
    """The same constraints and right-hand side with W = Q diag(lam) Q^T (Q Haar)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((inst.n, inst.n))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    W = (q * lam[None, :]) @ q.T
    inst.W = np.ascontiguousarray(0.5 * (W + W.T))
    return inst


def _solve(ctx, inst, **kw):
    P = problem_from(ctx, inst)
    opts = pk.opts(**kw)
    F = pk.Factor(P, to_dev(inst.W), inst.k, opts)
    y, ylo, st, info = F.solve(to_dev(inst.r), opts)
    return P, F, y, ylo, st, info


def test_equal_small_eigenvalues_one_iteration(ctx):
    inst = make_instance(80, 3, 700, 1e-2, seed=21)
    lam = np.concatenate([np.full(77, 0.02), [1.3, 1.6, 1.9]])
    inst = _with_spectrum(inst, lam, seed=22)
    P, F, y, ylo, st, info = _solve(ctx, inst, dd_mode=pk.LRSDP_DD_OFF)
    assert st == 0, info
    assert info["iters"] <= 2, info          # one in exact arithmetic
    assert abs(info["tau"] - 0.02) <= 1e-12
    H = hs.hessian_dense(inst.W, inst.a, inst.b, inst.val)
    assert rel(host(y), hs.solve_dense(H, inst.r)) <= 1e-8


def test_preconditioner_equals_dense_smw_solve(ctx):
    inst = make_instance(60, 2, 500, 1e-4, seed=23)
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), inst.k)
    ex = F.export(U=True, Z=True)
    # the preconditioner matrix from the oracle's own split with the same tau rule
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    Fo = alg1.factor(C, inst.W, inst.k, tau_rule="mean")
    Hp = alg1.precond_dense(Fo)              # tau^2 A^T A + bold U bold U^T
    v = np.random.default_rng(5).standard_normal(inst.m)
    z_ref = np.linalg.solve(Hp, v)
    z = host(F.precond_apply(to_dev(v)))
    # FP64 with an explicit inverse: a backward-stable-like error, u kappa(H~) times a margin
    assert rel(z, z_ref) <= 50 * np.finfo(float).eps * np.linalg.cond(Hp)
    assert abs(ex["tau"] - Fo.tau) <= 1e-12 * Fo.tau


@pytest.mark.parametrize("n,k,m,mu", [(97, 1, 900, 1e-4), (100, 16, 1500, 1e-2),
                                      (70, 2, 70, 1e-2), (65, 4, 640, 1e-6)])
def test_shapes(ctx, n, k, m, mu):
    inst = make_instance(n, k, m, mu, seed=n + k)
    P, F, y, ylo, st, info = _solve(ctx, inst)
    assert st == 0, info
    yh, yl = host(y), host(ylo)
    r_true, _ = ddo.true_relative_residual(inst.W, inst.a, inst.b, inst.val, inst.r, yh, yl)
    assert r_true <= 1e-8
    if mu >= 1e-4:
        H = hs.hessian_dense(inst.W, inst.a, inst.b, inst.val)
        assert rel(yh + yl, hs.solve_dense(H, inst.r)) <= 1e-6


def test_error_paths(ctx):
    inst = make_instance(40, 2, 200, 1e-2, seed=3)
    P = problem_from(ctx, inst)
    W = to_dev(inst.W)
    for bad_k in (0, 40, 17):
        with pytest.raises(pk.LrsdpError) as e:
            pk.Factor(P, W, bad_k)
        assert e.value.status == pk._lib.LRSDP_ERR_INVALID_ARG
    with pytest.raises(pk.LrsdpError) as e:       # not positive definite
        pk.Factor(P, to_dev(-inst.W), 2)
    assert e.value.status in (pk._lib.LRSDP_ERR_NOT_PD_W, pk._lib.LRSDP_ERR_CHOL_Z)
    with pytest.raises(pk.LrsdpError) as e:       # bad option value
        pk.Factor(P, W, 2, pk.opts(tau_rule=7))
    assert e.value.status == pk._lib.LRSDP_ERR_INVALID_ARG
    F = pk.Factor(P, W, 2)                        # the problem is still usable
    y, ylo, st, info = F.solve(to_dev(inst.r), pk.opts())
    assert st == 0


def test_zero_right_hand_side(ctx):
    inst = make_instance(50, 2, 300, 1e-2, seed=8)
    inst.r = np.zeros(inst.m)
    P, F, y, ylo, st, info = _solve(ctx, inst, dd_mode=pk.LRSDP_DD_OFF)
    assert st == 0
    assert np.all(host(y) == 0.0)


def test_gapless_w_takes_the_householder_fallback(ctx):
    """A scaling matrix with no spectral gap at k (evenly spread eigenvalues, as early
    interior-point iterates have): the subspace iteration of the default tau rule stalls and
    the factor falls back to Householder tridiagonalization, bisection and inverse iteration
    (eig_sweeps == 0).  tau is still the mean of the n - k smallest eigenvalues (Section 3.1),
    the k largest pairs are exact, and the solve matches the dense oracle."""
    inst = make_instance(200, 3, 2500, 1e-2, seed=61)
    lam = np.linspace(1.0, 2.0, 200)
    inst = _with_spectrum(inst, lam, seed=62)
    print("gapless W, n=200 k=3, default tau rule", flush=True)
    P, F, y, ylo, st, info = _solve(ctx, inst, dd_mode=pk.LRSDP_DD_OFF)
    assert st == 0, info
    assert info["eig_sweeps"] == 0, info           # the Householder path ran
    lam_w = np.linalg.eigvalsh(inst.W)
    tau = (np.trace(inst.W) - lam_w[-3:].sum()) / 197
    ex = F.export()
    assert abs(ex["tau"] - tau) <= 1e-12 * tau
    np.testing.assert_allclose(ex["lam"][1:], lam_w[-3:], rtol=1e-12)
    H = hs.hessian_dense(inst.W, inst.a, inst.b, inst.val)
    assert rel(host(y), hs.solve_dense(H, inst.r)) <= 1e-6
    F.close()
    P.close()


def test_mis_sized_arguments_are_refused(ctx):
    inst = make_instance(50, 2, 300, 1e-2, seed=5)
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), inst.k)
    short = torch.zeros(inst.m - 1, dtype=torch.float64, device="cuda")
    good = to_dev(inst.r)
    with pytest.raises(ValueError):
        F.solve(short)
    with pytest.raises(ValueError):
        F.precond_apply(short)
    with pytest.raises(ValueError):
        F.hessian_apply_split(short)
    with pytest.raises(ValueError):
        pk.lrsdp_residual_dd(F.handle, good, short)
    with pytest.raises(ValueError):
        P.hessian_apply(to_dev(inst.W[:49, :49]), good)
    with pytest.raises(ValueError):
        pk.Factor(P, to_dev(inst.W[:, :49]), inst.k)
    F.close()
    P.close()


def test_inputs_written_by_torch_just_before_the_call(ctx):
    """Inputs produced by a torch kernel still in flight on torch's default stream are read
    after it finishes: the context's own stream is ordered after the default stream."""
    inst = make_instance(100, 2, 1000, 1e-4, seed=1001)
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), inst.k)
    v = np.random.default_rng(11).standard_normal(inst.m)
    torch.cuda.synchronize()
    want_z = host(F.precond_apply(to_dev(v)))
    want_y = host(F.solve(to_dev(v), pk.opts(dd_mode=pk.LRSDP_DD_OFF), want_lo=False)[0])
    big = torch.randn(6144, 6144, device="cuda")
    for _ in range(3):
        vd = to_dev(v)
        slow = (big @ big @ big)[0, 0] * 0.0          # a long chain of kernels
        vin = vd + slow.to(torch.float64)             # v again, written after the chain
        got_z = host(F.precond_apply(vin))
        assert np.array_equal(got_z, want_z)
        vin2 = vd * 1.0 + (big @ big)[1, 1].to(torch.float64) * 0.0
        got_y = host(F.solve(vin2, pk.opts(dd_mode=pk.LRSDP_DD_OFF), want_lo=False)[0])
        assert np.array_equal(got_y, want_y)
    F.close()
    P.close()


def test_refactor_reusing_pooled_memory(ctx):
    """nk = 12000: the Cholesky's top-level products are large enough for 128-wide tiles with
    triangular operands.  A second factor of the same W in the same context gets the first
    one's pooled arrays back (L^{-1} with its transpose mirrored into the other triangle);
    the products must not read that triangle, so both solves agree bit for bit."""
    inst = make_instance(2400, 5, 60000, 1e-4, seed=77)
    P = problem_from(ctx, inst)
    out = []
    for rep in range(2):
        print(f"factor nk=12000, repetition {rep}", flush=True)
        F = pk.Factor(P, to_dev(inst.W), inst.k)
        y, _, st, info = F.solve(to_dev(inst.r), pk.opts(dd_mode=pk.LRSDP_DD_OFF), want_lo=False)
        assert st == 0, info
        out.append((host(y), info["iters"]))
        F.close()
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]
    assert out[0][1] <= 25
    P.close()
