"""HIP path vs the CPU oracle, through the C ABI (steps A0-A8)."""

import numpy as np
import pytest
import torch

from oracle import alg1, dd as ddo, hessian as hs, refine
from synth import make_instance

pytestmark = pytest.mark.gpu

pk = pytest.importorskip("paper_1703_10973_amd")
from gpu_util import DEV, host, problem_from, rel, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pk.Context(0)
    yield c
    c.close()


# ------------------------------------------------------------------ A0 ingest

def test_ingest_pattern_and_errors(ctx):
    inst = make_instance(50, 2, 300, 1e-2, seed=5)
    P = problem_from(ctx, inst)
    n, m, nnz = P.info()
    assert (n, m, nnz) == (50, 300, 50 + 2 * 250)
    con, row, col, val = inst.triplets()
    # duplicate pair
    row2, col2 = row.copy(), col.copy()
    row2[-1], col2[-1] = row[-2], col[-2]
    with pytest.raises(pk.LrsdpError) as e:
        pk.Problem(ctx, 50, 300, to_dev(con, torch.int32), to_dev(row2, torch.int32),
                   to_dev(col2, torch.int32), to_dev(val))
    assert e.value.status == pk._lib.LRSDP_ERR_DUPLICATE_PAIR
    # row > col
    row3, col3 = row.copy(), col.copy()
    row3[-1], col3[-1] = col[-1], row[-1]
    with pytest.raises(pk.LrsdpError) as e:
        pk.Problem(ctx, 50, 300, to_dev(con, torch.int32), to_dev(row3, torch.int32),
                   to_dev(col3, torch.int32), to_dev(val))
    assert e.value.status == pk._lib.LRSDP_ERR_INVALID_ARG
    # a constraint given twice (overlapping supports)
    con4 = con.copy()
    con4[-1] = 0
    with pytest.raises(pk.LrsdpError) as e:
        pk.Problem(ctx, 50, 300, to_dev(con4, torch.int32), to_dev(row, torch.int32),
                   to_dev(col, torch.int32), to_dev(val))
    assert e.value.status == pk._lib.LRSDP_ERR_UNSUPPORTED
    # the context is still usable
    P2 = problem_from(ctx, inst)
    assert P2.info()[2] == nnz


# ------------------------------------------------------------------ A5 H v

@pytest.mark.parametrize("shape", [(100, 2, 1000, 1e-4, 1001), (37, 3, 200, 1e-2, 3)])
def test_hessian_apply_matches_dense(ctx, shape):
    n, k, m, mu, seed = shape
    inst = make_instance(n, k, m, mu, seed)
    P = problem_from(ctx, inst)
    H = hs.hessian_dense(inst.W, inst.a, inst.b, inst.val)
    rng = np.random.default_rng(0)
    for _ in range(3):
        v = rng.standard_normal(m)
        got = host(P.hessian_apply(to_dev(inst.W), to_dev(v)))
        assert rel(got, H @ v) <= 1e-12


def test_hessian_apply_full_size(ctx):
    """The benchmark shape (n = 1000, m = 20000), against the oracle's matrix-free product."""
    inst = make_instance(1000, 5, 20000, 1e-4, seed=2001)
    P = problem_from(ctx, inst)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    v = np.random.default_rng(1).standard_normal(inst.m)
    got = host(P.hessian_apply(to_dev(inst.W), to_dev(v)))
    ref = alg1.hessian_apply_mf(C, inst.W, v)
    assert rel(got, ref) <= 1e-12
    # sampled outputs checked one by one against the closed form of H
    idx = np.random.default_rng(2).choice(inst.m, 40, replace=False)
    s = hs.half_scale(inst.a, inst.b, inst.val)
    W = inst.W
    for i in idx:
        a, b = inst.a[i], inst.b[i]
        row = 2 * s[i] * s * (W[a, inst.a] * W[b, inst.b] + W[a, inst.b] * W[b, inst.a])
        assert abs(got[i] - row @ v) <= 1e-12 * np.abs(row) @ np.abs(v)


# ------------------------------------------------------------------ A1-A4 factor

RULES = {"min": 0, "mean": 1}


def _w0_exact_sample(W, U, W0, count, seed):
    """Max error, in units of the last place, of sampled W0 entries against W - U U^T in
    exact rational arithmetic (W0 is rounded once from double-double)."""
    from fractions import Fraction
    n = W.shape[0]
    rng = np.random.default_rng(seed)
    worst = 0.0
    for _ in range(count):
        i, j = rng.integers(0, n, 2)
        ex = Fraction(W[i, j]) - sum(Fraction(U[i, l]) * Fraction(U[j, l])
                                     for l in range(U.shape[1]))
        err = abs(Fraction(W0[i, j]) - ex)
        ulp = np.spacing(abs(float(ex))) if ex != 0 else np.spacing(0.0)
        worst = max(worst, float(err) / ulp)
    return worst


@pytest.mark.parametrize("rule", ["min", "mean"])
@pytest.mark.parametrize("shape", [(100, 2, 1000, 1e-4, 1001), (64, 3, 600, 1e-2, 9),
                                   (130, 1, 900, 1e-6, 4)])
def test_factor_matches_oracle(ctx, shape, rule):
    n, k, m, mu, seed = shape
    inst = make_instance(n, k, m, mu, seed)
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), k, pk.opts(tau_rule=RULES[rule]))
    ex = F.export(U=True, W0=True, Z=True, Sinv=True)
    C = alg1.Constraints(n, inst.a, inst.b, inst.val)
    Fo = alg1.factor(C, inst.W, k, tau_rule=rule)
    nW = Fo.split.lam[-1]
    # tau: lambda_min, or the mean of the n - k smallest eigenvalues (Section 3.1)
    assert abs(ex["tau"] - Fo.tau) <= 1e-12 * Fo.tau + 1e-15 * nW * np.sqrt(n)
    np.testing.assert_allclose(ex["lam"][1:], Fo.split.lam[n - k:], rtol=1e-12)
    U = host(ex["U"]).T                                  # n x k
    np.testing.assert_allclose(U @ U.T, Fo.split.U @ Fo.split.U.T, atol=1e-10 * nW)
    # W0 = W - U U^T of the GPU's own U, rounded once (property of the split)
    W0 = host(ex["W0"])
    assert _w0_exact_sample(inst.W, U, W0, 60, seed) <= 1.0
    np.testing.assert_allclose(W0, Fo.split.W0, atol=1e-10 * nW)
    Z = host(ex["Z"])
    assert np.max(np.abs(np.triu(Z, 1))) == 0.0
    Zin = 2 * W0 + U @ U.T
    assert np.max(np.abs(Z @ Z.T - Zin)) <= 1e-13 * np.max(np.abs(Zin))
    # bold S^{-1} against the oracle's own (deflated) bold S.  Eigenvector signs are free
    # (U -> U D, D = diag(+-1)), and bold S transforms as (D x I) S (D x I) with the nk
    # index p + n j; align the oracle's signs with the GPU's before comparing.
    Sinv = host(ex["Sinv"])
    if k >= 2:
        assert abs(ex["shift"] - Fo.shift) <= 1e-10 * Fo.shift
    c = np.einsum("pj,pj->j", U, Fo.split.U)
    np.testing.assert_allclose(np.abs(c), np.einsum("pj,pj->j", U, U), rtol=1e-9)
    d = np.repeat(np.sign(c), n)
    So = d[:, None] * Fo.S * d[None, :]
    kap = np.linalg.cond(So)
    resid = np.linalg.norm(Sinv @ So - np.eye(n * k), 2)
    assert resid <= 1e-11 * kap


# ------------------------------------------------------------------ A6 preconditioner

@pytest.mark.parametrize("rule", ["min", "mean"])
@pytest.mark.parametrize("mu", [1e-2, 1e-4])
def test_precond_matches_oracle(ctx, mu, rule):
    """H~^{-1} v (eq SMW2) in all three modes (FP64 with the explicit bold S^{-1}, FP64 with
    one refinement step of t, double-double w and t) against the oracle's double-double
    preconditioner, to the 1e-9 relative error the SMW application admits at mu = 1e-4."""
    inst = make_instance(100, 2, 1000, mu, seed=1001)
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), inst.k, pk.opts(tau_rule=RULES[rule]))
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    Fo = alg1.factor(C, inst.W, inst.k, tau_rule=rule)
    v = np.random.default_rng(3).standard_normal(inst.m)
    zo = refine.dd_precond_apply(Fo, v)
    assert rel(alg1.precond_apply(Fo, v), zo) <= 1e-9      # the oracle's own two forms agree
    for mode in (0, 1, 2):
        z = host(F.precond_apply(to_dev(v), mode=mode))
        assert rel(z, zo) <= 1e-9, (mode, rel(z, zo))


@pytest.mark.parametrize("k", [1, 3, 7, 12])
def test_precond_all_widths_match_oracle(ctx, k):
    """Every column-count width of the reduction kernels (k <= 2, 4, 8, 16), FP64 and
    double-double, against the oracle's preconditioner (Section 3.2, eq SMW2)."""
    inst = make_instance(60, k, 600, 1e-2, seed=40 + k)
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), k, pk.opts(tau_rule=RULES["min"]))
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    Fo = alg1.factor(C, inst.W, k, tau_rule="min")
    v = np.random.default_rng(3).standard_normal(inst.m)
    zo = refine.dd_precond_apply(Fo, v)
    for mode in (0, 1, 2):
        assert rel(host(F.precond_apply(to_dev(v), mode=mode)), zo) <= 1e-9


@pytest.mark.parametrize("k", [1, 3, 7, 12])
def test_precond_dd_where_it_matters(ctx, k):
    """At mu = 1e-8 and v = bold U x (the range where the SMW form cancels), FP64 pieces lose
    about 1e-3 (Section 4's instability), while the double-double w and t keep the answer.
    The GPU's double-double preconditioner is held to 1e-6 of the oracle's; two oracle factors
    that differ only in their eigensolver agree to ~5e-9 here, and a lost low word of w or t
    shows up at the 1e-4..1e-2 level."""
    inst = make_instance(60, k, 600, 1e-8, seed=40 + k)
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), k)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    Fo = alg1.factor(C, inst.W, k, tau_rule="mean")
    x = np.random.default_rng(5).standard_normal(inst.n * k)
    v = alg1._Umul(Fo, x)
    zo = refine.dd_precond_apply(Fo, v)
    z64o = alg1.precond_apply(Fo, v)
    assert rel(z64o, zo) >= 1e-5                # FP64 pieces do lose accuracy here
    zd = host(F.precond_apply(to_dev(v), mode=1))
    assert rel(zd, zo) <= 1e-6, rel(zd, zo)


@pytest.mark.parametrize("k", [7, 12])
def test_refined_solve_wide_k(ctx, k):
    """The double-double refinement (every width of its double-double kernels) reaches the
    target true residual (Algorithm 1 step 3)."""
    inst = make_instance(60, k, 600, 1e-6, seed=50 + k)
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), k)
    y, ylo, st, info = F.solve(to_dev(inst.r), pk.opts(dd_mode=pk.LRSDP_DD_ON))
    assert st == 0, info
    r_true, _ = ddo.true_relative_residual(inst.W, inst.a, inst.b, inst.val, inst.r, host(y),
                                           host(ylo))
    assert r_true <= 1e-8


# ------------------------------------------------------------------ A7 split H v

@pytest.mark.parametrize("mu", [1e-2, 1e-6])
def test_split_hessian_apply(ctx, mu):
    inst = make_instance(100, 2, 1000, mu, seed=1001)
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), inst.k)
    H = hs.hessian_dense(inst.W, inst.a, inst.b, inst.val)
    v = np.random.default_rng(4).standard_normal(inst.m)
    ref = H @ v
    vd = to_dev(v)
    assert rel(host(F.hessian_apply_split(vd, pk.LRSDP_PREC_FP64)), ref) <= 1e-12
    assert rel(host(F.hessian_apply_split(vd, pk.LRSDP_PREC_FP32)), ref) <= 1e-5
    assert rel(host(F.hessian_apply_split(vd, pk.LRSDP_PREC_BF16)), ref) <= 3e-2


# ------------------------------------------------------------------ A8 residual and solve

def test_dd_residual_matches_oracle(ctx):
    inst = make_instance(100, 2, 1000, 1e-6, seed=1001)
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), inst.k)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    out = refine.refine(alg1.factor(C, inst.W, inst.k), inst.r, eps=1e-10)
    for yh, yl in [(out.yh, out.yl), (out.yh, None), (out.yh * (1 + 1e-9), None)]:
        ro, _ = ddo.true_relative_residual(inst.W, inst.a, inst.b, inst.val, inst.r, yh, yl)
        rg = F.residual_dd(to_dev(inst.r), to_dev(yh), None if yl is None else to_dev(yl))
        assert abs(rg - ro) <= 1e-6 * ro + 1e-15


@pytest.mark.parametrize("mu", [1e-2, 1e-4])
def test_solve_fp64(ctx, mu):
    inst = make_instance(100, 2, 1000, mu, seed=1001)
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), inst.k)
    y, ylo, st, info = F.solve(to_dev(inst.r), pk.opts(dd_mode=pk.LRSDP_DD_OFF))
    assert st == 0, info
    assert info["iters"] <= 25
    assert info["eig_sweeps"] > 0          # the default tau rule takes the subspace iteration
    # the setup phases are device time between events inside the setup's wall time
    assert all(t > 0.0 for t in info["phase_ms"]), info["phase_ms"]
    assert sum(info["phase_ms"]) <= info["setup_ms"] * 1.001 + 0.05, info
    y = host(y)
    H = hs.hessian_dense(inst.W, inst.a, inst.b, inst.val)
    ystar = hs.solve_dense(H, inst.r)
    assert rel(y, ystar) <= 1e-6
    r_true, _ = ddo.true_relative_residual(inst.W, inst.a, inst.b, inst.val, inst.r, y)
    assert r_true <= 1e-8


@pytest.mark.parametrize("mu,prec", [(1e-6, 0), (1e-8, 0), (1e-4, 1), (1e-4, 2), (1e-8, 1)])
def test_solve_refined(ctx, mu, prec):
    inst = make_instance(100, 2, 1000, mu, seed=1001)
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), inst.k)
    y, ylo, st, info = F.solve(to_dev(inst.r), pk.opts(dd_mode=pk.LRSDP_DD_ON, precision=prec))
    assert st == 0, info
    yh, yl = host(y), host(ylo)
    r_true, _ = ddo.true_relative_residual(inst.W, inst.a, inst.b, inst.val, inst.r, yh, yl)
    assert r_true <= 1e-8
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    ref = refine.refine(alg1.factor(C, inst.W, inst.k), inst.r, eps=1e-10)
    err = np.linalg.norm((yh - ref.yh) + (yl - ref.yl)) / np.linalg.norm(ref.yh)
    assert err <= 1e-6


def test_inner_tolerance_by_precision(ctx):
    """The refinement's inner PCG stops at 1e-2 with BF16 W0 products by default (inner_eps =
    0), and at a given inner_eps when one is set: both reach the 1e-8 target (the oracle's
    double-double true residual), and the tighter explicit tolerance takes at least as many
    inner iterations per outer step."""
    inst = make_instance(200, 3, 3000, 1e-8, seed=1201)
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), inst.k)
    runs = {}
    for name, ie in (("default", 0.0), ("explicit", 1e-3)):
        o = pk.opts(dd_mode=pk.LRSDP_DD_ON, precision=pk.LRSDP_PREC_BF16, inner_eps=ie)
        y, ylo, st, info = F.solve(to_dev(inst.r), o)
        assert st == 0, (name, info)
        r_true, _ = ddo.true_relative_residual(inst.W, inst.a, inst.b, inst.val, inst.r,
                                               host(y), host(ylo))
        assert r_true <= 1e-8, (name, r_true)
        runs[name] = info["iters"] / max(1, info["outer_iters"])
    assert runs["explicit"] >= runs["default"], runs
    with pytest.raises(pk.LrsdpError):  # a negative tolerance is refused
        F.solve(to_dev(inst.r), pk.opts(inner_eps=-1e-3))
    F.close()
    P.close()


# ------------------------------------------------------------------ large n: T rows outside LDS

def test_hessian_apply_large_n(ctx):
    """n = 2602 (>= 2048): the H v kernels and the double-double residual keep their rows of
    T in global scratch and only rows of W in LDS; the last workgroup covers a partial block.
    FP64 and split FP32 products against the oracle's matrix-free product, and the residual
    r - H (y + y_lo) on sampled constraints against the closed form of H in double-double."""
    from test_gpu_large import _sampled_residual
    inst = make_instance(2602, 3, 30000, 1e-6, seed=2602)
    P = problem_from(ctx, inst)
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(inst.m)
    ref = alg1.hessian_apply_mf(C, inst.W, v)
    assert rel(host(P.hessian_apply(to_dev(inst.W), to_dev(v))), ref) <= 1e-12
    F = pk.Factor(P, to_dev(inst.W), inst.k)
    vd = to_dev(v)
    assert rel(host(F.hessian_apply_split(vd, pk.LRSDP_PREC_FP64)), ref) <= 1e-12
    assert rel(host(F.hessian_apply_split(vd, pk.LRSDP_PREC_FP32)), ref) <= 1e-5
    yh = rng.standard_normal(inst.m)
    yl = yh * 1e-17 * rng.standard_normal(inst.m)
    res = torch.empty(inst.m, dtype=torch.float64, device="cuda")
    pk._lib.lrsdp_residual_dd(F.handle, to_dev(inst.r), to_dev(yh), to_dev(yl), res)
    idx = rng.choice(inst.m, 12, replace=False)
    want = _sampled_residual(inst, yh, yl, idx)
    got = host(res)[idx]
    assert np.max(np.abs(got - want)) <= 1e-12 * np.linalg.norm(inst.r), (got, want)
    F.close()
    P.close()


@pytest.mark.parametrize("precond", ["smw", "aug"])
def test_block_explicit_factor_matches_oracle(ctx, precond):
    """nk = 8400 is above the block-explicit size, and so are both of its blocks (4224 and 4176
    rows): the factor of bold S (or of the augmented trailing block) is kept as a tree whose four
    leaves (2112, 2112, 2112 and 2064 rows) hold explicit inverses, with L below them; the
    leading blocks' L21 are solved over the tree.  The exported inverse (the library then forms
    the full L^{-1}, children before their node), every preconditioner mode and the solve match
    the oracle.  (At this
    size the checks use a random block and the bound kappa <= lambda_max / lambda_min, with
    Gershgorin's bound on lambda_max and a lower bound on the smallest eigenvalue: tau^2 for deflated bold S, tau / 2 for the augmented block.)"""
    from oracle import aug
    inst = make_instance(2100, 4, 24000, 1e-2, seed=17)
    nk = inst.n * inst.k
    P = problem_from(ctx, inst)
    o = pk.opts(precond=1 if precond == "aug" else 0)
    F = pk.Factor(P, to_dev(inst.W), inst.k, o)
    ex = F.export(U=True, Sinv=True)
    U, tau = host(ex["U"]).T, ex["tau"]
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    Sinv = host(ex["Sinv"])
    g = C.g
    v = np.random.default_rng(3).standard_normal(inst.m)
    if precond == "aug":
        S = aug.trailing_schur(C, U, tau)
        lam_min = tau / 2
        B = aug.bold_B(C, U)
        t = np.linalg.solve(S, B.T @ (v / g))
        zo = (v - B @ t) / (tau * tau * g)
    else:
        Fo = alg1.factor(C, inst.W, inst.k, tau_rule="mean")
        c = np.einsum("pj,pj->j", U, Fo.split.U)
        d = np.repeat(np.sign(c), inst.n)
        S = d[:, None] * Fo.S * d[None, :]
        lam_min = tau * tau
        zo = alg1.precond_apply(Fo, v)
    X = np.random.default_rng(4).standard_normal((nk, 4))
    lam_max = np.max(np.abs(S).sum(axis=1))  # Gershgorin: an upper bound
    kap = lam_max / lam_min
    err = np.linalg.norm(Sinv @ (S @ X) - X) / np.linalg.norm(X)
    assert err <= 1e-12 * kap, (err, kap)
    modes = (0,) if precond == "aug" else (0, 1, 2)
    for mode in modes:
        assert rel(host(F.precond_apply(to_dev(v), mode=mode)), zo) <= 1e-10, mode
    y, ylo, st, info = F.solve(to_dev(inst.r), o)
    assert st == 0, info
    r_true, _ = ddo.true_relative_residual(inst.W, inst.a, inst.b, inst.val, inst.r, host(y),
                                           host(ylo))
    assert r_true <= 1e-8
    F.close()
    P.close()
