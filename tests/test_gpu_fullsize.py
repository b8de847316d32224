"""Full benchmark size (n = 1000, k = 5, m = 20000), in the configuration bench.py times."""

import numpy as np
import pytest
import torch

from oracle import alg1, dd as ddo, refine
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


@pytest.fixture(scope="module")
def problem(ctx):
    inst = make_instance(1000, 5, 20000, 1e-2, seed=2001)
    return problem_from(ctx, inst)


MODES = {"mixed": dict(precision=pk.LRSDP_PREC_AUTO, dd_mode=pk.LRSDP_DD_AUTO),
         "fp32-refined": dict(precision=pk.LRSDP_PREC_FP32, dd_mode=pk.LRSDP_DD_ON),
         "bf16-refined": dict(precision=pk.LRSDP_PREC_BF16, dd_mode=pk.LRSDP_DD_AUTO),
         "fp64": dict(precision=pk.LRSDP_PREC_FP64, dd_mode=pk.LRSDP_DD_AUTO)}


_REFS = {}


def _oracle_reference(inst):
    """The oracle's answer for one mu of the path, computed once per module: FP64 Algorithm 1
    where FP64 represents the answer (mu >= 1e-4), else the double-double refinement with the
    residual from the plain definition (mu <= 1e-6), both to 1e-10."""
    if inst.mu not in _REFS:
        C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
        Fo = alg1.factor(C, inst.W, inst.k, tau_rule="mean")
        if inst.mu >= 1e-4:
            _REFS[inst.mu] = alg1.solve(Fo, inst.r, eps=1e-10).y
        else:
            out = refine.refine(Fo, inst.r, eps=1e-10)
            assert out.relres <= 1e-10
            _REFS[inst.mu] = out.yh + out.yl
    return _REFS[inst.mu]


@pytest.mark.parametrize("mode", ["mixed", "fp32-refined", "bf16-refined", "fp64"])
@pytest.mark.parametrize("mu", [1e-2, 1e-4, 1e-6, 1e-8])
def test_full_size_solve_meets_target(problem, mode, mu):
    """Every mu of the benchmark's path, in each mode the benchmark can run: the oracle's
    double-double true residual of the returned answer (y + y_lo) meets 1e-8 and the answer
    is within 1e-6 of the oracle's."""
    inst = make_instance(1000, 5, 20000, mu, seed=2001)
    print(f"full-size solve mu={mu:g} mode={mode}", flush=True)
    F = pk.Factor(problem, to_dev(inst.W), inst.k)
    y, ylo, st, info = F.solve(to_dev(inst.r), pk.opts(**MODES[mode]))
    assert st == 0, info
    yh, yl = host(y), host(ylo)
    r_true, _ = ddo.true_relative_residual(inst.W, inst.a, inst.b, inst.val, inst.r, yh, yl)
    assert r_true <= 1e-8
    ref = _oracle_reference(inst)
    assert rel(yh + yl, ref) <= 1e-6
    assert info["iters"] <= 25 * max(1, info["outer_iters"])
    F.close()


@pytest.mark.parametrize("mu", [1e-2, 1e-8])
def test_full_size_augmented_preconditioner(problem, mu):
    """The benchmark shape with the augmented preconditioner of Section 4.2 (no Z, no double-
    double SMW pieces): the true residual (oracle, double-double) meets 1e-8 and the answer is
    the oracle's; the iteration counts are printed."""
    inst = make_instance(1000, 5, 20000, mu, seed=2001)
    o = pk.opts(precision=pk.LRSDP_PREC_AUTO, precond=pk.LRSDP_PRECOND_AUG)
    F = pk.Factor(problem, to_dev(inst.W), inst.k, o)
    y, ylo, st, info = F.solve(to_dev(inst.r), o)
    assert st == 0, info
    yh, yl = host(y), host(ylo)
    r_true, _ = ddo.true_relative_residual(inst.W, inst.a, inst.b, inst.val, inst.r, yh, yl)
    assert r_true <= 1e-8
    assert rel(yh + yl, _oracle_reference(inst)) <= 1e-6
    print(f"full-size aug mu={mu:g}: iters={info['iters']} outer={info['outer_iters']} "
          f"setup={info['setup_ms']:.2f} ms solve={info['solve_ms']:.2f} ms", flush=True)
    F.close()


@pytest.mark.parametrize("rule", ["min", "mean"])
def test_full_size_tau_and_top_eigenvalues(problem, rule):
    inst = make_instance(1000, 5, 20000, 1e-6, seed=2001)
    F = pk.Factor(problem, to_dev(inst.W), inst.k,
                  pk.opts(tau_rule={"min": 0, "mean": 1}[rule]))
    ex = F.export(U=True)
    lam = np.linalg.eigvalsh(inst.W)
    tau = lam[0] if rule == "min" else (np.trace(inst.W) - lam[-5:].sum()) / 995
    assert abs(ex["tau"] - tau) <= 1e-12 * tau + 1e-15 * lam[-1] * np.sqrt(1000)
    np.testing.assert_allclose(ex["lam"][1:], lam[-5:], rtol=1e-12)
    # the rows of U span the top invariant subspace: ||W u - u (lam + ...)|| small
    U = host(ex["U"])                                     # k x n
    V = U / np.linalg.norm(U, axis=1, keepdims=True)
    R = V @ inst.W - np.asarray(ex["lam"])[1:, None] * V
    assert np.max(np.linalg.norm(R, axis=1)) <= 1e-11 * lam[-1]
    F.close()
