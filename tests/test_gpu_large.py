"""The large configuration (n = 4000, k = 10, m = 400 000, mu = 1e-8): one full solve.

At this size the oracle cannot form H (1.28 TB) or run its double-double residual over all
constraints in test time, so the check is split: the library's double-double residual
r - H (y + y_lo) is compared with the oracle's plain-definition value on sampled constraints
(each one a sparse product in double-double), and the library's full-norm true residual
must then meet the 1e-8 target.
"""

import numpy as np
import pytest
import torch

from oracle import dd as ddo
from oracle import hessian as hs
from synth import CONFIG_C4, make_instance

pytestmark = pytest.mark.gpu

pk = pytest.importorskip("paper_1703_10973_amd")
from gpu_util import host, problem_from, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pk.Context(0)
    yield c
    c.close()


def _sampled_residual(inst, yh, yl, idx):
    """(r - H (yh + yl))_i for the constraints idx, from the closed form
    H_ij = 2 s_i s_j (W_{a_i a_j} W_{b_i b_j} + W_{a_i b_j} W_{b_i a_j}) (A_i = s_i (E_ab + E_ba)),
    every product and sum in double-double."""
    s = hs.half_scale(inst.a, inst.b, inst.val)
    out = []
    for i in idx:
        a, b = inst.a[i], inst.b[i]
        p1h, p1l = ddo.two_prod(inst.W[a, inst.a], inst.W[b, inst.b])
        p2h, p2l = ddo.two_prod(inst.W[a, inst.b], inst.W[b, inst.a])
        hh, hl = ddo.dd_add(p1h, p1l, p2h, p2l)
        hh, hl = ddo.dd_mul_d(hh, hl, s)
        th, tl = ddo.dd_mul(hh, hl, yh, yl)
        sh, sl = ddo.dd_sum_axis1(th[None, :], tl[None, :])
        sh, sl = ddo.dd_mul_d(sh, sl, 2.0 * s[i])
        rh, rl = ddo.dd_add_d(-sh, -sl, inst.r[i])
        out.append(rh[0] + rl[0])
    return np.array(out)


def test_large_config_solve(ctx):
    cfg = CONFIG_C4
    inst = make_instance(cfg["n"], cfg["k"], cfg["m"], cfg["mu"], seed=cfg["seed"])
    P = problem_from(ctx, inst)
    F = pk.Factor(P, to_dev(inst.W), inst.k)
    y, ylo, st, info = F.solve(to_dev(inst.r), pk.opts())
    assert st == 0, info
    assert info["dd_used"]
    res = torch.empty_like(y)
    d_r = to_dev(inst.r)
    rel = pk._lib.lrsdp_residual_dd(F.handle, d_r, y, ylo, res)
    assert rel <= 1e-8, rel
    yh, yl = host(y), host(ylo)
    idx = np.random.default_rng(7).choice(inst.m, 12, replace=False)
    ref = _sampled_residual(inst, yh, yl, idx)
    got = host(res)[idx]
    scale = np.linalg.norm(inst.r) * 1e-12
    assert np.max(np.abs(got - ref)) <= scale, (got, ref)
    F.close()
    P.close()
