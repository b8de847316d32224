"""The augmented system of Section 4.1 (eq aug_ex) on the device: lrsdp_aug_wtilde_solve against
the oracle (oracle/augsys.py), an extended-precision reference, and eq wsmf's backward error."""

import numpy as np
import pytest
import torch

from oracle import augsys as A

pytestmark = pytest.mark.gpu

pk = pytest.importorskip("paper_1703_10973_amd")
from gpu_util import host, to_dev  # noqa: E402

U_EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pk.Context(0)
    yield c
    c.close()


def _case(n, k, seed, in_range):
    rng = np.random.default_rng(seed)
    Ut = rng.standard_normal((k, n)) / np.sqrt(n) * np.linspace(3.0, 1.0, k)[:, None]
    b = Ut.T @ rng.standard_normal(k) if in_range else rng.standard_normal(n)
    return Ut, b


def _backward(Ut, tau, b, x):
    W = A.wtilde(Ut, tau)
    return np.linalg.norm(b - W @ x) / (np.linalg.norm(W, 2) * np.linalg.norm(x) +
                                        np.linalg.norm(b))


@pytest.mark.parametrize("in_range", [False, True])
@pytest.mark.parametrize("tau", [1e-2, 1e-6, 1e-10])
def test_aug_solve_backward_stable(ctx, tau, in_range):
    """n = 300, k = 4: the backward error stays at the rounding level for every tau, the
    forward error within kappa(W~) u of the extended-precision answer; where W~ is well
    conditioned (tau = 1e-2) the answer is the oracle's to 1e-12."""
    Ut, b = _case(300, 4, 11, in_range)
    print(f"aug solve n=300 k=4 tau={tau:g} in_range={in_range}", flush=True)
    x = host(ctx.aug_wtilde_solve(to_dev(Ut), tau, to_dev(b)))
    assert _backward(Ut, tau, b, x) <= 64 * U_EPS
    xe = A.exact_solve(Ut, tau, b)
    assert np.linalg.norm(x - xe) <= 100 * A.wtilde_cond(Ut, tau) * U_EPS * np.linalg.norm(xe)
    if tau >= 1e-2:
        xo = A.aug_solve(Ut, tau, b)
        assert np.linalg.norm(x - xo) <= 1e-12 * np.linalg.norm(xo)


def test_aug_solve_against_smw_at_the_headline_shape(ctx):
    """n = 1000, k = 5, tau = 1e-10, b in range(U): the device's augmented solve keeps the
    backward error at the rounding level where eq wsmf (FP64) has lost about u kappa(W~)."""
    Ut, b = _case(1000, 5, 13, True)
    tau = 1e-10
    print("aug solve n=1000 k=5 tau=1e-10", flush=True)
    x = host(ctx.aug_wtilde_solve(to_dev(Ut), tau, to_dev(b)))
    back_aug = _backward(Ut, tau, b, x)
    back_smw = _backward(Ut, tau, b, A.smw_solve(Ut, tau, b))
    assert back_aug <= 64 * U_EPS, back_aug
    assert back_smw >= 1e4 * back_aug and back_smw >= 1e-9, (back_smw, back_aug)


def test_aug_solve_smallest_and_refused(ctx):
    """n = 1, k = 1 (a 2 x 2 system); tau <= 0 and n + k above the limit are refused."""
    Ut = np.array([[2.0]])
    b = np.array([3.0])
    x = host(ctx.aug_wtilde_solve(to_dev(Ut), 0.5, to_dev(b)))
    assert abs(x[0] - 3.0 / 4.5) <= 1e-15
    for tau in (0.0, -1.0):
        with pytest.raises(pk.LrsdpError):
            ctx.aug_wtilde_solve(to_dev(Ut), tau, to_dev(b))
    big = torch.zeros((1, 16384), dtype=torch.float64, device="cuda")
    with pytest.raises(pk.LrsdpError):
        ctx.aug_wtilde_solve(big, 1.0, torch.zeros(16384, dtype=torch.float64, device="cuda"))
