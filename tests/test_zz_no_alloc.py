"""The allocation-free H v entry point against lrsdp_hessian_apply, through the C ABI.

Two calls in a row on the same device (the second with a smaller problem, so the fixed
scratch array still holds the first call's larger contents), each compared bit for bit with
the allocating entry point on the same inputs and against the oracle's product; a problem
larger than the array is refused before anything runs.
"""

import numpy as np
import pytest
import torch

from oracle import alg1
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


def _one(ctx, inst, seed):
    P = problem_from(ctx, inst)
    v = np.random.default_rng(seed).standard_normal(inst.m)
    W, vd = to_dev(inst.W), to_dev(v)
    h_ref = torch.empty_like(vd)
    pk.lrsdp_hessian_apply(P.handle, W, vd, h_ref)
    h = torch.full_like(vd, float("nan"))
    pk.lrsdp_hessian_apply_noalloc(P.handle, W, vd, h)
    assert np.array_equal(host(h), host(h_ref))
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    assert rel(host(h), alg1.hessian_apply_mf(C, inst.W, v)) <= 1e-12
    P.close()


def test_noalloc_matches_allocating_entry_point_twice(ctx):
    print("no-alloc H v: n=1000 m=20000, then n=150 m=1500", flush=True)
    _one(ctx, make_instance(1000, 5, 20000, 1e-4, seed=2001), seed=1)
    _one(ctx, make_instance(150, 3, 1500, 1e-2, seed=15), seed=2)


def test_noalloc_refuses_what_the_array_cannot_hold(ctx):
    inst = make_instance(2100, 2, 6000, 1e-2, seed=21)      # n >= 2048: rows of T in scratch
    P = problem_from(ctx, inst)
    h = torch.empty(inst.m, dtype=torch.float64, device="cuda")
    with pytest.raises(pk.LrsdpError) as e:
        pk.lrsdp_hessian_apply_noalloc(P.handle, to_dev(inst.W), to_dev(inst.r), h)
    assert e.value.status == pk._lib.LRSDP_ERR_SCRATCH
    P.close()
