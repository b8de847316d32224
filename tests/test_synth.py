"""The shared instance generator produces the shapes and spectra it promises."""

import math

import numpy as np

from synth import draw_batch_shape, draw_serving_shape, make_instance


def test_instance_structure():
    inst = make_instance(50, 3, 400, 1e-4, seed=9)
    assert inst.W.shape == (50, 50) and np.array_equal(inst.W, inst.W.T)
    np.testing.assert_allclose(np.linalg.eigvalsh(inst.W), inst.lam, rtol=1e-8, atol=1e-13)
    assert np.all(inst.a <= inst.b)
    assert np.array_equal(inst.a[:50], np.arange(50)) and np.array_equal(inst.b[:50], np.arange(50))
    pairs = set(zip(inst.a.tolist(), inst.b.tolist()))
    assert len(pairs) == inst.m
    off = list(zip(inst.a[50:].tolist(), inst.b[50:].tolist()))
    assert off == sorted(off)
    lam = inst.lam
    assert np.all((lam[:47] >= 1e-4) & (lam[:47] < 2e-4)) and np.all((lam[47:] >= 1) & (lam[47:] < 2))


def test_mu_path_reuses_draws():
    i1 = make_instance(30, 2, 100, 1e-2, seed=4)
    i2 = make_instance(30, 2, 100, 1e-6, seed=4)
    assert np.array_equal(i1.a, i2.a) and np.array_equal(i1.r, i2.r)
    np.testing.assert_allclose(i1.lam[:28] * 1e-4, i2.lam[:28], rtol=1e-12)


def test_batch_and_serving_shapes():
    for s in range(3000, 3020):
        n, k, m, mu = draw_batch_shape(s)
        assert 64 <= n <= 512 and 1 <= k <= 4 and mu == 1e-6
        assert m == min(n * (n + 1) // 2, math.ceil(3 * n * k * math.log(n)))
    for s in range(50000, 50020):
        n, k, m, mu = draw_serving_shape(s)
        assert 200 <= n <= 3000 and 1 <= k <= 8 and 1e-8 <= mu <= 1e-2
        assert n <= m <= n * (n + 1) // 2


def test_make_path_equals_make_instance():
    from synth import make_instance, make_path
    path = make_path(50, 2, 300, (1e-2, 1e-6), seed=17)
    for inst in path:
        ref = make_instance(50, 2, 300, inst.mu, seed=17)
        for f in ("a", "b", "val", "W", "r", "bvec", "lam"):
            assert np.array_equal(getattr(inst, f), getattr(ref, f)), f
