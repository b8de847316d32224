"""Random matrix-completion-shaped instances of the interior-point Hessian equation.

The paper tests on random matrix-completion SDPs (Section 5.1): the sampled set
Omega is drawn uniformly at random with a given cardinality and the low-rank
ground truth is a product of Gaussian factors.  The Hessian-equation workloads
used here keep that structure but take the symmetric form: every constraint
fixes one entry (a, b), a <= b, of the n x n matrix variable, all n diagonal
entries are fixed, and the scaling matrix W carries the spectrum that
Proposition "Weig" predicts near the end of an interior-point run: k eigenvalues
of order one and n - k eigenvalues of order mu.

Draw order for one seed (fixed, so that every consumer sees the same bits):
  1. Zgen  (n x k)  standard Gaussian        -- ground-truth factor
  2. the m - n off-diagonal pairs a < b, uniform without replacement
  3. the Haar orthogonal Q (QR of a Gaussian n x n, sign of diag(R) fixed)
  4. n - k uniforms U[1,2) for the small eigenvalues (scaled by mu)
  5. k uniforms U[1,2) for the large eigenvalues
  6. r ~ N(0, I_m)
Changing mu alone therefore reproduces every other draw (an "IPM path").

Constraint order: the n diagonal pairs (a ascending) then the off-diagonal
pairs in lexicographic order.  Constraint i is A_i = val_i (e_a e_b^T + e_b e_a^T)
for a != b and A_i = val_i e_a e_a^T for a == b; matrix completion uses
val = 1/2 off the diagonal and val = 1 on it, so that A_i . X = X_ab.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Paper-shaped workloads (sizes and spectra) used by the tests and the benchmark.
CONFIG_C1 = dict(n=100, k=2, m=1000, mu=1e-4, seed=1001)
CONFIG_C2 = dict(n=1000, k=5, m=20000, mus=(1e-2, 1e-4, 1e-6, 1e-8), seed=2001)
CONFIG_C4 = dict(n=4000, k=10, m=400000, mu=1e-8, seed=4001)


@dataclass
class Instance:
    n: int
    k: int
    m: int
    mu: float
    seed: int
    a: np.ndarray            # int32 (m,), row of the fixed entry, a <= b
    b: np.ndarray            # int32 (m,), column of the fixed entry
    val: np.ndarray          # float64 (m,), triplet value of A_i
    W: np.ndarray            # float64 (n, n) symmetric positive definite, C-contiguous
    r: np.ndarray            # float64 (m,) right-hand side
    bvec: np.ndarray         # float64 (m,) matrix-completion data (ZgenZgen^T)_ab
    lam: np.ndarray = field(default=None)  # eigenvalues used to build W (ascending)

    def triplets(self):
        """(con, row, col, val) with row <= col: (A_i)_{row,col} = (A_i)_{col,row} = val."""
        con = np.arange(self.m, dtype=np.int32)
        return con, self.a.copy(), self.b.copy(), self.val.copy()


def _pair_from_linear(t: np.ndarray, n: int):
    """Map linear indices of the strict upper triangle (row-major) to (a, b), a < b."""
    rows = np.arange(n, dtype=np.int64)
    start = rows * (n - 1) - rows * (rows - 1) // 2  # first linear index of row a
    a = np.searchsorted(start, t, side="right") - 1
    b = a + 1 + (t - start[a])
    return a.astype(np.int32), b.astype(np.int32)


def _haar(rng: np.random.Generator, n: int) -> np.ndarray:
    g = rng.standard_normal((n, n))
    q, rr = np.linalg.qr(g)
    d = np.sign(np.diag(rr))
    d[d == 0] = 1.0
    return q * d[None, :]


def make_instance(n: int, k: int, m: int, mu: float, seed: int) -> Instance:
    if not (1 <= k < n):
        raise ValueError("need 1 <= k < n")
    if m < n or m > n * (n + 1) // 2:
        raise ValueError("need n <= m <= n(n+1)/2 (all diagonals are fixed)")
    rng = np.random.default_rng(seed)
    zgen = rng.standard_normal((n, k))
    n_off = m - n
    t = np.sort(rng.choice(n * (n - 1) // 2, size=n_off, replace=False).astype(np.int64))
    a_off, b_off = _pair_from_linear(t, n)
    diag = np.arange(n, dtype=np.int32)
    a = np.concatenate([diag, a_off]).astype(np.int32)
    b = np.concatenate([diag, b_off]).astype(np.int32)
    val = np.where(a == b, 1.0, 0.5)
    q = _haar(rng, n)
    small = mu * rng.uniform(1.0, 2.0, size=n - k)
    large = rng.uniform(1.0, 2.0, size=k)
    lam = np.concatenate([small, large])
    W = (q * lam[None, :]) @ q.T
    W = 0.5 * (W + W.T)
    W = np.ascontiguousarray(W)
    r = rng.standard_normal(m)
    bvec = np.einsum("ij,ij->i", zgen[a], zgen[b])
    return Instance(n=n, k=k, m=m, mu=mu, seed=seed, a=a, b=b, val=val, W=W, r=r,
                    bvec=bvec, lam=np.sort(lam))


def make_path(n: int, k: int, m: int, mus, seed: int):
    """make_instance(n, k, m, mu, seed) for each mu in mus: every draw is shared (the same
    pattern, Q, uniforms and r), so only W changes, as along an interior-point path.  The QR
    of the Haar draw is done once."""
    rng = np.random.default_rng(seed)
    zgen = rng.standard_normal((n, k))
    n_off = m - n
    t = np.sort(rng.choice(n * (n - 1) // 2, size=n_off, replace=False).astype(np.int64))
    a_off, b_off = _pair_from_linear(t, n)
    diag = np.arange(n, dtype=np.int32)
    a = np.concatenate([diag, a_off]).astype(np.int32)
    b = np.concatenate([diag, b_off]).astype(np.int32)
    val = np.where(a == b, 1.0, 0.5)
    q = _haar(rng, n)
    u_small = rng.uniform(1.0, 2.0, size=n - k)
    large = rng.uniform(1.0, 2.0, size=k)
    r = rng.standard_normal(m)
    bvec = np.einsum("ij,ij->i", zgen[a], zgen[b])
    out = []
    for mu in mus:
        lam = np.concatenate([mu * u_small, large])
        W = (q * lam[None, :]) @ q.T
        W = np.ascontiguousarray(0.5 * (W + W.T))
        out.append(Instance(n=n, k=k, m=m, mu=mu, seed=seed, a=a, b=b, val=val, W=W, r=r,
                            bvec=bvec, lam=np.sort(lam)))
    return out


def draw_batch_shape(seed: int):
    """Shape of one instance of the batched workload: n log-uniform in [64, 512],
    k uniform in {1..4}, m = min(n(n+1)/2, ceil(3 n k ln n)), mu = 1e-6."""
    rng = np.random.default_rng(seed)
    n = int(round(math.exp(rng.uniform(math.log(64), math.log(512)))))
    k = int(rng.integers(1, 5))
    m = min(n * (n + 1) // 2, int(math.ceil(3 * n * k * math.log(n))))
    return n, k, max(m, n), 1e-6


def draw_serving_shape(seed: int):
    """Shape of one serving request: n log-uniform in [200, 3000], k uniform in
    {1..8}, m = ceil(3 n k ln n) clamped to n(n+1)/2, mu log-uniform in [1e-8, 1e-2]."""
    rng = np.random.default_rng(seed)
    n = int(round(math.exp(rng.uniform(math.log(200), math.log(3000)))))
    k = int(rng.integers(1, 9))
    m = min(n * (n + 1) // 2, int(math.ceil(3 * n * k * math.log(n))))
    mu = float(math.exp(rng.uniform(math.log(1e-8), math.log(1e-2))))
    return n, k, max(m, n), mu


def batch_instances(count: int = 256, base_seed: int = 3000):
    out = []
    for i in range(count):
        n, k, m, mu = draw_batch_shape(base_seed + i)
        out.append(make_instance(n, k, m, mu, seed=base_seed + i))
    return out


def serving_requests(count: int = 2000, base_seed: int = 50000, qps: float = 10.0,
                     arrival_seed: int = 59999):
    """Shapes and Poisson arrival times (seconds) of a serving stream."""
    rng = np.random.default_rng(arrival_seed)
    gaps = rng.exponential(1.0 / qps, size=count)
    t = np.cumsum(gaps) - gaps[0]
    shapes = [draw_serving_shape(base_seed + i) for i in range(count)]
    return shapes, t
