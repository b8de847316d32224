"""Writes tiny_exact.json: the 50-digit solution of one tiny Hessian equation.

Calls only the oracle (mpmath LU on the trace definition of H) and the shared
instance generator.  Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mp  # noqa: E402
from synth import make_instance  # noqa: E402

SPEC = dict(n=10, k=2, m=30, mu=1e-8, seed=41)

inst = make_instance(**SPEC)
_, y = mp.exact_solve(inst.W, inst.a, inst.b, inst.val, inst.r, dps=50)
hi, lo = mp.to_dd(y)
out = dict(SPEC, y_hi=hi.tolist(), y_lo=lo.tolist(),
           _note="exact solution of H y = r (50 digits, mpmath LU) split into FP64 hi + lo")
with open(os.path.join(HERE, "tiny_exact.json"), "w") as f:
    json.dump(out, f, indent=1)
print("wrote tiny_exact.json")
