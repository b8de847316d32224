"""Handle lifetimes through the C ABI, in a fresh process that must exit cleanly.

The child process creates handles, makes factor creation fail (W not positive definite, an
invalid k), destroys handles parent-first through the raw C calls (the library then defers
the parent's release to its last child), lets a garbage cycle holding a context with its
problem and factor be finalized in whatever order the collector picks, and leaves one
context with children open for the exit hook.  It must print its last line and exit with 0.
"""

import os
import subprocess
import sys
import textwrap

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent("""
    import gc, sys
    sys.path.insert(0, {root!r})
    sys.path.insert(0, {tests!r})
    import numpy as np, torch
    import paper_1703_10973_amd as pk
    from paper_1703_10973_amd import _lib
    from synth import make_instance
    from gpu_util import problem_from, to_dev
    inst = make_instance(60, 2, 400, 1e-2, seed=3)
    print("step 1: failed factor creates", flush=True)
    ctx = pk.Context(0)
    P = problem_from(ctx, inst)
    for bad in (lambda: pk.Factor(P, to_dev(-inst.W), 2), lambda: pk.Factor(P, to_dev(inst.W), 60)):
        try:
            bad()
        except pk.LrsdpError as e:
            keep = sys.exc_info()              # keep the traceback (and its frames) alive
    F = pk.Factor(P, to_dev(inst.W), 2)
    y, _, st, _ = F.solve(to_dev(inst.r), pk.opts(dd_mode=pk.LRSDP_DD_OFF), want_lo=False)
    assert st == 0
    print("step 2: parent-first destroys through the C calls", flush=True)
    c2 = _lib.lrsdp_ctx_create(0)
    con, row, col, val = inst.triplets()
    p2 = _lib.lrsdp_problem_create(c2, inst.n, inst.m, to_dev(con, torch.int32),
                                   to_dev(row, torch.int32), to_dev(col, torch.int32), to_dev(val))
    f2 = _lib.lrsdp_factor_create(p2, to_dev(inst.W), 2)
    _lib.lrsdp_ctx_destroy(c2)                 # deferred: the problem is alive
    _lib.lrsdp_problem_destroy(p2)             # deferred: the factor is alive
    z = torch.empty(inst.m, dtype=torch.float64, device="cuda")
    _lib.lrsdp_precond_apply(f2, to_dev(inst.r), z)   # the factor still works
    _lib.lrsdp_factor_destroy(f2)              # releases the factor, problem and context
    print("step 3: a garbage cycle with a context and its children", flush=True)
    c3 = pk.Context(0)
    P3 = problem_from(c3, inst)
    F3 = pk.Factor(P3, to_dev(inst.W), 2)
    cyc = [c3, P3, F3]
    cyc.append(cyc)
    c3.cycle = cyc
    del c3, P3, F3, cyc
    gc.collect()
    print("step 4: open handles left for the exit hook", flush=True)
    c4 = pk.Context(0)
    P4 = problem_from(c4, inst)
    F4 = pk.Factor(P4, to_dev(inst.W), 2)
    torch.cuda.synchronize()
    print("clean-exit-ok", flush=True)
""")


def test_failed_creates_and_any_destroy_order_exit_cleanly():
    code = CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"))
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       timeout=110)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-3000:]
    assert "clean-exit-ok" in p.stdout, out[-3000:]
