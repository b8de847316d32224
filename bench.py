"""Benchmark: Hessian-equation solves/s on one MI355X (matrix-completion shape n=1000, k=5,
m=20000, the duality-gap path mu = 1e-2, 1e-4, 1e-6, 1e-8).

One step = one pass of the whole hot path over one synthetic batch:
  A0  ingest of the constraint triplets (already in HBM),
  then for each mu of the path: A1-A4 (eigen-split, Z, bold S, its factor and inverse) and
  A5-A8 (PCG with the matrix-free H v and the SMW preconditioner, with double-double
  refinement where mu makes FP64 insufficient), to a true relative residual of 1e-8.
value = solves per second of the mixed-precision path (W0 part of H v in FP32 inside the
double-double refinement, which the small-mu solves need anyway; plain FP64 PCG where FP64
reaches the target); the all-FP64 path is timed the same way and reported beside it, with
p50 / p99 latency per solve.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Hessian-eq PCG solves/s at 1e-8 rel. residual, mixed vs FP64; p50/p99 ms"
N, K, M, SEED = 1000, 5, 20000, 2001
MUS = (1e-2, 1e-4, 1e-6, 1e-8)
HBM_PEAK = 8.0e12          # bytes/s (MI355X HBM3E)
FP64_PEAK = 78.6e12        # flop/s (MI355X FP64, matrix and vector)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving-with-resident-factors stream of the headline line")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--workload", default="mu-path",
                    choices=["mu-path", "batch", "serving", "serving-sessions", "large", "ipm", "hv",
                             "single", "copy-calibration", "augsys"],
                    help="mu-path (default): the headline line; batch: 256 independent "
                         "instances (n in [64, 512], k in 1..4, mu = 1e-6); serving: Poisson "
                         "request stream (n in [200, 3000], k in 1..8, mu in [1e-8, 1e-2]); "
                         "large: n=4000 k=10 m=400000 mu=1e-8; single: one mixed-mode solve "
                         "of the mu=1e-6 instance of the default workload, untimed (for counter "
                         "runs); copy-calibration: a plain device copy of known size, for "
                         "scaling HBM counters")
    ap.add_argument("--count", type=int, default=0, help="instances / requests (batch, serving)")
    ap.add_argument("--qps", type=float, default=4.0, help="serving arrival rate")
    ap.add_argument("--qps-sweep", action="store_true",
                    help="serving: measure capacity, then 0.25x to 1x of it")
    ap.add_argument("--workers", type=int, default=8,
                    help="host worker threads (streams) of the batch and serving workloads")
    ap.add_argument("--summarize-stats", metavar="DIR",
                    help="no GPU: print the top kernels of a rocprofv3 --kernel-trace --stats "
                         "-f csv output folder as a text table")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="no GPU: mean value per dispatch of every counter in rocprofv3 --pmc "
                         "output folders, per kernel")
    ap.add_argument("--summarize-traffic", nargs=4, metavar="DIR",
                    help="no GPU: read four rocprofv3 --pmc output folders (FETCH_SIZE and "
                         "WRITE_SIZE of --workload single, then of --workload "
                         "copy-calibration), print the per-kernel HBM table and write "
                         "profiles/hbm_traffic.json")
    return ap.parse_args()


# kernel class (as profiled by the library) -> (kernel-name prefixes whose launches are class
# launches, further prefixes whose bytes count in the class).  The method's GEMMs are the
# instances with a transposed operand; the explicit-inverse products have none.
TRAFFIC_CLASSES = {
    "gemm": (("k_gemm<true", "k_gemm<false, true"), ()),
    "gemm_inv": (("k_gemm<false, false",), ()),
    "hv": (("k_hv_fused",), ("k_scatter",)), "gemv": (("k_gemv_tri",), ("k_gemv_rect",)),
    "resdd": (("k_residual_dd",), ("k_scatter_dd",)), "bz": (("k_PJ",), ("k_dJL",)),
    "leaf": (("k_chol_leaf",), ()), "tile": (("k_rl_fused", "k_rl_panel"), ()),
}
CLASS_SOURCE = {"gemm": "dense.hip", "gemm_inv": "dense.hip", "hv": "hv.hip",
                "gemv": "dense.hip", "resdd": "hv.hip", "bz": "factor.hip", "leaf": "dense.hip",
                "tile": "dense.hip"}


def summarize_traffic(dirs):
    """HBM bytes per kernel of the second (warm) solve of --workload single, from FETCH_SIZE
    and WRITE_SIZE counter runs, each scaled by what the counter reads for a 1 GiB copy."""
    import csv
    import glob
    import hashlib
    import re

    def rows(d):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        with open(f) as fh:
            out = [(int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"]))
                   for r in csv.DictReader(fh)]
        return sorted(out)

    def short(name):
        name = name.replace("(anonymous namespace)::", "").replace("void ", "")
        return re.sub(r"\(.*", "", name.replace("lrsdp::", ""))

    def warm(rs):  # from the last problem validation on: the second solve
        start = max(i for i, r in enumerate(rs) if short(r[1]) == "k_validate")
        return rs[start:]

    fetch, write = warm(rows(dirs[0])), warm(rows(dirs[1]))
    copy_bytes = float(1 << 30)
    cf = sorted(v for _, _, v in rows(dirs[2]))[-5:]
    cw = sorted(v for _, _, v in rows(dirs[3]))[-5:]
    fscale = copy_bytes / (np.mean(cf) * 1024.0)
    wscale = copy_bytes / (np.mean(cw) * 1024.0)
    per = {}
    for tag, rs, sc in (("f", fetch, fscale), ("w", write, wscale)):
        for _, name, v in rs:
            k = short(name)
            e = per.setdefault(k, {"n": 0, "f": 0.0, "w": 0.0})
            if tag == "f":
                e["n"] += 1
            e[tag] += v * 1024.0 * sc
    print(f"# calibration: a 1 GiB device copy reads FETCH_SIZE {np.mean(cf):.1f} KiB and "
          f"WRITE_SIZE {np.mean(cw):.1f} KiB,")
    print(f"# so fetched bytes = FETCH_SIZE x 1024 x {fscale:.4f} and written bytes = "
          f"WRITE_SIZE x 1024 x {wscale:.4f}")
    print(f"{'kernel':40s} {'launches':>8s} {'fetch_MB':>10s} {'write_MB':>10s} {'MB/launch':>10s}")
    for k, e in sorted(per.items(), key=lambda kv: -(kv[1]["f"] + kv[1]["w"])):
        print(f"{k[:40]:40s} {e['n']:8d} {e['f'] / 1e6:10.2f} {e['w'] / 1e6:10.2f} "
              f"{(e['f'] + e['w']) / 1e6 / max(e['n'], 1):10.3f}")
    classes = {}
    def _m(k, nm):  # a kernel name, any of its template instances, or a template prefix
        return k == nm or k.startswith(nm + "<") or ("<" in nm and k.startswith(nm))

    for cls, (lnames, xnames) in TRAFFIC_CLASSES.items():
        hit = [(k, e) for k, e in per.items() if any(_m(k, nm) for nm in lnames + xnames)]
        launches = sum(e["n"] for k, e in hit if any(_m(k, nm) for nm in lnames))
        if not launches:
            continue
        src = os.path.join(ROOT, "paper_1703_10973_amd", "csrc", CLASS_SOURCE[cls])
        with open(src, "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
        classes[cls] = {
            "launches": launches,
            "fetch_bytes_per_launch": sum(e["f"] for _, e in hit) / launches,
            "write_bytes_per_launch": sum(e["w"] for _, e in hit) / launches,
            "source": CLASS_SOURCE[cls], "source_sha256": sha}
    with open(os.path.join(ROOT, "profiles", "hbm_traffic.json"), "w") as fh:
        json.dump({"fetch_scale": fscale, "write_scale": wscale, "classes": classes}, fh,
                  indent=1)


def summarize_counters(dirs):
    """Mean per-dispatch value of each counter, per kernel, over rocprofv3 --pmc folders."""
    import csv
    import glob
    import re
    per = {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    k = r["Kernel_Name"].replace("(anonymous namespace)::", "").replace("void ", "")
                    k = re.sub(r"\(.*", "", k.replace("lrsdp::", ""))
                    per.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(
                        float(r["Counter_Value"]))
    for k, cs in sorted(per.items()):
        print(k)
        for c, v in sorted(cs.items()):
            print(f"  {c:36s} {np.mean(v):16.1f}   ({len(v)} dispatches)")


def summarize_stats(d, top=30):
    """Top kernels by total time from a rocprofv3 kernel_stats.csv (durations in us)."""
    import csv
    import glob
    import re
    f = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)[0]
    with open(f) as fh:
        rows = list(csv.DictReader(fh))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    print(f"{'kernel':60s} {'calls':>7s} {'total_us':>11s} {'avg_us':>9s} {'min_us':>8s} "
          f"{'max_us':>8s} {'pct':>6s}")
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in rows[:top]:
        nm = r["Name"].replace("(anonymous namespace)::", "").replace("void ", "")
        nm = re.sub(r"\(.*", "", nm.replace("lrsdp::", ""))
        t = float(r["TotalDurationNs"])
        print(f"{nm[:60]:60s} {int(r['Calls']):7d} {t / 1e3:11.1f} "
              f"{float(r['AverageNs']) / 1e3:9.2f} {float(r['MinNs']) / 1e3:8.2f} "
              f"{float(r['MaxNs']) / 1e3:8.2f} {100 * t / tot:6.2f}")
    print(f"# all kernels: {tot / 1e6:.3f} ms in {sum(int(r['Calls']) for r in rows)} dispatches")


def main():
    args = parse()
    if args.summarize_stats:
        return summarize_stats(args.summarize_stats)
    if args.summarize_traffic:
        return summarize_traffic(args.summarize_traffic)
    if args.summarize_counters:
        return summarize_counters(args.summarize_counters)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the per-GPU "
              "shard of this workload is one independent instance stream", file=sys.stderr)
        sys.exit(2)
    if args.workload != "mu-path":
        return {"batch": run_batch, "serving": run_serving, "large": run_large, "ipm": run_ipm,
                "hv": run_hv,
                "serving-sessions": run_serving_sessions, "single": run_single,
                "copy-calibration": run_copy, "augsys": run_augsys}[args.workload](args)
    import torch

    import paper_1703_10973_amd as pk
    from synth import make_instance

    dev = torch.device("cuda", 0)
    insts = [make_instance(N, K, M, mu, SEED) for mu in MUS]
    t = lambda x, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=dev)  # noqa: E731
    con, row, col, val = insts[0].triplets()
    d_con, d_row, d_col, d_val = (t(con, torch.int32), t(row, torch.int32),
                                  t(col, torch.int32), t(val))
    d_W = [t(i.W) for i in insts]
    d_r = t(insts[0].r)
    ctx = pk.Context(0)
    modes = {
        # mixed: FP32 for the W0 part of H v wherever the solve refines in double-double
        # (mu <= ~2e-5); plain FP64 PCG where FP64 alone reaches the target
        "mixed": pk.opts(precision=pk.LRSDP_PREC_AUTO, dd_mode=pk.LRSDP_DD_AUTO),
        "fp64": pk.opts(precision=pk.LRSDP_PREC_FP64, dd_mode=pk.LRSDP_DD_AUTO),
        # the low-precision W0 product at every mu (refinement at every mu, with the residual
        # in double-double), FP32 and BF16 operands with FP32 accumulation
        "fp32_all": pk.opts(precision=pk.LRSDP_PREC_FP32, dd_mode=pk.LRSDP_DD_AUTO),
        "bf16_all": pk.opts(precision=pk.LRSDP_PREC_BF16, dd_mode=pk.LRSDP_DD_AUTO),
    }

    def one_step(opts, keep=False):
        lat, infos, outs = [], [], []
        P = pk.Problem(ctx, N, M, d_con, d_row, d_col, d_val)
        for W in d_W:
            t0 = time.perf_counter()
            F = pk.Factor(P, W, K)
            y, ylo, st, info = F.solve(d_r, opts)
            lat.append((time.perf_counter() - t0) * 1e3)
            info["status"] = st
            infos.append(info)
            if keep:
                outs.append((F, y, ylo))
            else:
                F.close()
        if not keep:
            P.close()
        return lat, infos, outs, P

    # ---- dominant kernel class (one profiled pass, untimed)
    ctx.profile(-1)
    one_step(modes["mixed"])
    prof = ctx.profile_read()
    dom = max(prof, key=lambda k: prof[k]["ms"])
    dom_id = pk.LRSDP_K_NAMES.index(dom)
    ctx.profile(0)

    results = {}
    for name, opts in modes.items():
        for _ in range(args.warmup):
            one_step(opts)
        torch.cuda.synchronize()
        lat_all, infos_all = [], []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            lat, infos, _, _ = one_step(opts)
            lat_all += lat
            infos_all += infos
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        results[name] = dict(elapsed=elapsed, lat=lat_all, infos=infos_all)

    # ---- the dominant kernel class, timed live with HIP events on the library's stream over
    #      a further timed region of the same steps (mixed mode); kept apart from the region
    #      that gives `value` because the events add host work per launch
    hv_id = pk.LRSDP_K_NAMES.index("hv")
    gm_id = pk.LRSDP_K_NAMES.index("gemm")
    gi_id = pk.LRSDP_K_NAMES.index("gemm_inv")
    ctx.profile((1 << dom_id) | (1 << hv_id) | (1 << gm_id) | (1 << gi_id))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(modes["mixed"])
    torch.cuda.synchronize()
    prof_ms_per_step = (time.perf_counter() - t0) / args.steps * 1e3
    pstat = ctx.profile_read()
    dstat, hstat = pstat[dom], pstat["hv"]
    nsolves_prof = args.steps * len(MUS)
    ctx.profile(0)

    # ---- accuracy of the returned answers (untimed): GPU double-double true residual
    # ---- PCG only, with the factors resident (several right-hand sides per W): each kept
    #      factor solves the same right-hand side `reps` times
    checks, pcg_only, answers = {}, {}, {}
    reps = 5
    for name, opts in modes.items():
        _, infos, outs, P = one_step(opts, keep=True)
        rr = []
        for (F, y, ylo) in outs:
            rr.append(F.residual_dd(d_r, y, ylo))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for (F, _, _) in outs:
            for _ in range(reps):
                F.solve(d_r, opts)
        torch.cuda.synchronize()
        pcg_only[name] = len(outs) * reps / (time.perf_counter() - t0)
        if name == "mixed":
            answers = {mu: (y.cpu().numpy(), ylo.cpu().numpy())
                       for mu, (_, y, ylo) in zip(MUS, outs)}
        for (F, _, _) in outs:
            F.close()
        P.close()
        checks[name] = dict(relres=rr, iters=[i["iters"] for i in infos],
                            outer=[i["outer_iters"] for i in infos],
                            status=[i["status"] for i in infos])

    def summ(name):
        r = results[name]
        nsolve = len(r["lat"])
        setup = [i["setup_ms"] for i in r["infos"]]
        solve = [i["solve_ms"] for i in r["infos"]]
        return dict(value=nsolve / r["elapsed"], p50_ms=float(np.percentile(r["lat"], 50)),
                    p99_ms=float(np.percentile(r["lat"], 99)),
                    setup_ms_mean=float(np.mean(setup)), pcg_ms_mean=float(np.mean(solve)),
                    phase_ms_mean=dict(zip(("eig", "split_and_Z", "S_formation", "S_factor"),
                                           np.mean([i["phase_ms"] for i in r["infos"]],
                                                   axis=0).round(4).tolist())),
                    ms_per_step=r["elapsed"] / args.steps * 1e3,
                    relres_max=float(max(checks[name]["relres"])),
                    iters=checks[name]["iters"], outer=checks[name]["outer"],
                    status=checks[name]["status"])

    mixed, fp64 = summ("mixed"), summ("fp64")
    low = {name: summ(name) for name in ("fp32_all", "bf16_all")}

    # ---- roofline of the dominant kernel class, from the events of the timed region.  The
    #      flops are algorithmic: the method's own (bold S formation, the Cholesky's panel
    #      solves and trailing updates, deflation), counted on structurally nonzero operand
    #      entries; the products that form the explicit inverse L^{-1} are a class of their own
    #      and are reported beside it, not counted.
    def mfma_record(st, name):
        n_l = max(st["launches"], 1)
        a_ms = st["ms"] / n_l
        ach = st["flops"] / n_l / (a_ms * 1e-3) / 1e12 if a_ms > 0 else 0.0
        return dict(bound="mfma", achieved=ach, peak=FP64_PEAK / 1e12, unit="TFLOP/s",
                    frac=ach / (FP64_PEAK / 1e12), traffic=None, kernel=name,
                    launches=st["launches"], avg_us=a_ms * 1e3,
                    flops_per_launch=st["flops"] / n_l,
                    flops_per_solve=st["flops"] / nsolves_prof,
                    ms_per_solve=st["ms"] / nsolves_prof)

    avg_ms = dstat["ms"] / max(dstat["launches"], 1)
    if dom in ("gemm", "tile", "gemm_inv", "leaf"):
        roof = mfma_record(dstat, dom)
        roof["profiled_ms_per_step"] = prof_ms_per_step
    else:
        per = dstat["bytes"] / max(dstat["launches"], 1)
        achieved = per / (avg_ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK / 1e9, unit="GB/s",
                    frac=achieved / (HBM_PEAK / 1e9), traffic=None, kernel=dom,
                    launches=dstat["launches"], avg_us=avg_ms * 1e3,
                    profiled_ms_per_step=prof_ms_per_step)

    roof["traffic"] = hbm_traffic(dom)

    # ---- H v (A5/A7) against the HBM roof: its compulsory bytes per launch (W once, the
    #      pattern, and per constraint its owner entry, coefficient and output) over the
    #      event-timed launch duration, in the same timed region
    hv_ms = hstat["ms"] / max(hstat["launches"], 1)
    hv_ach = hstat["bytes"] / max(hstat["launches"], 1) / (hv_ms * 1e-3) / 1e9
    hv_roof = dict(bound="hbm", achieved=hv_ach, peak=HBM_PEAK / 1e9, unit="GB/s",
                   frac=hv_ach / (HBM_PEAK / 1e9), traffic=hbm_traffic("hv"), kernel="hv",
                   launches=hstat["launches"], avg_us=hv_ms * 1e3,
                   bytes_per_launch=hstat["bytes"] / max(hstat["launches"], 1),
                   tflops=hstat["flops"] / max(hstat["ms"], 1e-9) / 1e9)

    # ---- the whole solve against its roofline: setup flops at the FP64 matrix peak plus,
    #      per PCG iteration (inner iterations and outer residual evaluations), the compulsory
    #      bytes of H v, two passes over L^{-1}, Z twice and ~10 m-vectors at the HBM peak
    nnz = 2 * M - N
    nk = N * K
    f_setup = nk ** 3 / 3 + N ** 3 / 3 + K * (K + 1) / 2 * 2 * N ** 3 + 2 * nnz * N * K
    b_hv = 32 * N * N + 24 * M + 20 * nnz
    b_iter = b_hv + 8 * nk * nk + 16 * N * N + 80 * M
    t_roof = [f_setup / FP64_PEAK + (it + out) * b_iter / HBM_PEAK
              for it, out in zip(mixed["iters"], mixed["outer"])]
    t_meas = [i["setup_ms"] + i["solve_ms"] for i in results["mixed"]["infos"]]
    t_meas = [float(np.mean(t_meas[j::len(MUS)])) * 1e-3 for j in range(len(MUS))]
    solve_roof = dict(t_roof_ms=[round(x * 1e3, 4) for x in t_roof],
                      t_measured_ms=[round(x * 1e3, 4) for x in t_meas],
                      frac=float(np.sum(t_roof) / np.sum(t_meas)),
                      setup_flops=f_setup, bytes_per_iter=b_iter)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(insts, args.cpu_seconds, answers)

    # ---- serving with resident factors (the serving configuration's 2000 requests)
    serving = None
    if not args.no_serving:
        try:
            serving = serving_sessions(pk, torch, count=2000, workers=args.workers,
                                       log=lambda x: print(x, file=sys.stderr, flush=True))
        except Exception as e:  # reported, never hides the headline line
            serving = {"error": repr(e)}

    line = {
        "metric": METRIC,
        "value": mixed["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64+dd",
        "data": "synthetic",
        "config": {"workload": "matrix-completion Hessian equation n=1000 k=5 m=20000, "
                               "mu path 1e-2,1e-4,1e-6,1e-8 (A0 + 4 x Alg.1 per step)",
                   "n": N, "k": K, "m": M, "mus": list(MUS), "seed": SEED,
                   "precision": "W0 part of H v in FP32 inside double-double refinement (mu <= 1e-6), "
                                "FP64 PCG elsewhere"},
        "p50_ms": mixed["p50_ms"],
        "p99_ms": mixed["p99_ms"],
        "relres_max": mixed["relres_max"],
        "pcg_iters": mixed["iters"],
        "outer_iters": mixed["outer"],
        "setup_ms_mean": mixed["setup_ms_mean"],
        "setup_phase_ms_mean": mixed["phase_ms_mean"],
        "pcg_ms_mean": mixed["pcg_ms_mean"],
        "fp64": {k: fp64[k] for k in ("value", "p50_ms", "p99_ms", "ms_per_step", "relres_max",
                                      "iters", "outer", "setup_ms_mean", "pcg_ms_mean")},
        "mixed_over_fp64": mixed["value"] / fp64["value"],
        "low_precision_everywhere": {
            name: dict({k: low[name][k] for k in ("value", "p50_ms", "p99_ms", "relres_max",
                                                  "iters", "outer", "pcg_ms_mean")},
                       over_fp64=low[name]["value"] / fp64["value"],
                       pcg_only_over_fp64=pcg_only[name] / pcg_only["fp64"])
            for name in low},
        "pcg_only_solves_per_s": {k: v for k, v in pcg_only.items()},
        "kernel_profile_ms": {k: round(v["ms"], 3) for k, v in prof.items()},
        "roofline": roof,
        "gemm_method_roofline": mfma_record(pstat["gemm"], "gemm"),
        "explicit_inverse_gemm": {k: v for k, v in mfma_record(pstat["gemm_inv"], "gemm_inv").items()
                                  if k in ("launches", "avg_us", "flops_per_solve",
                                           "ms_per_solve", "achieved")},
        "hv_roofline": hv_roof,
        "solve_roofline": solve_roof,
        "cpu_baseline": cpu,
        "serving_resident": serving,
    }
    print(json.dumps(line))


def hbm_traffic(kernel_class):
    """HBM bytes per launch of a kernel class from the committed hardware-counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), or None when the class
    was not measured or its source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)["classes"][kernel_class]
        src = os.path.join(ROOT, "paper_1703_10973_amd", "csrc", rec["source"])
        with open(src, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
                return None
        return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def _device_inputs(inst, torch, dev):
    t = lambda x, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=dev)  # noqa: E731
    con, row, col, val = inst.triplets()
    return dict(n=inst.n, k=inst.k, con=t(con, torch.int32), row=t(row, torch.int32),
                col=t(col, torch.int32), val=t(val), W=t(inst.W), r=t(inst.r),
                y=torch.zeros(inst.m, dtype=torch.float64, device=dev),
                y_lo=torch.zeros(inst.m, dtype=torch.float64, device=dev))


def _sample_residuals(insts, devs, count):
    """The oracle's double-double true residual of a few returned answers (untimed)."""
    from oracle import dd as ddo
    out = []
    for inst, d in list(zip(insts, devs))[:count]:
        yh, yl = d["y"].cpu().numpy(), d["y_lo"].cpu().numpy()
        out.append(ddo.true_relative_residual(inst.W, inst.a, inst.b, inst.val, inst.r, yh, yl)[0])
    return out


def run_batch(args):
    """Batched workload: 256 independent instances, each A0 + Algorithm 1, all inputs
    resident in HBM; value = instances / wall second of one lrsdp_solve_batch call (the median
    of five, the precisions taking turns)."""
    import torch

    import paper_1703_10973_amd as pk
    from synth import batch_instances
    count = args.count or 256
    dev = torch.device("cuda", 0)
    insts = batch_instances(count, base_seed=3000)
    devs = [_device_inputs(i, torch, dev) for i in insts]
    ctx = pk.Context(0)
    # the batched configuration's products are BF16 (FP32 accumulation, residuals in
    # double-double); FP32 operands and plain FP64 run beside it
    modes = {"bf16": pk.opts(precision=pk.LRSDP_PREC_BF16, dd_mode=pk.LRSDP_DD_AUTO),
             "fp32": pk.opts(precision=pk.LRSDP_PREC_FP32, dd_mode=pk.LRSDP_DD_AUTO),
             "fp64": pk.opts(precision=pk.LRSDP_PREC_FP64, dd_mode=pk.LRSDP_DD_AUTO)}
    out = {}
    # warm-up: the same batch once per mode (kernels loaded; the batch's worker contexts keep
    # their memory pools between calls, as a serving loop over interior-point steps would)
    for opts in modes.values():
        pk.solve_batch(ctx, devs, opts, workers=args.workers)
    torch.cuda.synchronize()
    # timed calls, the modes taking turns (so that drift of the box hits them alike); a mode's
    # value is the median call
    reps = 5
    times = {name: [] for name in modes}
    for rep in range(reps):
        for name, opts in modes.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, info = pk.solve_batch(ctx, devs, opts, workers=args.workers)
            torch.cuda.synchronize()
            times[name].append(time.perf_counter() - t0)
            if rep == reps - 1:
                rr = _sample_residuals(insts, devs, 8)
                el = float(np.median(times[name]))
                out[name] = dict(value=count / el, ms_total=el * 1e3,
                                 ms_calls=[round(t * 1e3, 1) for t in times[name]],
                                 statuses_ok=int(sum(1 for x in st if x == 0)),
                                 relres_sampled_max=max(rr),
                                 iters_mean=float(np.mean([i["iters"] for i in info])),
                                 outer_mean=float(np.mean([i["outer_iters"] for i in info])))
    m = out["bf16"]
    print(json.dumps({
        "metric": "batched Hessian-eq solves/s (A0 + Alg.1 each) at 1e-8 rel. residual",
        "value": m["value"], "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
        "ms_total": m["ms_total"], "ms_calls": m["ms_calls"], "workers": args.workers,
        "dtype": "bf16+f32+f64+dd",
        "data": "synthetic", "statuses_ok": m["statuses_ok"],
        "relres_sampled_max": m["relres_sampled_max"], "iters_mean": m["iters_mean"],
        "outer_mean": m["outer_mean"], "fp32": out["fp32"], "fp64": out["fp64"],
        "mixed_over_fp64": m["value"] / out["fp64"]["value"],
        "fp32_over_fp64": out["fp32"]["value"] / out["fp64"]["value"],
        "config": {"workload": f"{count} instances, n log-uniform [64,512], k 1..4, "
                               "m = min(n(n+1)/2, 3nk ln n), mu=1e-6, seeds 3000+",
                   "precision": "W0 part of H v with BF16 operands (FP32 accumulation) inside "
                                "double-double refinement"}}))
    ctx.close()


def _serve_stream(pk, ctx, devs, arrive, opts, workers):
    """Submits request i at arrive[i] seconds after the start and polls until all are done;
    returns the latencies (completion - arrival, ms) and the wall time to the last result."""
    import time as _t
    count = len(devs)
    srv = pk.Server(ctx, workers=workers)
    t0 = _t.perf_counter()
    pending, done_t, lat = {}, {}, {}
    nxt = 0
    while len(done_t) < count:
        now = _t.perf_counter() - t0
        while nxt < count and arrive[nxt] <= now:
            d = devs[nxt]
            pending[srv.submit(d["n"], d["k"], d["con"], d["row"], d["col"], d["val"], d["W"],
                               d["r"], d["y"], d["y_lo"], opts)] = nxt
            nxt += 1
        for tk in list(pending):
            out = srv.poll(tk)
            if out is not None:
                i = pending.pop(tk)
                done_t[i] = _t.perf_counter() - t0
                lat[i] = (done_t[i] - arrive[i]) * 1e3
                assert out[0] == 0, out
        _t.sleep(0.0005)
    srv.close()
    return np.array([lat[i] for i in range(count)]), max(done_t.values())


def run_serving(args):
    """Serving workload: requests arrive as a Poisson stream and are submitted at their
    arrival times; latency = completion - arrival.  Inputs are placed in HBM beforehand.
    With --qps-sweep: capacity first (every request submitted at once), then the stream at
    0.25, 0.5, 0.75 and 1.0 times that rate."""
    import torch

    import paper_1703_10973_amd as pk
    from synth import make_instance, serving_requests
    count = args.count or 48
    dev = torch.device("cuda", 0)
    shapes, arrive = serving_requests(count, base_seed=50000, qps=1.0)  # unit-rate arrivals
    insts = [make_instance(n, k, m, mu, seed=50000 + i) for i, (n, k, m, mu) in enumerate(shapes)]
    devs = [_device_inputs(i, torch, dev) for i in insts]
    ctx = pk.Context(0)
    opts = pk.opts(precision=pk.LRSDP_PREC_AUTO, dd_mode=pk.LRSDP_DD_AUTO)
    torch.cuda.synchronize()
    cfg = {"workload": f"{count} requests, Poisson arrivals, n log-uniform [200,3000], k 1..8, "
                       "m = min(n(n+1)/2, 3nk ln n), mu log-uniform [1e-8,1e-2], seeds 50000+, "
                       "arrivals seed 59999"}
    if args.qps_sweep:
        _, el = _serve_stream(pk, ctx, devs, np.zeros(count), opts, args.workers)
        cap = count / el
        points = []
        for frac in (0.25, 0.5, 0.75, 1.0):
            q = frac * cap
            L, el = _serve_stream(pk, ctx, devs, arrive / q, opts, args.workers)
            points.append(dict(qps=q, load=frac, p50_ms=float(np.percentile(L, 50)),
                               p99_ms=float(np.percentile(L, 99)), solves_per_s=count / el))
            print(f"# qps {q:.2f}: p50 {points[-1]['p50_ms']:.1f} ms, p99 "
                  f"{points[-1]['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
        rr = _sample_residuals(insts, devs, 6)
        print(json.dumps({
            "metric": "serving Hessian-eq solves: latency p50/p99 ms against arrival rate",
            "value": points[-1]["p50_ms"], "unit": "ms (p50 latency at capacity)",
            "n_gpus": 1, "higher_is_better": False, "capacity_solves_per_s": cap,
            "points": points, "requests": count, "workers": args.workers,
            "dtype": "f32+f64+dd", "data": "synthetic", "relres_sampled_max": max(rr),
            "config": cfg}))
        ctx.close()
        return
    L, el = _serve_stream(pk, ctx, devs, arrive / args.qps, opts, args.workers)
    rr = _sample_residuals(insts, devs, 6)
    print(json.dumps({
        "metric": "serving Hessian-eq solves: latency p50/p99 ms at a Poisson arrival rate",
        "value": float(np.percentile(L, 50)), "unit": "ms (p50 latency)", "n_gpus": 1,
        "higher_is_better": False, "p99_ms": float(np.percentile(L, 99)),
        "solves_per_s": count / el, "qps": args.qps, "requests": count,
        "workers": args.workers, "dtype": "f32+f64+dd", "data": "synthetic",
        "relres_sampled_max": max(rr), "config": cfg}))
    ctx.close()


def serving_sessions(pk, torch, count=2000, sessions=32, rhs_per_step=2, qps=None,
                     workers=8, log=None):
    """Serving with resident factors: `count` requests in a Poisson stream over `sessions`
    SDPs of the serving shapes (n log-uniform [200,3000], k 1..8, m = min(n(n+1)/2,
    3nk ln n), mu log-uniform [1e-8,1e-2], seeds 50000+).  Each session keeps its problem and
    current factor resident on the server; its requests are interior-point steps: a factor
    request for the step's W (the session's draws at mu, mu/10, mu/100 in turn, an IPM path)
    followed by `rhs_per_step` solve requests against it.  Returns the capacity run (every
    request submitted at once) and the stream at 0.5 and 0.9 of that capacity, with p50/p99
    latency (completion - arrival) over all requests and over the solve requests."""
    from synth import draw_serving_shape, make_path
    dev = torch.device("cuda", 0)
    t_gen = time.perf_counter()
    sess = []
    for s in range(sessions):
        n, k, m, mu = draw_serving_shape(50000 + s)
        mus = [max(mu * f, 1e-8) for f in (1.0, 1e-1, 1e-2)]
        path = make_path(n, k, m, mus, seed=50000 + s)
        t = lambda x, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=dev)  # noqa: E731
        con, row, col, val = path[0].triplets()
        rng = np.random.default_rng(59000 + s)
        sess.append(dict(n=n, k=k, m=m, insts=path, con=t(con, torch.int32), row=t(row, torch.int32),
                         col=t(col, torch.int32), val=t(val), W=[t(i.W) for i in path],
                         r=[t(rng.standard_normal(m)) for _ in range(rhs_per_step)]))
    gen_s = time.perf_counter() - t_gen
    # the request list: per session, steps of (factor, solve x rhs_per_step), sessions
    # interleaved in a seeded random order that keeps each session's own order
    per = [[] for _ in range(sessions)]
    rng = np.random.default_rng(59999)
    order = rng.integers(0, sessions, size=count)
    for s in order:
        q = per[s]
        step, pos = divmod(len(q), rhs_per_step + 1)
        q.append(("factor", step % 3) if pos == 0 else ("solve", pos - 1))
    reqs = []
    cursor = [0] * sessions
    for s in order:
        reqs.append((int(s),) + per[s][cursor[s]])
        cursor[s] += 1
    opts = pk.opts(precision=pk.LRSDP_PREC_AUTO, dd_mode=pk.LRSDP_DD_AUTO)

    def stream(arrive):
        srv = pk.Server(pk_ctx, workers=workers)
        sid = []
        for d in sess:
            s_id, t_open = srv.open_session(d["n"], d["m"], d["con"], d["row"], d["col"], d["val"])
            sid.append(s_id)
            assert srv.poll(t_open, wait=True)[0] == 0
        outs = [torch.empty(d["m"], dtype=torch.float64, device=dev) for d in sess]
        outl = [torch.empty(d["m"], dtype=torch.float64, device=dev) for d in sess]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pending, lat, kind, nxt = {}, {}, {}, 0
        while len(lat) < len(reqs):
            now = time.perf_counter() - t0
            while nxt < len(reqs) and arrive[nxt] <= now:
                s, what, arg = reqs[nxt]
                d = sess[s]
                if what == "factor":
                    tk = srv.submit_factor(sid[s], d["W"][arg], d["k"], opts)
                else:
                    tk = srv.submit_solve(sid[s], d["r"][arg], outs[s], outl[s], opts)
                pending[tk] = nxt
                kind[nxt] = what
                nxt += 1
            for tk in list(pending):
                out = srv.poll(tk)
                if out is not None:
                    i = pending.pop(tk)
                    lat[i] = (time.perf_counter() - t0 - arrive[i]) * 1e3
                    if out[0] != 0:
                        raise RuntimeError(f"request {i} ({reqs[i]}) failed: {out}")
            time.sleep(0.0002)
        wall = time.perf_counter() - t0
        for s_id in sid:
            srv.poll(srv.close_session(s_id), wait=True)
        srv.close()
        L = np.array([lat[i] for i in range(len(reqs))])
        Ls = np.array([lat[i] for i in range(len(reqs)) if kind[i] == "solve"])
        Lf = np.array([lat[i] for i in range(len(reqs)) if kind[i] == "factor"])
        return dict(requests_per_s=len(reqs) / wall, wall_s=wall,
                    p50_ms=float(np.percentile(L, 50)), p99_ms=float(np.percentile(L, 99)),
                    solve_p50_ms=float(np.percentile(Ls, 50)),
                    solve_p99_ms=float(np.percentile(Ls, 99)),
                    factor_p50_ms=float(np.percentile(Lf, 50)),
                    factor_p99_ms=float(np.percentile(Lf, 99)))

    pk_ctx = pk.Context(0)
    unit = np.cumsum(np.random.default_rng(59998).exponential(1.0, size=len(reqs)))
    unit -= unit[0]
    cap = stream(np.zeros(len(reqs)))
    if log:
        log(f"# serving sessions: capacity {cap['requests_per_s']:.1f} requests/s")
    points = []
    for load in (0.5, 0.9):
        q = load * cap["requests_per_s"] if qps is None else qps
        pt = stream(unit / q)
        pt.update(qps=q, load=load)
        points.append(pt)
        if log:
            log(f"# serving sessions at {q:.1f}/s: p50 {pt['p50_ms']:.1f} ms p99 {pt['p99_ms']:.1f} ms")
    # accuracy of a few answers (untimed): solve again alone and check the oracle's residual
    checks = []
    for d in sess:
        if d["n"] > 600 or len(checks) >= 3:
            continue
        inst = d["insts"][0]
        P = pk.Problem(pk_ctx, d["n"], d["m"], d["con"], d["row"], d["col"], d["val"])
        F = pk.Factor(P, d["W"][0], d["k"], opts)
        y, ylo, st, _ = F.solve(d["r"][0], opts)
        from oracle import dd as ddo
        checks.append(ddo.true_relative_residual(inst.W, inst.a, inst.b, inst.val,
                                                 d["r"][0].cpu().numpy(), y.cpu().numpy(),
                                                 ylo.cpu().numpy())[0])
        F.close()
        P.close()
    pk_ctx.close()
    return dict(requests=len(reqs), sessions=sessions, rhs_per_step=rhs_per_step,
                workers=workers, capacity=cap, points=points,
                relres_sampled_max=max(checks) if checks else None,
                input_generation_s=round(gen_s, 2),
                config="C5 serving shapes as resident sessions: each request is an interior-point "
                       "step (factor of a new W on the resident problem) or a further right-hand "
                       "side against the resident factor; Poisson arrivals, seeds 50000+, "
                       "arrivals 59998/59999")


def run_serving_sessions(args):
    import torch

    import paper_1703_10973_amd as pk
    out = serving_sessions(pk, torch, count=args.count or 2000, workers=args.workers,
                           log=lambda x: print(x, file=sys.stderr, flush=True))
    pt = out["points"][-1]
    print(json.dumps({"metric": "serving with resident factors: requests/s and p50/p99 ms",
                      "value": out["capacity"]["requests_per_s"], "unit": "requests/s",
                      "n_gpus": 1, "higher_is_better": True, "p50_ms": pt["p50_ms"],
                      "p99_ms": pt["p99_ms"], "dtype": "f32+f64+dd", "data": "synthetic",
                      "detail": out}))


def run_ipm(args):
    """The interior-point method on the device (lrsdp_ipm_solve) on random bipartite
    matrix-completion SDPs (Section 5: Omega uniform, M = G1 G2^T Gaussian): the instance of the
    paper's comparison with SVT (p = q = 500, rank 4, m = 20 000) and two of its first problem
    set's shape (m = 25 n, rank 3, n = 2000 and 4000), with the rank estimated from W
    (k_max = 6, eta = 10), the solve tolerance kept in proportion to mu and the centering by
    the predictor rule.  Reports iterations, time per iteration and its parts, the final
    measures and the recovery error of M; the oracle's method (dense Newton solves) is timed
    beside the device on the small instance it can handle."""
    import torch

    import paper_1703_10973_amd as pk
    from oracle import ipm as oipm
    dev = torch.device("cuda", 0)
    ctx = pk.Context(0)
    out = {}
    for (p, k, m, seed) in ((40, 3, 900, 8), (500, 4, 20000, 11), (1000, 3, 50000, 12),
                            (2000, 3, 100000, 13)):
        n = 2 * p
        inst = oipm.matcomp_instance(p, p, k, m, seed)
        t = lambda x, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=dev)  # noqa: E731
        P = pk.Problem(ctx, n, m, t(np.arange(m), torch.int32), t(inst["a"], torch.int32),
                       t(inst["b"], torch.int32), t(inst["val"]))
        b = t(inst["bvec"])
        kw = dict(k=6, rank_eta=10.0, tol=1e-8, pcg_eps=1e-10, pcg_eps_mu=1e-3)
        P.ipm_solve(b, max_iter=2, **kw)  # warm-up (kernels loaded, pools filled)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, y, S, st, info, recs = P.ipm_solve(b, **kw)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        Xh = X.cpu().numpy()
        rec = float(np.linalg.norm(Xh[:p, p:] - inst["Mtrue"]) / np.linalg.norm(inst["Mtrue"]))
        steps = max(1, len(recs))
        row = {"n": n, "m": m, "k_true": k, "status": st, "iters": info["iters"],
               "seconds": el, "ms_per_iter": el * 1e3 / steps,
               "factor_ms_per_iter": float(np.mean([r["factor_ms"] for r in recs])),
               "solve_ms_per_iter": float(np.mean([r["solve_ms"] for r in recs])),
               "scaling_ms_per_iter": float(np.mean([r["scaling_ms"] for r in recs])),
               "rank_ms_per_iter": float(np.mean([r["rank_ms"] for r in recs])),
               "steps_ms_per_iter": float(np.mean([r["steps_ms"] for r in recs])),
               "predictor_ms_per_iter": float(np.mean([r["pred_ms"] for r in recs])),
               "pcg_iters_per_step": [r["pcg_iters"] for r in recs],
               "predictor_pcg_iters_per_step": [r["pred_pcg_iters"] for r in recs],
               "sigma": [round(r["sigma"], 4) for r in recs],
               "k_used": [r["k"] for r in recs],
               "ns_iters": [r["ns_iters"] for r in recs],
               "pinf": info["pinf"], "dinf": info["dinf"], "gap": info["gap"],
               "recovery_rel_err": rec}
        if p == 40:
            t0 = time.perf_counter()
            ref = oipm.run(inst, tol=1e-8)
            row["oracle_seconds"] = time.perf_counter() - t0
            row["oracle_iters"] = ref.iters
            row["oracle_note"] = ("oracle: numpy FP64, dense Hessian and dense Newton solves, "
                                  "plus its own PCG comparison per step")
        out[f"n{n}_m{m}"] = row
        print(f"# ipm n={n} m={m}: {info['iters']} iterations, {el:.2f} s, "
              f"recovery {rec:.1e}", file=sys.stderr)
        P.close()
    big = out["n1000_m20000"]
    print(json.dumps({
        "metric": "interior-point iterations/s on the device (matrix completion, NT scaling, "
                  "Algorithm 1 per Newton system)",
        "value": big["iters"] / big["seconds"], "unit": "iterations/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "f64+dd", "data": "synthetic",
        "config": {"workload": "bipartite matrix completion p=q=500 (n=1000), m=20000, rank 4, "
                               "tol 1e-8 (value); n=2000 m=50000 and n=4000 m=100000 rank 3; "
                               "p=q=40 (n=80), m=900 against the oracle"},
        "detail": out}))
    ctx.close()


def run_large(args):
    """The large configuration n=4000 k=10 m=400000 mu=1e-8: one end-to-end solve (after a
    warm-up solve), with the setup and PCG times the library reports."""
    import torch

    import paper_1703_10973_amd as pk
    from synth import CONFIG_C4, make_instance
    cfg = CONFIG_C4
    dev = torch.device("cuda", 0)
    inst = make_instance(cfg["n"], cfg["k"], cfg["m"], cfg["mu"], seed=cfg["seed"])
    d = _device_inputs(inst, torch, dev)
    ctx = pk.Context(0)
    # FP32 H v inside the FP64 / double-double refinement, as the configuration specifies
    opts = pk.opts(precision=pk.LRSDP_PREC_AUTO, dd_mode=pk.LRSDP_DD_AUTO)
    P = pk.Problem(ctx, inst.n, inst.m, d["con"], d["row"], d["col"], d["val"])
    res = []
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = pk.Factor(P, d["W"], inst.k, opts)
        y, ylo, st, info = F.solve(d["r"], opts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rel = F.residual_dd(d["r"], y, ylo)
        res.append((el, info, st, rel))
        F.close()
    el, info, st, rel = res[-1]
    print(json.dumps({
        "metric": "Hessian-eq solve time (setup + PCG) at 1e-8 rel. residual", "value": el * 1e3,
        "unit": "ms", "n_gpus": 1, "higher_is_better": False, "status": st,
        "setup_ms": info["setup_ms"], "pcg_ms": info["solve_ms"], "iters": info["iters"],
        "outer_iters": info["outer_iters"], "relres": rel,
        "precision": "W0 part of H v in FP32 inside double-double refinement",
        "setup_phase_ms": dict(zip(("eig", "split_and_Z", "S_formation", "S_factor"),
                                   info["phase_ms"])),
        "pcg_ms_per_inner_iter": info["solve_ms"] / max(info["iters"], 1),
        "dtype": "f32+f64+dd", "data": "synthetic",
        "config": {"workload": "n=4000 k=10 m=400000 mu=1e-8 seed 4001"}}))
    P.close()
    ctx.close()


def run_augsys(args):
    """Section 4.1: W~ x = b (W~ = tau I + U U^T) through the augmented system of eq aug_ex on
    the device (LU with partial pivoting), at the headline shape n = 1000, k = 5, over tau from
    1e-2 to 1e-12.  U = V_l (Lambda_l - t)^{1/2} from the top five eigenpairs of the headline
    generator's W at mu = 1e-8 (t the mean of the other eigenvalues); b = U c, the right-hand
    side on which eq wsmf cancels.  value = device solves/s (mean over tau); the backward
    errors ||b - W~ x|| / (||W~|| ||x|| + ||b||) of the device's answers; the cpu_baseline leg
    times the oracle's pivoted solve and gives eq wsmf's backward errors and the device
    answers' forward errors against a 50-digit reference."""
    import torch

    import paper_1703_10973_amd as pk
    from synth import make_instance
    dev = torch.device("cuda", 0)
    inst = make_instance(1000, 5, 20000, 1e-8, seed=2001)
    lam, V = np.linalg.eigh(inst.W)
    n, k = 1000, 5
    t = float(lam[:n - k].mean())
    Ut = (V[:, n - k:] * np.sqrt(lam[n - k:] - t)).T.copy()  # k x n
    b = Ut.T @ np.random.default_rng(2002).standard_normal(k)
    taus = [1e-2, 1e-4, 1e-6, 1e-8, 1e-10, 1e-12]
    ctx = pk.Context(0)
    dUt, db = torch.as_tensor(Ut, device=dev), torch.as_tensor(b, device=dev)
    ms, back, xs = [], [], []
    for tau in taus:
        x = ctx.aug_wtilde_solve(dUt, tau, db)  # warm-up
        torch.cuda.synchronize()
        runs = []
        for _ in range(3):
            t0 = time.perf_counter()
            x = ctx.aug_wtilde_solve(dUt, tau, db)
            torch.cuda.synchronize()
            runs.append(time.perf_counter() - t0)
        ms.append(float(np.median(runs)) * 1e3)
        xh = x.cpu().numpy()
        xs.append(xh)
        W = tau * np.eye(n) + Ut.T @ Ut
        back.append(float(np.linalg.norm(b - W @ xh) /
                          (np.linalg.norm(W, 2) * np.linalg.norm(xh) + np.linalg.norm(b))))
    N = n + k
    bytes_per_solve = 16.0 * (N - 1) * N * (2 * N - 1) / 6.0 + 8.0 * N * N
    mean_ms = float(np.mean(ms))
    line = {
        "metric": "augmented-system solves of W~ x = b (Section 4.1, eq aug_ex) at n=1000 k=5",
        "value": 1e3 / mean_ms, "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f64", "data": "synthetic", "taus": taus, "ms_per_solve": ms,
        "backward_error_device": back,
        "roofline": {"bound": "hbm", "achieved": bytes_per_solve / (mean_ms * 1e-3) / 1e9,
                     "peak": 8000.0, "unit": "GB/s",
                     "frac": bytes_per_solve / (mean_ms * 1e-3) / 1e9 / 8000.0,
                     "traffic": None, "bytes_per_solve": bytes_per_solve,
                     "kernel": "k_aug_update (trailing block read and written per column)"},
        "config": {"workload": "n=1000 k=5, U from the top eigenpairs of the mu=1e-8 headline W, "
                               "b in range(U), tau 1e-2..1e-12"}}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = _augsys_cpu_baseline(Ut, b, taus, xs)
    print(json.dumps(line))
    ctx.close()


def _augsys_cpu_baseline(Ut, b, taus, xs):
    """The oracle's pivoted solve of eq aug_ex (LAPACK LU, host threads) timed over the same taus;
    eq wsmf's backward errors in FP64; the device answers' forward errors against the oracle's
    50-digit answer, beside kappa(W~) u."""
    from oracle import augsys as A
    n = Ut.shape[1]
    total, smw_back, fwd, kw = 0.0, [], [], []
    for tau, x in zip(taus, xs):
        t0 = time.perf_counter()
        A.aug_solve(Ut, tau, b)
        total += time.perf_counter() - t0
        W = A.wtilde(Ut, tau)
        xs_ = A.smw_solve(Ut, tau, b)
        smw_back.append(float(np.linalg.norm(b - W @ xs_) /
                              (np.linalg.norm(W, 2) * np.linalg.norm(xs_) + np.linalg.norm(b))))
        xe = A.exact_solve(Ut, tau, b)
        fwd.append(float(np.linalg.norm(x - xe) / np.linalg.norm(xe)))
        kw.append(A.wtilde_cond(Ut, tau) * np.finfo(np.float64).eps)
    return {"value": len(taus) / total, "unit": "solves/s", "cores": os.cpu_count(),
            "kind": "oracle", "sample": f"the oracle's LU solve of eq aug_ex (n + k = {n + 5}) at "
                                        f"each of the {len(taus)} taus",
            "seconds": total, "smw_backward_error": smw_back,
            "device_forward_error_vs_50_digits": fwd, "kappa_wtilde_times_u": kw}


def run_hv(args):
    """H v of the default workload's mu = 1e-2 instance (n=1000 k=5 m=20000): 20 FP64 products
    with W and 20 split products with the W0 part in FP32 (for counter runs)."""
    import torch

    import paper_1703_10973_amd as pk
    from synth import make_instance
    dev = torch.device("cuda", 0)
    inst = make_instance(N, K, M, MUS[0], SEED)
    d = _device_inputs(inst, torch, dev)
    ctx = pk.Context(0)
    P = pk.Problem(ctx, inst.n, inst.m, d["con"], d["row"], d["col"], d["val"])
    F = pk.Factor(P, d["W"], inst.k)
    v = torch.as_tensor(np.random.default_rng(1).standard_normal(inst.m), device=dev)
    out = torch.empty_like(v)
    for _ in range(20):
        P.hessian_apply(d["W"], v, out)
    for _ in range(20):
        F.hessian_apply_split(v, pk.LRSDP_PREC_FP32)
    torch.cuda.synchronize()
    print(json.dumps({"hv_fp64": 20, "hv_split_fp32": 20}))
    F.close()
    P.close()
    ctx.close()


def run_single(args):
    """One mixed-mode solve (A0 + Algorithm 1) of the mu = 1e-6 instance of the default
    workload, after one warm-up solve; prints its status (for hardware-counter runs)."""
    import torch

    import paper_1703_10973_amd as pk
    from synth import make_instance
    dev = torch.device("cuda", 0)
    inst = make_instance(N, K, M, MUS[2], SEED)
    d = _device_inputs(inst, torch, dev)
    ctx = pk.Context(0)
    opts = pk.opts(precision=pk.LRSDP_PREC_AUTO, dd_mode=pk.LRSDP_DD_AUTO)
    for _ in range(2):
        P = pk.Problem(ctx, inst.n, inst.m, d["con"], d["row"], d["col"], d["val"])
        F = pk.Factor(P, d["W"], inst.k, opts)
        y, ylo, st, info = F.solve(d["r"], opts)
        F.close()
        P.close()
    torch.cuda.synchronize()
    print(json.dumps({"status": st, "iters": info["iters"], "outer_iters": info["outer_iters"]}))
    ctx.close()


def run_copy(args):
    """A plain device copy of 1 GiB, five times (scale reference for HBM byte counters)."""
    import torch
    x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8,
                      "launches": 5}))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_solve(inst):
    """One oracle solve of an instance of the mu path: FP64 Algorithm 1 where FP64 represents
    the answer (mu >= 1e-4), else the double-double refinement (mu <= 1e-6).  Returns the
    answer as one FP64 vector and the wall time."""
    from oracle import alg1, refine
    t0 = time.perf_counter()
    C = alg1.Constraints(inst.n, inst.a, inst.b, inst.val)
    F = alg1.factor(C, inst.W, inst.k, tau_rule="mean")
    if inst.mu >= 1e-4:
        y = alg1.solve(F, inst.r, eps=1e-8).y
    else:
        out = refine.refine(F, inst.r, eps=1e-8)
        y = out.yh + out.yl
    return y, time.perf_counter() - t0


def cpu_baseline(insts, budget_s, answers=None):
    """The oracle on the host CPU, on the same instances as one GPU step: one solve per mu of
    the path (FP64 Algorithm 1 at 1e-2 and 1e-4, the double-double refinement at 1e-6 and
    1e-8), with every host BLAS thread, and a one-thread leg on the FP64 solves.  Also the
    oracle's double-double true residual of the GPU's answers and their distance from the
    oracle's."""
    from oracle import dd as ddo
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_info = threadpool_limits = None
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1]) \
        if threadpool_info else os.cpu_count()
    per_mu, err, gpu_relres = {}, {}, {}
    total = 0.0
    for inst in insts:
        y, el = _oracle_solve(inst)
        total += el
        per_mu[f"{inst.mu:g}"] = round(el, 3)
        if answers and inst.mu in answers:
            yh, yl = answers[inst.mu]
            err[f"{inst.mu:g}"] = float(np.linalg.norm(yh + yl - y) / np.linalg.norm(y))
            if inst.mu <= 1e-6:
                gpu_relres[f"{inst.mu:g}"] = ddo.true_relative_residual(
                    inst.W, inst.a, inst.b, inst.val, inst.r, yh, yl)[0]
    one = None
    if threadpool_limits is not None:
        easy = [i for i in insts if i.mu >= 1e-4]
        with threadpool_limits(limits=1):
            t1 = sum(_oracle_solve(i)[1] for i in easy)
        one = {"value": len(easy) / t1, "unit": "solves/s", "cores": 1,
               "sample": "the FP64 Algorithm-1 solves (mu = 1e-2, 1e-4) only", "seconds": t1}
    return {"value": len(insts) / total, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"one oracle solve (setup + PCG) per mu of the n=1000 k=5 m=20000 path: "
                      f"numpy/scipy FP64 Algorithm 1 at mu=1e-2,1e-4, the double-double "
                      f"refinement at mu=1e-6,1e-8; all host BLAS threads",
            "seconds": total, "seconds_per_mu": per_mu, "cpu_model": _cpu_model(),
            "os_cpu_count": os.cpu_count(), "blas_threads": threads, "one_thread": one,
            "gpu_rel_err_vs_oracle": err, "gpu_true_relres_oracle_dd": gpu_relres}


if __name__ == "__main__":
    main()
