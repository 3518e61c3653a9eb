#!/usr/bin/env python3
"""Benchmark of the TSFCDE time-level solver on one MI355X.

Workload (the configuration the headline metric is quoted on): alpha = 0.7,
beta = 1.8, n = 2^20 interior unknowns, M = 512 time levels on [0,1]x[0,1],
gamma = -(1+t)/2, d_+ = 1+t, d_- = (1+t)/2, manufactured solution
u = t^2 x^2 (1-x)^2 (A0 + A1 x + A2 x^2) with seeded amplitudes; FP64; CGS
stopped at |r_k| <= 1e-10 |g| from a zero initial guess (the plain method).

One step = one whole march of M levels (right-hand side with the history sum
and the preconditioned Krylov solve at every level).  value = levels solved
per second over the timed steps.  Source vectors f(x_i, t_{j+sigma}) for all
levels are built on the device before timing (inputs resident in HBM).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Algorithmic HBM bytes per launch of each kernel class, FP64, for n unknowns
# (reads + writes the kernel must make, counting each vector once):
#   history at level j: reads u^0..u^j (8n(j+1)), writes H (8n)
#   matvec middle pass (k_mid, product mode): reads the N = n complex buffer
#     (16n) and the stored spectrum (16n), writes the buffer (16n): 48n
#   preconditioner middle pass (k_mid, solve mode): the same on N = n/2: 24n
def history_bytes(n, j):
    return 8 * n * (j + 1) + 8 * n if j >= 1 else 0


KCLASS = {"history": 0, "col_passes": 1, "mid_matvec": 2, "cgs_chunks": 3, "mid_precond": 4, "fused_cols": 5}


def build_sources(prob, device):
    import numpy as np
    import torch
    prof, coef = prob.source_profiles()
    P = torch.as_tensor(prof, dtype=torch.float64, device=device)
    Cf = torch.as_tensor(coef, dtype=torch.float64, device=device)
    F = Cf @ P  # (M x 4) @ (4 x n): f(x_i, t_{j+sigma}) for every level
    torch.cuda.synchronize()
    return F


def cpu_baseline(n_full, M_full, budget_s=12.0):
    """Time the CPU oracle (dense LU per level, FP64) on a bounded sample."""
    import numpy as np
    import oracle as O
    import workloads as W
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threads = os.cpu_count()
    n_s = 2048
    prob = W.config_large(n=n_s, M=M_full)
    U = np.zeros((prob.M + 1, n_s))
    U[0] = prob.initial_vector()
    t0 = time.perf_counter()
    levels = 0
    while levels < prob.M and time.perf_counter() - t0 < budget_s:
        U[levels + 1] = O.level_solve(prob, U, levels, prob.source_level(levels))
        levels += 1
    dt = time.perf_counter() - t0
    rate_s = levels / dt
    scale = (n_s / n_full) ** 3  # dense LU is O(n^3) per level
    return {
        "value": rate_s * scale,
        "unit": "level-solves/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"dense-LU oracle, first {levels} levels at n={n_s} (M={M_full} grid), "
                   f"{rate_s:.3f} level-solves/s measured in {dt:.1f}s; value extrapolated to "
                   f"n={n_full} by (n_s/n)^3"),
        "measured_value": rate_s,
        "measured_n": n_s,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--M", type=int, default=512)
    ap.add_argument("--levels", type=int, default=0, help="levels per step (default: all M)")
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--warm-start", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the warm-started forms")
    ap.add_argument("--profile-class", default="mid_matvec", choices=sorted(KCLASS))
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run three plain device copies of MIB MiB (reference for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    import paper_1603_00279_amd as P

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calibration > 0:
        src = torch.rand(args.copy_calibration << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {args.copy_calibration} MiB")
        del src, dst
    prob = W.config_large(n=args.n, M=args.M)
    levels = args.levels if args.levels > 0 else prob.M
    log(f"workload n={prob.n} M={prob.M} levels/step={levels} alpha={prob.alpha} beta={prob.beta}")
    F = build_sources(prob, dev)
    log("sources built")
    s = P.TimeLevelSolver.from_problem(prob, rtol=args.rtol, warm_start=args.warm_start)
    u0 = s.history()[0].clone()
    log(f"plan ready, workspace {s.workspace_bytes / 2**30:.2f} GiB")

    def one_step(stats_out=None):
        s.set_state(0, u0.view(1, -1))
        for j in range(levels):
            st = s.step(F[j])
            if stats_out is not None:
                stats_out.append(st)

    for w in range(args.warmup):
        one_step()
        log(f"warmup step {w + 1}/{args.warmup} done")

    cls = KCLASS[args.profile_class]
    s.profile(cls, True)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_step(stats if k == 0 else None)
        log(f"timed step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launches, kms = s.profile_read(cls)
    s.profile(cls, False)

    total_levels = levels * args.steps
    value = total_levels / elapsed
    iters = [st["iters"] for st in stats]
    n = prob.n
    # roofline of the dominant kernel (HBM-bound; algorithmic bytes per launch)
    if args.profile_class == "history":
        bytes_step = sum(history_bytes(n, j) for j in range(levels))
        per_launch = bytes_step / max(1, levels - 1)
    elif args.profile_class == "mid_matvec":
        per_launch = 48 * n   # buffer in (16n) + spectrum (16n) + buffer out (16n)
    elif args.profile_class == "mid_precond":
        per_launch = 24 * n   # the same on n/2 complex values
    else:
        per_launch = float("nan")
    # launches skipped after convergence exit at once; count the ones that did
    # the work: two products per CGS iteration plus the right-hand side's one
    real = launches
    if args.profile_class == "mid_matvec":
        real = args.steps * (2 * sum(iters) + levels)
    elif args.profile_class == "mid_precond":
        real = args.steps * 2 * sum(iters)
    avg_ms = kms / max(1, real)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if launches else float("nan")
    peak = 8000.0
    out = {
        "metric": "time-level solves/s at N=2^20 to rel-res 1e-10",
        "value": value,
        "unit": "level-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded manufactured solution; no dataset)",
        "config": {"workload": f"single instance n={n}, M={prob.M}, alpha={prob.alpha}, beta={prob.beta}, "
                               f"gamma=-(1+t)/2, d+=1+t, d-=(1+t)/2, zero initial guess, rtol={args.rtol}",
                   "n": n, "M": prob.M, "levels_per_step": levels, "rtol": args.rtol,
                   "warm_start": "previous level" if args.warm_start else "zero"},
        "roofline": {"bound": "hbm", "kernel": args.profile_class, "achieved": achieved, "peak": peak,
                     "unit": "GB/s", "frac": achieved / peak, "traffic": None,
                     "launches": launches, "working_launches": real, "avg_launch_us": 1e3 * avg_ms,
                     "algorithmic_bytes_per_launch": per_launch},
        "cgs_iterations": {"mean": float(np.mean(iters)), "min": int(min(iters)), "max": int(max(iters))},
    }
    # the same march with the warm-started forms (one timed step each)
    if not args.no_forms:
        forms = {}
        for ws, name in ((P.TSFCDE_WS_PREV, "previous_level"), (P.TSFCDE_WS_EXTRAP, "extrapolated")):
            sw = P.TimeLevelSolver.from_problem(prob, rtol=args.rtol, warm_start=ws)
            stw = []
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sw.set_state(0, u0.view(1, -1))
            for j in range(levels):
                stw.append(sw.step(F[j]))
            torch.cuda.synchronize()
            dtw = time.perf_counter() - t1
            forms[name] = {"value": levels / dtw, "unit": "level-solves/s",
                           "cgs_iterations_mean": float(np.mean([st["iters"] for st in stw])),
                           "speedup_vs_plain": (levels / dtw) / value}
            sw.close()
            log(f"form {name}: {levels / dtw:.1f} level-solves/s")
        out["forms"] = forms
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(n, prob.M)
    print(json.dumps(out), flush=True)
    s.close()


if __name__ == "__main__":
    main()
