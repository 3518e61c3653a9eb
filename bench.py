#!/usr/bin/env python3
"""Benchmark of the TSFCDE time-level solver on one MI355X.

Workload (the configuration the headline metric is quoted on): alpha = 0.7,
beta = 1.8, n = 2^20 interior unknowns, M = 512 time levels on [0,1]x[0,1],
gamma = -(1+t)/2, d_+ = 1+t, d_- = (1+t)/2, manufactured solution
u = t^2 x^2 (1-x)^2 (A0 + A1 x + A2 x^2) with seeded amplitudes; FP64; CGS
stopped at |r_k| <= 1e-10 |g| from a zero initial guess (the plain method).

One step = one whole march of M levels (right-hand side with the history sum
and the preconditioned Krylov solve at every level), run by the library's
tsfcde_solve (a partial march, --levels < M, steps level by level through
tsfcde_step).  value = levels solved
per second over the timed steps.  Source vectors f(x_i, t_{j+sigma}) for all
levels are built on the device before timing (inputs resident in HBM), at
the plan's own nodes and sampling instants.  Every timed level must pass the
library's acceptance test; the line records the largest backward error and
true residual, the restarts and the failed levels, and the script exits
non-zero when a level failed.

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
#   history: one sweep per block of HB levels (reads u^0..u^{b-1}, writes the
#     block's sums) and a catch-up per later level (reads the newest levels of
#     the block and its sum, writes P); see history_bytes
#   matvec middle pass (k_mid, product mode): reads the N = n complex buffer
#     (16n) and the stored spectrum (16n), writes the buffer (16n): 48n
#   preconditioner middle pass (k_mid, solve mode): the same on N = n/2: 24n
HB = 8  # levels per history block (one sweep over the stored levels per block)


def path_bytes(n, M, levels, iters):
    """Algorithmic HBM bytes of one march step, FP64, by the method's byte
    model: a CGS iteration makes two Toeplitz products (three passes over the
    transform: 12 * 8n each), two preconditioner solves (7 * 8n each) and the
    fused vector updates and reductions (14 * 8n), 416n in all; a level adds
    its right-hand side (one product shared with r0, f read, g written:
    14 * 8n) and its share of the history sum (history_bytes)."""
    hist, _ = history_bytes(n, M, levels)
    return 416 * n * sum(iters) + 112 * n * levels + hist


def fused_bytes(n, M, levels, iters):
    """The same march's bytes as the fused power-of-two path moves them: 45
    units of 8n per CGS iteration (ten passes, the vector updates folded into
    them), 20 units per level (right-hand side and acceptance products with
    their epilogues), plus the history."""
    hist, _ = history_bytes(n, M, levels)
    return 360 * n * sum(iters) + 160 * n * levels + hist


def history_bytes(n, M, levels):
    """Algorithmic HBM bytes and launches of the history kernels over levels
    0..levels-1: at a block's first level b the sweep reads u^0..u^{b-1} and
    writes the block's sums; at a later level L of the block the catch-up
    reads u^{b-1}..u^{L-1} and the block sum Q_L and writes P_L."""
    total, launches = 0, 0
    for L in range(1, levels):
        b = 1 + HB * ((L - 1) // HB)
        if L == b:
            total += 8 * n * (b + min(HB, M - b))
        else:
            total += 8 * n * ((L - b + 1) + 2)
        launches += 1
    return total, launches


KCLASS = {"history": 0, "col_passes": 1, "mid_matvec": 2, "cgs_chunks": 3, "mid_precond": 4, "fused_cols": 5}


def build_sources(prob, solver):
    """f at the plan's nodes x_i and instants t_{j+sigma} for every level: one
    (M x 4) @ (4 x n) product of the manufactured source's separable form."""
    import torch
    import workloads as W
    F = W.device_sources(prob, solver.nodes(), solver.level_times(), solver.device)
    torch.cuda.synchronize()
    return F


def acceptance(stats):
    """Acceptance summary of per-level stats (a list of records, or a numpy
    structured array with a status field): the largest backward error and
    true residual met, total restarts, failed levels."""
    if hasattr(stats, "dtype"):
        import numpy as np
        st = stats.reshape(-1)
        bw, tr = st["backward_err"], st["relres_true"]
        bw, tr = bw[bw >= 0], tr[tr >= 0]
        return {"levels": int(st.size), "failed_levels": int(np.count_nonzero(st["status"] != 0)),
                "max_backward_err": float(bw.max()) if bw.size else None,
                "max_relres_true": float(tr.max()) if tr.size else None, "restarts": int(st["restarts"].sum())}
    bw = [st["backward_err"] for st in stats if st["backward_err"] >= 0]
    tr = [st["relres_true"] for st in stats if st["relres_true"] >= 0]
    return {"levels": len(stats), "failed_levels": sum(1 for st in stats if (st["code"] if "code" in st else st["status"]) != 0),
            "max_backward_err": max(bw) if bw else None, "max_relres_true": max(tr) if tr else None,
            "restarts": sum(st["restarts"] for st in stats)}


def committed_traffic(kclass, n):
    """HBM bytes per launch of the profiled kernel from the committed counter
    summary (FETCH_SIZE / WRITE_SIZE scaled by a plain copy), if there is one
    for this kernel and size."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kclass}_n{n}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    return {"bytes_per_launch": d["fetch_bytes"] + d["write_bytes"], "source": os.path.relpath(path, ROOT)}


def timed_march(solver, F, u0, levels, torch):
    """Wall time and per-level stats of one march from level 0."""
    solver.set_state(0, u0.view(1, -1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [solver.step(F[j], raise_on_error=False) for j in range(levels)]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, stats


def forms(args, P, W, prob, F, u0, levels, plain_value, dev):
    """The other forms, each beside the plain FP64 path on its own workload."""
    import numpy as np
    import torch
    res = {}
    if args.form in ("all", "warm"):
        warm_forms(args, P, prob, F, u0, levels, plain_value, res)
    if args.form in ("all", "fp32"):
        fp32_forms(args, P, W, prob, F, u0, levels, plain_value, dev, res)
    if args.form in ("all", "batched"):
        res["batched"] = batched_form(args, P, W, dev)
    if args.form in ("all", "learned"):
        res["learned"] = learned_form(args, P, W, dev)
    if args.form in ("all", "krylov"):
        res["krylov"] = krylov_forms(args, P, prob, F, u0, levels, plain_value)
    if args.form in ("all", "gsf"):
        res["constant_gsf"] = gsf_form(args, P, W, dev)
    if args.form in ("all", "history"):
        res["fast_history"] = history_form(args, P, prob, F, u0, levels, plain_value)
    if args.form in ("all", "2d"):
        res["two_dimensional"] = nd_form(args, P, W, dev, 2)
    if args.form in ("all", "3d"):
        res["three_dimensional"] = nd_form(args, P, W, dev, 3)
    return res


def path_bytes_nd(d, N, levels, iters, restarts=0):
    """Algorithmic HBM bytes of a march of ``levels`` levels of the d-axis
    solver (d = 2, 3) on N unknowns, FP64, as its kernels move them (units of
    8N).  A CGS iteration: the first preconditioner solve (fast-axis forward
    pass with the u/p update: r, q, p in, u, p and the half spectrum out, 6;
    then 2 per further pass: the middle axis twice in 3D, the division pass,
    the inverse fast-axis pass), the product (fast axis 2, middle axis 3, the
    slow axis with rt.vhat 4), the second solve (forward pass with the q
    update: u, vhat in, q and the spectrum out, 4; then as before, its last
    pass also updating x: 2 more) and the product with the r update (slow
    axis: uhat, w, rt, r in, r out, 5): 33 units in 2D, 47 in 3D.  A level
    adds its right-hand side and one acceptance check per (re)start
    (products of 3d - 1 units each, the right-hand side kernel 6, the zero
    guess 1, the residual 5) and the history (j + 2 units at level j >= 1,
    the whole sum; the blocked sum moves fewer)."""
    per_iter = {2: 33, 3: 47}[d]
    hist = sum(j + 2 for j in range(1, levels))
    prod = 3 * d - 1
    return 8 * N * (per_iter * sum(iters) + (prod + 7) * levels + (prod + 5) * (levels + restarts) + hist)


ND_FORMS = {2: dict(ns=(1024, 1024), M=32), 3: dict(ns=(256, 256, 256), M=8)}
# the largest grid of each family measured beside it (zero guess, a few levels)
ND_LARGE = {2: dict(ns=(2048, 2048), M=4), 3: dict(ns=(512, 512, 512), M=2)}


def nd_large(args, P, W, dev, d):
    """One march of the d-axis solver on its largest measured grid (2D:
    2048^2 = 2^22 unknowns, 3D: 512^3 = 2^27, 1 GiB per vector, well beyond
    the Infinity Cache) after a warm-up march: level-solves/s, the time per
    CGS iteration and the byte-model rate."""
    import numpy as np
    import torch
    cfg = ND_LARGE[d]
    ns, M = cfg["ns"], cfg["M"]
    prob = W.problem_2d(*ns, M) if d == 2 else W.problem_3d(*ns, M)
    Solver = P.TimeLevelSolver2D if d == 2 else P.TimeLevelSolver3D
    src = W.device_sources_2d if d == 2 else W.device_sources_3d
    N = int(np.prod(ns))
    with Solver.from_problem(prob, rtol=args.rtol) as sv:
        F = src(prob, *sv.nodes(), sv.level_times(), dev)
        u0 = sv.history()[0].clone()
        dts = []
        for _ in range(2):  # the first march warms up
            sv.set_state(0, u0.view((1,) + tuple(ns)))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            code, st = sv.solve(F, raise_on_error=False)
            torch.cuda.synchronize()
            dts.append(time.perf_counter() - t0)
        del F
    dt = dts[-1]
    iters = [int(q["iters"]) for q in st]
    nbytes = path_bytes_nd(d, N, M, iters, int(sum(int(q["restarts"]) for q in st)))
    out = {"workload": f"{'x'.join(str(n) for n in ns)}, M={M}, zero guess", "value": M / dt,
           "unit": "level-solves/s", "code": int(code), "cgs_iterations_mean": float(np.mean(iters)),
           "ms_per_cgs_iteration": 1e3 * dt / max(1, sum(iters)),
           "path_roofline": {"bound": "hbm", "achieved": nbytes / dt / 1e9, "peak": 8000.0, "unit": "GB/s",
                             "frac": nbytes / dt / 1e9 / 8000.0},
           "acceptance": acceptance(st)}
    log(f"form {d}d at {out['workload']}: {out['value']:.2f} level-solves/s, {out['ms_per_cgs_iteration']:.3f} ms "
        f"per CGS iteration, {out['path_roofline']['achieved']:.0f} GB/s by the byte model")
    return out


def nd_form(args, P, W, dev, d):
    """The d-axis extension (d = 2: nx = ny = 1024, N = 2^20 unknowns, the
    headline's count, M = 32; d = 3: 256^3, N = 2^24, M = 8) on its seeded
    family (alpha = 0.6, one order per axis), zero initial guess, rtol as
    the headline; sources on the device before timing.  Two timed marches
    after a warm-up march; the faster counts.  The same with the quadratic
    extrapolation as each level's initial guess, and (2D) one march of the
    headline's M = 512 levels with that guess.  At 2^20 unknowns the working
    set (about 20 vectors of 8 MiB) fits in the 256 MiB Infinity Cache, so the
    byte rate is not bounded by HBM; at 2^24 it is."""
    import numpy as np
    import torch
    cfg = ND_FORMS[d]
    ns, M = cfg["ns"], cfg["M"]
    if d == 2:
        prob = W.problem_2d(*ns, M)
        Solver, src = P.TimeLevelSolver2D, W.device_sources_2d
    else:
        prob = W.problem_3d(*ns, M)
        Solver, src = P.TimeLevelSolver3D, W.device_sources_3d
    N = int(np.prod(ns))
    F = None

    def run(warm):
        nonlocal F
        with Solver.from_problem(prob, rtol=args.rtol, warm_start=warm) as sv:
            if F is None:
                F = src(prob, *sv.nodes(), sv.level_times(), dev)
            u0 = sv.history()[0].clone()
            dts, st, code = [], None, 0
            for _ in range(3):  # the first march warms up
                sv.set_state(0, u0.view((1,) + tuple(ns)))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                code, st = sv.solve(F, raise_on_error=False)
                torch.cuda.synchronize()
                dts.append(time.perf_counter() - t0)
        return min(dts[1:]), st, code

    dt, st, code = run(P.TSFCDE_WS_ZERO)
    dtx, stx, codex = run(P.TSFCDE_WS_EXTRAP)
    del F
    long = None
    if d == 2:
        # the headline's M = 512 levels (tau = 1/512, history sums over up to
        # 512 levels, blocked), extrapolated guess: one timed march
        probl = W.problem_2d(*ns, 512)
        with Solver.from_problem(probl, rtol=args.rtol, warm_start=P.TSFCDE_WS_EXTRAP) as sv:
            Fl = src(probl, *sv.nodes(), sv.level_times(), dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            codel, stl = sv.solve(Fl, raise_on_error=False)
            torch.cuda.synchronize()
            dtl = time.perf_counter() - t0
            del Fl
        long = {"workload": f"{'x'.join(str(n) for n in ns)}, M=512, extrapolated guess", "value": 512 / dtl,
                "unit": "level-solves/s", "code": int(codel),
                "cgs_iterations_mean": float(np.mean([int(q["iters"]) for q in stl])), "acceptance": acceptance(stl)}
        log(f"form 2d, M=512, extrapolated guess: {512 / dtl:.1f} level-solves/s")
    iters = [int(q["iters"]) for q in st]
    restarts = int(sum(int(q["restarts"]) for q in st))
    nbytes = path_bytes_nd(d, N, M, iters, restarts)
    out = {"workload": f"{'x'.join(str(n) for n in ns)}, M={M}, alpha={prob.alpha}, "
                       f"betas={(prob.beta_x, prob.beta_y) if d == 2 else prob.betas}, "
                       "seeded manufactured solution, zero guess, multi-level circulant Strang preconditioner",
           "value": M / dt, "unit": "level-solves/s", "code": int(code),
           "cgs_iterations": {"mean": float(np.mean(iters)), "min": int(min(iters)), "max": int(max(iters))},
           "ms_per_cgs_iteration": 1e3 * dt / max(1, sum(iters)),
           "path_roofline": {"bound": "hbm", "bytes_per_march": nbytes, "achieved": nbytes / dt / 1e9,
                             "peak": 8000.0, "unit": "GB/s", "frac": nbytes / dt / 1e9 / 8000.0,
                             "model": f"{ {2: 33, 3: 47}[d]} x 8N B per CGS iteration, "
                                      f"{6 * d + 10} x 8N B per level plus the history"},
           "acceptance": acceptance(st),
           "extrapolated": {"value": M / dtx, "unit": "level-solves/s", "code": int(codex),
                            "cgs_iterations_mean": float(np.mean([int(q["iters"]) for q in stx])),
                            "speedup_vs_zero_guess": dt / dtx, "acceptance": acceptance(stx)}}
    if long is not None:
        out["long_march_extrapolated"] = long
    out["largest"] = nd_large(args, P, W, dev, d)
    log(f"form {d}d extrapolated guess: {M / dtx:.2f} level-solves/s, "
        f"{out['extrapolated']['cgs_iterations_mean']:.1f} iterations")
    log(f"form {d}d: {M / dt:.2f} level-solves/s, {np.mean(iters):.1f} iterations, "
        f"{out['ms_per_cgs_iteration']:.3f} ms per iteration, {out['path_roofline']['achieved']:.0f} GB/s "
        "by the byte model")
    return out


def history_form(args, P, prob, F, u0, levels, plain_value):
    """The headline march with the fast history (the L2-1sigma weights as a
    fitted sum of exponentials, tolerance 1e-12) beside the exact one; the
    largest per-level difference between the two marches is reported."""
    import numpy as np
    import torch
    out = {"workload": "headline", "history_tol": 1e-12}
    Us = {}
    for name, ht in (("exact", 0.0), ("fast", 1e-12)):
        with P.TimeLevelSolver.from_problem(prob, rtol=args.rtol, history_tol=ht) as sh:
            timed_march(sh, F, u0, min(levels, 16), torch)  # warm-up
            dt, st = timed_march(sh, F, u0, levels, torch)
            Us[name] = sh.history()[: levels + 1].clone()
        out[name] = {"value": levels / dt, "unit": "level-solves/s", "acceptance": acceptance(st)}
        log(f"history {name}: {levels / dt:.1f} level-solves/s")
    d = (Us["fast"] - Us["exact"]).norm(dim=1) / Us["exact"].norm(dim=1).clamp_min(1e-300)
    out["max_level_rel_diff"] = float(d.max())
    out["speedup_vs_exact"] = out["fast"]["value"] / out["exact"]["value"]
    del Us
    return out


def krylov_forms(args, P, prob, F, u0, levels, plain_value):
    """The headline march with the other Krylov method and the other
    circulant preconditioner, beside the plain PCGS with Strang's."""
    import numpy as np
    import torch
    out = {"workload": "headline"}
    for name, kr, pc in (("bicgstab_strang", P.TSFCDE_KRYLOV_BICGSTAB, P.TSFCDE_PREC_STRANG),
                         ("cgs_tchan", P.TSFCDE_KRYLOV_CGS, P.TSFCDE_PREC_TCHAN),
                         ("bicgstab_tchan", P.TSFCDE_KRYLOV_BICGSTAB, P.TSFCDE_PREC_TCHAN)):
        with P.TimeLevelSolver.from_problem(prob, rtol=args.rtol, krylov=kr, preconditioner=pc) as sk:
            timed_march(sk, F, u0, min(levels, 16), torch)  # warm-up
            dt, st = timed_march(sk, F, u0, levels, torch)
        out[name] = {"value": levels / dt, "unit": "level-solves/s",
                     "iterations_mean": float(np.mean([x["iters"] for x in st])),
                     "speedup_vs_plain": (levels / dt) / plain_value, "acceptance": acceptance(st)}
        log(f"form {name}: {levels / dt:.1f} level-solves/s, {out[name]['iterations_mean']:.2f} iterations")
    return out


def gsf_form(args, P, W, dev):
    """Constant coefficients at the headline size (Example 1's gamma, d_+-,
    n = 2^20, M = 512): Algorithm 3 with the Gohberg-Semencul formula against
    the plain PCGS march of the same problem."""
    import numpy as np
    import torch
    prob = W.config_large_constant(n=args.n, M=args.M)
    out = {"workload": f"n={prob.n}, M={prob.M}, alpha={prob.alpha}, beta={prob.beta}, gamma=-0.1, d+=0.8, d-=0.5"}
    F = None
    for name, flags in (("pcgs", 0), ("gsf", P.TSFCDE_FLAG_CONSTANT_GSF)):
        with P.TimeLevelSolver.from_problem(prob, rtol=args.rtol, flags=flags) as sg:
            if F is None:
                F = build_sources(prob, sg)
            u0 = sg.history()[0].clone()
            timed_march(sg, F, u0, prob.M, torch)  # warm-up (and, for gsf, the solves (3.4))
            dt, st = timed_march(sg, F, u0, prob.M, torch)
        out[name] = {"value": prob.M / dt, "unit": "level-solves/s", "acceptance": acceptance(st),
                     "iterations_mean": float(np.mean([x["iters"] for x in st]))}
        log(f"constant coefficients, {name}: {prob.M / dt:.1f} level-solves/s")
    out["speedup_vs_plain"] = out["gsf"]["value"] / out["pcgs"]["value"]
    out["note"] = ("timed march after a warm-up march; the two solves (3.4) run once per plan, before its first "
                   "level j >= 1 (in the warm-up)")
    del F
    return out


def warm_forms(args, P, prob, F, u0, levels, plain_value, res):
    import numpy as np
    import torch
    for ws, name in ((P.TSFCDE_WS_PREV, "previous_level"), (P.TSFCDE_WS_EXTRAP, "extrapolated")):
        with P.TimeLevelSolver.from_problem(prob, rtol=args.rtol, warm_start=ws) as sw:
            dt, st = timed_march(sw, F, u0, levels, torch)
        res[name] = {"workload": "headline", "value": levels / dt, "unit": "level-solves/s",
                     "cgs_iterations_mean": float(np.mean([x["iters"] for x in st])),
                     "speedup_vs_plain": (levels / dt) / plain_value, "acceptance": acceptance(st)}
        log(f"form {name}: {levels / dt:.1f} level-solves/s")


def fp32_forms(args, P, W, prob, F, u0, levels, plain_value, dev, res):
    """FP32-refined: on the headline workload the rounding-error model keeps
    FP64; inside the envelope it refines in FP32."""
    import numpy as np
    import torch
    with P.TimeLevelSolver.from_problem(prob, rtol=args.rtol, precision=P.TSFCDE_FP32_REFINED) as sw:
        dt, st = timed_march(sw, F, u0, levels, torch)
    share = float(np.mean([x["precision_used"] == P.TSFCDE_FP32_REFINED for x in st]))
    res["fp32_refined"] = {"workload": "headline", "value": levels / dt, "unit": "level-solves/s",
                           "levels_refined_in_fp32": share, "acceptance": acceptance(st),
                           "note": "the rounding-error model keeps every level of this workload in FP64 "
                                   "(eps32 log2(L) |A|/eta is far above 0.1 at n = 2^20), so this is the FP64 "
                                   "path; no speedup is claimed"}
    small = W.config_large(n=args.fp32_n, M=args.M)
    rates = {}
    Fs = None
    for prec in (P.TSFCDE_FP64, P.TSFCDE_FP32_REFINED):
        with P.TimeLevelSolver.from_problem(small, rtol=args.rtol, precision=prec) as sw:
            if Fs is None:
                Fs = build_sources(small, sw)
            us = sw.history()[0].clone()
            timed_march(sw, Fs, us, small.M, torch)  # warm-up
            dt, st = timed_march(sw, Fs, us, small.M, torch)
            rates[prec] = (small.M / dt, st)
    st32 = rates[P.TSFCDE_FP32_REFINED][1]
    res["fp32_refined_in_envelope"] = {
        "workload": f"n={small.n}, M={small.M}, headline coefficients",
        "value": rates[P.TSFCDE_FP32_REFINED][0], "plain_value": rates[P.TSFCDE_FP64][0], "unit": "level-solves/s",
        "speedup_vs_plain": rates[P.TSFCDE_FP32_REFINED][0] / rates[P.TSFCDE_FP64][0],
        "levels_refined_in_fp32": float(np.mean([x["precision_used"] == P.TSFCDE_FP32_REFINED for x in st32])),
        "true_relres_max": float(max(x["relres_true"] for x in st32)), "acceptance": acceptance(st32),
        "inner_iterations_mean": float(np.mean([x["iters"] for x in st32])),
        "outer_sweeps_mean": float(np.mean([x["outer_iters"] for x in st32]))}
    del Fs
    log(f"form fp32_refined: headline {res['fp32_refined']['value']:.1f} (fp32 share {share:.2f}); "
        f"n={small.n}: {res['fp32_refined_in_envelope']['speedup_vs_plain']:.2f}x plain")


def batched_form(args, P, W, dev):
    """512 instances of uneven n, alpha, beta (n log-uniform in [2^10, 2^16],
    M = 128) advanced together; the plain comparison runs single-instance
    plans one after another on a sample of the instances."""
    import numpy as np
    import torch
    from paper_1603_00279_amd import warmnet as WN
    probs = W.batched_instances(count=args.batch_count, M=args.batch_M)
    ns = [p.n for p in probs]
    out = {"workload": f"{len(probs)} instances, n log-uniform in [2^10, 2^16] (sum {sum(ns)}), M={args.batch_M}"}
    Fall = None
    for ws, key, flags in ((P.TSFCDE_WS_ZERO, "zero_guess", 0), (P.TSFCDE_WS_ZERO, "zero_guess_graphs", P.TSFCDE_FLAG_GRAPHS),
                           (P.TSFCDE_WS_EXTRAP, "extrapolated", 0)):
        with P.BatchSolver(probs, rtol=args.rtol, warm_start=ws, flags=flags) as bs:
            if Fall is None:  # (M x n) per instance at its own nodes and instants
                Fall = [W.device_sources(p, bs.nodes(i), bs.level_times(i), dev) for i, p in enumerate(probs)]
            zeros = [torch.zeros(n, dtype=torch.float64, device=dev) for n in ns]
            bs.reset(zeros)
            torch.cuda.synchronize()
            # every level of every instance in one call (instances advance on their own)
            t0 = time.perf_counter()
            code, st = bs.solve(Fall, raise_on_error=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if code in (P.TSFCDE_EDEVICE, P.TSFCDE_EINVAL, P.TSFCDE_ENOMEM, P.TSFCDE_EDONE):
                raise RuntimeError(f"batched form ({key}): tsfcde_batch_solve returned {code}")
        out[key] = {"value": len(probs) * args.batch_M / dt, "unit": "instance-levels/s",
                    "unknown_levels_per_s": sum(ns) * args.batch_M / dt,
                    "cgs_iterations_mean": float(st["iters"].mean()), "acceptance": acceptance(st)}
        log(f"batched ({key}): {out[key]['value']:.0f} instance-levels/s")
    sub = list(range(0, len(probs), max(1, len(probs) // 32)))
    tot = 0.0
    for i in sub:
        with P.TimeLevelSolver.from_problem(probs[i], rtol=args.rtol) as s1:
            u0 = s1.history()[0].clone()
            dt, _ = timed_march(s1, Fall[i], u0, args.batch_M, torch)
            tot += dt
    seq = len(sub) * args.batch_M / tot
    out["sequential_single_plans"] = {"value": seq, "unit": "instance-levels/s",
                                      "sample": f"{len(sub)} of the instances, one plan after another"}
    out["speedup_vs_plain"] = out["zero_guess"]["value"] / seq
    log(f"batched: {out['speedup_vs_plain']:.1f}x sequential single-instance plans")
    return out


def iteration_summary(its):
    """Mean and distribution of per-level CGS iteration counts."""
    import numpy as np
    a = np.asarray(its, dtype=float)
    return {"mean": float(a.mean()), "p50": float(np.percentile(a, 50)), "p90": float(np.percentile(a, 90)),
            "max": float(a.max())}


def net_cost_iterations(prev, extrap, net):
    """The network's cost per level in CGS-iteration equivalents.  Each
    argument is (seconds per level, mean CGS iterations per level); the
    previous-level and extrapolated guesses (both checked by the same
    acceptance product, neither with inference) fix the line
    seconds = c + t_it * iterations, and the network's excess over that line,
    divided by t_it, is its cost.  None when the two guesses take the same
    iterations (no slope)."""
    (tp, ip), (te, ie), (tn, i_n) = prev, extrap, net
    if abs(ip - ie) < 1e-9:
        return None
    t_it = (tp - te) / (ip - ie)
    if t_it <= 0.0:
        return None
    c = te - t_it * ie
    return (tn - (c + t_it * i_n)) / t_it


def learned_form(args, P, W, dev):
    """The learned warm start with the committed parameters (trained by
    paper_1603_00279_amd.warmnet on 2000 trajectories at n = 2^14, M = 256)
    on held-out (alpha, beta) at n = 2^14 and 2^18, against the plain,
    previous-level and extrapolated guesses: level-solves/s, the distribution
    of CGS iterations per level and the network's cost in iteration
    equivalents."""
    import numpy as np
    import torch
    from paper_1603_00279_amd import warmnet as WN
    path = os.path.join(ROOT, "paper_1603_00279_amd", "data", "warmnet_c4.npz")
    theta = np.load(path)["theta"]
    M = 256
    out = {"workload": f"held-out (alpha, beta), n=16384 (and 262144), M={M}, Example-2 time dependence",
           "parameters": os.path.relpath(path, ROOT)}
    for n, key_n in ((1 << 14, None), (1 << 18, "n_2p18")):
        held = W.warmstart_instances(2, n, M, seed=W.SEED_BASE + 77, held_out=True)
        rec = {} if key_n else out
        if key_n:
            rec["workload"] = f"held-out (alpha, beta), n={n}, M={M}, Example-2 time dependence"
        with P.WarmStartNet(max_points=n, max_batch=1) as net:
            net.set_params(theta)
            for ws, key in ((P.TSFCDE_WS_ZERO, "plain"), (P.TSFCDE_WS_PREV, "previous_level"),
                            (P.TSFCDE_WS_EXTRAP, "extrapolated"), (P.TSFCDE_WS_NET, "network")):
                tot, its, kept = 0.0, [], []
                for prob in held:
                    with P.TimeLevelSolver.from_problem(prob, rtol=args.rtol, warm_start=ws) as s1:
                        F = WN.device_sources(prob, s1)
                        if ws == P.TSFCDE_WS_NET:
                            net.attach(s1)
                        u0 = s1.history()[0].clone()
                        timed_march(s1, F, u0, M, torch)
                        dt, st = timed_march(s1, F, u0, M, torch)
                        del F
                    tot += dt
                    its += [x["iters"] for x in st[2:]]
                    kept += [x["guess"] == P.TSFCDE_WS_NET for x in st[2:]]
                rec[key] = {"value": len(held) * M / tot, "unit": "level-solves/s",
                            "cgs_iterations_mean": float(np.mean(its)), "cgs_iterations": iteration_summary(its)}
                if ws == P.TSFCDE_WS_NET:
                    rec[key]["levels_using_network_guess"] = float(np.mean(kept))
                log(f"learned form n={n} ({key}): {rec[key]['value']:.1f} level-solves/s, {np.mean(its):.2f} iterations")
        pt = {k: (1.0 / rec[k]["value"], rec[k]["cgs_iterations_mean"]) for k in ("previous_level", "extrapolated", "network")}
        rec["network_cost_iterations"] = net_cost_iterations(pt["previous_level"], pt["extrapolated"], pt["network"])
        rec["speedup_vs_plain"] = rec["network"]["value"] / rec["plain"]["value"]
        if key_n:
            out[key_n] = rec
    return out


def host_cores():
    """CPU threads this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(n_full, M_full, rtol, budget_s=15.0, lu_sizes=(64, 256, 1024, 2048, 4096), lu_reps=5):
    """Time the CPU oracle on a bounded sample of the same march.

    Value: the oracle's FFT route (embedding products, Strang solve,
    preconditioned CGS, Sec. 4) at the full n on the first levels of the
    march.  numpy's FFT and vector operations run on one thread whatever the
    thread pools allow (a single 1-D transform is not split over cores), so
    this leg uses one core.  Beside it, the dense-LU oracle (LAPACK dgesv
    through numpy, BLAS on every host core) per level at n in lu_sizes with
    M = 64: the median of lu_reps timings of its first levels, and its
    (4096/n)^3 extrapolation to the full n."""
    import numpy as np
    import oracle as O
    import workloads as W
    from threadpoolctl import threadpool_info, threadpool_limits
    cores = host_cores()
    with threadpool_limits(limits=1):
        prob = W.config_large(n=n_full, M=M_full)
        U = [O.initial_level(prob)]
        its = []
        t0 = time.perf_counter()
        while len(its) < prob.M and time.perf_counter() - t0 < budget_s:
            j = len(its)
            u, k = O.level_solve_pcgs(prob, np.array(U), j, O.source_level(prob, j), rtol=rtol)
            U.append(u)
            its.append(k)
        dt = time.perf_counter() - t0
    sweep = []
    with threadpool_limits(limits=cores):
        blas = [f"{d.get('internal_api')} ({d.get('num_threads')} threads)" for d in threadpool_info()
                if d.get("user_api") == "blas"]
        for n_s in lu_sizes:
            small = W.config_large(n=n_s, M=64)
            per = 2 if n_s >= 4096 else 3
            times = []
            for _ in range(lu_reps):
                V = np.zeros((small.M + 1, n_s))
                V[0] = O.initial_level(small)
                t1 = time.perf_counter()
                for j in range(per):
                    V[j + 1] = O.level_solve(small, V, j, O.source_level(small, j))
                times.append((time.perf_counter() - t1) / per)
            med = float(np.median(times))
            sweep.append({"n": n_s, "seconds_per_level": med, "level_solves_per_s": 1.0 / med,
                          "levels_timed": per, "repeats": lu_reps})
            log(f"cpu baseline: dense LU n={n_s}: {1e3 * med:.1f} ms per level")
    big = sweep[-1]
    return {
        "value": len(its) / dt,
        "unit": "level-solves/s",
        "cores": 1,
        "host_cores": cores,
        "kind": "oracle",
        "sample": (f"FFT-PCGS oracle (numpy FFT, one thread: its transforms and vector operations are "
                   f"single-threaded), first {len(its)} levels of the same march "
                   f"(n={n_full}, M={M_full}, rtol={rtol}, zero initial guess) in {dt:.1f}s, "
                   f"CGS iterations {its}"),
        "dense_lu": {"cores": cores, "blas": blas, "M": 64, "sweep": sweep,
                     "value_extrapolated": big["level_solves_per_s"] * (big["n"] / n_full) ** 3,
                     "note": (f"dense-LU oracle per level (assembly of A and B plus dgesv), median of "
                              f"{lu_reps}; at the full n only the ({big['n']}/n)^3 extrapolation of the "
                              f"largest measured size")},
    }


def cpu_baseline_nd(rtol, its=(6, 3)):
    """The 2D and 3D oracles' FFT route (numpy FFTs, one thread) on a bounded
    sample: the right-hand side and its[0] (2D, 1024 x 1024, the bench form's
    size) or its[1] (3D, at 128^3: a 256^3 iteration takes tens of seconds on
    one core) CGS iterations of level 0; seconds per CGS iteration."""
    import numpy as np
    import oracle.ids2d_oracle as O2
    import oracle.ids3d_oracle as O3
    import workloads as W
    from threadpoolctl import threadpool_limits
    out = {}
    with threadpool_limits(limits=1):
        for d, prob, mod, k in ((2, W.problem_2d(1024, 1024, ND_FORMS[2]["M"]), O2, its[0]),
                                (3, W.problem_3d(128, 128, 128, ND_FORMS[3]["M"]), O3, its[1])):
            U = np.array([mod.initial_level(prob)])
            f = mod.source_level(prob, 0)
            solve = O2.level_solve_pcgs2 if d == 2 else O3.level_solve_pcgs3
            t0 = time.perf_counter()
            _, done = solve(prob, U, 0, f, rtol=rtol, maxit=k)
            dt = time.perf_counter() - t0
            size = "x".join(str(v) for v in ((prob.nx, prob.ny) if d == 2 else prob.ns))
            out[f"{d}d"] = {"grid": size, "cgs_iterations": int(done), "seconds": dt,
                            "seconds_per_cgs_iteration": dt / max(1, done), "cores": 1, "kind": "oracle",
                            "sample": f"level 0 of the {d}D family at {size}: right-hand side, spectra and "
                                      f"{done} CGS iterations of the FFT-route oracle"}
            log(f"cpu baseline {d}D oracle at {size}: {dt / max(1, done):.2f} s per CGS iteration")
    return out


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
    ap.add_argument("--no-large-leg", action="store_true", help="skip the n = 2^24 roofline leg")
    ap.add_argument("--profile-class", default="mid_matvec", choices=sorted(KCLASS))
    ap.add_argument("--profile-period", type=int, default=7,
                    help="events on every k-th launch of the profiled class (1 = all)")
    ap.add_argument("--fp32-n", type=int, default=2048, help="grid of the FP32-refined form inside its envelope")
    ap.add_argument("--form", default="all", choices=["all", "warm", "fp32", "batched", "learned", "krylov", "gsf", "history", "2d", "3d"],
                    help="which of the other forms to run (for profiling one of them)")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-M", type=int, default=128)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run three plain device copies of MIB MiB (reference for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1 (how the march would shard "
                                   "over several GPUs is described, not implemented)",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    import paper_1603_00279_amd as P

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calibration > 0:
        # reference for the HBM counters: plain copies of a source larger than
        # the 256 MB Infinity Cache, evicted before each copy by writing a
        # second buffer of the same size
        src = torch.rand(args.copy_calibration << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        evict = torch.empty_like(src)
        for _ in range(3):
            evict.fill_(1.0)
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {args.copy_calibration} MiB, each after a {args.copy_calibration} MiB fill")
        del src, dst, evict
    prob = W.config_large(n=args.n, M=args.M)
    levels = args.levels if args.levels > 0 else prob.M
    log(f"workload n={prob.n} M={prob.M} levels/step={levels} alpha={prob.alpha} beta={prob.beta}")
    s = P.TimeLevelSolver.from_problem(prob, rtol=args.rtol, warm_start=args.warm_start)
    u0 = s.history()[0].clone()
    log(f"plan ready, workspace {s.workspace_bytes / 2**30:.2f} GiB")
    F = build_sources(prob, s)
    log("sources built")

    def one_step(stats_out):
        s.set_state(0, u0.view(1, -1))
        if levels == prob.M:  # the whole march in one library call (tsfcde_solve)
            _, st = s.solve(F, raise_on_error=False)
            stats_out.extend(st)
            return
        for j in range(levels):
            stats_out.append(s.step(F[j], raise_on_error=False))

    for w in range(args.warmup):
        one_step([])
        log(f"warmup step {w + 1}/{args.warmup} done")

    cls = KCLASS[args.profile_class]
    # events on a sample of the class's launches: a launch that carries them
    # idles the stream for a few microseconds on either side (the history sum,
    # one launch per level of growing size, is timed at every launch)
    period = 1 if args.profile_class == "history" else args.profile_period
    s.profile(cls, True, period)
    all_stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_step(all_stats)
        log(f"timed step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launches, kms = s.profile_read(cls)
    issued = s.profile_issued(cls)
    s.profile(cls, False)

    total_levels = levels * args.steps
    value = total_levels / elapsed
    stats = all_stats[:levels]  # the first timed march (all marches take the same iterations)
    iters = [st["iters"] for st in stats]
    accept = acceptance(all_stats)
    log(f"acceptance: {accept}")
    n = prob.n
    # roofline of the dominant kernel (HBM-bound; algorithmic bytes per launch)
    if args.profile_class == "history":
        bytes_step, nl_step = history_bytes(n, prob.M, levels)
        per_launch = bytes_step / max(1, nl_step)
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
    # mean over the sampled launches, scaled to every issued launch, per working launch
    avg_ms = kms / max(1, launches) * issued / max(1, real)
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
        "path_roofline": {"bound": "hbm", "bytes_per_step": path_bytes(n, prob.M, levels, iters),
                          "achieved": path_bytes(n, prob.M, levels, iters) * args.steps / elapsed / 1e9,
                          "peak": peak, "unit": "GB/s",
                          "frac": path_bytes(n, prob.M, levels, iters) * args.steps / elapsed / 1e9 / peak,
                          "model": "416n B per CGS iteration, 112n B per right-hand side, plus the history",
                          "fused_bytes_per_step": fused_bytes(n, prob.M, levels, iters),
                          "fused_frac": fused_bytes(n, prob.M, levels, iters) * args.steps / elapsed / 1e9 / peak},
        "roofline": {"bound": "hbm", "kernel": args.profile_class, "achieved": achieved, "peak": peak,
                     "unit": "GB/s", "frac": achieved / peak, "traffic": None,
                     "sampled_launches": launches, "sample_period": period, "issued_launches": issued,
                     "working_launches": real, "avg_launch_us": 1e3 * avg_ms,
                     "algorithmic_bytes_per_launch": per_launch},
        "cgs_iterations": {"mean": float(np.mean(iters)), "min": int(min(iters)), "max": int(max(iters))},
        "acceptance": accept,
    }
    traffic = committed_traffic(args.profile_class, n)
    if traffic is not None:
        out["roofline"]["traffic"] = traffic["bytes_per_launch"]
        out["roofline"]["traffic_source"] = traffic["source"]
    s.close()
    if not args.no_large_leg:
        out["roofline_n2p24"] = large_leg(args, P, W, dev)
    if not args.no_forms:
        out["forms"] = forms(args, P, W, prob, F, u0, levels, value, dev)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(n, prob.M, args.rtol)
        if not args.no_forms and args.form in ("all", "2d", "3d"):
            nd = cpu_baseline_nd(args.rtol)
            for d, key in ((2, "two_dimensional"), (3, "three_dimensional")):
                form = out.get("forms", {}).get(key)
                if form and d == 2:
                    # same grid: the oracle's level at the GPU's mean iteration count
                    nd["2d"]["level_solves_per_s_at_gpu_iterations"] = 1.0 / (
                        nd["2d"]["seconds_per_cgs_iteration"] * form["cgs_iterations"]["mean"])
                    nd["2d"]["gpu_over_oracle"] = form["value"] / nd["2d"]["level_solves_per_s_at_gpu_iterations"]
            out["cpu_baseline"]["nd"] = nd
    print(json.dumps(out), flush=True)
    if accept["failed_levels"]:
        log(f"{accept['failed_levels']} timed levels failed the acceptance test")
        sys.exit(3)


def large_leg(args, P, W, dev, n=1 << 24, M=8):
    """The product middle pass at n = 2^24 (transform buffers of 256 MiB, the
    same as the Infinity Cache, spectrum and buffer 512 MiB together): a
    march of M levels of the headline family with events on every 7th launch
    of the class; working launches as in the headline leg."""
    import numpy as np
    import torch
    prob = W.config_large(n=n, M=M)
    with P.TimeLevelSolver.from_problem(prob, rtol=args.rtol) as sl:
        F = build_sources(prob, sl)
        u0 = sl.history()[0].clone()
        timed_march(sl, F, u0, 2, torch)  # warm-up
        sl.profile(KCLASS["mid_matvec"], True, 7)
        dt, st = timed_march(sl, F, u0, M, torch)
        launches, kms = sl.profile_read(KCLASS["mid_matvec"])
        issued = sl.profile_issued(KCLASS["mid_matvec"])
        sl.profile(KCLASS["mid_matvec"], False)
    iters = [x["iters"] for x in st]
    real = 2 * sum(iters) + M
    avg_ms = kms / max(1, launches) * issued / max(1, real)
    achieved = 48 * n / (avg_ms * 1e-3) / 1e9
    cgs_bytes = 416 * n * sum(iters)
    out = {"workload": f"n={n}, M={M}, headline coefficients and solution family, zero guess",
           "kernel": "mid_matvec", "bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
           "frac": achieved / 8000.0, "avg_launch_us": 1e3 * avg_ms, "algorithmic_bytes_per_launch": 48 * n,
           "level_solves_per_s": M / dt, "cgs_iterations_mean": float(np.mean(iters)),
           "path_frac_lower_bound": (path_bytes(n, M, M, iters)) / dt / 1e9 / 8000.0,
           "cgs_iteration_bytes": cgs_bytes, "acceptance": acceptance(st)}
    traffic = committed_traffic("mid_matvec", n)
    out["traffic"] = traffic["bytes_per_launch"] if traffic else None
    if traffic:
        out["traffic_source"] = traffic["source"]
    log(f"n=2^24 leg: mid_matvec {achieved:.0f} GB/s ({out['frac']:.3f}), {M / dt:.1f} level-solves/s")
    del F
    return out


if __name__ == "__main__":
    main()
