"""Learned Krylov warm start: a thin binding of the network kernels behind
the C ABI (tsfcde_net_*) and a training driver over trajectories that the
solver itself produces.

The network (include/tsfcde.h, "learned warm start") predicts level j+1 from
levels j, j-1, j-2 as a correction to quadratic extrapolation in t; a plan
with warm_start = TSFCDE_WS_NET and an attached network uses the prediction
as CGS's initial guess whenever its true residual beats the previous level's.
Every step of training and inference runs in the library's kernels; this
module only marshals pointers and arrays.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _native as N
from .solver import BatchSolver, TimeLevelSolver


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class WarmStartNet:
    """The network in a torch-allocated device workspace sized for batches of
    up to ``max_batch`` samples and ``max_points`` grid points in all."""

    def __init__(self, max_points: int, max_batch: int = 64, device: Optional[torch.device] = None,
                 stream: Optional[torch.cuda.Stream] = None):
        self._lib = N.lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.max_points, self.max_batch = int(max_points), int(max_batch)
        nb = ctypes.c_size_t(0)
        N.check(self._lib.tsfcde_net_workspace_bytes(self.max_points, self.max_batch, ctypes.byref(nb)),
                "tsfcde_net_workspace_bytes")
        self._ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            N.check(self._lib.tsfcde_net_create(ctypes.c_void_p(base + off), nb.value, self.max_points,
                                                self.max_batch, ctypes.c_void_p(self.stream.cuda_stream),
                                                ctypes.byref(h)), "tsfcde_net_create")
        self._net = h
        self.param_count = int(self._lib.tsfcde_net_param_count())

    def set_params(self, theta: np.ndarray):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        assert theta.size == self.param_count
        N.check(self._lib.tsfcde_net_set_params(self._net, _fptr(theta)), "tsfcde_net_set_params")

    def get_params(self) -> np.ndarray:
        out = np.empty(self.param_count, dtype=np.float32)
        N.check(self._lib.tsfcde_net_get_params(self._net, _fptr(out)), "tsfcde_net_get_params")
        return out

    def train_step(self, samples: Sequence[N.tsfcde_net_sample], n: int, lr: float, want_grad: bool = False):
        arr = (N.tsfcde_net_sample * len(samples))(*samples)
        loss = ctypes.c_double(0.0)
        grad = np.empty(self.param_count, dtype=np.float32) if want_grad else None
        N.check(self._lib.tsfcde_net_train_step(self._net, arr, len(samples), n, lr, ctypes.byref(loss),
                                                _fptr(grad) if want_grad else None), "tsfcde_net_train_step")
        return loss.value, grad

    def predict(self, sample: N.tsfcde_net_sample, n: int) -> torch.Tensor:
        x0 = torch.empty(n, dtype=torch.float64, device=self.device)
        N.check(self._lib.tsfcde_net_predict(self._net, ctypes.byref(sample), n, ctypes.c_void_p(x0.data_ptr())),
                "tsfcde_net_predict")
        return x0

    def attach(self, solver: TimeLevelSolver):
        N.check(self._lib.tsfcde_plan_set_net(solver._plan, self._net), "tsfcde_plan_set_net")

    def close(self):
        if getattr(self, "_net", None):
            self._lib.tsfcde_net_destroy(self._net)
            self._net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def make_sample(plan_handle, hist_ptr: int, ld: int, j: int, target: bool = True) -> N.tsfcde_net_sample:
    """Sample for level j (needs j >= 2) of the stored levels at hist_ptr
    (row stride ld doubles); the level's features come from the plan."""
    lib = N.lib()
    s = N.tsfcde_net_sample()
    row = lambda k: ctypes.c_void_p(hist_ptr + 8 * ld * k)  # noqa: E731
    s.u_next = row(j + 1) if target else None
    s.u0, s.u1, s.u2 = row(j), row(j - 1), row(j - 2)
    N.check(lib.tsfcde_level_features(plan_handle, j, s.feat), "tsfcde_level_features")
    return s


def device_sources(prob, solver: TimeLevelSolver) -> torch.Tensor:
    """f at the plan's nodes and sampling instants t_{j+sigma} for every
    level, built on the device (M x n)."""
    import workloads as W
    return W.device_sources(prob, solver.nodes(), solver.level_times(), solver.device)


class Trajectories:
    """Whole marches of many instances of one grid size, solved together by
    the batched form; their stored levels are the training data.  Each
    level's sources are formed for all instances at once from the
    separable manufactured source (profiles x coefficients)."""

    def __init__(self, problems, rtol: float = 1e-10, warm_start: int = N.TSFCDE_WS_EXTRAP, log=None):
        assert len({p.n for p in problems}) == 1 and len({p.M for p in problems}) == 1
        self.problems = problems
        self.n, self.M = problems[0].n, problems[0].M
        self.batch = BatchSolver(problems, rtol=rtol, warm_start=warm_start)
        dev = self.batch.device
        profs, coefs = zip(*(p.source_matrix(self.batch.nodes(i), self.batch.level_times(i))
                             for i, p in enumerate(problems)))
        prof = torch.as_tensor(np.stack(profs), dtype=torch.float64, device=dev)      # (count, 4, n)
        coef = torch.as_tensor(np.stack(coefs), dtype=torch.float64, device=dev)      # (count, M, 4)
        self.iters = []
        for j in range(self.M):
            Fj = torch.bmm(coef[:, j:j + 1, :].contiguous(), prof)[:, 0, :].contiguous()  # (count, n)
            _, stats = self.batch.step([Fj[i] for i in range(len(problems))])
            self.iters.append(float(np.mean([st["iters"] for st in stats])))
            if log and (j % max(1, self.M // 8) == 0 or j == self.M - 1):
                log(f"trajectories: level {j + 1}/{self.M}, mean CGS iterations {self.iters[-1]:.2f}")
        del prof, coef
        lib = N.lib()
        self.members = [self.batch.member(i) for i in range(len(problems))]
        self.hist = [int(lib.tsfcde_history(h)) for h in self.members]
        self.ld = [int(lib.tsfcde_history_ld(h)) for h in self.members]

    def sample(self, i: int, j: int, target: bool = True) -> N.tsfcde_net_sample:
        return make_sample(self.members[i], self.hist[i], self.ld[i], j, target)

    def random_samples(self, rng: np.random.Generator, count: int) -> List[N.tsfcde_net_sample]:
        ii = rng.integers(0, len(self.problems), count)
        jj = rng.integers(2, self.M, count)  # j + 1 <= M
        return [self.sample(int(i), int(j)) for i, j in zip(ii, jj)]

    def close(self):
        self.batch.close()


def initial_params(seed: int = 0) -> np.ndarray:
    """Fan-in scaled random hidden layers and a zero output layer, so that an
    untrained network predicts the quadratic extrapolation exactly."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in ((7, 32), (32, 32), (32, 32), (32, 1)):
        w = rng.normal(0, 1.0 / np.sqrt(ci * 5), co * ci * 5) if co > 1 else np.zeros(co * ci * 5)
        parts.append(np.concatenate([w, np.zeros(co)]))
    return np.concatenate(parts).astype(np.float32)


def train(net: WarmStartNet, data: Trajectories, steps: int, batch: int, lr: float = 1e-3, seed: int = 0,
          lr_final: Optional[float] = None, log=None) -> List[float]:
    """Adam on random (instance, level) samples; the learning rate decays
    geometrically from lr to lr_final (default lr / 10).  Returns the losses."""
    rng = np.random.default_rng(seed)
    lr_final = lr / 10 if lr_final is None else lr_final
    losses = []
    for k in range(steps):
        rate = lr * (lr_final / lr) ** (k / max(1, steps - 1))
        loss, _ = net.train_step(data.random_samples(rng, batch), data.n, rate)
        losses.append(loss)
        if log and (k % max(1, steps // 10) == 0 or k == steps - 1):
            log(f"step {k}/{steps} loss {loss:.4e} lr {rate:.2e}")
    return losses


def march_iterations(prob, warm_start: int, net: Optional[WarmStartNet] = None, rtol: float = 1e-10,
                     F: Optional[torch.Tensor] = None):
    """CGS iterations (per level) of a whole march with the given warm start,
    and the guesses the levels used."""
    with TimeLevelSolver.from_problem(prob, rtol=rtol, warm_start=warm_start) as s:
        if net is not None:
            net.attach(s)
        F = device_sources(prob, s) if F is None else F
        code, stats = s.solve(F)
        N.check(code, "march")
        return [st["iters"] for st in stats], [st["guess"] for st in stats]


def main(argv=None):
    """Train on solver trajectories and compare the guesses on held-out
    (alpha, beta).  Defaults: 2000 trajectories at n = 2^14, M = 256;
    held-out evaluation at n = 2^14 and 2^18."""
    import argparse
    import json
    import sys
    import time

    import workloads as W

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--count", type=int, default=2000)
    ap.add_argument("--n", type=int, default=1 << 14)
    ap.add_argument("--M", type=int, default=256)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=1e-5)
    ap.add_argument("--eval-n", type=int, nargs="*", default=[1 << 14, 1 << 18])
    ap.add_argument("--eval-count", type=int, default=4)
    ap.add_argument("--out", default="warmnet_params.npz")
    ap.add_argument("--report", default=None)
    args = ap.parse_args(argv)

    def log(msg):
        print(f"[warmnet] {msg}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    train_set = W.warmstart_instances(args.count, args.n, args.M)
    data = Trajectories(train_set, log=log)
    t_gen = time.perf_counter() - t0
    log(f"{args.count} trajectories in {t_gen:.1f} s")
    report = {"train": {"count": args.count, "n": args.n, "M": args.M, "steps": args.steps, "batch": args.batch,
                        "lr": args.lr, "trajectory_seconds": t_gen}}
    with WarmStartNet(max_points=args.batch * args.n, max_batch=args.batch) as net:
        net.set_params(initial_params(0))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        losses = train(net, data, args.steps, args.batch, args.lr, seed=1, lr_final=args.lr_final, log=log)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t1
        report["train"].update({"seconds": t_train, "loss_first": float(np.mean(losses[:50])),
                                "loss_last": float(np.mean(losses[-50:]))})
        data.close()
        theta = net.get_params()
        np.savez(args.out, theta=theta, losses=np.asarray(losses))
        log(f"trained in {t_train:.1f} s; loss {report['train']['loss_first']:.3e} -> "
            f"{report['train']['loss_last']:.3e}; parameters in {args.out}")
        report["eval"] = {}
        for n in args.eval_n:
            held = W.warmstart_instances(args.eval_count, n, args.M, seed=W.SEED_BASE + 40 + n % 97, held_out=True)
            big = WarmStartNet(max_points=n, max_batch=1)
            big.set_params(theta)
            res = {"prev": [], "extrap": [], "net": [], "net_levels_using_net": 0, "levels": 0}
            for prob in held:
                for key, ws, nt in (("prev", N.TSFCDE_WS_PREV, None), ("extrap", N.TSFCDE_WS_EXTRAP, None),
                                    ("net", N.TSFCDE_WS_NET, big)):
                    it, g = march_iterations(prob, ws, nt)
                    res[key] += it[2:]
                    if key == "net":
                        res["net_levels_using_net"] += sum(1 for x in g[2:] if x == N.TSFCDE_WS_NET)
                        res["levels"] += len(g) - 2
            big.close()
            summary = {k: float(np.mean(v)) for k, v in res.items() if isinstance(v, list)}
            summary["net_share"] = res["net_levels_using_net"] / max(1, res["levels"])
            report["eval"][str(n)] = summary
            log(f"held-out n={n}: mean CGS iterations prev {summary['prev']:.2f}, extrap {summary['extrap']:.2f}, "
                f"net {summary['net']:.2f} (net guess kept at {100 * summary['net_share']:.0f}% of levels)")
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(report, fh, indent=1)
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()
