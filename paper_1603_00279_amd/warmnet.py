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


def device_sources(prob, device) -> torch.Tensor:
    """f(x_i, t_{j+sigma}) for every level, built on the device (M x n)."""
    prof, coef = prob.source_profiles()
    return torch.as_tensor(coef, dtype=torch.float64, device=device) @ torch.as_tensor(prof, dtype=torch.float64,
                                                                                       device=device)


class Trajectories:
    """Whole marches of many instances of one grid size, solved together by
    the batched form; their stored levels are the training data."""

    def __init__(self, problems, rtol: float = 1e-10, warm_start: int = N.TSFCDE_WS_EXTRAP):
        assert len({p.n for p in problems}) == 1 and len({p.M for p in problems}) == 1
        self.problems = problems
        self.n, self.M = problems[0].n, problems[0].M
        self.batch = BatchSolver(problems, rtol=rtol, warm_start=warm_start)
        dev = self.batch.device
        srcs = [device_sources(p, dev) for p in problems]
        for j in range(self.M):
            self.batch.step([F[j] for F in srcs])
        del srcs
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
        F = device_sources(prob, s.device) if F is None else F
        code, stats = s.solve(F)
        N.check(code, "march")
        return [st["iters"] for st in stats], [st["guess"] for st in stats]
