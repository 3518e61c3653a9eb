"""Thin Python wrapper around the C ABI: one plan per TimeLevelSolver.

PyTorch supplies the device workspace and the stream; the wrapper only
marshals arguments.  Every numerical step runs in the HIP kernels of
libtsfcde.so.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _native as N


def _dptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("contiguous float64 tensor expected")
    return ctypes.c_void_p(t.data_ptr())


class TimeLevelSolver:
    """A plan of the TSFCDE time-level solver (problem (1.1), Algorithm 2).

    Coefficients are given as samples at t_{j+sigma}, j = 0..M-1 (arrays of
    length M).  The initial level u^0 is given with ``set_state(0, u0)`` (or
    left at zero).
    """

    def __init__(self, *, alpha: float, beta: float, n: int, M: int,
                 gamma_at: Sequence[float], dplus_at: Sequence[float], dminus_at: Sequence[float],
                 a: float = 0.0, b: float = 1.0, T: float = 1.0, rtol: float = 1e-10, maxit: int = 500,
                 warm_start: int = N.TSFCDE_WS_ZERO, flags: int = 0, precision: int = N.TSFCDE_FP64,
                 device: Optional[torch.device] = None, stream: Optional[torch.cuda.Stream] = None):
        self._lib = N.lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.n, self.M = int(n), int(M)
        self._g = np.ascontiguousarray(gamma_at, dtype=np.float64)
        self._dp = np.ascontiguousarray(dplus_at, dtype=np.float64)
        self._dm = np.ascontiguousarray(dminus_at, dtype=np.float64)
        if not (len(self._g) == len(self._dp) == len(self._dm) == self.M):
            raise ValueError("coefficient samples must have length M")
        dptr = ctypes.POINTER(ctypes.c_double)
        self.problem = N.tsfcde_problem(
            alpha=alpha, beta=beta, a=a, b=b, T=T, n=self.n, M=self.M,
            gamma=N.COEF_FN(), dplus=N.COEF_FN(), dminus=N.COEF_FN(), coef_user=None,
            gamma_at=self._g.ctypes.data_as(dptr), dplus_at=self._dp.ctypes.data_as(dptr),
            dminus_at=self._dm.ctypes.data_as(dptr), phi=N.IC_FN(), phi_user=None,
            rtol=rtol, maxit=maxit, precision=precision, warm_start=warm_start, flags=flags)
        nbytes = ctypes.c_size_t(0)
        N.check(self._lib.tsfcde_workspace_bytes(ctypes.byref(self.problem), ctypes.byref(nbytes)),
                "tsfcde_workspace_bytes")
        self.workspace_bytes = nbytes.value
        # over-allocate by 256 bytes so the plan can start on a 256-byte boundary
        self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_off = (-base) % 256
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            N.check(self._lib.tsfcde_plan(ctypes.byref(self.problem), ctypes.c_void_p(base + self._ws_off),
                                          self.workspace_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                                          ctypes.byref(handle)), "tsfcde_plan")
        self._plan = handle

    # ------------------------------------------------------------------
    @classmethod
    def from_problem(cls, prob, **kw):
        """Build from an object with alpha, beta, n, M, a, b, T and
        ``coefficient_samples()`` / ``initial_vector()`` (see workloads)."""
        g, dp, dm = prob.coefficient_samples()
        s = cls(alpha=prob.alpha, beta=prob.beta, n=prob.n, M=prob.M, gamma_at=g, dplus_at=dp, dminus_at=dm,
                a=prob.a, b=prob.b, T=prob.T, **kw)
        u0 = torch.as_tensor(prob.initial_vector(), dtype=torch.float64, device=s.device)
        s.set_state(0, u0.reshape(1, -1))
        return s

    def close(self):
        if getattr(self, "_plan", None):
            self._lib.tsfcde_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------
    @property
    def level(self) -> int:
        return int(self._lib.tsfcde_level(self._plan))

    def history(self) -> torch.Tensor:
        """View of the stored levels U ((M+1) x n, row stride ld) inside the workspace."""
        ptr = self._lib.tsfcde_history(self._plan)
        ld = int(self._lib.tsfcde_history_ld(self._plan))
        off = ptr - self._ws.data_ptr()
        flat = self._ws[off: off + 8 * (self.M + 1) * ld].view(torch.float64)
        return flat.view(self.M + 1, ld)[:, : self.n]

    def set_state(self, level: int, U: torch.Tensor):
        U = U.contiguous()
        if U.numel() != (level + 1) * self.n:
            raise ValueError("U must hold level+1 rows of n values")
        N.check(self._lib.tsfcde_set_state(self._plan, level, _dptr(U)), "tsfcde_set_state")

    def step(self, f: Optional[torch.Tensor] = None, u_out: Optional[torch.Tensor] = None, raise_on_error=True):
        st = N.tsfcde_stats()
        code = self._lib.tsfcde_step(self._plan, _dptr(f), _dptr(u_out), ctypes.byref(st))
        if raise_on_error:
            N.check(code, "tsfcde_step")
        d = st.as_dict()
        d["code"] = code
        return d

    def solve(self, F: Optional[torch.Tensor] = None, U_out: Optional[torch.Tensor] = None, raise_on_error=True):
        stats = (N.tsfcde_stats * self.M)()
        ld = F.shape[1] if F is not None else self.n
        code = self._lib.tsfcde_solve(self._plan, _dptr(F), ld, _dptr(U_out), stats)
        if raise_on_error:
            N.check(code, "tsfcde_solve")
        return code, [s.as_dict() for s in stats]

    def apply(self, op: int, j: int, x: torch.Tensor) -> torch.Tensor:
        y = torch.empty_like(x)
        N.check(self._lib.tsfcde_apply(self._plan, op, j, _dptr(x), _dptr(y)), "tsfcde_apply")
        return y

    def rhs(self, j: int, f: Optional[torch.Tensor] = None) -> torch.Tensor:
        g = torch.empty(self.n, dtype=torch.float64, device=self.device)
        N.check(self._lib.tsfcde_rhs(self._plan, j, _dptr(f), _dptr(g)), "tsfcde_rhs")
        return g

    def weights(self) -> torch.Tensor:
        w = torch.empty(self.n + 1, dtype=torch.float64, device=self.device)
        N.check(self._lib.tsfcde_weights(self._plan, _dptr(w)), "tsfcde_weights")
        return w

    @property
    def embedding_length(self) -> int:
        return int(self._lib.tsfcde_embedding_length(self._plan))

    def spectrum(self, which: int) -> torch.Tensor:
        cnt = self.embedding_length // 2 + 1 if which == N.TSFCDE_SPEC_EMBED else self.n // 2 + 1
        out = torch.empty(2 * cnt, dtype=torch.float64, device=self.device)
        N.check(self._lib.tsfcde_spectrum(self._plan, which, _dptr(out)), "tsfcde_spectrum")
        return torch.view_as_complex(out.view(cnt, 2))

    def profile(self, kernel_class: int, enable: bool = True, period: int = 1):
        """Start (enable) or stop recording one kernel class; events ride on
        every ``period``-th launch of the class."""
        if period < 1:
            raise ValueError("period must be >= 1")
        N.check(self._lib.tsfcde_profile(self._plan, kernel_class, period if enable else 0), "tsfcde_profile")

    def profile_issued(self, kernel_class: int) -> int:
        cnt = ctypes.c_int64(0)
        N.check(self._lib.tsfcde_profile_issued(self._plan, kernel_class, ctypes.byref(cnt)), "tsfcde_profile_issued")
        return cnt.value

    def profile_read(self, kernel_class: int):
        cnt = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        N.check(self._lib.tsfcde_profile_read(self._plan, kernel_class, ctypes.byref(cnt), ctypes.byref(ms)),
                "tsfcde_profile_read")
        return cnt.value, ms.value


class BatchSolver:
    """Many independent instances advanced level by level with grouped
    launches (tsfcde_plan_batch / tsfcde_batch_step).  ``problems`` are
    objects with alpha, beta, n, M, a, b, T, coefficient_samples() and
    initial_vector(); all share M."""

    def __init__(self, problems, *, rtol: float = 1e-10, maxit: int = 500, warm_start: int = N.TSFCDE_WS_ZERO,
                 precision: int = N.TSFCDE_FP64, flags: int = 0, device: Optional[torch.device] = None,
                 stream: Optional[torch.cuda.Stream] = None):
        self._lib = N.lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.count = len(problems)
        self.M = problems[0].M
        self.ns = [p.n for p in problems]
        dptr = ctypes.POINTER(ctypes.c_double)
        self._keep = []
        arr = (N.tsfcde_problem * self.count)()
        for i, prob in enumerate(problems):
            g, dp, dm = (np.ascontiguousarray(v, dtype=np.float64) for v in prob.coefficient_samples())
            self._keep += [g, dp, dm]
            arr[i] = N.tsfcde_problem(
                alpha=prob.alpha, beta=prob.beta, a=prob.a, b=prob.b, T=prob.T, n=prob.n, M=prob.M,
                gamma=N.COEF_FN(), dplus=N.COEF_FN(), dminus=N.COEF_FN(), coef_user=None,
                gamma_at=g.ctypes.data_as(dptr), dplus_at=dp.ctypes.data_as(dptr), dminus_at=dm.ctypes.data_as(dptr),
                phi=N.IC_FN(), phi_user=None, rtol=rtol, maxit=maxit, precision=precision,
                warm_start=warm_start, flags=flags)
        self._arr = arr
        nbytes = ctypes.c_size_t(0)
        N.check(self._lib.tsfcde_batch_workspace_bytes(arr, self.count, ctypes.byref(nbytes)),
                "tsfcde_batch_workspace_bytes")
        self.workspace_bytes = nbytes.value
        self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            N.check(self._lib.tsfcde_plan_batch(arr, self.count, ctypes.c_void_p(base + off), self.workspace_bytes,
                                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)),
                    "tsfcde_plan_batch")
        self._batch = handle
        for i, prob in enumerate(problems):
            u0 = torch.as_tensor(prob.initial_vector(), dtype=torch.float64, device=self.device)
            N.check(self._lib.tsfcde_set_state(self.member(i), 0, ctypes.c_void_p(u0.data_ptr())), "tsfcde_set_state")
        torch.cuda.synchronize(self.device)

    def member(self, i: int):
        return self._lib.tsfcde_batch_member(self._batch, i)

    def history(self, i: int) -> torch.Tensor:
        """Copy of instance i's stored levels ((M+1) x n)."""
        h = self.member(i)
        ptr = self._lib.tsfcde_history(h)
        ld = int(self._lib.tsfcde_history_ld(h))
        n = self.ns[i]
        off = ptr - self._ws.data_ptr()
        flat = self._ws[off: off + 8 * (self.M + 1) * ld].view(torch.float64)
        return flat.view(self.M + 1, ld)[:, :n].clone()

    def reset(self, u0s):
        """Set every instance back to level 0 with the given initial vectors."""
        for i, u0 in enumerate(u0s):
            N.check(self._lib.tsfcde_set_state(self.member(i), 0, ctypes.c_void_p(u0.data_ptr())), "tsfcde_set_state")
        N.check(self._lib.tsfcde_batch_set_level(self._batch, 0), "tsfcde_batch_set_level")

    def step(self, fs=None, raise_on_error=True):
        """fs: list of device tensors (f of each instance at this level) or None."""
        ptrs = None
        if fs is not None:
            ptrs = (ctypes.c_void_p * self.count)(*[f.data_ptr() if f is not None else None for f in fs])
        stats = (N.tsfcde_stats * self.count)()
        code = self._lib.tsfcde_batch_step(self._batch, ptrs, stats)
        if raise_on_error:
            N.check(code, "tsfcde_batch_step")
        return code, [st.as_dict() for st in stats]

    def close(self):
        if getattr(self, "_batch", None):
            self._lib.tsfcde_batch_destroy(self._batch)
            self._batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
