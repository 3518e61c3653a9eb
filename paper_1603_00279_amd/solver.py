"""Thin Python wrapper around the C ABI: one plan per TimeLevelSolver.

PyTorch supplies the device workspace and the stream; the wrapper only
marshals arguments.  Every numerical step runs in the HIP kernels of
libtsfcde.so.
"""
from __future__ import annotations

import ctypes
from typing import Callable, Optional

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


def _coef_fields(gamma, dplus, dminus, keep: list):
    """ctypes fields of gamma, d_+, d_-: each either a callable of t (wrapped
    as a C callback, which the library samples at its own t_{j+sigma}) or a
    sequence of the M samples."""
    out = {}
    dptr = ctypes.POINTER(ctypes.c_double)
    for name, v in (("gamma", gamma), ("dplus", dplus), ("dminus", dminus)):
        if callable(v):
            cb = N.COEF_FN(lambda t, _u, fn=v: float(fn(t)))
            keep.append(cb)
            out[name] = cb
            out[name + "_at"] = None
        else:
            arr = np.ascontiguousarray(v, dtype=np.float64)
            keep.append(arr)
            out[name] = N.COEF_FN()
            out[name + "_at"] = arr.ctypes.data_as(dptr)
    return out


def _problem(*, alpha, beta, n, M, a, b, T, gamma, dplus, dminus, phi, f, rtol, maxit, precision, warm_start,
             flags, keep: list, krylov=N.TSFCDE_KRYLOV_CGS, preconditioner=N.TSFCDE_PREC_STRANG,
             history_tol=0.0):
    """A tsfcde_problem; the Python callables and arrays it points to are
    appended to ``keep`` (they must outlive every library call that uses it)."""
    fields = _coef_fields(gamma, dplus, dminus, keep)
    if phi is not None:
        phi_cb = N.IC_FN(lambda x, _u, fn=phi: float(fn(x)))
        keep.append(phi_cb)
    else:
        phi_cb = N.IC_FN()
    if f is not None:
        f_cb = N.SRC_FN(lambda x, t, _u, fn=f: float(fn(x, t)))
        keep.append(f_cb)
    else:
        f_cb = N.SRC_FN()
    return N.tsfcde_problem(
        alpha=alpha, beta=beta, a=a, b=b, T=T, n=int(n), M=int(M), coef_user=None, phi=phi_cb, phi_user=None,
        rtol=rtol, maxit=maxit, precision=precision, warm_start=warm_start, flags=flags, f=f_cb, f_user=None,
        krylov=krylov, preconditioner=preconditioner, history_tol=history_tol, **fields)


def _scalar_phi(prob):
    return lambda x: float(np.asarray(prob.phi(np.array([x], dtype=np.float64)))[0])


def _scalar_f(prob):
    return lambda x, t: float(np.asarray(prob.f(np.array([x], dtype=np.float64), t))[0])


class TimeLevelSolver:
    """A plan of the TSFCDE time-level solver (problem (1.1), Algorithm 2).

    gamma, dplus, dminus: callables of t, sampled by the library at its own
    t_{j+sigma}, or sequences of those M samples.  phi: optional callable of
    x (the library evaluates it at its nodes; otherwise u^0 = 0 until
    ``set_state``).  f: optional callable of (x, t), evaluated by the library
    for every level stepped without a device source.
    """

    def __init__(self, *, alpha: float, beta: float, n: int, M: int, gamma, dplus, dminus,
                 phi: Optional[Callable] = None, f: Optional[Callable] = None,
                 a: float = 0.0, b: float = 1.0, T: float = 1.0, rtol: float = 1e-10, maxit: int = 500,
                 warm_start: int = N.TSFCDE_WS_ZERO, flags: int = 0, precision: int = N.TSFCDE_FP64,
                 krylov: int = N.TSFCDE_KRYLOV_CGS, preconditioner: int = N.TSFCDE_PREC_STRANG,
                 history_tol: float = 0.0,
                 device: Optional[torch.device] = None, stream: Optional[torch.cuda.Stream] = None):
        self._lib = N.lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.n, self.M = int(n), int(M)
        for v in (gamma, dplus, dminus):
            if not callable(v) and len(v) != self.M:
                raise ValueError("coefficient samples must have length M")
        self._keep = []
        self.problem = _problem(alpha=alpha, beta=beta, n=n, M=M, a=a, b=b, T=T, gamma=gamma, dplus=dplus,
                                dminus=dminus, phi=phi, f=f, rtol=rtol, maxit=maxit, precision=precision,
                                warm_start=warm_start, flags=flags, keep=self._keep, krylov=krylov,
                                preconditioner=preconditioner, history_tol=history_tol)
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
    def from_problem(cls, prob, callbacks: bool = False, **kw):
        """Build from a problem description (workloads.Problem: alpha, beta,
        n, M, a, b, T and the callables gamma, dplus, dminus, phi(x), f(x, t)).
        The coefficients go to the library as callbacks.  u^0 is phi at the
        plan's nodes, set from one vectorised call; with ``callbacks`` phi and
        f go to the library as scalar callbacks too (one host call per node,
        for small n), and steps without a device source take f from there."""
        s = cls(alpha=prob.alpha, beta=prob.beta, n=prob.n, M=prob.M, gamma=prob.gamma, dplus=prob.dplus,
                dminus=prob.dminus, phi=_scalar_phi(prob) if callbacks else None,
                f=_scalar_f(prob) if callbacks else None, a=prob.a, b=prob.b, T=prob.T, **kw)
        if not callbacks:
            u0 = torch.as_tensor(np.asarray(prob.phi(s.nodes()), dtype=np.float64), device=s.device)
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

    def level_time(self, j: int) -> float:
        """t_{j+sigma} of level j as the plan samples it."""
        return float(self._lib.tsfcde_level_time(self._plan, j))

    def level_times(self) -> np.ndarray:
        return np.array([self.level_time(j) for j in range(self.M)])

    def nodes(self) -> np.ndarray:
        """The plan's interior nodes x_1..x_n."""
        x = np.empty(self.n, dtype=np.float64)
        N.check(self._lib.tsfcde_nodes(self._plan, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                "tsfcde_nodes")
        return x

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
    """Many independent instances advanced with grouped launches
    (tsfcde_plan_batch / tsfcde_batch_step level by level, or
    tsfcde_batch_solve for every remaining level).  ``problems`` are
    problem descriptions as for TimeLevelSolver.from_problem, all with the
    same M; coefficients go to the library as callbacks, u^0 is phi at each
    member's nodes, and with ``callbacks`` f is a callback too."""

    def __init__(self, problems, *, rtol: float = 1e-10, maxit: int = 500, warm_start: int = N.TSFCDE_WS_ZERO,
                 precision: int = N.TSFCDE_FP64, flags: int = 0, callbacks: bool = False,
                 preconditioner: int = N.TSFCDE_PREC_STRANG, krylov: int = N.TSFCDE_KRYLOV_CGS,
                 device: Optional[torch.device] = None, stream: Optional[torch.cuda.Stream] = None):
        self._lib = N.lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.count = len(problems)
        self.M = problems[0].M
        self.ns = [p.n for p in problems]
        self._keep = []
        arr = (N.tsfcde_problem * self.count)()
        for i, prob in enumerate(problems):
            arr[i] = _problem(alpha=prob.alpha, beta=prob.beta, n=prob.n, M=prob.M, a=prob.a, b=prob.b, T=prob.T,
                              gamma=prob.gamma, dplus=prob.dplus, dminus=prob.dminus, phi=None,
                              f=_scalar_f(prob) if callbacks else None, rtol=rtol, maxit=maxit,
                              precision=precision, warm_start=warm_start, flags=flags, keep=self._keep,
                              krylov=krylov, preconditioner=preconditioner)
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
            u0 = torch.as_tensor(np.asarray(prob.phi(self.nodes(i)), dtype=np.float64), device=self.device)
            N.check(self._lib.tsfcde_set_state(self.member(i), 0, ctypes.c_void_p(u0.data_ptr())), "tsfcde_set_state")
        torch.cuda.synchronize(self.device)

    def member(self, i: int):
        return self._lib.tsfcde_batch_member(self._batch, i)

    def groups(self):
        """[(L, members, values per lane of the middle passes)] per group."""
        out = []
        for g in range(int(self._lib.tsfcde_batch_group_count(self._batch))):
            L, m, e = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
            N.check(self._lib.tsfcde_batch_group_info(self._batch, g, ctypes.byref(L), ctypes.byref(m),
                                                      ctypes.byref(e)), "tsfcde_batch_group_info")
            out.append((L.value, m.value, e.value))
        return out

    def nodes(self, i: int) -> np.ndarray:
        """Member i's interior nodes."""
        x = np.empty(self.ns[i], dtype=np.float64)
        N.check(self._lib.tsfcde_nodes(self.member(i), x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                "tsfcde_nodes")
        return x

    def level_times(self, i: int) -> np.ndarray:
        """Member i's sampling instants t_{j+sigma}, j = 0..M-1."""
        h = self.member(i)
        return np.array([float(self._lib.tsfcde_level_time(h, j)) for j in range(self.M)])

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

    def solve(self, Fs=None, raise_on_error=True):
        """Every remaining level of every instance in one call
        (tsfcde_batch_solve): instances advance on their own.  Fs: list of
        device tensors, entry i holding f of instance i at level j in row j
        (M x ld, ld >= n), or None (entries may be None) for the f callback.
        Returns (code, stats) with stats a numpy structured array of shape
        (count, levels) with the fields of tsfcde_stats."""
        nlev = self.M - int(self._level())
        ptrs = lds = None
        if Fs is not None:
            ptrs = (ctypes.c_void_p * self.count)(*[F.data_ptr() if F is not None else None for F in Fs])
            lds = (ctypes.c_int64 * self.count)(*[F.stride(0) if F is not None else 0 for F in Fs])
        stats = (N.tsfcde_stats * (self.count * max(nlev, 1)))()
        code = self._lib.tsfcde_batch_solve(self._batch, ptrs, lds, stats)
        if raise_on_error:
            N.check(code, "tsfcde_batch_solve")
        arr = np.frombuffer(stats, dtype=N.STATS_DTYPE).reshape(self.count, max(nlev, 1))[:, :nlev].copy()
        return code, arr

    def _level(self):
        return self._lib.tsfcde_level(self.member(0))

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
