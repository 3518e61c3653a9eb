"""Thin Python wrapper around the two-dimensional C ABI (include/tsfcde2d.h):
one plan per TimeLevelSolver2D.  PyTorch supplies the device workspace and
the stream; the wrapper only marshals arguments.  Every numerical step runs in
the HIP kernels of libtsfcde.so."""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _native as N
from .solver import _dptr


class TimeLevelSolver2D:
    """The implicit difference scheme in two space dimensions: one plan,
    levels advanced by step / solve.  Arrays are (nx, ny) FP64 device tensors
    (x along axis 0).  Coefficients are callables of t (sampled by the library
    at its own t_{j+sigma}); phi(x, y) and f(x, y, t) callables of scalars are
    optional (the initial level is 0 without phi; levels stepped without a
    source use f, or 0).  warm_start: TSFCDE_WS_ZERO, _PREV or _EXTRAP."""

    def __init__(self, *, alpha, beta_x, beta_y, nx, ny, M, gamma_x, gamma_y, dplus_x, dminus_x, dplus_y,
                 dminus_y, a=0.0, b=1.0, c=0.0, d=1.0, T=1.0, phi=None, f=None, rtol=1e-10, maxit=500, warm_start=0,
                 device: Optional[torch.device] = None, stream: Optional[torch.cuda.Stream] = None):
        self._lib = N.lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.nx, self.ny, self.M = int(nx), int(ny), int(M)
        self._keep = []
        p = N.tsfcde2d_problem(alpha=alpha, beta_x=beta_x, beta_y=beta_y, a=a, b=b, c=c, d=d, T=T, nx=nx, ny=ny,
                               M=M, rtol=rtol, maxit=maxit, warm_start=warm_start)
        for name, fn in (("gamma_x", gamma_x), ("gamma_y", gamma_y), ("dplus_x", dplus_x), ("dminus_x", dminus_x),
                         ("dplus_y", dplus_y), ("dminus_y", dminus_y)):
            cb = N.COEF_FN(lambda t, _u, fn=fn: float(fn(t)))
            self._keep.append(cb)
            setattr(p, name, cb)
        if phi is not None:
            cb = N.IC2_FN(lambda x, y, _u, fn=phi: float(fn(x, y)))
            self._keep.append(cb)
            p.phi = cb
        if f is not None:
            cb = N.SRC2_FN(lambda x, y, t, _u, fn=f: float(fn(x, y, t)))
            self._keep.append(cb)
            p.f = cb
        self._prob = p
        nbytes = ctypes.c_size_t(0)
        N.check(self._lib.tsfcde2d_workspace_bytes(ctypes.byref(p), ctypes.byref(nbytes)), "tsfcde2d_workspace_bytes")
        self.workspace_bytes = nbytes.value
        self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            N.check(self._lib.tsfcde2d_plan(ctypes.byref(p), ctypes.c_void_p(base + off), self.workspace_bytes,
                                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)),
                    "tsfcde2d_plan")
        self._plan = handle

    @classmethod
    def from_problem(cls, prob, with_phi: bool = True, **kw):
        """A plan for a workloads.Problem2D; u^0 = phi at the plan's own nodes."""
        s = cls(alpha=prob.alpha, beta_x=prob.beta_x, beta_y=prob.beta_y, nx=prob.nx, ny=prob.ny, M=prob.M,
                gamma_x=prob.gamma_x, gamma_y=prob.gamma_y, dplus_x=prob.dplus_x, dminus_x=prob.dminus_x,
                dplus_y=prob.dplus_y, dminus_y=prob.dminus_y, a=prob.a, b=prob.b, c=prob.c, d=prob.d, T=prob.T,
                **kw)
        if with_phi:
            x, y = s.nodes()
            u0 = torch.as_tensor(np.asarray(prob.phi(x, y), dtype=np.float64), device=s.device).contiguous()
            s.set_state(0, u0.view(1, s.nx, s.ny))
        return s

    # --- queries ----------------------------------------------------------
    def nodes(self):
        x = np.empty(self.nx)
        y = np.empty(self.ny)
        dp = ctypes.POINTER(ctypes.c_double)
        N.check(self._lib.tsfcde2d_nodes(self._plan, x.ctypes.data_as(dp), y.ctypes.data_as(dp)), "tsfcde2d_nodes")
        return x, y

    def level_times(self) -> np.ndarray:
        return np.array([float(self._lib.tsfcde2d_level_time(self._plan, j)) for j in range(self.M)])

    @property
    def level(self) -> int:
        return int(self._lib.tsfcde2d_level(self._plan))

    def history(self) -> torch.Tensor:
        """Copy of the stored levels, (M+1, nx, ny)."""
        ptr = self._lib.tsfcde2d_history(self._plan)
        off = ptr - self._ws.data_ptr()
        n = (self.M + 1) * self.nx * self.ny
        return self._ws[off: off + 8 * n].view(torch.float64).view(self.M + 1, self.nx, self.ny).clone()

    # --- work ---------------------------------------------------------------
    def set_state(self, level: int, U: torch.Tensor):
        U = U.contiguous()
        if U.numel() != (level + 1) * self.nx * self.ny:
            raise ValueError("U must hold level+1 arrays of nx*ny values")
        N.check(self._lib.tsfcde2d_set_state(self._plan, level, _dptr(U)), "tsfcde2d_set_state")

    def step(self, f: Optional[torch.Tensor] = None, u_out: Optional[torch.Tensor] = None, raise_on_error=True):
        if f is not None and f.numel() != self.nx * self.ny:
            raise ValueError("f must hold nx*ny values")
        if u_out is not None and u_out.numel() != self.nx * self.ny:
            raise ValueError("u_out must hold nx*ny values")
        st = N.tsfcde_stats()
        code = self._lib.tsfcde2d_step(self._plan, _dptr(f.contiguous() if f is not None else None), _dptr(u_out),
                                       ctypes.byref(st))
        if raise_on_error:
            N.check(code, "tsfcde2d_step")
        d = st.as_dict()
        d["code"] = code
        return d

    def solve(self, F: Optional[torch.Tensor] = None, raise_on_error=True):
        """Every remaining level; F: (M, nx, ny) device sources or None."""
        nlev = self.M - self.level
        if F is not None and F.numel() != self.M * self.nx * self.ny:
            raise ValueError("F must hold M arrays of nx*ny values (row j for level j)")
        stats = (N.tsfcde_stats * max(nlev, 1))()
        ld = self.nx * self.ny
        code = self._lib.tsfcde2d_solve(self._plan, _dptr(F.contiguous() if F is not None else None), ld, None, stats)
        if raise_on_error:
            N.check(code, "tsfcde2d_solve")
        return code, [stats[k].as_dict() for k in range(nlev)]

    def apply(self, op: int, j: int, x: torch.Tensor) -> torch.Tensor:
        if x.numel() != self.nx * self.ny:
            raise ValueError("x must hold nx*ny values")
        x = x.contiguous()
        y = torch.empty_like(x)
        N.check(self._lib.tsfcde2d_apply(self._plan, op, j, _dptr(x), _dptr(y)), "tsfcde2d_apply")
        return y

    def close(self):
        if getattr(self, "_plan", None):
            self._lib.tsfcde2d_destroy(self._plan)
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
