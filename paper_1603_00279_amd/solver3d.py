"""Thin Python wrapper around the three-dimensional C ABI (include/tsfcde3d.h):
one plan per TimeLevelSolver3D.  PyTorch supplies the device workspace and
the stream; the wrapper only marshals arguments.  Every numerical step runs in
the HIP kernels of libtsfcde.so."""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _native as N
from .solver import _dptr


class TimeLevelSolver3D:
    """The implicit difference scheme in three space dimensions: one plan,
    levels advanced by step / solve.  Arrays are (nx, ny, nz) FP64 device
    tensors (z fastest).  Per-axis arguments are sequences in the order x, y,
    z; coefficients are callables of t (sampled by the library at its own
    t_{j+sigma}); phi(x, y, z) and f(x, y, z, t) callables of scalars are
    optional.  warm_start: TSFCDE_WS_ZERO, _PREV or _EXTRAP."""

    def __init__(self, *, alpha, betas, ns, M, gammas, dpluses, dminuses, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                 T=1.0, phi=None, f=None, rtol=1e-10, maxit=500, warm_start=0, device: Optional[torch.device] = None,
                 stream: Optional[torch.cuda.Stream] = None):
        self._lib = N.lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ns = tuple(int(n) for n in ns)
        self.N = int(np.prod(self.ns))
        self.M = int(M)
        self._keep = []
        p = N.tsfcde3d_problem(alpha=alpha, T=T, M=M, rtol=rtol, maxit=maxit, warm_start=warm_start)
        for k in range(3):
            p.beta[k] = float(betas[k])
            p.lo[k] = float(lo[k])
            p.hi[k] = float(hi[k])
            p.n[k] = self.ns[k]
            for arr, fn in ((p.gamma, gammas[k]), (p.dplus, dpluses[k]), (p.dminus, dminuses[k])):
                cb = N.COEF_FN(lambda t, _u, fn=fn: float(fn(t)))
                self._keep.append(cb)
                arr[k] = cb
        if phi is not None:
            cb = N.IC3_FN(lambda x, y, z, _u, fn=phi: float(fn(x, y, z)))
            self._keep.append(cb)
            p.phi = cb
        if f is not None:
            cb = N.SRC3_FN(lambda x, y, z, t, _u, fn=f: float(fn(x, y, z, t)))
            self._keep.append(cb)
            p.f = cb
        self._prob = p
        nbytes = ctypes.c_size_t(0)
        N.check(self._lib.tsfcde3d_workspace_bytes(ctypes.byref(p), ctypes.byref(nbytes)), "tsfcde3d_workspace_bytes")
        self.workspace_bytes = nbytes.value
        self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            N.check(self._lib.tsfcde3d_plan(ctypes.byref(p), ctypes.c_void_p(base + off), self.workspace_bytes,
                                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)),
                    "tsfcde3d_plan")
        self._plan = handle

    @classmethod
    def from_problem(cls, prob, with_phi: bool = True, **kw):
        """A plan for a workloads.Problem3D; u^0 = phi at the plan's own nodes."""
        s = cls(alpha=prob.alpha, betas=prob.betas, ns=prob.ns, M=prob.M, gammas=prob.gammas,
                dpluses=prob.dpluses, dminuses=prob.dminuses, lo=prob.lo, hi=prob.hi, T=prob.T, **kw)
        if with_phi:
            x, y, z = s.nodes()
            u0 = torch.as_tensor(np.asarray(prob.phi(x, y, z), dtype=np.float64), device=s.device).contiguous()
            s.set_state(0, u0.view((1,) + s.ns))
        return s

    # --- queries ----------------------------------------------------------
    def nodes(self):
        out = [np.empty(n) for n in self.ns]
        dp = ctypes.POINTER(ctypes.c_double)
        N.check(self._lib.tsfcde3d_nodes(self._plan, *(a.ctypes.data_as(dp) for a in out)), "tsfcde3d_nodes")
        return tuple(out)

    def level_times(self) -> np.ndarray:
        return np.array([float(self._lib.tsfcde3d_level_time(self._plan, j)) for j in range(self.M)])

    @property
    def level(self) -> int:
        return int(self._lib.tsfcde3d_level(self._plan))

    def history(self) -> torch.Tensor:
        """Copy of the stored levels, (M+1, nx, ny, nz)."""
        ptr = self._lib.tsfcde3d_history(self._plan)
        off = ptr - self._ws.data_ptr()
        n = (self.M + 1) * self.N
        return self._ws[off: off + 8 * n].view(torch.float64).view((self.M + 1,) + self.ns).clone()

    # --- work ---------------------------------------------------------------
    def set_state(self, level: int, U: torch.Tensor):
        U = U.contiguous()
        if U.numel() != (level + 1) * self.N:
            raise ValueError("U must hold level+1 arrays of nx*ny*nz values")
        N.check(self._lib.tsfcde3d_set_state(self._plan, level, _dptr(U)), "tsfcde3d_set_state")

    def step(self, f: Optional[torch.Tensor] = None, u_out: Optional[torch.Tensor] = None, raise_on_error=True):
        if f is not None and f.numel() != self.N:
            raise ValueError("f must hold nx*ny*nz values")
        if u_out is not None and u_out.numel() != self.N:
            raise ValueError("u_out must hold nx*ny*nz values")
        st = N.tsfcde_stats()
        code = self._lib.tsfcde3d_step(self._plan, _dptr(f.contiguous() if f is not None else None), _dptr(u_out),
                                       ctypes.byref(st))
        if raise_on_error:
            N.check(code, "tsfcde3d_step")
        d = st.as_dict()
        d["code"] = code
        return d

    def solve(self, F: Optional[torch.Tensor] = None, raise_on_error=True):
        """Every remaining level; F: (M, nx, ny, nz) device sources or None."""
        nlev = self.M - self.level
        if F is not None and F.numel() != self.M * self.N:
            raise ValueError("F must hold M arrays of nx*ny*nz values (row j for level j)")
        stats = (N.tsfcde_stats * max(nlev, 1))()
        code = self._lib.tsfcde3d_solve(self._plan, _dptr(F.contiguous() if F is not None else None), self.N, None,
                                        stats)
        if raise_on_error:
            N.check(code, "tsfcde3d_solve")
        return code, [stats[k].as_dict() for k in range(nlev)]

    def apply(self, op: int, j: int, x: torch.Tensor) -> torch.Tensor:
        if x.numel() != self.N:
            raise ValueError("x must hold nx*ny*nz values")
        x = x.contiguous()
        y = torch.empty_like(x)
        N.check(self._lib.tsfcde3d_apply(self._plan, op, j, _dptr(x), _dptr(y)), "tsfcde3d_apply")
        return y

    def close(self):
        if getattr(self, "_plan", None):
            self._lib.tsfcde3d_destroy(self._plan)
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
