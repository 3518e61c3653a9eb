"""Problem statements and manufactured solutions for the TSFCDE (1.1).

Conventions (shared by the oracle and the GPU path):

* ``n`` is the number of interior unknowns and ``M`` the number of time
  steps; where the grid points and sampling instants lie is the solver's
  business (the CPU oracle and the library each compute their own).
* Coefficients gamma(t), d_+(t), d_-(t), the source f(x, t) and the initial
  condition phi(x) are plain callables of continuous x and t.

Manufactured solutions have the separable form u(x, t) = theta(t) * P(x),
with theta a finite sum of powers of t and P a polynomial carrying a double
root at both ends of [a, b].  The source f is then closed form:

  Caputo derivative of t^e (e > 0):  Gamma(e+1)/Gamma(e+1-alpha) t^(e-alpha)
  left RL derivative of (x-a)^k:      Gamma(k+1)/Gamma(k+1-beta) (x-a)^(k-beta)
  right RL derivative of (b-x)^k:     Gamma(k+1)/Gamma(k+1-beta) (b-x)^(k-beta)

(definitions (1.2)-(1.4)), and f = D_t^alpha u - gamma u_x - d_+ D_left u
- d_- D_right u by (1.1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 20160301


@dataclass
class ManufacturedSolution:
    """u(x, t) = theta(t) * P(x).

    ``theta_terms``: list of (coefficient, exponent) pairs, theta(t) = sum c t^e.
    ``poly_s``: coefficients of P in powers of s = x - a (ascending order);
    entries for s^0 and s^1 must vanish (double root at x = a), and the
    polynomial must have a double root at x = b too.
    """

    theta_terms: Sequence[Tuple[float, float]]
    poly_s: np.ndarray
    a: float = 0.0
    b: float = 1.0

    def __post_init__(self):
        p = np.asarray(self.poly_s, dtype=np.float64)
        self.poly_s = p
        # Coefficients of P in powers of r = b - x: substitute s = (b-a) - r.
        ell = self.b - self.a
        deg = len(p) - 1
        q = np.zeros(deg + 1)
        for k, pk in enumerate(p):
            # ((b-a) - r)^k = sum_m C(k,m) (b-a)^(k-m) (-r)^m
            for m in range(k + 1):
                q[m] += pk * math.comb(k, m) * ell ** (k - m) * (-1.0) ** m
        # P has a double root at x = b by construction; the r^0, r^1
        # coefficients are zero in exact arithmetic and are set so here, so
        # that no rounding residue multiplies the singular (b-x)^(k-beta).
        q[:2] = 0.0
        if abs(p[0]) > 0 or abs(p[1]) > 0:
            raise ValueError("P must have a double root at x = a")
        self.poly_r = q

    # --- time factor -----------------------------------------------------
    def theta(self, t):
        return sum(c * (t ** e if e != 0 else 1.0) for c, e in self.theta_terms)

    def caputo_theta(self, t, alpha):
        out = 0.0
        for c, e in self.theta_terms:
            if e == 0:
                continue
            out += c * math.gamma(e + 1.0) / math.gamma(e + 1.0 - alpha) * t ** (e - alpha)
        return out

    # --- space factor ----------------------------------------------------
    def P(self, x):
        s = np.asarray(x, dtype=np.float64) - self.a
        return np.polynomial.polynomial.polyval(s, self.poly_s)

    def dP(self, x):
        s = np.asarray(x, dtype=np.float64) - self.a
        return np.polynomial.polynomial.polyval(s, np.polynomial.polynomial.polyder(self.poly_s))

    def rl_left(self, x, beta):
        s = np.asarray(x, dtype=np.float64) - self.a
        out = np.zeros_like(s)
        for k, pk in enumerate(self.poly_s):
            if pk == 0.0:
                continue
            out += pk * math.gamma(k + 1.0) / math.gamma(k + 1.0 - beta) * s ** (k - beta)
        return out

    def rl_right(self, x, beta):
        r = self.b - np.asarray(x, dtype=np.float64)
        out = np.zeros_like(r)
        for k, qk in enumerate(self.poly_r):
            if qk == 0.0:
                continue
            out += qk * math.gamma(k + 1.0) / math.gamma(k + 1.0 - beta) * r ** (k - beta)
        return out

    def u(self, x, t):
        return self.theta(t) * self.P(x)

    def profiles(self, x, beta):
        """The four x-profiles [P, P', D_left P, D_right P] (shape 4 x len(x))."""
        return np.stack([self.P(x), self.dP(x), self.rl_left(x, beta), self.rl_right(x, beta)])

    def profile_coeffs(self, t, alpha, gamma, dplus, dminus):
        """Scalars c(t) with f(x, t) = sum_k c_k(t) * profiles_k(x)."""
        th = self.theta(t)
        return np.array([self.caputo_theta(t, alpha), -th * gamma(t), -th * dplus(t), -th * dminus(t)])


@dataclass
class Problem:
    """Problem (1.1) with its discretisation sizes.

    f(x, t) takes an array x and a scalar t; phi(x) an array x.
    """

    alpha: float
    beta: float
    n: int
    M: int
    gamma: Callable[[float], float]
    dplus: Callable[[float], float]
    dminus: Callable[[float], float]
    a: float = 0.0
    b: float = 1.0
    T: float = 1.0
    solution: Optional[ManufacturedSolution] = None
    phi_fn: Optional[Callable] = None
    f_fn: Optional[Callable] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    # --- data ------------------------------------------------------------
    def phi(self, x) -> np.ndarray:
        if self.phi_fn is not None:
            return np.asarray(self.phi_fn(x), dtype=np.float64)
        if self.solution is not None:
            return self.solution.u(x, 0.0)
        return np.zeros_like(np.asarray(x, dtype=np.float64))

    def f(self, x, t) -> np.ndarray:
        if self.f_fn is not None:
            return np.asarray(self.f_fn(x, t), dtype=np.float64)
        if self.solution is None:
            return np.zeros_like(np.asarray(x, dtype=np.float64))
        sol = self.solution
        return (sol.caputo_theta(t, self.alpha) * sol.P(x)
                - sol.theta(t) * (self.gamma(t) * sol.dP(x)
                                  + self.dplus(t) * sol.rl_left(x, self.beta)
                                  + self.dminus(t) * sol.rl_right(x, self.beta)))

    def exact(self, x, t) -> np.ndarray:
        if self.solution is None:
            raise ValueError("no closed-form solution for this problem")
        return self.solution.u(x, t)

    # --- separable sources -----------------------------------------------
    def source_matrix(self, x, ts):
        """(profiles[4, len(x)], coeffs[len(ts), 4]) with f(x, t_k) =
        coeffs[k] @ profiles for a manufactured problem without a custom f:
        all sources at the nodes x and the instants ts come from one small
        matrix product.  The caller chooses x and ts."""
        if self.solution is None or self.f_fn is not None:
            raise ValueError("separable source only for manufactured problems")
        prof = self.solution.profiles(np.asarray(x, dtype=np.float64), self.beta)
        co = np.stack([self.solution.profile_coeffs(float(t), self.alpha, self.gamma, self.dplus, self.dminus)
                       for t in ts])
        return prof, co


def device_sources(prob: Problem, x, ts, device):
    """f(x_i, t_k) for every instant t_k in ``ts`` (rows) at the nodes ``x``,
    as an FP64 torch tensor on ``device``, from the separable form of a
    manufactured source (one (K x 4) @ (4 x n) product)."""
    import torch
    prof, co = prob.source_matrix(x, ts)
    return (torch.as_tensor(co, dtype=torch.float64, device=device)
            @ torch.as_tensor(prof, dtype=torch.float64, device=device)).contiguous()


def _x2_one_minus_x2(extra=(1.0,)):
    """Coefficients in s = x of x^2 (1-x)^2 * (e0 + e1 x + e2 x^2 ...) on [0, 1]."""
    base = np.array([0.0, 0.0, 1.0, -2.0, 1.0])
    return np.polynomial.polynomial.polymul(base, np.asarray(extra, dtype=np.float64))


def example1(alpha: float, beta: float, N: int, M: Optional[int] = None) -> Problem:
    """Example 1 of Sec. 4: d_+ = 0.8, d_- = 0.5, gamma = -0.1 on [0,1]x[0,1],
    u = (t^(2+alpha) + 1) x^2 (1-x)^2.  ``N`` is the paper's number of
    subintervals; ``M`` (time steps) defaults to N."""
    M = N if M is None else M
    sol = ManufacturedSolution([(1.0, 2.0 + alpha), (1.0, 0.0)], _x2_one_minus_x2())
    return Problem(alpha=alpha, beta=beta, n=N - 1, M=M,
                   gamma=lambda t: -0.1, dplus=lambda t: 0.8, dminus=lambda t: 0.5,
                   solution=sol, name=f"example1(alpha={alpha},beta={beta},N={N},M={M})")


def example2(alpha: float, beta: float, N: int, M: Optional[int] = None) -> Problem:
    """Example 2 of Sec. 4: d_+ = 9 sin t, d_- = 4 sin t, gamma = -t, same
    solution family as Example 1 (the exact solution printed there drops the
    '+1' that its initial condition and source require)."""
    M = N if M is None else M
    sol = ManufacturedSolution([(1.0, 2.0 + alpha), (1.0, 0.0)], _x2_one_minus_x2())
    return Problem(alpha=alpha, beta=beta, n=N - 1, M=M,
                   gamma=lambda t: -t, dplus=lambda t: 9.0 * math.sin(t),
                   dminus=lambda t: 4.0 * math.sin(t),
                   solution=sol, name=f"example2(alpha={alpha},beta={beta},N={N},M={M})")


def config_small(n: int = 64, M: int = 64, alpha: float = 0.5, beta: float = 1.5) -> Problem:
    """Small plain-method case: alpha=0.5, beta=1.5, n=64 interior points, M=64,
    gamma = -(1+t)/2, d_+ = 1+t, d_- = 0.5(1+t), u = t^2 x^2 (1-x)^2, phi = 0."""
    sol = ManufacturedSolution([(1.0, 2.0)], _x2_one_minus_x2())
    return Problem(alpha=alpha, beta=beta, n=n, M=M,
                   gamma=lambda t: -(1.0 + t) / 2.0, dplus=lambda t: 1.0 + t,
                   dminus=lambda t: 0.5 * (1.0 + t), solution=sol,
                   name=f"small(n={n},M={M},alpha={alpha},beta={beta})")


def config_large(n: int = 1 << 20, M: int = 512, alpha: float = 0.7, beta: float = 1.8,
                 seed: int = SEED_BASE + 1) -> Problem:
    """Large single-instance case: alpha=0.7, beta=1.8, n=2^20, M=512, the
    coefficient family of ``config_small`` and
    u = t^2 x^2 (1-x)^2 (A0 + A1 x + A2 x^2) with A_i ~ U(0.5, 2) drawn from
    ``numpy.random.default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    amps = rng.uniform(0.5, 2.0, size=3)
    sol = ManufacturedSolution([(1.0, 2.0)], _x2_one_minus_x2(amps))
    return Problem(alpha=alpha, beta=beta, n=n, M=M,
                   gamma=lambda t: -(1.0 + t) / 2.0, dplus=lambda t: 1.0 + t,
                   dminus=lambda t: 0.5 * (1.0 + t), solution=sol,
                   name=f"large(n={n},M={M},alpha={alpha},beta={beta})",
                   meta={"amplitudes": amps.tolist(), "seed": seed})


def config_large_constant(n: int = 1 << 20, M: int = 512, alpha: float = 0.7, beta: float = 1.8,
                          seed: int = SEED_BASE + 1) -> Problem:
    """The large single-instance case with Example 1's constant coefficients
    (gamma = -0.1, d_+ = 0.8, d_- = 0.5) in place of the time-dependent ones,
    the same seeded solution family: the workload of the constant-coefficient
    path (Algorithm 3)."""
    rng = np.random.default_rng(seed)
    amps = rng.uniform(0.5, 2.0, size=3)
    sol = ManufacturedSolution([(1.0, 2.0)], _x2_one_minus_x2(amps))
    return Problem(alpha=alpha, beta=beta, n=n, M=M,
                   gamma=lambda t: -0.1, dplus=lambda t: 0.8, dminus=lambda t: 0.5, solution=sol,
                   name=f"large_constant(n={n},M={M},alpha={alpha},beta={beta})",
                   meta={"amplitudes": amps.tolist(), "seed": seed})


def batched_instances(count: int = 512, M: int = 128, nmin: int = 1 << 10, nmax: int = 1 << 16,
                      seed: int = SEED_BASE + 3):
    """Independent instances of uneven size: n = round(exp(U(ln nmin, ln nmax))),
    alpha ~ U(0.1, 0.95), beta ~ U(1.1, 1.95), d_+- = c_+-(1+t) with
    c_+- ~ U(0.2, 2), gamma = g (1+t) with g ~ U(-1, 1), and a per-instance
    solution u = A t^2 x^2 (1-x)^2 with A ~ U(0.5, 2)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        alpha = float(rng.uniform(0.1, 0.95))
        beta = float(rng.uniform(1.1, 1.95))
        cp, cm = (float(v) for v in rng.uniform(0.2, 2.0, size=2))
        g = float(rng.uniform(-1.0, 1.0))
        A = float(rng.uniform(0.5, 2.0))
        sol = ManufacturedSolution([(A, 2.0)], _x2_one_minus_x2())
        out.append(Problem(alpha=alpha, beta=beta, n=n, M=M,
                           gamma=(lambda t, g=g: g * (1.0 + t)),
                           dplus=(lambda t, c=cp: c * (1.0 + t)),
                           dminus=(lambda t, c=cm: c * (1.0 + t)),
                           solution=sol, name=f"batch[{k}](n={n})",
                           meta={"c_plus": cp, "c_minus": cm, "g": g, "A": A}))
    return out


HELD_OUT = ((0.45, 0.6), (1.45, 1.6))  # (alpha, beta) rectangle kept out of training


def warmstart_instances(count: int, n: int, M: int, seed: int = SEED_BASE + 4, held_out: bool = False):
    """Instances for the learned warm start: the batched family's parameter
    distributions at one grid size n, with (alpha, beta) outside the held-out
    rectangle HELD_OUT (training) or inside it (held-out evaluation), and
    Example 2's time dependence u = A (t^{2+alpha} + 1) x^2 (1-x)^2, whose
    third time difference (of order step^3 t^{alpha-1}) leaves quadratic extrapolation
    a smooth error to correct (for a solution quadratic in t it would be
    exact).  Rejection sampling keeps the two sets disjoint for any seed."""
    rng = np.random.default_rng(seed)
    (a0, a1), (b0, b1) = HELD_OUT
    out = []
    while len(out) < count:
        if held_out:
            alpha, beta = float(rng.uniform(a0, a1)), float(rng.uniform(b0, b1))
        else:
            alpha, beta = float(rng.uniform(0.1, 0.95)), float(rng.uniform(1.1, 1.95))
            if a0 <= alpha <= a1 and b0 <= beta <= b1:
                continue
        cp, cm = (float(v) for v in rng.uniform(0.2, 2.0, size=2))
        g = float(rng.uniform(-1.0, 1.0))
        A = float(rng.uniform(0.5, 2.0))
        k = len(out)
        sol = ManufacturedSolution([(A, 2.0 + alpha), (A, 0.0)], _x2_one_minus_x2())
        out.append(Problem(alpha=alpha, beta=beta, n=n, M=M,
                           gamma=(lambda t, g=g: g * (1.0 + t)),
                           dplus=(lambda t, c=cp: c * (1.0 + t)),
                           dminus=(lambda t, c=cm: c * (1.0 + t)),
                           solution=sol, name=f"warm[{k}](n={n})",
                           meta={"c_plus": cp, "c_minus": cm, "g": g, "A": A}))
    return out


# ---------------------------------------------------------------------------
# Two space dimensions (the extension the paper names as future work):
#   D_t^alpha u = gx u_x + gy u_y + dxp D_{a+,x}^bx u + dxm D_{x,b-}^bx u
#                 + dyp D_{c+,y}^by u + dym D_{y,d-}^by u + f   on [a,b] x [c,d],
# u = 0 on the boundary, u(x, y, 0) = phi(x, y).
# ---------------------------------------------------------------------------

@dataclass
class Problem2D:
    """Problem (1.1) in two space dimensions with its discretisation sizes.

    Arrays of the solution are (nx, ny): x along axis 0, y along axis 1.
    A manufactured solution is u = theta(t) Px(x) Py(y) with Px from
    ``sol_x`` (its theta is used) and Py from ``sol_y``."""

    alpha: float
    beta_x: float
    beta_y: float
    nx: int
    ny: int
    M: int
    gamma_x: Callable[[float], float]
    gamma_y: Callable[[float], float]
    dplus_x: Callable[[float], float]
    dminus_x: Callable[[float], float]
    dplus_y: Callable[[float], float]
    dminus_y: Callable[[float], float]
    a: float = 0.0
    b: float = 1.0
    c: float = 0.0
    d: float = 1.0
    T: float = 1.0
    sol_x: Optional[ManufacturedSolution] = None
    sol_y: Optional[ManufacturedSolution] = None
    name: str = ""

    def axis(self, which: str) -> Problem:
        """The one-dimensional problem along x or y (coefficients, order,
        interval and grid of that axis; no source)."""
        if which == "x":
            return Problem(alpha=self.alpha, beta=self.beta_x, n=self.nx, M=self.M, gamma=self.gamma_x,
                           dplus=self.dplus_x, dminus=self.dminus_x, a=self.a, b=self.b, T=self.T)
        return Problem(alpha=self.alpha, beta=self.beta_y, n=self.ny, M=self.M, gamma=self.gamma_y,
                       dplus=self.dplus_y, dminus=self.dminus_y, a=self.c, b=self.d, T=self.T)

    def swapped(self) -> "Problem2D":
        """The same problem with the roles of x and y exchanged."""
        return Problem2D(alpha=self.alpha, beta_x=self.beta_y, beta_y=self.beta_x, nx=self.ny, ny=self.nx,
                         M=self.M, gamma_x=self.gamma_y, gamma_y=self.gamma_x, dplus_x=self.dplus_y,
                         dminus_x=self.dminus_y, dplus_y=self.dplus_x, dminus_y=self.dminus_x, a=self.c,
                         b=self.d, c=self.a, d=self.b, T=self.T,
                         sol_x=None if self.sol_y is None else ManufacturedSolution(
                             self.sol_x.theta_terms, self.sol_y.poly_s, self.sol_y.a, self.sol_y.b),
                         sol_y=None if self.sol_x is None else ManufacturedSolution(
                             [(1.0, 0.0)], self.sol_x.poly_s, self.sol_x.a, self.sol_x.b),
                         name=self.name + " (x<->y)")

    def theta(self, t):
        return self.sol_x.theta(t)

    def phi(self, x, y) -> np.ndarray:
        if self.sol_x is None:
            return np.zeros((len(x), len(y)))
        return self.theta(0.0) * np.outer(self.sol_x.P(x), self.sol_y.P(y))

    def exact(self, x, y, t) -> np.ndarray:
        return self.theta(t) * np.outer(self.sol_x.P(x), self.sol_y.P(y))

    def source_terms(self, x, y, t):
        """(coeffs[7], X[7, nx], Y[7, ny]) with f(x_i, y_k, t) =
        sum_m coeffs[m] X[m, i] Y[m, k] (the closed-form derivatives of
        the separable manufactured solution)."""
        sx, sy = self.sol_x, self.sol_y
        th = self.theta(t)
        Px, Py = sx.P(x), sy.P(y)
        X = np.stack([Px, sx.dP(x), Px, sx.rl_left(x, self.beta_x), sx.rl_right(x, self.beta_x), Px, Px])
        Y = np.stack([Py, Py, sy.dP(y), Py, Py, sy.rl_left(y, self.beta_y), sy.rl_right(y, self.beta_y)])
        co = np.array([sx.caputo_theta(t, self.alpha), -th * self.gamma_x(t), -th * self.gamma_y(t),
                       -th * self.dplus_x(t), -th * self.dminus_x(t), -th * self.dplus_y(t),
                       -th * self.dminus_y(t)])
        return co, X, Y

    def f(self, x, y, t) -> np.ndarray:
        if self.sol_x is None:
            return np.zeros((len(x), len(y)))
        co, X, Y = self.source_terms(x, y, t)
        return (co[:, None] * X).T @ Y


def device_sources_2d(prob: Problem2D, x, y, ts, device):
    """f at the nodes x (axis 0), y (axis 1) and every instant in ``ts`` as an
    FP64 torch tensor (len(ts), nx, ny) on ``device``, from the separable form."""
    import torch
    out = []
    for t in ts:
        co, X, Y = prob.source_terms(np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64), float(t))
        Xd = torch.as_tensor((co[:, None] * X).T, dtype=torch.float64, device=device)
        out.append(Xd @ torch.as_tensor(Y, dtype=torch.float64, device=device))
    return torch.stack(out).contiguous()


def problem_2d(nx: int, ny: int, M: int, alpha: float = 0.6, beta_x: float = 1.7, beta_y: float = 1.4,
               seed: int = SEED_BASE + 5) -> Problem2D:
    """A 2D instance of the headline family: gamma_x = -(1+t)/2, gamma_y =
    (1+t)/4, d_+-^x = c_+-^x (1+t), d_+-^y = c_+-^y (1+t) with seed-drawn
    c ~ U(0.5, 2) and amplitude A ~ U(0.5, 2); u = A t^2 x^2 (1-x)^2 y^2 (1-y)^2."""
    rng = np.random.default_rng(seed)
    cxp, cxm, cyp, cym, A = (float(v) for v in rng.uniform(0.5, 2.0, size=5))
    return Problem2D(alpha=alpha, beta_x=beta_x, beta_y=beta_y, nx=nx, ny=ny, M=M,
                     gamma_x=lambda t: -(1.0 + t) / 2.0, gamma_y=lambda t: (1.0 + t) / 4.0,
                     dplus_x=lambda t, c=cxp: c * (1.0 + t), dminus_x=lambda t, c=cxm: c * (1.0 + t),
                     dplus_y=lambda t, c=cyp: c * (1.0 + t), dminus_y=lambda t, c=cym: c * (1.0 + t),
                     sol_x=ManufacturedSolution([(A, 2.0)], _x2_one_minus_x2()),
                     sol_y=ManufacturedSolution([(1.0, 0.0)], _x2_one_minus_x2()),
                     name=f"2d(nx={nx}, ny={ny}, M={M})")


# ---------------------------------------------------------------------------
# Three space dimensions: the same operator on each of x, y, z,
#   D_t^alpha u = sum_axes [ g u_axis + dp D_{lo+}^b u + dm D_{hi-}^b u ] + f
# on a box, u = 0 on its boundary, u(., 0) = phi.
# ---------------------------------------------------------------------------

@dataclass
class Problem3D:
    """Problem (1.1) in three space dimensions with its discretisation sizes.

    Per-axis data are tuples in axis order (x, y, z); arrays of the solution
    are (nx, ny, nz), z fastest when flattened.  A manufactured solution is
    u = theta(t) Px(x) Py(y) Pz(z) from ``sols`` (theta from sols[0])."""

    alpha: float
    betas: Tuple[float, float, float]
    ns: Tuple[int, int, int]
    M: int
    gammas: Tuple[Callable[[float], float], ...]
    dpluses: Tuple[Callable[[float], float], ...]
    dminuses: Tuple[Callable[[float], float], ...]
    lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    T: float = 1.0
    sols: Optional[Tuple[ManufacturedSolution, ...]] = None
    name: str = ""

    @property
    def N(self) -> int:
        return int(self.ns[0] * self.ns[1] * self.ns[2])

    def axis(self, k: int) -> Problem:
        """The one-dimensional problem along axis k (coefficients, order,
        interval and grid of that axis; no source)."""
        return Problem(alpha=self.alpha, beta=self.betas[k], n=self.ns[k], M=self.M, gamma=self.gammas[k],
                       dplus=self.dpluses[k], dminus=self.dminuses[k], a=self.lo[k], b=self.hi[k], T=self.T)

    def permuted(self, perm) -> "Problem3D":
        """The same problem with its axes reordered: new axis k is old axis
        perm[k] (the solution array is transposed by perm)."""
        pk = lambda v: tuple(v[p] for p in perm)  # noqa: E731
        sols = None
        if self.sols is not None:
            theta = self.sols[0].theta_terms
            sols = tuple(ManufacturedSolution(theta if k == 0 else [(1.0, 0.0)], self.sols[p].poly_s,
                                              self.sols[p].a, self.sols[p].b) for k, p in enumerate(perm))
        return Problem3D(alpha=self.alpha, betas=pk(self.betas), ns=pk(self.ns), M=self.M, gammas=pk(self.gammas),
                         dpluses=pk(self.dpluses), dminuses=pk(self.dminuses), lo=pk(self.lo), hi=pk(self.hi),
                         T=self.T, sols=sols, name=self.name + f" (axes {tuple(perm)})")

    def theta(self, t):
        return self.sols[0].theta(t)

    def _outer(self, a, b, c):
        return a[:, None, None] * b[None, :, None] * c[None, None, :]

    def phi(self, x, y, z) -> np.ndarray:
        if self.sols is None:
            return np.zeros((len(x), len(y), len(z)))
        return self.theta(0.0) * self._outer(self.sols[0].P(x), self.sols[1].P(y), self.sols[2].P(z))

    def exact(self, x, y, z, t) -> np.ndarray:
        return self.theta(t) * self._outer(self.sols[0].P(x), self.sols[1].P(y), self.sols[2].P(z))

    def source_terms(self, x, y, z, t):
        """(coeffs[10], (X[10, nx], Y[10, ny], Z[10, nz])) with f(x_i, y_k, z_l, t)
        = sum_m coeffs[m] X[m, i] Y[m, k] Z[m, l]: the Caputo derivative of
        theta times P, then per axis the convection and the two Riemann-
        Liouville terms (closed forms of the separable solution)."""
        pts = (x, y, z)
        th = self.theta(t)
        P = [s.P(q) for s, q in zip(self.sols, pts)]
        co = [self.sols[0].caputo_theta(t, self.alpha)]
        fac = [list(P)]
        for k in range(3):
            s, q, b = self.sols[k], pts[k], self.betas[k]
            for c, Fk in ((-th * self.gammas[k](t), s.dP(q)), (-th * self.dpluses[k](t), s.rl_left(q, b)),
                          (-th * self.dminuses[k](t), s.rl_right(q, b))):
                co.append(c)
                row = list(P)
                row[k] = Fk
                fac.append(row)
        co = np.array(co)
        return co, tuple(np.stack([r[k] for r in fac]) for k in range(3))

    def f(self, x, y, z, t) -> np.ndarray:
        if self.sols is None:
            return np.zeros((len(x), len(y), len(z)))
        co, (X, Y, Z) = self.source_terms(x, y, z, t)
        return np.einsum("m,mi,mk,ml->ikl", co, X, Y, Z)


def device_sources_3d(prob: Problem3D, x, y, z, ts, device):
    """f at the nodes (x, y, z) and every instant in ``ts`` as an FP64 torch
    tensor (len(ts), nx, ny, nz) on ``device``, from the separable form."""
    import torch
    out = []
    for t in ts:
        co, (X, Y, Z) = prob.source_terms(np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64),
                                          np.asarray(z, dtype=np.float64), float(t))
        Xd = torch.as_tensor(co[:, None] * X, dtype=torch.float64, device=device)
        Yd = torch.as_tensor(Y, dtype=torch.float64, device=device)
        Zd = torch.as_tensor(Z, dtype=torch.float64, device=device)
        XY = (Xd[:, :, None] * Yd[:, None, :]).reshape(len(co), -1)  # (m, nx*ny)
        out.append((XY.T @ Zd).reshape(len(x), len(y), len(z)))
    return torch.stack(out).contiguous()


def problem_3d(nx: int, ny: int, nz: int, M: int, alpha: float = 0.6, betas=(1.7, 1.4, 1.85),
               seed: int = SEED_BASE + 6) -> Problem3D:
    """A 3D instance of the headline family: gamma = (-(1+t)/2, (1+t)/4,
    -(1+t)/3) per axis, d_+- = c_+- (1+t) with seed-drawn c ~ U(0.5, 2) per
    axis and side, amplitude A ~ U(0.5, 2); u = A t^2 prod_axes s^2 (1-s)^2."""
    rng = np.random.default_rng(seed)
    c = [float(v) for v in rng.uniform(0.5, 2.0, size=7)]
    A = c[6]
    sol = lambda theta: ManufacturedSolution(theta, _x2_one_minus_x2())  # noqa: E731
    return Problem3D(alpha=alpha, betas=tuple(float(b) for b in betas), ns=(nx, ny, nz), M=M,
                     gammas=(lambda t: -(1.0 + t) / 2.0, lambda t: (1.0 + t) / 4.0, lambda t: -(1.0 + t) / 3.0),
                     dpluses=tuple((lambda t, cc=c[2 * k]: cc * (1.0 + t)) for k in range(3)),
                     dminuses=tuple((lambda t, cc=c[2 * k + 1]: cc * (1.0 + t)) for k in range(3)),
                     sols=(sol([(A, 2.0)]), sol([(1.0, 0.0)]), sol([(1.0, 0.0)])),
                     name=f"3d(nx={nx}, ny={ny}, nz={nz}, M={M})")
