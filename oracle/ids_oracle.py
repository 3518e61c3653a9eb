"""Plain FP64 CPU oracle for the implicit difference scheme (IDS).

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; never by the product path.

Paper: Gu, Huang, Ji, Carpentieri, Alikhanov, "Fast iterative method with a
second order implicit difference scheme for time-space fractional
convection-diffusion equations", arXiv:1603.00279.

What is computed, and where it is defined:

* Grunwald coefficients g_k = (-1)^k binom(beta, k)  -- Lemma 2, computed with
  the recurrence of Lemma 3.
* WSGD weights omega_k from lambda_1, lambda_0, lambda_-1  -- Lemma 2.
* L2-1sigma coefficients a_l, b_l, c_m^(alpha,sigma,j)  -- Lemma 1.
* The matrices Q and W_beta  -- (3.2);  A^(j+sigma), B^(j+sigma), eta_j  --
  (3.1) and (3.3).
* The history term  tau^-alpha/Gamma(2-alpha) sum_{s<j} c_{j-s}(u^{s+1}-u^s),
  entering the right-hand side with a minus sign  -- (3.1).
* One time level: g = B u^j - history + f^{j+sigma};  u^{j+1} = A^{-1} g by
  dense Gaussian elimination (LAPACK dgesv)  -- Algorithm 2 with the direct
  solver the paper uses as its baseline (Sec. 3.2).
* The Strang circulant preconditioner P^(j+sigma) as a dense matrix, and
  the eigenvalues of circulants  -- (3.7), Lemma 8, Sec. 3.2.
* Row-by-row evaluation of (A u)_i and g_i by direct O(n) sums, for checks at
  sizes where no dense matrix fits.
* Constant coefficients: Algorithm 3, with A^-1 applied by the
  Gohberg-Semencul formula of Sec. 3.1 (Algorithm 1) from the two solves
  (3.4), all with dense matrices.

Every function is pinned by ``tests/test_oracle_*.py`` against closed forms,
library special cases, the numbers printed in the paper's tables, and an
independent all-levels-at-once assembly of the scheme.

Readings of the paper taken here (each is also listed in the design notes):

* n = interior unknowns, h = (b-a)/(n+1) (the paper's N is n+1).
* The history term enters (3.3) with the minus sign of (3.1).
* gamma, d_+-, f are sampled at t_{j+sigma}.
* Strang circulant of a Toeplitz matrix with lags t_m:  c_k = t_k for
  0 <= k <= floor(n/2), c_k = t_{k-n} otherwise; s(W^T) is taken as s(W)^T,
  whose eigenvalues are the conjugates of those of s(W) as Sec. 3.2 states.
* DFT sign convention lambda_k = sum_m c_m exp(-2 pi i m k / n).
"""
from __future__ import annotations

import math
from typing import Iterable, Optional

import numpy as np

__all__ = [
    "mesh_h", "time_step", "sigma_of", "t_sigma", "nodes", "initial_level", "source_level",
    "grunwald_weights", "wsgd_lambdas", "wsgd_weights", "l21s_a", "l21s_b", "l21s_c",
    "l21s_kappa", "eta", "matrix_Q", "toeplitz_W", "level_scalars", "level_L", "level_A",
    "level_B", "history_term", "rhs", "level_solve", "march", "error_norms",
    "strang_column", "circulant", "preconditioner_matrix", "circulant_eigenvalues",
    "embedding_column", "apply_A_rows", "apply_P_rows", "rhs_rows", "caputo_l21s",
    "embedding_eigenvalues", "embedding_product", "strang_eigenvalues", "strang_solve", "rhs_fft",
    "level_solve_pcgs", "level_solve_pbicgstab", "tchan_column", "coefficients_constant", "history_perturbation_bound", "gsf_generators", "gsf_matrices", "gsf_apply", "march_gsf",
]


# ---------------------------------------------------------------------------
# The grid of Sec. 2.1 and the sampling instant of Lemma 1.
# ---------------------------------------------------------------------------

def mesh_h(prob) -> float:
    """h = (b - a)/(n + 1): n interior nodes, the paper's N = n + 1
    subintervals (Sec. 2.1)."""
    return (prob.b - prob.a) / (prob.n + 1)


def time_step(prob) -> float:
    """tau = T/M (Sec. 2.1)."""
    return prob.T / prob.M


def sigma_of(alpha: float) -> float:
    """sigma = 1 - alpha/2, the offset of the L2-1sigma formula (Lemma 1)."""
    return 1.0 - alpha / 2.0


def t_sigma(prob, j: int) -> float:
    """t_{j+sigma} = (j + sigma) tau, where level j samples gamma, d_+-, f
    (Lemma 1; the scheme's coefficients gamma^(j+sigma), D_+-^(j+sigma),
    f^(j+sigma) of Sec. 2.1)."""
    return (j + sigma_of(prob.alpha)) * time_step(prob)


def nodes(prob) -> np.ndarray:
    """Interior nodes x_i = a + i h, i = 1..n (Sec. 2.1)."""
    return prob.a + mesh_h(prob) * np.arange(1, prob.n + 1, dtype=np.float64)


def initial_level(prob) -> np.ndarray:
    """u^0_i = phi(x_i) (Sec. 2.1)."""
    return np.asarray(prob.phi(nodes(prob)), dtype=np.float64)


def source_level(prob, j: int) -> np.ndarray:
    """f(x_i, t_{j+sigma}) on the interior nodes ((3.1))."""
    return np.asarray(prob.f(nodes(prob), t_sigma(prob, j)), dtype=np.float64)


# ---------------------------------------------------------------------------
# Space discretisation: Lemma 2 (WSGD) with the recurrence of Lemma 3.
# ---------------------------------------------------------------------------

def grunwald_weights(beta: float, K: int) -> np.ndarray:
    """g_k^(beta) = (-1)^k binom(beta, k) for k = 0..K (Lemma 2), evaluated by
    the recurrence g_0 = 1, g_k = (1 - (beta+1)/k) g_{k-1} of Lemma 3."""
    factors = np.empty(K + 1, dtype=np.float64)
    factors[0] = 1.0
    k = np.arange(1, K + 1, dtype=np.float64)
    factors[1:] = 1.0 - (beta + 1.0) / k
    return np.cumprod(factors)


def wsgd_lambdas(beta: float):
    """lambda_1, lambda_0, lambda_-1 of Lemma 2."""
    lam1 = (beta * beta + 3.0 * beta + 2.0) / 12.0
    lam0 = (4.0 - beta * beta) / 6.0
    lamm1 = (beta * beta - 3.0 * beta + 2.0) / 12.0
    return lam1, lam0, lamm1


def wsgd_weights(beta: float, K: int) -> np.ndarray:
    """omega_k^(beta), k = 0..K (Lemma 2):
    omega_0 = l1 g_0, omega_1 = l1 g_1 + l0 g_0,
    omega_k = l1 g_k + l0 g_{k-1} + l_-1 g_{k-2} (k >= 2)."""
    g = grunwald_weights(beta, K)
    lam1, lam0, lamm1 = wsgd_lambdas(beta)
    w = lam1 * g
    if K >= 1:
        w[1:] += lam0 * g[:-1]
    if K >= 2:
        w[2:] += lamm1 * g[:-2]
    return w


# ---------------------------------------------------------------------------
# Time discretisation: the L2-1sigma formula of Lemma 1.
# ---------------------------------------------------------------------------

def l21s_a(alpha: float, L: int) -> np.ndarray:
    """a_0 = sigma^(1-alpha); a_l = (l+sigma)^(1-alpha) - (l-1+sigma)^(1-alpha)
    for l = 1..L (Lemma 1)."""
    sigma = 1.0 - alpha / 2.0
    a = np.empty(L + 1, dtype=np.float64)
    a[0] = sigma ** (1.0 - alpha)
    for l in range(1, L + 1):
        a[l] = (l + sigma) ** (1.0 - alpha) - (l - 1 + sigma) ** (1.0 - alpha)
    return a


def l21s_b(alpha: float, L: int) -> np.ndarray:
    """b_l for l = 1..L (index 0 unused, set to 0) (Lemma 1):
    b_l = [(l+sigma)^(2-alpha) - (l-1+sigma)^(2-alpha)]/(2-alpha)
          - [(l+sigma)^(1-alpha) + (l-1+sigma)^(1-alpha)]/2."""
    sigma = 1.0 - alpha / 2.0
    b = np.zeros(L + 1, dtype=np.float64)
    for l in range(1, L + 1):
        b[l] = (((l + sigma) ** (2.0 - alpha) - (l - 1 + sigma) ** (2.0 - alpha)) / (2.0 - alpha)
                - 0.5 * ((l + sigma) ** (1.0 - alpha) + (l - 1 + sigma) ** (1.0 - alpha)))
    return b


def l21s_c(alpha: float, j: int) -> np.ndarray:
    """c_m^(alpha,sigma,j) for m = 0..j (Lemma 1).

    j = 0: c_0 = a_0.  j >= 1: c_0 = a_0 + b_1; c_m = a_m + b_{m+1} - b_m for
    1 <= m <= j-1; c_j = a_j - b_j."""
    a = l21s_a(alpha, j + 1)
    b = l21s_b(alpha, j + 1)
    c = np.empty(j + 1, dtype=np.float64)
    if j == 0:
        c[0] = a[0]
        return c
    c[0] = a[0] + b[1]
    for m in range(1, j):
        c[m] = a[m] + b[m + 1] - b[m]
    c[j] = a[j] - b[j]
    return c


def l21s_kappa(alpha: float, tau: float) -> float:
    """tau^-alpha / Gamma(2 - alpha), the prefactor of Lemma 1."""
    return tau ** (-alpha) / math.gamma(2.0 - alpha)


def caputo_l21s(alpha: float, tau: float, values: np.ndarray, j: int) -> float:
    """Delta^alpha_{0,t_{j+sigma}} u of Lemma 1 for u sampled at t_0..t_{j+1}."""
    c = l21s_c(alpha, j)
    acc = 0.0
    for s in range(j + 1):
        acc += c[j - s] * (values[s + 1] - values[s])
    return l21s_kappa(alpha, tau) * acc


def eta(alpha: float, tau: float, j: int) -> float:
    """eta_j = c_0^(alpha,sigma,j) / (tau^alpha Gamma(2-alpha))  (Sec. 3, after (3.1))."""
    return l21s_kappa(alpha, tau) * l21s_c(alpha, j)[0]


# ---------------------------------------------------------------------------
# Matrix form (3.1)-(3.3).
# ---------------------------------------------------------------------------

def matrix_Q(n: int) -> np.ndarray:
    """Q of (3.2): +1 on the superdiagonal, -1 on the subdiagonal."""
    Q = np.zeros((n, n))
    i = np.arange(n - 1)
    Q[i, i + 1] = 1.0
    Q[i + 1, i] = -1.0
    return Q


def toeplitz_W(beta: float, n: int) -> np.ndarray:
    """W_beta of (3.2): W[i, k] = omega_{i-k+1} for i - k + 1 >= 0, else 0."""
    w = wsgd_weights(beta, n)
    lag = np.arange(n)[:, None] - np.arange(n)[None, :] + 1
    return np.where(lag >= 0, w[np.clip(lag, 0, n)], 0.0)


def level_scalars(prob, j: int):
    """(eta_j, gamma^(j+sigma), D_+^(j+sigma), D_-^(j+sigma)) for level j."""
    t = t_sigma(prob, j)
    return eta(prob.alpha, time_step(prob), j), prob.gamma(t), prob.dplus(t), prob.dminus(t)


def level_L(prob, j: int) -> np.ndarray:
    """gamma/(2h) Q + D_+/h^beta W + D_-/h^beta W^T at t_{j+sigma}."""
    _, gam, dp, dm = level_scalars(prob, j)
    n, h, beta = prob.n, mesh_h(prob), prob.beta
    W = toeplitz_W(beta, n)
    return gam / (2.0 * h) * matrix_Q(n) + dp / h ** beta * W + dm / h ** beta * W.T


def level_A(prob, j: int) -> np.ndarray:
    """A^(j+sigma) = eta_j I - sigma L  (3.3)."""
    e = level_scalars(prob, j)[0]
    return e * np.eye(prob.n) - sigma_of(prob.alpha) * level_L(prob, j)


def level_B(prob, j: int) -> np.ndarray:
    """B^(j+sigma) = eta_j I + (1 - sigma) L  (3.3)."""
    e = level_scalars(prob, j)[0]
    return e * np.eye(prob.n) + (1.0 - sigma_of(prob.alpha)) * level_L(prob, j)


def history_term(prob, U: np.ndarray, j: int) -> np.ndarray:
    """tau^-alpha/Gamma(2-alpha) * sum_{s=0}^{j-1} c_{j-s}^(j) (u^{s+1} - u^s),
    the delta u^(j) of (3.3) (zero for j = 0)."""
    n = U.shape[1]
    acc = np.zeros(n)
    if j == 0:
        return acc
    c = l21s_c(prob.alpha, j)
    for s in range(j):
        acc += c[j - s] * (U[s + 1] - U[s])
    return l21s_kappa(prob.alpha, time_step(prob)) * acc


def rhs(prob, U: np.ndarray, j: int, f_j: np.ndarray) -> np.ndarray:
    """g^(j+1) = B^(j+sigma) u^j - history + f^(j+sigma)  ((3.1), Algorithm 2)."""
    return level_B(prob, j) @ U[j] - history_term(prob, U, j) + f_j


def level_solve(prob, U: np.ndarray, j: int, f_j: np.ndarray) -> np.ndarray:
    """u^{j+1} = (A^(j+sigma))^{-1} g^(j+1) by Gaussian elimination."""
    return np.linalg.solve(level_A(prob, j), rhs(prob, U, j, f_j))


def march(prob, f_levels: Optional[Iterable[np.ndarray]] = None, levels: Optional[int] = None,
          u0: Optional[np.ndarray] = None) -> np.ndarray:
    """Algorithm 2 with a dense direct solve at every level.

    Returns U with U[j] = u^j on the interior nodes, j = 0..levels."""
    M = prob.M if levels is None else levels
    U = np.zeros((M + 1, prob.n))
    U[0] = initial_level(prob) if u0 is None else u0
    flist = list(f_levels) if f_levels is not None else None
    for j in range(M):
        f_j = flist[j] if flist is not None else source_level(prob, j)
        U[j + 1] = level_solve(prob, U, j, f_j)
    return U


def error_norms(prob, U: np.ndarray):
    """(max_j ||E^j||_0, max_{i,j} |E_i^j|) with ||v||_0 = sqrt(h sum v_i^2)
    (Sec. 2.2 and the tables of Sec. 4)."""
    x = nodes(prob)
    l2 = 0.0
    cmax = 0.0
    for j in range(U.shape[0]):
        E = U[j] - prob.exact(x, j * time_step(prob))
        l2 = max(l2, math.sqrt(mesh_h(prob) * float(E @ E)))
        cmax = max(cmax, float(np.max(np.abs(E))))
    return l2, cmax


# ---------------------------------------------------------------------------
# Circulant preconditioner (3.7) and circulant spectra (Sec. 3.2, Lemma 8).
# ---------------------------------------------------------------------------

def strang_column(lag_value, n: int) -> np.ndarray:
    """First column of the Strang circulant of a Toeplitz matrix whose entry
    at lag m = i - k is lag_value(m):  c_k = t_k (0 <= k <= floor(n/2)),
    c_k = t_{k-n} (floor(n/2) < k < n)."""
    c = np.zeros(n)
    for k in range(n):
        c[k] = lag_value(k) if k <= n // 2 else lag_value(k - n)
    return c


def tchan_column(lag_value, n: int) -> np.ndarray:
    """First column of T. Chan's optimal circulant of a Toeplitz matrix whose
    entry at lag m = i - k is lag_value(m): c_k = ((n - k) t_k + k t_{k-n}) / n
    (T. Chan, SIAM J. Sci. Stat. Comput. 9 (1988); the circulant nearest to
    the Toeplitz matrix in the Frobenius norm)."""
    c = np.zeros(n)
    for k in range(n):
        c[k] = ((n - k) * lag_value(k) + (k * lag_value(k - n) if k > 0 else 0.0)) / n
    return c


def circulant(col: np.ndarray) -> np.ndarray:
    """Dense circulant C[i, k] = col[(i - k) mod n]."""
    n = len(col)
    i = np.arange(n)[:, None]
    k = np.arange(n)[None, :]
    return col[(i - k) % n]


def _W_lag(beta: float, n: int):
    w = wsgd_weights(beta, n + 1)

    def lag(m):
        return w[m + 1] if m >= -1 else 0.0
    return lag


def _Q_lag(m):
    return -1.0 if m == 1 else (1.0 if m == -1 else 0.0)


def preconditioner_matrix(prob, j: int, kind: str = "strang") -> np.ndarray:
    """P^(j+sigma) = eta_j I - sigma (gamma/(2h) s(Q) + D_+/h^beta s(W)
    + D_-/h^beta s(W)^T)  (3.7), as a dense matrix; kind "tchan" puts T.
    Chan's circulant c(.) in place of Strang's s(.) (c(W^T) = c(W)^T
    exactly)."""
    e, gam, dp, dm = level_scalars(prob, j)
    n, h, beta = prob.n, mesh_h(prob), prob.beta
    col = {"strang": strang_column, "tchan": tchan_column}[kind]
    sQ = circulant(col(_Q_lag, n))
    sW = circulant(col(_W_lag(beta, n), n))
    return e * np.eye(n) - sigma_of(prob.alpha) * (gam / (2.0 * h) * sQ + dp / h ** beta * sW
                                         + dm / h ** beta * sW.T)


def circulant_eigenvalues(col: np.ndarray) -> np.ndarray:
    """lambda_k = sum_m col_m exp(-2 pi i m k / n): the eigenvalues of the
    circulant with first column col, via the library FFT."""
    return np.fft.fft(col)


def embedding_column(beta: float, n: int, L: int) -> np.ndarray:
    """First column of a length-L (L >= 2n - 1) circulant whose leading n x n
    block is W_beta: c_m = omega_{m+1} (0 <= m < n), c_{L-1} = omega_0, else 0."""
    if L < 2 * n - 1:
        raise ValueError("embedding length must be at least 2n - 1")
    w = wsgd_weights(beta, n)
    c = np.zeros(L)
    c[:n] = w[1:n + 1]
    c[L - 1] += w[0]
    return c


# ---------------------------------------------------------------------------
# Row-by-row evaluation for large n (no dense matrix).
# ---------------------------------------------------------------------------

def apply_A_rows(prob, j: int, u: np.ndarray, rows: np.ndarray, which: str = "A") -> np.ndarray:
    """(A^(j+sigma) u)_i (or B) for the given 0-based rows by direct sums:
    (Q u)_i = u_{i+1} - u_{i-1};  (W u)_i = sum_{m <= i+1} omega_{i-m+1} u_m;
    (W^T u)_i = sum_{m >= i-1} omega_{m-i+1} u_m."""
    e, gam, dp, dm = level_scalars(prob, j)
    n, h, beta, sigma = prob.n, mesh_h(prob), prob.beta, sigma_of(prob.alpha)
    w = wsgd_weights(beta, n + 1)
    out = np.empty(len(rows))
    for r, i in enumerate(rows):
        i = int(i)
        qu = (u[i + 1] if i + 1 < n else 0.0) - (u[i - 1] if i >= 1 else 0.0)
        hi = min(i + 1, n - 1)
        # W row: m = 0..hi, weight omega_{i-m+1}
        wu = float(np.dot(w[i + 1 - hi:i + 2][::-1], u[0:hi + 1]))
        lo = max(i - 1, 0)
        # W^T row: m = lo..n-1, weight omega_{m-i+1}
        wtu = float(np.dot(w[lo - i + 1:n - i + 1], u[lo:n]))
        Lu = gam / (2.0 * h) * qu + dp / h ** beta * wu + dm / h ** beta * wtu
        out[r] = e * u[i] - sigma * Lu if which == "A" else e * u[i] + (1.0 - sigma) * Lu
    return out


def apply_P_rows(prob, j: int, y: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """(P^(j+sigma) y)_i of the Strang preconditioner (3.7) for the given
    0-based rows: a circulant with first column c acts as
    (C y)_i = sum_k c_{(i-k) mod n} y_k, its transpose with c_{(k-i) mod n}."""
    e, gam, dp, dm = level_scalars(prob, j)
    n, h, beta, sigma = prob.n, mesh_h(prob), prob.beta, sigma_of(prob.alpha)
    cQ = strang_column(_Q_lag, n)
    cW = strang_column(_W_lag(beta, n), n)
    k = np.arange(n)
    out = np.empty(len(rows))
    for r, i in enumerate(rows):
        i = int(i)
        fwd = (i - k) % n
        bwd = (k - i) % n
        Ly = (gam / (2.0 * h) * float(np.dot(cQ[fwd], y)) + dp / h ** beta * float(np.dot(cW[fwd], y))
              + dm / h ** beta * float(np.dot(cW[bwd], y)))
        out[r] = e * y[i] - sigma * Ly
    return out


def rhs_rows(prob, U: np.ndarray, j: int, f_j: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """g_i^(j+1) for the given rows (same definition as ``rhs``)."""
    Bu = apply_A_rows(prob, j, U[j], rows, which="B")
    if j == 0:
        return Bu + f_j[rows]
    c = l21s_c(prob.alpha, j)
    acc = np.zeros(len(rows))
    for s in range(j):
        acc += c[j - s] * (U[s + 1][rows] - U[s][rows])
    return Bu - l21s_kappa(prob.alpha, time_step(prob)) * acc + f_j[rows]


# ---------------------------------------------------------------------------
# The paper's fast level solve for large n (Sec. 3.2 and Algorithm 2 with
# PCGS): Toeplitz products through a circulant embedding and the Strang
# preconditioner, both with the library FFT, and preconditioned CGS as in
# Barrett et al., Templates (1994).  Plain NumPy, independent of the GPU path.
# ---------------------------------------------------------------------------

def embedding_eigenvalues(prob) -> np.ndarray:
    """Eigenvalues of the circulant embedding of W (length L = the next power
    of two >= 2n)."""
    L = 1
    while L < 2 * prob.n:
        L *= 2
    return circulant_eigenvalues(embedding_column(prob.beta, prob.n, L))


def embedding_product(prob, j: int, x: np.ndarray, which: str = "A", lam=None) -> np.ndarray:
    """A^(j+sigma) x (or B^(j+sigma) x) with W x and W^T x from a circulant
    embedding of length L = the next power of two >= 2n: the embedding's
    eigenvalues lam = DFT(column) (embedding_eigenvalues) act on the
    zero-padded x, and W^T, the transpose of a real circulant, has the
    eigenvalues conj(lam)."""
    e, gam, dp, dm = level_scalars(prob, j)
    n, h, beta, sigma = prob.n, mesh_h(prob), prob.beta, sigma_of(prob.alpha)
    if lam is None:
        lam = embedding_eigenvalues(prob)
    L = lam.size
    X = np.fft.fft(np.concatenate([x, np.zeros(L - n)]))
    wx = np.fft.ifft(lam * X).real[:n]
    wtx = np.fft.ifft(np.conj(lam) * X).real[:n]
    qx = np.concatenate([x[1:], [0.0]]) - np.concatenate([[0.0], x[:-1]])
    Lx = gam / (2.0 * h) * qx + dp / h ** beta * wx + dm / h ** beta * wtx
    return e * x - sigma * Lx if which == "A" else e * x + (1.0 - sigma) * Lx


def strang_eigenvalues(prob, j: int, kind: str = "strang") -> np.ndarray:
    """Eigenvalues of the Strang preconditioner (3.7): eta_j - sigma (gamma/(2h)
    lam(s(Q)) + D+/h^beta lam(s(W)) + D-/h^beta conj lam(s(W))); kind
    "tchan" for T. Chan's circulants instead."""
    e, gam, dp, dm = level_scalars(prob, j)
    n, h, beta, sigma = prob.n, mesh_h(prob), prob.beta, sigma_of(prob.alpha)
    col = {"strang": strang_column, "tchan": tchan_column}[kind]
    lq = circulant_eigenvalues(col(_Q_lag, n))
    lw = circulant_eigenvalues(col(_W_lag(beta, n), n))
    return e - sigma * (gam / (2.0 * h) * lq + dp / h ** beta * lw + dm / h ** beta * np.conj(lw))


def strang_solve(prob, j: int, y: np.ndarray, lam=None) -> np.ndarray:
    """(P^(j+sigma))^{-1} y, a division by the circulant's eigenvalues."""
    if lam is None:
        lam = strang_eigenvalues(prob, j)
    return np.fft.ifft(np.fft.fft(y) / lam).real


def rhs_fft(prob, U: np.ndarray, j: int, f_j: np.ndarray, lam=None) -> np.ndarray:
    """g^(j) of (3.3) (same definition as ``rhs``) with B^(j+sigma) u^j
    through the embedding product."""
    g = embedding_product(prob, j, U[j], "B", lam) + f_j
    if j == 0:
        return g
    c = l21s_c(prob.alpha, j)
    acc = np.zeros(prob.n)
    for s_ in range(j):
        acc += c[j - s_] * (U[s_ + 1] - U[s_])
    return g - l21s_kappa(prob.alpha, time_step(prob)) * acc


def level_solve_pcgs(prob, U: np.ndarray, j: int, f_j: np.ndarray, rtol: float = 1e-10, maxit: int = 500,
                     kind: str = "strang"):
    """u^{j+1} by preconditioned CGS on A^(j+sigma) u = g (3.3) from x0 = 0,
    stopped when the recursive residual falls to rtol |g| (Sec. 4).  Returns
    (u, iterations)."""
    lam_e = embedding_eigenvalues(prob)
    lam_p = strang_eigenvalues(prob, j, kind)
    g = rhs_fft(prob, U, j, f_j, lam_e)
    A = lambda v: embedding_product(prob, j, v, "A", lam_e)  # noqa: E731
    Pinv = lambda v: strang_solve(prob, j, v, lam_p)  # noqa: E731
    x = np.zeros(prob.n)
    r = g.copy()
    rt = r.copy()
    gnorm = np.linalg.norm(g)
    rho_old, q, p = 1.0, None, None
    for it in range(1, maxit + 1):
        rho = float(rt @ r)
        if rho == 0.0:
            return x, it
        if it == 1:
            u = r.copy()
            p = u.copy()
        else:
            beta = rho / rho_old
            u = r + beta * q
            p = u + beta * (q + beta * p)
        vhat = A(Pinv(p))
        alpha = rho / float(rt @ vhat)
        q = u - alpha * vhat
        uhat = Pinv(u + q)
        x = x + alpha * uhat
        r = r - alpha * A(uhat)
        if np.linalg.norm(r) <= rtol * gnorm:
            return x, it
        rho_old = rho
    return x, maxit



# ---------------------------------------------------------------------------
# Constant coefficients: Algorithm 3 with the Gohberg-Semencul formula of
# Sec. 3.1 ((3.4), the formula after it, and Algorithm 1).  With gamma, d_+-
# constant, A^(j+sigma) = A for every j >= 1 (eta_j is the same for j >= 1),
# so A^-1 is reconstructed from two solves, A x = e_1 and A y = e_n.
# ---------------------------------------------------------------------------

def level_solve_pbicgstab(prob, U: np.ndarray, j: int, f_j: np.ndarray, rtol: float = 1e-10, maxit: int = 500,
                          kind: str = "strang"):
    """u^{j+1} by right-preconditioned BiCGSTAB (van der Vorst 1992, in the
    form of Barrett et al., Templates 1994) on A^(j+sigma) u = g from x0 = 0,
    with the circulant preconditioner of the given kind, stopped when the
    residual falls to rtol |g|.  Returns (u, iterations)."""
    lam_e = embedding_eigenvalues(prob)
    lam_p = strang_eigenvalues(prob, j, kind)
    g = rhs_fft(prob, U, j, f_j, lam_e)
    A = lambda v: embedding_product(prob, j, v, "A", lam_e)  # noqa: E731
    Pinv = lambda v: strang_solve(prob, j, v, lam_p)  # noqa: E731
    x = np.zeros(prob.n)
    r = g.copy()
    rt = r.copy()
    gnorm = np.linalg.norm(g)
    rho_old = alpha = omega = 1.0
    p = v = np.zeros(prob.n)
    for it in range(1, maxit + 1):
        rho = float(rt @ r)
        if rho == 0.0:
            return x, it
        if it == 1:
            p = r.copy()
        else:
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
        phat = Pinv(p)
        v = A(phat)
        alpha = rho / float(rt @ v)
        s = r - alpha * v
        shat = Pinv(s)
        t = A(shat)
        tt = float(t @ t)
        omega = float(t @ s) / tt if tt > 0 else 0.0
        x = x + alpha * phat + omega * shat
        r = s - omega * t
        if np.linalg.norm(r) <= rtol * gnorm:
            return x, it
        if omega == 0.0:
            return x, it
        rho_old = rho
    return x, maxit


def coefficients_constant(prob) -> bool:
    """gamma, d_+- take the same values at every sampling instant."""
    vals = {(prob.gamma(t_sigma(prob, j)), prob.dplus(t_sigma(prob, j)), prob.dminus(t_sigma(prob, j)))
            for j in range(prob.M)}
    return len(vals) == 1


def gsf_generators(prob):
    """(x, y) of (3.4): A x = e_1 and A y = e_n for the level matrix of
    levels j >= 1, by Gaussian elimination."""
    A = level_A(prob, 1 if prob.M > 1 else 0)
    n = prob.n
    e1 = np.zeros(n)
    e1[0] = 1.0
    en = np.zeros(n)
    en[-1] = 1.0
    return np.linalg.solve(A, e1), np.linalg.solve(A, en)


def gsf_matrices(x: np.ndarray, y: np.ndarray):
    """The four triangular Toeplitz factors of the Gohberg-Semencul formula,
    as printed after (3.4):
      L_p  lower, first column (xi_0, ..., xi_{n-1});
      R_p  upper, first row (eta_{n-1}, ..., eta_0);
      L0_p strictly lower, first column (0, eta_0, ..., eta_{n-2});
      R0_p strictly upper, first row (0, xi_{n-1}, ..., xi_1)."""
    n = len(x)
    d = np.arange(n)[:, None] - np.arange(n)[None, :]  # i - k
    Lp = np.where(d >= 0, x[np.clip(d, 0, n - 1)], 0.0)
    Rp = np.where(d <= 0, y[np.clip(n - 1 + d, 0, n - 1)], 0.0)
    L0 = np.where(d >= 1, y[np.clip(d - 1, 0, n - 1)], 0.0)
    R0 = np.where(d <= -1, x[np.clip(n + d, 0, n - 1)], 0.0)
    return Lp, Rp, L0, R0


def gsf_apply(x: np.ndarray, y: np.ndarray, v: np.ndarray) -> np.ndarray:
    """z = A^-1 v by Algorithm 1: z1 = R0_p v, z2 = R_p v, z3 = L0_p z1,
    z4 = L_p z2, z = (z4 - z3) / xi_0 (requires xi_0 != 0)."""
    Lp, Rp, L0, R0 = gsf_matrices(x, y)
    z1 = R0 @ v
    z2 = Rp @ v
    z3 = L0 @ z1
    z4 = Lp @ z2
    return (z4 - z3) / x[0]


def march_gsf(prob, f_levels: Optional[Iterable[np.ndarray]] = None) -> np.ndarray:
    """Algorithm 3: level 0 solves A^(sigma) u^1 = g^(1) by Gaussian
    elimination; every later level forms g^(j+1) (with the history entering
    with the minus sign of (3.1)) and applies A^-1 by Algorithm 1."""
    if not coefficients_constant(prob):
        raise ValueError("Algorithm 3 needs constant gamma, d_+-")
    U = np.zeros((prob.M + 1, prob.n))
    U[0] = initial_level(prob)
    flist = list(f_levels) if f_levels is not None else None
    x, y = gsf_generators(prob)
    for j in range(prob.M):
        f_j = flist[j] if flist is not None else source_level(prob, j)
        if j == 0:
            U[1] = level_solve(prob, U, 0, f_j)
        else:
            U[j + 1] = gsf_apply(x, y, rhs(prob, U, j, f_j))
    return U


def history_perturbation_bound(prob, U: np.ndarray, j: int, rel_tol: float) -> np.ndarray:
    """Elementwise bound on how far a history term whose weights c_m
    (2 <= m <= j-1) each carry a relative error of at most rel_tol can move
    from the exact one of (3.3):  kappa rel_tol sum_{m=2}^{j-1} c_m |u^{j-m+1} - u^{j-m}|
    (the weights of Lemma 1 are positive).  Zero for j <= 2."""
    n = U.shape[1]
    acc = np.zeros(n)
    if j <= 2:
        return acc
    c = l21s_c(prob.alpha, j)
    for m in range(2, j):
        acc += abs(c[m]) * np.abs(U[j - m + 1] - U[j - m])
    return l21s_kappa(prob.alpha, time_step(prob)) * rel_tol * acc
