"""Plain FP64 CPU oracle of the implicit difference scheme in two space
dimensions.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/`` and the two-dimensional
leg of ``bench.py``; never by the product path.

The paper (arXiv:1603.00279) solves (1.1) in one space dimension and names
the two- and three-dimensional problems, with block-Toeplitz systems and
multi-dimensional FFTs, as future work (Sec. 5).  The scheme here is the
direct extension, each step of it the paper's one-dimensional step on one
axis:

* L2-1sigma in time with the same tables, sampling instant t_{j+sigma} and
  history sum (Lemma 1, (3.1)).
* The space operator is the Kronecker sum  L = L_x (x) I_y + I_x (x) L_y,
  where L_x = gx/(2hx) Q + dxp/hx^bx W_bx + dxm/hx^bx W_bx^T is the
  one-dimensional operator of (3.2)-(3.3) on the x grid (and L_y likewise):
  shifted Grunwald (WSGD) differences along each axis (Lemma 2) and central
  differences for the convection.
* A = eta_j I - sigma L, B = eta_j I + (1 - sigma) L: the arrays u[i, k] =
  u(x_{i+1}, y_{k+1}) of shape (nx, ny), flattened row-major (y fastest), so
  that L_x (x) I_y acts along axis 0.
* The preconditioner is the block-circulant-with-circulant-blocks (BCCB)
  analogue of (3.7):  P = eta_j I - sigma (s(L_x) (x) I + I (x) s(L_y)) with
  Strang's circulants s(.), diagonalised by the two-dimensional DFT.

Functions reuse the one-dimensional oracle (``ids_oracle``) for every
per-axis quantity.  Pinned by ``tests/test_oracle_2d.py``: reduction to the
one-dimensional oracle line by line when one axis's operator vanishes,
exchange of the axes, observed second-order convergence to a manufactured
solution, the FFT route against dense linear algebra, and the point-wise
direct sums against the dense rows.
"""
from __future__ import annotations

import numpy as np

from . import ids_oracle as O

__all__ = [
    "axes", "mesh", "nodes", "t_sigma", "time_step", "initial_level", "source_level", "level_L2", "level_A2",
    "level_B2", "history_term2", "rhs2", "level_solve2", "march2", "error_norms2", "axis_L_product",
    "product2", "bccb_eigenvalues", "bccb_solve", "bccb_matrix", "level_solve_pcgs2", "apply_A2_points",
    "rhs2_points", "anorm2",
]


def axes(prob):
    """(x-axis problem, y-axis problem): the one-dimensional problems whose
    operators L_x, L_y make up the Kronecker sum."""
    return prob.axis("x"), prob.axis("y")


def mesh(prob):
    """(hx, hy) = ((b-a)/(nx+1), (d-c)/(ny+1))."""
    px, py = axes(prob)
    return O.mesh_h(px), O.mesh_h(py)


def nodes(prob):
    """Interior nodes (x_1..x_nx, y_1..y_ny)."""
    px, py = axes(prob)
    return O.nodes(px), O.nodes(py)


def time_step(prob) -> float:
    return O.time_step(axes(prob)[0])


def t_sigma(prob, j: int) -> float:
    return O.t_sigma(axes(prob)[0], j)


def initial_level(prob) -> np.ndarray:
    x, y = nodes(prob)
    return np.asarray(prob.phi(x, y), dtype=np.float64)


def source_level(prob, j: int) -> np.ndarray:
    """f(x_i, y_k, t_{j+sigma}) as an (nx, ny) array."""
    x, y = nodes(prob)
    return np.asarray(prob.f(x, y, t_sigma(prob, j)), dtype=np.float64)


# ---------------------------------------------------------------------------
# Dense matrices: the Kronecker sum and the level's direct solve.
# ---------------------------------------------------------------------------

def level_L2(prob, j: int) -> np.ndarray:
    """L = L_x (x) I_ny + I_nx (x) L_y at t_{j+sigma} (dense, nx*ny square)."""
    px, py = axes(prob)
    return np.kron(O.level_L(px, j), np.eye(prob.ny)) + np.kron(np.eye(prob.nx), O.level_L(py, j))


def _eta(prob, j: int) -> float:
    return O.level_scalars(axes(prob)[0], j)[0]


def level_A2(prob, j: int) -> np.ndarray:
    """A = eta_j I - sigma L."""
    return _eta(prob, j) * np.eye(prob.nx * prob.ny) - O.sigma_of(prob.alpha) * level_L2(prob, j)


def level_B2(prob, j: int) -> np.ndarray:
    """B = eta_j I + (1 - sigma) L."""
    return _eta(prob, j) * np.eye(prob.nx * prob.ny) + (1.0 - O.sigma_of(prob.alpha)) * level_L2(prob, j)


def history_term2(prob, U: np.ndarray, j: int) -> np.ndarray:
    """kappa sum_{s<j} c_{j-s}^(j) (u^{s+1} - u^s) of (3.1) on the 2D grid."""
    acc = np.zeros((prob.nx, prob.ny))
    if j == 0:
        return acc
    c = O.l21s_c(prob.alpha, j)
    for s in range(j):
        acc += c[j - s] * (U[s + 1] - U[s])
    return O.l21s_kappa(prob.alpha, time_step(prob)) * acc


def rhs2(prob, U: np.ndarray, j: int, f_j: np.ndarray) -> np.ndarray:
    """g = B u^j - history + f^{j+sigma} (as (nx, ny))."""
    Bu = (level_B2(prob, j) @ U[j].reshape(-1)).reshape(prob.nx, prob.ny)
    return Bu - history_term2(prob, U, j) + f_j


def level_solve2(prob, U: np.ndarray, j: int, f_j: np.ndarray) -> np.ndarray:
    """u^{j+1} = A^{-1} g by Gaussian elimination."""
    g = rhs2(prob, U, j, f_j)
    return np.linalg.solve(level_A2(prob, j), g.reshape(-1)).reshape(prob.nx, prob.ny)


def march2(prob, f_levels=None, levels=None, u0=None) -> np.ndarray:
    """Every level by dense direct solves; U[j] = u^j, shape (levels+1, nx, ny)."""
    M = prob.M if levels is None else levels
    U = np.zeros((M + 1, prob.nx, prob.ny))
    U[0] = initial_level(prob) if u0 is None else u0
    flist = list(f_levels) if f_levels is not None else None
    for j in range(M):
        f_j = flist[j] if flist is not None else source_level(prob, j)
        U[j + 1] = level_solve2(prob, U, j, f_j)
    return U


def error_norms2(prob, U: np.ndarray):
    """(max_j sqrt(hx hy sum E^2), max |E|) against the manufactured solution."""
    x, y = nodes(prob)
    hx, hy = mesh(prob)
    l2 = cmax = 0.0
    for j in range(U.shape[0]):
        E = U[j] - prob.exact(x, y, j * time_step(prob))
        l2 = max(l2, float(np.sqrt(hx * hy * np.sum(E * E))))
        cmax = max(cmax, float(np.max(np.abs(E))))
    return l2, cmax


# ---------------------------------------------------------------------------
# FFT route: Toeplitz products along each axis through circulant embeddings,
# the BCCB Strang preconditioner through the 2D DFT, preconditioned CGS.
# ---------------------------------------------------------------------------

def axis_L_product(p1, j: int, V: np.ndarray, axis: int) -> np.ndarray:
    """L_axis applied along ``axis`` of V: the one-dimensional operator of the
    axis problem p1 on every line, W and W^T through the length-L embedding
    (L the next power of two >= 2n) and Q by differences."""
    _, gam, dp, dm = O.level_scalars(p1, j)
    n, h, beta = p1.n, O.mesh_h(p1), p1.beta
    lam = O.embedding_eigenvalues(p1)
    Lemb = lam.size
    Vt = np.moveaxis(V, axis, -1)
    pad = np.concatenate([Vt, np.zeros(Vt.shape[:-1] + (Lemb - n,))], axis=-1)
    X = np.fft.fft(pad, axis=-1)
    wx = np.fft.ifft(lam * X, axis=-1).real[..., :n]
    wtx = np.fft.ifft(np.conj(lam) * X, axis=-1).real[..., :n]
    z = np.zeros(Vt.shape[:-1] + (1,))
    qx = np.concatenate([Vt[..., 1:], z], axis=-1) - np.concatenate([z, Vt[..., :-1]], axis=-1)
    Lv = gam / (2.0 * h) * qx + dp / h ** beta * wx + dm / h ** beta * wtx
    return np.moveaxis(Lv, -1, axis)


def product2(prob, j: int, V: np.ndarray, which: str = "A") -> np.ndarray:
    """A V (or B V) for an (nx, ny) array through the FFT route."""
    px, py = axes(prob)
    LV = axis_L_product(px, j, V, 0) + axis_L_product(py, j, V, 1)
    e, sg = _eta(prob, j), O.sigma_of(prob.alpha)
    return e * V - sg * LV if which == "A" else e * V + (1.0 - sg) * LV


def _strang_symbol(p1, j: int) -> np.ndarray:
    """Eigenvalues of s(L_axis): gx/(2h) lam(s(Q)) + dp/h^b lam(s(W)) + dm/h^b conj lam(s(W))."""
    _, gam, dp, dm = O.level_scalars(p1, j)
    n, h, beta = p1.n, O.mesh_h(p1), p1.beta
    lq = O.circulant_eigenvalues(O.strang_column(O._Q_lag, n))
    lw = O.circulant_eigenvalues(O.strang_column(O._W_lag(beta, n), n))
    return gam / (2.0 * h) * lq + dp / h ** beta * lw + dm / h ** beta * np.conj(lw)


def bccb_eigenvalues(prob, j: int) -> np.ndarray:
    """Eigenvalues of P = eta I - sigma (s(L_x) (x) I + I (x) s(L_y)) on the 2D
    DFT grid: eta - sigma (mu_x[kx] + mu_y[ky])."""
    px, py = axes(prob)
    return _eta(prob, j) - O.sigma_of(prob.alpha) * (_strang_symbol(px, j)[:, None] + _strang_symbol(py, j)[None, :])


def bccb_solve(prob, j: int, V: np.ndarray, eig=None) -> np.ndarray:
    """P^{-1} V by the 2D DFT."""
    if eig is None:
        eig = bccb_eigenvalues(prob, j)
    return np.fft.ifft2(np.fft.fft2(V) / eig).real


def bccb_matrix(prob, j: int) -> np.ndarray:
    """P as a dense matrix (circulants built from Strang's columns)."""
    px, py = axes(prob)

    def sL(p1):
        _, gam, dp, dm = O.level_scalars(p1, j)
        n, h, beta = p1.n, O.mesh_h(p1), p1.beta
        sQ = O.circulant(O.strang_column(O._Q_lag, n))
        sW = O.circulant(O.strang_column(O._W_lag(beta, n), n))
        return gam / (2.0 * h) * sQ + dp / h ** beta * sW + dm / h ** beta * sW.T

    Lc = np.kron(sL(px), np.eye(prob.ny)) + np.kron(np.eye(prob.nx), sL(py))
    return _eta(prob, j) * np.eye(prob.nx * prob.ny) - O.sigma_of(prob.alpha) * Lc


def level_solve_pcgs2(prob, U: np.ndarray, j: int, f_j: np.ndarray, rtol: float = 1e-10, maxit: int = 500):
    """u^{j+1} by right-preconditioned CGS (Barrett et al., Templates) on the
    FFT route, from x0 = 0, stopped at |r| <= rtol |g|.  Returns (u, iterations)."""
    eig = bccb_eigenvalues(prob, j)
    Bu = product2(prob, j, U[j], "B")
    g = Bu - history_term2(prob, U, j) + f_j
    A = lambda v: product2(prob, j, v, "A")  # noqa: E731
    Pinv = lambda v: bccb_solve(prob, j, v, eig)  # noqa: E731
    x = np.zeros_like(g)
    r = g.copy()
    rt = r.copy()
    gnorm = np.linalg.norm(g)
    rho_old, q, p = 1.0, None, None
    for it in range(1, maxit + 1):
        rho = float(np.sum(rt * r))
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
        alpha = rho / float(np.sum(rt * vhat))
        q = u - alpha * vhat
        uhat = Pinv(u + q)
        x = x + alpha * uhat
        r = r - alpha * A(uhat)
        if np.linalg.norm(r) <= rtol * gnorm:
            return x, it
        rho_old = rho
    return x, maxit


# ---------------------------------------------------------------------------
# Point-wise direct sums (sizes where no dense matrix fits).
# ---------------------------------------------------------------------------

def apply_A2_points(prob, j: int, V: np.ndarray, pts, which: str = "A") -> np.ndarray:
    """(A V)_{ik} (or B) at the points (i, k): the one-dimensional direct sums
    of the x line through the point and of the y line, combined."""
    px, py = axes(prob)
    e, sg = _eta(prob, j), O.sigma_of(prob.alpha)
    out = np.empty(len(pts))
    for r, (i, k) in enumerate(pts):
        i, k = int(i), int(k)
        # L_axis u at one index = (B - A) u there (the 1D direct sums)
        Lx = O.apply_A_rows(px, j, V[:, k], [i], "B")[0] - O.apply_A_rows(px, j, V[:, k], [i], "A")[0]
        Ly = O.apply_A_rows(py, j, V[i, :], [k], "B")[0] - O.apply_A_rows(py, j, V[i, :], [k], "A")[0]
        Lv = Lx + Ly
        out[r] = e * V[i, k] - sg * Lv if which == "A" else e * V[i, k] + (1.0 - sg) * Lv
    return out


def rhs2_points(prob, U: np.ndarray, j: int, f_j: np.ndarray, pts) -> np.ndarray:
    """g at the points (i, k) (same definition as ``rhs2``)."""
    Bu = apply_A2_points(prob, j, U[j], pts, "B")
    H = np.zeros(len(pts))
    if j >= 1:
        c = O.l21s_c(prob.alpha, j)
        kap = O.l21s_kappa(prob.alpha, time_step(prob))
        for r, (i, k) in enumerate(pts):
            H[r] = kap * sum(c[j - s] * (U[s + 1][i, k] - U[s][i, k]) for s in range(j))
    return Bu - H + np.array([f_j[int(i), int(k)] for i, k in pts])


def anorm2(prob, j: int) -> float:
    """An upper bound of |A|_2: eta + sigma (bound of |L_x|_2 + bound of |L_y|_2),
    each axis's |L| <= |gamma|/h + (d_+ + d_-) h^-beta sum_k |omega_k|."""
    tot = 0.0
    for p1 in axes(prob):
        _, gam, dp, dm = O.level_scalars(p1, j)
        h = O.mesh_h(p1)
        w = O.wsgd_weights(p1.beta, p1.n + 1)
        tot += abs(gam) / h + (dp + dm) * h ** (-p1.beta) * float(np.sum(np.abs(w)))
    return _eta(prob, j) + O.sigma_of(prob.alpha) * tot
