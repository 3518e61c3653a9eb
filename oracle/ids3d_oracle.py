"""Plain FP64 CPU oracle of the implicit difference scheme in three space
dimensions.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/`` and the three-dimensional
leg of ``bench.py``; never by the product path.

The paper (arXiv:1603.00279) names the two- and three-dimensional problems,
with block-Toeplitz systems and multi-dimensional FFTs, as future work
(Sec. 5).  The scheme here is the direct extension of its one-dimensional
scheme, as the two-dimensional oracle (``ids2d_oracle``) is, with one more
axis:

* L2-1sigma in time: the same tables, sampling instant t_{j+sigma} and
  history sum (Lemma 1, (3.1)).
* The space operator is the Kronecker sum
      L = L_x (x) I_y (x) I_z + I_x (x) L_y (x) I_z + I_x (x) I_y (x) L_z,
  each L_axis the one-dimensional operator of (3.2)-(3.3) on that axis's
  grid (WSGD differences, Lemma 2, and central convection differences).
  Arrays u[i, k, l] = u(x_{i+1}, y_{k+1}, z_{l+1}) of shape (nx, ny, nz) are
  flattened row-major (z fastest), so L_x acts along axis 0.
* A = eta_j I - sigma L and B = eta_j I + (1 - sigma) L.
* The preconditioner is the three-level block-circulant analogue of (3.7),
      P = eta_j I - sigma (s(L_x) (x) I (x) I + I (x) s(L_y) (x) I + I (x) I (x) s(L_z)),
  with Strang's circulants s(.), diagonalised by the three-dimensional DFT.

Per-axis quantities come from the one-dimensional oracle (``ids_oracle``),
and the FFT route along one axis from ``ids2d_oracle.axis_L_product``.
Pinned by ``tests/test_oracle_3d.py``: a z axis with a vanishing operator
reduces the march to the two-dimensional oracle's plane by plane; exchanging
axes permutes the solution; the Kronecker sum on separable arrays equals the
sum of the one-dimensional products; observed second-order convergence to a
manufactured solution; the FFT routes against dense linear algebra; the
point-wise direct sums against the dense rows.
"""
from __future__ import annotations

import numpy as np

from . import ids_oracle as O
from . import ids2d_oracle as O2

__all__ = [
    "axes", "mesh", "nodes", "t_sigma", "time_step", "initial_level", "source_level", "level_L3", "level_A3",
    "level_B3", "history_term3", "rhs3", "level_solve3", "march3", "error_norms3", "product3",
    "bccb3_eigenvalues", "bccb3_solve", "bccb3_matrix", "pcgs", "level_solve_pcgs3", "march_pcgs3",
    "apply_A3_points", "rhs3_points", "anorm3",
]


def axes(prob):
    """The one-dimensional problems of the three axes (x, y, z)."""
    return [prob.axis(k) for k in range(3)]


def mesh(prob):
    """(hx, hy, hz), h = (hi - lo)/(n + 1) per axis."""
    return tuple(O.mesh_h(p) for p in axes(prob))


def nodes(prob):
    """Interior nodes of each axis."""
    return tuple(O.nodes(p) for p in axes(prob))


def time_step(prob) -> float:
    return O.time_step(axes(prob)[0])


def t_sigma(prob, j: int) -> float:
    return O.t_sigma(axes(prob)[0], j)


def initial_level(prob) -> np.ndarray:
    return np.asarray(prob.phi(*nodes(prob)), dtype=np.float64)


def source_level(prob, j: int) -> np.ndarray:
    """f at the nodes and t_{j+sigma} as an (nx, ny, nz) array."""
    return np.asarray(prob.f(*nodes(prob), t_sigma(prob, j)), dtype=np.float64)


def _eta(prob, j: int) -> float:
    return O.level_scalars(axes(prob)[0], j)[0]


def _shape(prob):
    return tuple(int(n) for n in prob.ns)


# ---------------------------------------------------------------------------
# Dense matrices: the Kronecker sum and the level's direct solve.
# ---------------------------------------------------------------------------

def level_L3(prob, j: int) -> np.ndarray:
    """L = L_x (x) I (x) I + I (x) L_y (x) I + I (x) I (x) L_z at t_{j+sigma}
    (dense, N x N with N = nx ny nz)."""
    nx, ny, nz = _shape(prob)
    px, py, pz = axes(prob)
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    return (np.kron(np.kron(O.level_L(px, j), Iy), Iz) + np.kron(np.kron(Ix, O.level_L(py, j)), Iz)
            + np.kron(np.kron(Ix, Iy), O.level_L(pz, j)))


def level_A3(prob, j: int) -> np.ndarray:
    """A = eta_j I - sigma L."""
    return _eta(prob, j) * np.eye(prob.N) - O.sigma_of(prob.alpha) * level_L3(prob, j)


def level_B3(prob, j: int) -> np.ndarray:
    """B = eta_j I + (1 - sigma) L."""
    return _eta(prob, j) * np.eye(prob.N) + (1.0 - O.sigma_of(prob.alpha)) * level_L3(prob, j)


def history_term3(prob, U: np.ndarray, j: int) -> np.ndarray:
    """kappa sum_{s<j} c_{j-s}^(j) (u^{s+1} - u^s) of (3.1) on the 3D grid."""
    acc = np.zeros(_shape(prob))
    if j == 0:
        return acc
    c = O.l21s_c(prob.alpha, j)
    for s in range(j):
        acc += c[j - s] * (U[s + 1] - U[s])
    return O.l21s_kappa(prob.alpha, time_step(prob)) * acc


def rhs3(prob, U: np.ndarray, j: int, f_j: np.ndarray) -> np.ndarray:
    """g = B u^j - history + f^{j+sigma} (dense B)."""
    Bu = (level_B3(prob, j) @ U[j].reshape(-1)).reshape(_shape(prob))
    return Bu - history_term3(prob, U, j) + f_j


def level_solve3(prob, U: np.ndarray, j: int, f_j: np.ndarray) -> np.ndarray:
    """u^{j+1} = A^{-1} g by Gaussian elimination."""
    g = rhs3(prob, U, j, f_j)
    return np.linalg.solve(level_A3(prob, j), g.reshape(-1)).reshape(_shape(prob))


def march3(prob, f_levels=None, levels=None, u0=None) -> np.ndarray:
    """Every level by dense direct solves; U[j] = u^j, shape (levels+1, nx, ny, nz)."""
    M = prob.M if levels is None else levels
    U = np.zeros((M + 1,) + _shape(prob))
    U[0] = initial_level(prob) if u0 is None else u0
    flist = list(f_levels) if f_levels is not None else None
    for j in range(M):
        f_j = flist[j] if flist is not None else source_level(prob, j)
        U[j + 1] = level_solve3(prob, U, j, f_j)
    return U


def error_norms3(prob, U: np.ndarray):
    """(max_j sqrt(hx hy hz sum E^2), max |E|) against the manufactured solution."""
    x, y, z = nodes(prob)
    hx, hy, hz = mesh(prob)
    l2 = cmax = 0.0
    for j in range(U.shape[0]):
        E = U[j] - prob.exact(x, y, z, j * time_step(prob))
        l2 = max(l2, float(np.sqrt(hx * hy * hz * np.sum(E * E))))
        cmax = max(cmax, float(np.max(np.abs(E))))
    return l2, cmax


# ---------------------------------------------------------------------------
# FFT route: Toeplitz products along each axis through circulant embeddings,
# the three-level circulant Strang preconditioner through the 3D DFT,
# preconditioned CGS.
# ---------------------------------------------------------------------------

def product3(prob, j: int, V: np.ndarray, which: str = "A") -> np.ndarray:
    """A V (or B V) for an (nx, ny, nz) array through the FFT route."""
    LV = sum(O2.axis_L_product(p1, j, V, k) for k, p1 in enumerate(axes(prob)))
    e, sg = _eta(prob, j), O.sigma_of(prob.alpha)
    return e * V - sg * LV if which == "A" else e * V + (1.0 - sg) * LV


def bccb3_eigenvalues(prob, j: int) -> np.ndarray:
    """Eigenvalues of P on the 3D DFT grid: eta - sigma (mu_x[kx] + mu_y[ky] + mu_z[kz])."""
    mx, my, mz = (O2._strang_symbol(p1, j) for p1 in axes(prob))
    mu = mx[:, None, None] + my[None, :, None] + mz[None, None, :]
    return _eta(prob, j) - O.sigma_of(prob.alpha) * mu


def bccb3_solve(prob, j: int, V: np.ndarray, eig=None) -> np.ndarray:
    """P^{-1} V by the 3D DFT."""
    if eig is None:
        eig = bccb3_eigenvalues(prob, j)
    return np.fft.ifftn(np.fft.fftn(V) / eig).real


def bccb3_matrix(prob, j: int) -> np.ndarray:
    """P as a dense matrix, from the circulants of Strang's columns."""
    nx, ny, nz = _shape(prob)

    def sL(p1):
        _, gam, dp, dm = O.level_scalars(p1, j)
        n, h, beta = p1.n, O.mesh_h(p1), p1.beta
        sQ = O.circulant(O.strang_column(O._Q_lag, n))
        sW = O.circulant(O.strang_column(O._W_lag(beta, n), n))
        return gam / (2.0 * h) * sQ + dp / h ** beta * sW + dm / h ** beta * sW.T

    px, py, pz = axes(prob)
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    Lc = (np.kron(np.kron(sL(px), Iy), Iz) + np.kron(np.kron(Ix, sL(py)), Iz) + np.kron(np.kron(Ix, Iy), sL(pz)))
    return _eta(prob, j) * np.eye(prob.N) - O.sigma_of(prob.alpha) * Lc


def pcgs(A, Pinv, g: np.ndarray, rtol: float = 1e-10, maxit: int = 500):
    """Right-preconditioned CGS (Barrett et al., Templates) for A x = g from
    x0 = 0, stopped at |r| <= rtol |g|.  Returns (x, iterations)."""
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


def level_solve_pcgs3(prob, U: np.ndarray, j: int, f_j: np.ndarray, rtol: float = 1e-10, maxit: int = 500):
    """u^{j+1} by PCGS on the FFT route.  Returns (u, iterations)."""
    eig = bccb3_eigenvalues(prob, j)
    g = product3(prob, j, U[j], "B") - history_term3(prob, U, j) + f_j
    return pcgs(lambda v: product3(prob, j, v, "A"), lambda v: bccb3_solve(prob, j, v, eig), g, rtol, maxit)


def march_pcgs3(prob, f_levels=None, levels=None, u0=None, rtol: float = 1e-12):
    """Every level by PCGS on the FFT route; (U, iterations per level)."""
    M = prob.M if levels is None else levels
    U = np.zeros((M + 1,) + _shape(prob))
    U[0] = initial_level(prob) if u0 is None else u0
    flist = list(f_levels) if f_levels is not None else None
    its = []
    for j in range(M):
        f_j = flist[j] if flist is not None else source_level(prob, j)
        U[j + 1], it = level_solve_pcgs3(prob, U, j, f_j, rtol)
        its.append(it)
    return U, its


# ---------------------------------------------------------------------------
# Point-wise direct sums (sizes where no dense matrix fits).
# ---------------------------------------------------------------------------

def apply_A3_points(prob, j: int, V: np.ndarray, pts, which: str = "A") -> np.ndarray:
    """(A V) (or B V) at the points (i, k, l): the one-dimensional direct sums
    along the x, y and z lines through each point, combined."""
    px, py, pz = axes(prob)
    e, sg = _eta(prob, j), O.sigma_of(prob.alpha)

    def L1(p1, line, idx):
        # L_axis u at one index = (B - A) u there (the 1D direct sums)
        return (O.apply_A_rows(p1, j, line, [idx], "B")[0] - O.apply_A_rows(p1, j, line, [idx], "A")[0])

    out = np.empty(len(pts))
    for r, (i, k, l) in enumerate(pts):
        i, k, l = int(i), int(k), int(l)
        Lv = L1(px, V[:, k, l], i) + L1(py, V[i, :, l], k) + L1(pz, V[i, k, :], l)
        out[r] = e * V[i, k, l] - sg * Lv if which == "A" else e * V[i, k, l] + (1.0 - sg) * Lv
    return out


def rhs3_points(prob, U: np.ndarray, j: int, f_j: np.ndarray, pts) -> np.ndarray:
    """g at the points (i, k, l) (same definition as ``rhs3``)."""
    Bu = apply_A3_points(prob, j, U[j], pts, "B")
    H = np.zeros(len(pts))
    if j >= 1:
        c = O.l21s_c(prob.alpha, j)
        kap = O.l21s_kappa(prob.alpha, time_step(prob))
        for r, (i, k, l) in enumerate(pts):
            H[r] = kap * sum(c[j - s] * (U[s + 1][i, k, l] - U[s][i, k, l]) for s in range(j))
    return Bu - H + np.array([f_j[int(i), int(k), int(l)] for i, k, l in pts])


def anorm3(prob, j: int) -> float:
    """An upper bound of |A|_2: eta + sigma sum over the axes of
    |gamma|/h + (d_+ + d_-) h^-beta sum_k |omega_k|."""
    tot = 0.0
    for p1 in axes(prob):
        _, gam, dp, dm = O.level_scalars(p1, j)
        h = O.mesh_h(p1)
        w = O.wsgd_weights(p1.beta, p1.n + 1)
        tot += abs(gam) / h + (dp + dm) * h ** (-p1.beta) * float(np.sum(np.abs(w)))
    return _eta(prob, j) + O.sigma_of(prob.alpha) * tot
