"""Pins of the two-dimensional oracle against the one-dimensional oracle
(itself pinned), against exchange of the axes, against a manufactured
solution (observed second order), and between its dense and FFT routes."""
import numpy as np
import pytest

import oracle as O1
import oracle.ids2d_oracle as O2
import workloads as W


def _prob(nx, ny, M, **kw):
    return W.problem_2d(nx, ny, M, **kw)


def _zero_axis(prob, axis):
    """The problem with one axis's operator removed (gamma = d_+- = 0 there)."""
    z = lambda t: 0.0  # noqa: E731
    p = W.Problem2D(**{k: getattr(prob, k) for k in (
        "alpha", "beta_x", "beta_y", "nx", "ny", "M", "gamma_x", "gamma_y", "dplus_x", "dminus_x",
        "dplus_y", "dminus_y", "a", "b", "c", "d", "T", "sol_x", "sol_y")})
    if axis == "y":
        p.gamma_y = p.dplus_y = p.dminus_y = z
    else:
        p.gamma_x = p.dplus_x = p.dminus_x = z
    return p


@pytest.mark.parametrize("axis", ["x", "y"])
def test_reduces_to_the_1d_oracle_line_by_line(axis):
    """With the other axis's operator zero the system is block diagonal: every
    line along `axis` follows the one-dimensional scheme with the 2D source
    sampled on that line."""
    prob = _zero_axis(_prob(9, 7, 6), "y" if axis == "x" else "x")
    U = O2.march2(prob)
    F = [O2.source_level(prob, j) for j in range(prob.M)]
    p1 = prob.axis(axis)
    nlines = prob.ny if axis == "x" else prob.nx
    for line in range(nlines):
        take = (lambda A: A[:, line]) if axis == "x" else (lambda A: A[line, :])  # noqa: E731
        U1 = O1.march(p1, f_levels=[take(f) for f in F], u0=take(U[0]))
        got = np.stack([take(U[j]) for j in range(prob.M + 1)])
        assert np.max(np.abs(got - U1)) <= 1e-12 * max(1.0, np.max(np.abs(U1))), (axis, line)


def test_exchanging_the_axes_transposes_the_solution():
    prob = _prob(7, 11, 5, beta_x=1.3, beta_y=1.8)
    U = O2.march2(prob)
    Us = O2.march2(prob.swapped())
    assert Us.shape == (prob.M + 1, prob.ny, prob.nx)
    assert np.max(np.abs(Us - np.transpose(U, (0, 2, 1)))) <= 1e-12 * np.max(np.abs(U))


def test_second_order_convergence_to_the_manufactured_solution():
    """Errors against u = A t^2 x^2(1-x)^2 y^2(1-y)^2 fall by about four per
    halving of h and tau together (second order in time and space)."""
    errs = []
    for N in (8, 16, 32):
        prob = _prob(N - 1, N - 1, N, alpha=0.5, beta_x=1.6, beta_y=1.4)
        errs.append(O2.error_norms2(prob, O2.march2(prob))[0])
    orders = [np.log2(errs[k] / errs[k + 1]) for k in range(2)]
    print("2D errors", errs, "orders", orders)
    assert min(orders) > 1.75, (errs, orders)


def test_fft_route_against_dense():
    """Products, the BCCB preconditioner's solve and the PCGS level against
    dense matrices."""
    prob = _prob(16, 8, 8, beta_x=1.8, beta_y=1.2)
    rng = np.random.default_rng(3)
    V = rng.standard_normal((prob.nx, prob.ny))
    for j in (0, 3):
        for which, Mat in (("A", O2.level_A2), ("B", O2.level_B2)):
            ref = (Mat(prob, j) @ V.reshape(-1)).reshape(V.shape)
            assert np.max(np.abs(O2.product2(prob, j, V, which) - ref)) <= 1e-12 * np.max(np.abs(ref))
        P = O2.bccb_matrix(prob, j)
        Y = O2.bccb_solve(prob, j, V)
        assert np.max(np.abs((P @ Y.reshape(-1)).reshape(V.shape) - V)) <= 1e-11 * np.max(np.abs(V))
    U = O2.march2(prob, levels=3)
    f = O2.source_level(prob, 3)
    u_pcgs, its = O2.level_solve_pcgs2(prob, U, 3, f, rtol=1e-13)
    u_lu = O2.level_solve2(prob, U, 3, f)
    assert its < 60
    assert np.max(np.abs(u_pcgs - u_lu)) <= 1e-10 * np.max(np.abs(u_lu))


def test_points_match_dense_rows():
    prob = _prob(8, 16, 4)
    rng = np.random.default_rng(4)
    U = rng.standard_normal((3, prob.nx, prob.ny))
    f = rng.standard_normal((prob.nx, prob.ny))
    pts = [(0, 0), (7, 15), (3, 9), (0, 15), (7, 0), (4, 4)]
    for j in (0, 2):
        A = O2.level_A2(prob, j)
        ref = (A @ U[j].reshape(-1)).reshape(prob.nx, prob.ny)
        got = O2.apply_A2_points(prob, j, U[j], pts, "A")
        assert np.allclose(got, [ref[i, k] for i, k in pts], rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))
        g = O2.rhs2(prob, U, j, f)
        assert np.allclose(O2.rhs2_points(prob, U, j, f, pts), [g[i, k] for i, k in pts], rtol=1e-12,
                           atol=1e-12 * np.max(np.abs(g)))


def test_anorm_bounds_the_norm():
    prob = _prob(8, 8, 4)
    for j in (0, 3):
        assert np.linalg.norm(O2.level_A2(prob, j), 2) <= O2.anorm2(prob, j)
