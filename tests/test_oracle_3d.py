"""Pins of the three-dimensional oracle: against the two-dimensional oracle
(itself pinned against the one-dimensional one) plane by plane, against
permutations of the axes, against the one-dimensional operators on separable
arrays, against a manufactured solution (observed second order), and between
its dense and FFT routes."""
import dataclasses

import numpy as np
import pytest

import oracle as O1
import oracle.ids2d_oracle as O2
import oracle.ids3d_oracle as O3
import workloads as W


def _zero_axis(prob, k):
    """The problem with axis k's operator removed (gamma = d_+- = 0 there)."""
    z = lambda t: 0.0  # noqa: E731
    rep = lambda v: tuple(z if q == k else v[q] for q in range(3))  # noqa: E731
    return dataclasses.replace(prob, gammas=rep(prob.gammas), dpluses=rep(prob.dpluses), dminuses=rep(prob.dminuses))


def _plane_problem(prob, keep):
    """The two-dimensional problem on the two axes in ``keep`` (in order)."""
    a, b = keep
    return W.Problem2D(alpha=prob.alpha, beta_x=prob.betas[a], beta_y=prob.betas[b], nx=prob.ns[a], ny=prob.ns[b],
                       M=prob.M, gamma_x=prob.gammas[a], gamma_y=prob.gammas[b], dplus_x=prob.dpluses[a],
                       dminus_x=prob.dminuses[a], dplus_y=prob.dpluses[b], dminus_y=prob.dminuses[b],
                       a=prob.lo[a], b=prob.hi[a], c=prob.lo[b], d=prob.hi[b], T=prob.T)


@pytest.mark.parametrize("zero", [2, 0])
def test_reduces_to_the_2d_oracle_plane_by_plane(zero):
    """With one axis's operator zero the system is block diagonal: every plane
    across that axis follows the two-dimensional scheme with the 3D source
    and initial level sampled on the plane."""
    prob = _zero_axis(W.problem_3d(5, 6, 4, 4, betas=(1.5, 1.8, 1.3)), zero)
    U = O3.march3(prob)
    F = [O3.source_level(prob, j) for j in range(prob.M)]
    keep = tuple(k for k in range(3) if k != zero)
    p2 = _plane_problem(prob, keep)
    for plane in range(prob.ns[zero]):
        take = lambda A: np.take(A, plane, axis=zero)  # noqa: E731
        U2 = O2.march2(p2, f_levels=[take(f) for f in F], u0=take(U[0]))
        got = np.stack([take(U[j]) for j in range(prob.M + 1)])
        assert np.max(np.abs(got - U2)) <= 1e-12 * max(1.0, np.max(np.abs(U2))), (zero, plane)


@pytest.mark.parametrize("perm", [(2, 0, 1), (1, 0, 2), (0, 2, 1)])
def test_permuting_the_axes_transposes_the_solution(perm):
    prob = W.problem_3d(4, 5, 6, 3, betas=(1.3, 1.9, 1.6))
    U = O3.march3(prob)
    Up = O3.march3(prob.permuted(perm))
    ref = np.transpose(U, (0,) + tuple(p + 1 for p in perm))
    assert Up.shape == ref.shape
    assert np.max(np.abs(Up - ref)) <= 1e-12 * np.max(np.abs(U))


def test_kronecker_sum_on_separable_arrays():
    """L (a (x) b (x) c) = (L_x a) (x) b (x) c + a (x) (L_y b) (x) c + a (x) b (x) (L_z c)
    with the one-dimensional oracle's matrices, for the dense and FFT routes."""
    prob = W.problem_3d(6, 5, 7, 4, betas=(1.2, 1.7, 1.95))
    rng = np.random.default_rng(11)
    a, b, c = (rng.standard_normal(n) for n in prob.ns)
    V = np.einsum("i,k,l->ikl", a, b, c)
    px, py, pz = (prob.axis(k) for k in range(3))
    for j in (0, 3):
        ref = (np.einsum("i,k,l->ikl", O1.level_L(px, j) @ a, b, c) + np.einsum("i,k,l->ikl", a, O1.level_L(py, j) @ b, c)
               + np.einsum("i,k,l->ikl", a, b, O1.level_L(pz, j) @ c))
        got = (O3.level_L3(prob, j) @ V.reshape(-1)).reshape(V.shape)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
        e, sg = O1.level_scalars(px, j)[0], O1.sigma_of(prob.alpha)
        assert np.max(np.abs(O3.product3(prob, j, V, "A") - (e * V - sg * ref))) <= 1e-12 * np.max(np.abs(ref))


def test_second_order_convergence_to_the_manufactured_solution():
    """Errors against u = A t^2 prod s^2(1-s)^2 fall by about four per halving
    of h and tau together (second order in time and space); the larger
    grids run the FFT route (pinned against the dense one below)."""
    errs = []
    for N in (8, 16, 32):
        prob = W.problem_3d(N - 1, N - 1, N - 1, N, alpha=0.5, betas=(1.6, 1.4, 1.8))
        U = O3.march3(prob) if N < 16 else O3.march_pcgs3(prob, rtol=1e-12)[0]
        errs.append(O3.error_norms3(prob, U)[0])
    orders = [np.log2(errs[k] / errs[k + 1]) for k in range(2)]
    print("3D errors", errs, "orders", orders)
    assert min(orders) > 1.75, (errs, orders)


def test_fft_route_against_dense():
    """Products, the three-level circulant preconditioner's solve and the PCGS
    level against dense matrices."""
    prob = W.problem_3d(8, 4, 16, 6, betas=(1.8, 1.2, 1.5))
    rng = np.random.default_rng(3)
    V = rng.standard_normal(prob.ns)
    for j in (0, 4):
        for which, Mat in (("A", O3.level_A3), ("B", O3.level_B3)):
            ref = (Mat(prob, j) @ V.reshape(-1)).reshape(V.shape)
            assert np.max(np.abs(O3.product3(prob, j, V, which) - ref)) <= 1e-12 * np.max(np.abs(ref))
        P = O3.bccb3_matrix(prob, j)
        Y = O3.bccb3_solve(prob, j, V)
        assert np.max(np.abs((P @ Y.reshape(-1)).reshape(V.shape) - V)) <= 1e-11 * np.max(np.abs(V))
    U = O3.march3(prob, levels=3)
    f = O3.source_level(prob, 3)
    u_pcgs, its = O3.level_solve_pcgs3(prob, U, 3, f, rtol=1e-13)
    u_lu = O3.level_solve3(prob, U, 3, f)
    assert its < 60
    assert np.max(np.abs(u_pcgs - u_lu)) <= 1e-10 * np.max(np.abs(u_lu))


def test_points_match_dense_rows():
    prob = W.problem_3d(4, 8, 6, 4)
    rng = np.random.default_rng(4)
    U = rng.standard_normal((3,) + prob.ns)
    f = rng.standard_normal(prob.ns)
    pts = [(0, 0, 0), (3, 7, 5), (1, 4, 2), (0, 7, 0), (3, 0, 5), (2, 2, 2)]
    for j in (0, 2):
        ref = (O3.level_A3(prob, j) @ U[j].reshape(-1)).reshape(prob.ns)
        got = O3.apply_A3_points(prob, j, U[j], pts, "A")
        assert np.allclose(got, [ref[p] for p in pts], rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))
        g = O3.rhs3(prob, U, j, f)
        assert np.allclose(O3.rhs3_points(prob, U, j, f, pts), [g[p] for p in pts], rtol=1e-12,
                           atol=1e-12 * np.max(np.abs(g)))


def test_anorm_bounds_the_norm():
    prob = W.problem_3d(4, 6, 5, 4)
    for j in (0, 3):
        assert np.linalg.norm(O3.level_A3(prob, j), 2) <= O3.anorm3(prob, j)


def test_source_matches_the_manufactured_solution_pointwise():
    """The separable source equals the closed-form terms evaluated one point at
    a time (the Caputo term and, per axis, convection and the two
    Riemann-Liouville terms)."""
    prob = W.problem_3d(5, 4, 6, 4)
    x, y, z = O3.nodes(prob)
    t = 0.37
    F = prob.f(x, y, z, t)
    s = prob.sols
    for (i, k, l) in [(0, 0, 0), (4, 3, 5), (2, 1, 3)]:
        P = [s[0].P(x[i]), s[1].P(y[k]), s[2].P(z[l])]
        pt = (x[i], y[k], z[l])
        th = prob.theta(t)
        val = s[0].caputo_theta(t, prob.alpha) * P[0] * P[1] * P[2]
        for a in range(3):
            rest = np.prod([P[q] for q in range(3) if q != a])
            val -= th * rest * (prob.gammas[a](t) * s[a].dP(pt[a]) + prob.dpluses[a](t) * s[a].rl_left(pt[a], prob.betas[a])
                                + prob.dminuses[a](t) * s[a].rl_right(pt[a], prob.betas[a]))
        assert abs(F[i, k, l] - val) <= 1e-13 * max(1.0, abs(val))
