"""Pins of the oracle's preconditioner and solver parts against what the
paper fixes, independently of the oracle's own assembly of P:

* Sec. 3.2 defines P as the Strang circulant of the level matrix: for odd n
  the oracle's P (3.7) equals s(A) built from the central diagonals of the
  dense A^(j+sigma) of (3.3); for even n they differ only on the lag-n/2
  circulant diagonal, by the documented reading s(W^T) := s(W)^T.
* Theorem 3.1: every eigenvalue of P has a positive real part.
* Sec. 4 (and Sec. 3.2): PCGS needs few iterations per level on Example 2.
* Adam's bias correction (Kingma and Ba 2015) at steps 2 and 3, by closed
  forms for constant and alternating gradients.
"""
import math

import numpy as np
import pytest

import oracle as O
import oracle.warmnet_oracle as NO
import workloads as W


def strang_of_dense(A):
    """Strang circulant of a Toeplitz matrix given densely: lag m = i - k
    read off the first column (m >= 0) and the first row (m < 0); column
    c_k = t_k for k <= floor(n/2), t_{k-n} beyond."""
    n = A.shape[0]
    t = lambda m: A[m, 0] if m >= 0 else A[0, -m]  # noqa: E731
    col = np.array([t(k) if k <= n // 2 else t(k - n) for k in range(n)])
    idx = (np.arange(n)[:, None] - np.arange(n)[None, :]) % n
    return col[idx]


def _problems(n):
    # gamma != 0 of both signs and d+ != d-, so that a slip in the sign or
    # the factor of the convection term or of the D_- term changes P
    yield W.Problem(alpha=0.6, beta=1.7, n=n, M=8, gamma=lambda t: -0.8 - t, dplus=lambda t: 1.0 + t,
                    dminus=lambda t: 0.25 + 2.0 * t)
    yield W.Problem(alpha=0.9, beta=1.2, n=n, M=8, gamma=lambda t: 1.5, dplus=lambda t: 0.3,
                    dminus=lambda t: 1.7)


@pytest.mark.parametrize("n", [5, 31, 63, 127])
def test_P_is_strang_of_A_for_odd_n(n):
    for prob in _problems(n):
        for j in (0, 3):
            A = O.level_A(prob, j)
            P = O.preconditioner_matrix(prob, j)
            S = strang_of_dense(A)
            assert np.max(np.abs(P - S)) <= 1e-13 * np.max(np.abs(A)), (j, np.max(np.abs(P - S)))


@pytest.mark.parametrize("n", [8, 32, 64])
def test_P_differs_from_strang_of_A_by_one_lag_for_even_n(n):
    """For even n the Strang column takes the lag +n/2 entry at k = n/2, so
    s(W^T) has W's lag -n/2 (zero) there while s(W)^T has W's lag +n/2,
    omega_{n/2+1}: P - s(A) is -sigma D_- h^-beta omega_{n/2+1} on the
    circulant diagonal (i - k) mod n = n/2 and zero elsewhere."""
    for prob in _problems(n):
        j = 2
        A = O.level_A(prob, j)
        P = O.preconditioner_matrix(prob, j)
        D = P - strang_of_dense(A)
        _, gam, dp, dm = O.level_scalars(prob, j)
        h = O.mesh_h(prob)
        w = O.wsgd_weights(prob.beta, n + 1)
        expect = -O.sigma_of(prob.alpha) * dm * h ** (-prob.beta) * w[n // 2 + 1]
        diag = (np.arange(n)[:, None] - np.arange(n)[None, :]) % n == n // 2
        scale = np.max(np.abs(A))
        assert np.max(np.abs(D[~diag])) <= 1e-13 * scale
        assert np.max(np.abs(D[diag] - expect)) <= 1e-13 * scale
        assert abs(expect) > 1e-9 * scale  # the difference is really there


@pytest.mark.parametrize("n", [7, 16, 63, 100])
@pytest.mark.parametrize("alpha,beta", [(0.5, 1.5), (0.9, 1.05), (0.2, 1.95), (1.0, 2.0)])
def test_theorem_3_1_real_parts_positive(n, alpha, beta):
    """Re lambda(P) > 0, computed from the dense P by LAPACK's general
    eigenvalue routine (not from the circulant formula): with D_+- >= 0 the
    symmetric part of the Grunwald part of P is negative semidefinite and
    s(Q) is skew, so Re lambda >= eta_j."""
    prob = W.Problem(alpha=alpha, beta=beta, n=n, M=4, gamma=lambda t: -3.0 + t, dplus=lambda t: 2.0 * t,
                     dminus=lambda t: 0.7 + t)
    for j in range(prob.M):
        lam = np.linalg.eigvals(O.preconditioner_matrix(prob, j))
        e = O.level_scalars(prob, j)[0]
        assert np.min(lam.real) > 0.0
        assert np.min(lam.real) >= e * (1.0 - 1e-10), (j, np.min(lam.real), e)


@pytest.mark.parametrize("N", [32, 64, 128, 256, 512, 1024])
def test_pcgs_iterations_on_example2(N):
    """Example 2 (alpha = 0.9, beta = 1.5, h = tau = 1/N, n = N - 1): PCGS from
    x0 = 0 to a recursive residual of 1e-12 |g| takes the handful of
    iterations Sec. 4 reports (between 4 and 10), at the first levels and at
    the middle and last ones, where d_+- = (9, 4) sin t are largest.  The
    iteration count depends on A and g, not on the history, which is left
    at zero beyond u^0 here."""
    prob = W.example2(0.9, 1.5, N)
    its = []
    for j in (0, 1, N // 2, N - 1):
        U = np.zeros((j + 1, prob.n))
        U[0] = O.initial_level(prob)
        _, k = O.level_solve_pcgs(prob, U, j, O.source_level(prob, j), rtol=1e-12)
        its.append(k)
    assert 4 <= min(its) and max(its) <= 10, its


def _wrong_strang_eigenvalues(sign_dplus, sign_dminus):
    def lam(p, j, kind="strang"):
        e, gam, dp, dm = O.level_scalars(p, j)
        lw = O.circulant_eigenvalues(O.strang_column(O.ids_oracle._W_lag(p.beta, p.n), p.n))
        lq = O.circulant_eigenvalues(O.strang_column(O.ids_oracle._Q_lag, p.n))
        h, s = O.mesh_h(p), O.sigma_of(p.alpha)
        return e - s * (gam / (2 * h) * lq + sign_dplus * dp / h ** p.beta * lw
                        + sign_dminus * dm / h ** p.beta * np.conj(lw))
    return lam


@pytest.mark.parametrize("signs", [(1.0, -1.0), (-1.0, 1.0)])
def test_pcgs_iterations_grow_with_a_wrong_preconditioner(monkeypatch, signs):
    """The iteration pin has teeth: at N = 256, last level, flipping the sign
    of the D_- or of the D_+ term of P drives the count far beyond 10.  (The
    convection term is small beside h^-beta in Example 2; the Strang-of-A
    pins above catch its sign.)"""
    prob = W.example2(0.9, 1.5, 256)
    j = prob.M - 1
    U = np.zeros((j + 1, prob.n))
    U[0] = O.initial_level(prob)
    _, k_good = O.level_solve_pcgs(prob, U, j, O.source_level(prob, j), rtol=1e-12)
    monkeypatch.setattr(O.ids_oracle, "strang_eigenvalues", _wrong_strang_eigenvalues(*signs))
    _, k_bad = O.level_solve_pcgs(prob, U, j, O.source_level(prob, j), rtol=1e-12)
    assert k_good <= 10 and k_bad > 30, (k_good, k_bad)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_adam_constant_gradient_steps_are_lr_sign(sign):
    """With a constant gradient the bias-corrected moments are exact at every
    step (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so steps 1, 2 and 3 each
    move by lr sign(g).  Dropping the power of t in either correction makes
    step 2 move by lr (1 + b1)/sqrt(1 + b2) ~ 1.344 lr instead."""
    g = sign * np.array([0.5, 2.0, 1e-3])
    th = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    lr = 1e-2
    for t in (1, 2, 3):
        new, m, v = NO.adam_step(th, m, v, g, t, lr, eps=0.0)
        assert np.allclose(th - new, lr * np.sign(g), rtol=1e-12, atol=0), t
        th = new


def test_adam_alternating_gradient_steps():
    """g, -g, g: m_2 = -(1 - b1)^2 g, v_2 = (1 - b2)(1 + b2) g^2, so step 2
    moves theta by +lr (1 - b1)/(1 + b1) sign(g) = lr/19 sign(g) (b1 = 0.9);
    m_3 = (1 - b1)(1 - b1 (1 - b1)) g, v_3 = (1 - b2)(1 + b2 + b2^2) g^2, so
    step 3 moves it by -lr (0.1 * 0.91 / 0.271) sign(g)."""
    g = np.array([0.3, -4.0])
    lr = 1e-2
    th, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    th1, m, v = NO.adam_step(th, m, v, g, 1, lr, eps=0.0)
    th2, m, v = NO.adam_step(th1, m, v, -g, 2, lr, eps=0.0)
    assert np.allclose(th2 - th1, lr / 19.0 * np.sign(g), rtol=1e-12, atol=0)
    th3, m, v = NO.adam_step(th2, m, v, g, 3, lr, eps=0.0)
    assert np.allclose(th3 - th2, -lr * (0.1 * 0.91 / 0.271) * np.sign(g), rtol=1e-12, atol=0)
    assert math.isclose(0.1 * 0.91 / 0.271, 0.33579335793357934, rel_tol=1e-15)


def _optimal_circulant(T):
    """The circulant nearest to T in the Frobenius norm: its first column
    averages T over each wrapped diagonal, c_k = mean of T[i, l] with
    (i - l) mod n = k (the minimisation over the n circulant parameters)."""
    n = T.shape[0]
    d = (np.arange(n)[:, None] - np.arange(n)[None, :]) % n
    col = np.array([T[d == k].mean() for k in range(n)])
    return col[d]


@pytest.mark.parametrize("n", [5, 8, 31, 64])
def test_tchan_is_the_frobenius_optimal_circulant_of_A(n):
    """T. Chan's preconditioner is the optimal circulant of A itself (the
    identity, Q, W and W^T parts each averaged over wrapped diagonals), for
    odd and even n alike, and it is the Frobenius minimiser: any change of one
    circulant parameter moves it further from A."""
    for prob in _problems(n):
        j = 3
        A = O.level_A(prob, j)
        P = O.preconditioner_matrix(prob, j, "tchan")
        C = _optimal_circulant(A)
        assert np.max(np.abs(P - C)) <= 1e-13 * np.max(np.abs(A))
        d = (np.arange(n)[:, None] - np.arange(n)[None, :]) % n
        base = np.linalg.norm(P - A)
        for k in (0, 1, n - 1):
            bumped = P + 1e-3 * np.max(np.abs(A)) * (d == k)
            assert np.linalg.norm(bumped - A) > base


@pytest.mark.parametrize("n", [7, 64])
def test_tchan_eigenvalues_and_theorem_3_1(n):
    """The FFT eigenvalues of the T. Chan preconditioner are those of its
    dense matrix, and their real parts are positive (the argument of
    Theorem 3.1 carries over: c(Q) is skew, c(W) + c(W)^T is negative
    semidefinite for D_+- >= 0)."""
    prob = W.Problem(alpha=0.6, beta=1.7, n=n, M=4, gamma=lambda t: -3.0 + t, dplus=lambda t: 2.0 * t,
                     dminus=lambda t: 0.7 + t)
    for j in range(prob.M):
        lam = O.strang_eigenvalues(prob, j, "tchan")
        dense = np.linalg.eigvals(O.preconditioner_matrix(prob, j, "tchan"))
        tol = 1e-9 * np.abs(lam).max()
        assert np.max(np.min(np.abs(lam[:, None] - dense[None, :]), axis=1)) <= tol
        assert np.max(np.min(np.abs(dense[:, None] - lam[None, :]), axis=1)) <= tol
        assert np.min(lam.real) > 0


@pytest.mark.parametrize("kind", ["strang", "tchan"])
@pytest.mark.parametrize("n", [63, 64, 255])
def test_pbicgstab_reaches_the_lu_solution(kind, n):
    """BiCGSTAB with either circulant preconditioner converges, in a handful
    of iterations, to the dense-LU solution of the level (brute force)."""
    prob = W.config_large(n=n, M=8, alpha=0.6, beta=1.7)
    rng = np.random.default_rng(n)
    U = rng.standard_normal((prob.M + 1, n))
    f = rng.standard_normal(n)
    for j in (0, 5):
        A = O.level_A(prob, j)
        ref = O.level_solve(prob, U, j, f)
        u, its = O.level_solve_pbicgstab(prob, U, j, f, rtol=1e-13, kind=kind)
        bound = max(1e-10, 8 * 2.2e-16 * np.linalg.cond(A, 1))
        assert np.linalg.norm(u - ref) <= bound * np.linalg.norm(ref), (j, its)
        assert its <= 30
        u2, its2 = O.level_solve_pcgs(prob, U, j, f, rtol=1e-13, kind=kind)
        assert np.linalg.norm(u2 - ref) <= bound * np.linalg.norm(ref), (j, its2)
