"""Pins of the oracle's constant-coefficient path (Algorithm 3 with the
Gohberg-Semencul formula, Algorithm 1) against the definition of the inverse
and against the plain dense march: the formula's four triangular Toeplitz
factors rebuild A^-1 exactly (up to rounding), xi_0 is (A^-1)_{00}, and the
march by Algorithm 3 equals the march by Algorithm 2 level by level."""
import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.mark.parametrize("n", [4, 5, 31, 64])
@pytest.mark.parametrize("alpha,beta", [(0.9, 1.8), (0.1, 1.2), (1.0, 2.0)])
def test_gsf_rebuilds_the_inverse(n, alpha, beta):
    prob = W.example1(alpha, beta, n + 1)
    A = O.level_A(prob, 1)
    x, y = O.gsf_generators(prob)
    Ainv = np.linalg.inv(A)
    assert abs(x[0] - Ainv[0, 0]) <= 1e-13 * abs(Ainv[0, 0])
    assert np.allclose(x, Ainv[:, 0], rtol=0, atol=1e-13 * np.abs(Ainv).max())
    assert np.allclose(y, Ainv[:, -1], rtol=0, atol=1e-13 * np.abs(Ainv).max())
    Lp, Rp, L0, R0 = O.gsf_matrices(x, y)
    # triangular Toeplitz structure as printed
    assert np.array_equal(Lp, np.tril(Lp)) and np.array_equal(Rp, np.triu(Rp))
    assert np.array_equal(L0, np.tril(L0, -1)) and np.array_equal(R0, np.triu(R0, 1))
    assert np.all(np.diag(Rp) == y[-1]) and np.all(np.diag(Lp) == x[0])
    G = (Lp @ Rp - L0 @ R0) / x[0]
    assert np.max(np.abs(G - Ainv)) <= 1e-11 * np.abs(Ainv).max()
    v = np.random.default_rng(n).standard_normal(n)
    z = O.gsf_apply(x, y, v)
    assert np.linalg.norm(A @ z - v) <= 1e-12 * np.linalg.norm(v) * np.linalg.cond(A)


@pytest.mark.parametrize("alpha,beta,N", [(0.9, 1.2, 32), (0.5, 1.8, 64), (0.1, 1.5, 32), (0.99, 1.8, 16)])
def test_algorithm3_march_equals_algorithm2(alpha, beta, N):
    """Example 1 (constant coefficients) on the paper's grids: Algorithm 3
    level by level equals Algorithm 2 with Gaussian elimination."""
    prob = W.example1(alpha, beta, N)
    assert O.coefficients_constant(prob)
    U2 = O.march(prob)
    U3 = O.march_gsf(prob)
    for j in range(1, prob.M + 1):
        assert np.linalg.norm(U3[j] - U2[j]) <= 1e-12 * np.linalg.norm(U2[j]), j


def test_algorithm3_refuses_varying_coefficients():
    with pytest.raises(ValueError):
        O.march_gsf(W.example2(0.5, 1.5, 16))
