"""Pins for the oracle's space discretisation (Lemmas 2-4, Lemma 8, Remark 3.1).

Each check compares against something other than the oracle's own formula:
high-precision binomials, closed-form partial sums, the generating function
(lambda_1 + lambda_0 z + lambda_-1 z^2)(1 - z)^beta, exact special cases and
the sign/sum properties stated in the lemmas.
"""
import mpmath
import numpy as np
import pytest

import oracle as O

BETAS = [1.1, 1.3, 1.5, 1.8, 1.95, 2.0]


@pytest.mark.parametrize("beta", BETAS)
def test_grunwald_matches_high_precision_binomial(beta):
    # g_k = (-1)^k binom(beta, k)  (Lemma 2)
    mpmath.mp.dps = 40
    K = 600
    g = O.grunwald_weights(beta, K)
    for k in [0, 1, 2, 3, 7, 50, 123, 599, 600]:
        ref = float((-1) ** k * mpmath.binomial(mpmath.mpf(beta), k))
        if ref == 0.0:
            assert abs(g[k]) < 1e-300
        else:
            assert abs(g[k] - ref) <= 1e-13 * abs(ref), (k, g[k], ref)


@pytest.mark.parametrize("beta", [1.2, 1.5, 1.9])
def test_grunwald_partial_sums_closed_form(beta):
    # sum_{k<=m} (-1)^k binom(beta,k) = (-1)^m binom(beta-1, m)
    mpmath.mp.dps = 40
    g = O.grunwald_weights(beta, 400)
    cs = np.cumsum(g)
    for m in [1, 2, 5, 40, 399]:
        ref = float((-1) ** m * mpmath.binomial(mpmath.mpf(beta) - 1, m))
        assert abs(cs[m] - ref) <= 1e-13 * max(abs(ref), 1e-3), (m, cs[m], ref)


@pytest.mark.parametrize("beta", [1.2, 1.5, 1.8])
def test_grunwald_lemma3_properties(beta):
    g = O.grunwald_weights(beta, 2000)
    assert g[0] == 1.0 and g[1] == pytest.approx(-beta, rel=1e-15)
    assert np.all(np.diff(g[2:]) < 0) and np.all(g[2:] > 0)      # g_2 > g_3 > ... > 0
    for N in [2, 10, 100, 2000]:
        assert g[: N + 1].sum() < 0                                  # partial sums negative
    # decay O(k^-(beta+1))
    ratio = g[2000] / g[1000]
    assert abs(ratio - 2.0 ** (-(beta + 1))) < 2e-3


@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("z", [0.5, -0.5, 0.3 + 0.4j])
def test_wsgd_generating_function(beta, z):
    # sum_k omega_k z^k = (lambda_1 + lambda_0 z + lambda_-1 z^2) (1 - z)^beta; a wrong
    # lambda or a shifted index changes this identity.
    K = 400
    w = O.wsgd_weights(beta, K)
    lhs = np.polynomial.polynomial.polyval(z, w)
    l1 = (beta ** 2 + 3 * beta + 2) / 12
    l0 = (4 - beta ** 2) / 6
    lm1 = (beta ** 2 - 3 * beta + 2) / 12
    mpmath.mp.dps = 30
    rhs = complex((l1 + l0 * z + lm1 * z * z) * mpmath.power(1 - mpmath.mpc(z), beta))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(rhs))


def test_wsgd_beta2_is_three_point_laplacian():
    w = O.wsgd_weights(2.0, 10)
    assert np.array_equal(w, np.array([1.0, -2.0, 1.0] + [0.0] * 8))


@pytest.mark.parametrize("beta", [1.1, 1.4, 1.7, 1.99])
def test_wsgd_lemma4_properties(beta):
    w = O.wsgd_weights(beta, 5000)
    assert w[1] < 0
    assert np.all(w[3:] > 0)
    assert w[0] + w[2] >= 0
    # omega_0 = lambda_1 (the printed 'omega_0 = 1' holds only at beta = 2)
    assert w[0] == pytest.approx((beta ** 2 + 3 * beta + 2) / 12, rel=1e-15)
    for N in [2, 5, 100, 5000]:
        assert w[: N + 1].sum() < 0
    # sum to infinity is 0: the partial sums approach 0 like K^-beta
    assert abs(w.sum()) < 5.0 * 5000.0 ** (-beta)


@pytest.mark.parametrize("beta", [1.1, 1.2, 1.5, 1.7, 1.8, 1.95])
@pytest.mark.parametrize("n", [64, 1023, 1024])
def test_strang_spectrum_gershgorin_and_remark(beta, n):
    # Remark 3.1 (1) / Theorem 3.1: every eigenvalue of s(W) has negative real part.
    # Lemma 8 (disc |z - omega_1| < -omega_1, centre omega_1 < 0) and Remark 3.1 (2)
    # (|lambda| <= 2|omega_1|) follow from Gershgorin only when omega_k >= 0 for all
    # k != 1, i.e. when omega_2 >= 0; below that beta the disc bound does not hold.
    w = O.wsgd_weights(beta, n + 1)
    col = O.strang_column(lambda m: w[m + 1] if m >= -1 else 0.0, n)
    lam = O.circulant_eigenvalues(col)
    assert np.all(lam.real < 0)
    if w[2] >= 0:
        assert np.all(np.abs(lam - w[1]) < -w[1])
        assert np.all(np.abs(lam) <= 2 * abs(w[1]) * (1 + 1e-14))
    else:
        assert np.max(np.abs(lam - w[1])) > -w[1]


@pytest.mark.parametrize("n", [8, 31, 64])
def test_strang_Q_eigenvalues_closed_form(n):
    # s(Q) has eigenvalues 2 i sin(2 pi k / n) with the DFT convention of the oracle.
    col = O.strang_column(lambda m: -1.0 if m == 1 else (1.0 if m == -1 else 0.0), n)
    lam = O.circulant_eigenvalues(col)
    k = np.arange(n)
    assert np.allclose(lam, 2j * np.sin(2 * np.pi * k / n), atol=1e-14)


@pytest.mark.parametrize("n", [5, 16, 33])
def test_circulant_eigenvalues_match_dense_eig(n):
    rng = np.random.default_rng(n)
    col = rng.standard_normal(n)
    lam = O.circulant_eigenvalues(col)
    ref = np.linalg.eigvals(O.circulant(col))
    # same multiset: each eigenvalue has a partner in the other set, both ways
    d = np.abs(lam[:, None] - ref[None, :])
    assert d.min(axis=1).max() < 1e-12 and d.min(axis=0).max() < 1e-12


@pytest.mark.parametrize("n", [4, 9, 16])
def test_strang_column_copies_central_diagonals(n):
    # Strang: keep the central diagonals of the Toeplitz matrix, wrap them around.
    rng = np.random.default_rng(7)
    t = {m: rng.standard_normal() for m in range(-n + 1, n)}
    col = O.strang_column(lambda m: t[m], n)
    C = O.circulant(col)
    lo, hi = -(n - 1 - n // 2), n // 2
    for i in range(n):
        for k in range(n):
            if lo <= i - k <= hi:
                assert C[i, k] == t[i - k]


@pytest.mark.parametrize("n,L", [(5, 9), (8, 16), (13, 32)])
def test_embedding_column_reproduces_W(n, L):
    beta = 1.6
    c = O.embedding_column(beta, n, L)
    C = O.circulant(c)
    assert np.array_equal(C[:n, :n], O.toeplitz_W(beta, n))
    # and the transpose embedding is the reversed column (conjugate spectrum)
    rev = np.roll(c[::-1], 1)
    assert np.array_equal(O.circulant(rev)[:n, :n], O.toeplitz_W(beta, n).T)
    assert np.allclose(np.fft.fft(rev), np.conj(np.fft.fft(c)), atol=1e-13)
