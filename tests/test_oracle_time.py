"""Pins for the oracle's time discretisation (Lemma 1, the L2-1sigma formula).

The formula is exact for polynomials of degree <= 2 in t (checked against the
Gamma-function closed form of the Caputo derivative), degrades to the stated
O(tau^(3-alpha)) for t^3, and reduces to the backward difference quotient
(Crank-Nicolson in time) at alpha = 1.
"""
import math

import numpy as np
import pytest

import oracle as O


def caputo_power(p, alpha, t):
    # Caputo derivative of t^p (p > 0):  Gamma(p+1)/Gamma(p+1-alpha) t^(p-alpha)   (1.2)
    return math.gamma(p + 1) / math.gamma(p + 1 - alpha) * t ** (p - alpha)


@pytest.mark.parametrize("alpha", [0.1, 0.5, 0.7, 0.9, 0.99])
@pytest.mark.parametrize("j", [0, 1, 2, 5, 17, 60])
@pytest.mark.parametrize("p", [1, 2])
def test_l21s_exact_for_quadratics(alpha, j, p):
    tau = 0.05
    sigma = 1 - alpha / 2
    t = np.arange(j + 2) * tau
    approx = O.caputo_l21s(alpha, tau, t ** p, j)
    exact = caputo_power(p, alpha, (j + sigma) * tau)
    assert abs(approx - exact) <= 1e-12 * abs(exact), (approx, exact)


@pytest.mark.parametrize("alpha", [0.3, 0.8])
def test_l21s_constant_gives_zero(alpha):
    assert O.caputo_l21s(alpha, 0.1, np.ones(12), 10) == 0.0


@pytest.mark.parametrize("alpha", [0.3, 0.8])
def test_l21s_cubic_is_third_order(alpha):
    # not exact for t^3; error at fixed t shrinks like tau^(3 - alpha)
    errs = []
    for M in (20, 40, 80):
        tau = 1.0 / M
        j = M // 2
        sigma = 1 - alpha / 2
        t = np.arange(j + 2) * tau
        errs.append(abs(O.caputo_l21s(alpha, tau, t ** 3, j) - caputo_power(3, alpha, (j + sigma) * tau)))
    assert errs[0] > 1e-8
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    for r in rates:
        assert 3 - alpha - 0.3 < r < 3 - alpha + 0.3, rates


def test_l21s_alpha_one_is_difference_quotient():
    # alpha = 1: sigma = 1/2, a_l = b_l = 0 for l >= 1, c = (1, 0, ..., 0), kappa = 1/tau
    c = O.l21s_c(1.0, 9)
    assert c[0] == 1.0 and np.all(c[1:] == 0.0)
    assert O.l21s_kappa(1.0, 0.25) == 4.0


@pytest.mark.parametrize("alpha", [0.2, 0.6, 0.95])
def test_l21s_coefficient_signs(alpha):
    # c_0 > c_1 > ... > 0 style positivity used by the stability analysis (Lemma 7 setting):
    # all c_m^(j) are positive and eta_j > 0.
    for j in (1, 2, 10, 100):
        c = O.l21s_c(alpha, j)
        assert np.all(c > 0)
        assert O.eta(alpha, 0.01, j) > 0
