"""The fast history's fit (the library's host-side construction, no device
work) against the L2-1sigma weights of Lemma 1 evaluated in 40-digit
arithmetic, and the oracle's perturbation bound against its definition."""
import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as W


def _fit(alpha, M, tol):
    from paper_1603_00279_amd import _native as N
    K = ctypes.c_int32()
    err = ctypes.c_double()
    rho = np.zeros(512)
    w = np.zeros(512)
    poly = np.zeros(4)
    rc = N.lib().tsfcde_history_soe_fit(alpha, M, tol, 512, ctypes.byref(K), rho.ctypes.data, w.ctypes.data,
                                        poly.ctypes.data, ctypes.byref(err))
    return rc, K.value, rho[:K.value], w[:K.value], poly, err.value


def _c_exact(alpha, m):
    import mpmath as mp
    mp.mp.dps = 40
    al = mp.mpf(alpha)
    sg = 1 - al / 2
    a = lambda l: (l + sg) ** (1 - al) - (l - 1 + sg) ** (1 - al)  # noqa: E731
    b = lambda l: ((l + sg) ** (2 - al) - (l - 1 + sg) ** (2 - al)) / (2 - al) - ((l + sg) ** (1 - al)  # noqa: E731
                                                                                 + (l - 1 + sg) ** (1 - al)) / 2
    return float(a(m) + b(m + 1) - b(m))


@pytest.mark.parametrize("alpha", [0.1, 0.5, 0.7, 0.95])
@pytest.mark.parametrize("M,tol", [(64, 1e-12), (512, 1e-12), (4096, 1e-12), (512, 1e-8), (65536, 1e-6)])
def test_fit_meets_its_tolerance(alpha, M, tol):
    rc, K, rho, w, poly, err = _fit(alpha, M, tol)
    assert rc == 0 and err <= tol and 0 < K <= 128, (rc, K, err)
    assert np.all((rho > 0) & (rho < 1))
    ms = sorted({2, 3, 7, 31, M // 3, M // 2, M - 3, M - 2})
    for m in ms:
        approx = poly[0] + m * (poly[1] + m * (poly[2] + m * poly[3])) + float(np.sum(w * rho ** m))
        ce = _c_exact(alpha, m)
        assert abs(approx - ce) <= 1.01 * tol * abs(ce) + 1e-300, (m, approx, ce)


def test_fit_weights_match_lemma_1_in_double():
    """At moderate m the closed form of Lemma 1 is accurate in FP64, and the
    oracle's l21s_c (written from it) agrees with the fit to its tolerance."""
    rc, K, rho, w, poly, err = _fit(0.6, 200, 1e-12)
    c = O.l21s_c(0.6, 200)
    for m in range(2, 60):
        approx = poly[0] + m * (poly[1] + m * (poly[2] + m * poly[3])) + float(np.sum(w * rho ** m))
        assert abs(approx - c[m]) <= 2e-12 * abs(c[m]), m


def test_fit_rejects_bad_arguments():
    from paper_1603_00279_amd import _native as N
    K = ctypes.c_int32()
    err = ctypes.c_double()
    L = N.lib()
    assert L.tsfcde_history_soe_fit(0.0, 64, 1e-8, 0, ctypes.byref(K), None, None, None, ctypes.byref(err)) == -1
    assert L.tsfcde_history_soe_fit(0.5, 64, 0.0, 0, ctypes.byref(K), None, None, None, ctypes.byref(err)) == -1
    assert L.tsfcde_history_soe_fit(0.5, 64, 1e-30, 0, ctypes.byref(K), None, None, None, ctypes.byref(err)) == -8


def test_history_perturbation_bound_definition():
    """The bound is kappa tol sum c_m |delta|: scaling the weights' error
    changes the exact history by exactly that much at most, checked with the
    extreme perturbation (every weight moved by +tol relative)."""
    prob = W.config_large(n=9, M=12, alpha=0.6, beta=1.7)
    rng = np.random.default_rng(3)
    U = rng.standard_normal((prob.M + 1, prob.n))
    j = 9
    tol = 1e-3
    c = O.l21s_c(prob.alpha, j)
    kap = O.l21s_kappa(prob.alpha, O.time_step(prob))
    exact = O.history_term(prob, U, j)
    moved = exact.copy()
    for m in range(2, j):
        s = j - m
        moved += kap * tol * c[m] * np.sign(U[s + 1] - U[s]) * (U[s + 1] - U[s])
    bound = O.history_perturbation_bound(prob, U, j, tol)
    assert np.allclose(np.abs(moved - exact), bound, rtol=1e-12, atol=0)
