"""The library's own sampling, through the C ABI's callbacks: gamma, d_+-
at t_{j+sigma} during tsfcde_plan, phi at the plan's nodes, and f(x_i,
t_{j+sigma}) per level when a step has no device source (problem (1.1),
Lemma 1, Sec. 2.1).  Nothing here hands the library a sampled value: the
oracle samples the same problem by itself, and the two marches must agree
to the method's bar.  Also the acceptance status of a level that cannot
meet the strict true-residual test."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import banner, host, need_gpu, relerr, sources, t64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1603_00279_amd as P
    P.lib()


CASES = {
    "small_n64_M64": lambda: W.config_small(),
    "n1000_M8": lambda: W.config_large(n=1000, M=8, alpha=0.45, beta=1.65),
    "example2_N32": lambda: W.example2(0.9, 1.5, 32),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_march_through_callbacks_matches_oracle(case):
    """Every input through a callback (tsfcde_solve with no device source);
    per level the bar is 1e-10 normwise and elementwise against max|u|."""
    import paper_1603_00279_amd as P
    banner(f"callbacks {case}")
    prob = CASES[case]()
    Uref = O.march(prob)
    with P.TimeLevelSolver.from_problem(prob, callbacks=True, rtol=1e-13) as s:
        code, stats = s.solve(None)
        U = host(s.history())
        t_lib = s.level_times()
        x_lib = s.nodes()
    assert code == 0, stats
    # the plan's instants and nodes are the paper's: t_{j+sigma} = (j + 1 - alpha/2) tau, x_i = a + i h
    assert np.allclose(t_lib, [O.t_sigma(prob, j) for j in range(prob.M)], rtol=1e-15, atol=0)
    assert np.allclose(x_lib, O.nodes(prob), rtol=1e-15, atol=0)
    worst = 0.0
    for j in range(prob.M + 1):
        if np.linalg.norm(Uref[j]) == 0:
            assert np.all(U[j] == 0), j
            continue
        e_norm = relerr(U[j], Uref[j])
        e_elem = float(np.max(np.abs(U[j] - Uref[j])) / np.max(np.abs(Uref[j])))
        worst = max(worst, e_norm, e_elem)
        assert e_norm < 1e-10 and e_elem < 1e-10, (j, e_norm, e_elem)
    print(f"[callbacks {case}] worst per-level error vs oracle {worst:.2e}", flush=True)


def test_callbacks_equal_arrays_bitwise():
    """gamma, d_+- sampled by the plan's callbacks give the same march, bit
    for bit, as the same functions sampled by the caller at the plan's own
    instants and passed as arrays; the f callback gives what the device
    sources of the same instants give, to rounding."""
    import paper_1603_00279_amd as P
    banner("callbacks vs arrays")
    prob = W.config_large(n=256, M=12, alpha=0.6, beta=1.7)
    with P.TimeLevelSolver.from_problem(prob, rtol=1e-13) as s:
        ts = s.level_times()
        F = sources(s, prob)
        s.solve(F)
        U_cb = host(s.history())
    g = np.array([prob.gamma(t) for t in ts])
    dp = np.array([prob.dplus(t) for t in ts])
    dm = np.array([prob.dminus(t) for t in ts])
    with P.TimeLevelSolver(alpha=prob.alpha, beta=prob.beta, n=prob.n, M=prob.M, gamma=g, dplus=dp, dminus=dm,
                           rtol=1e-13) as s:
        s.set_state(0, t64(prob.phi(s.nodes())[None, :]))
        s.solve(F)
        U_arr = host(s.history())
    assert np.array_equal(U_cb, U_arr)
    with P.TimeLevelSolver.from_problem(prob, callbacks=True, rtol=1e-13) as s:
        s.solve(None)
        U_f = host(s.history())
    assert relerr(U_f, U_cb) < 1e-12


def test_strict_residual_level_reports_eaccept():
    """n = 2^14, C1 coefficients, rtol = 1e-14 with TSFCDE_FLAG_STRICT_RESIDUAL:
    the recursive residual converges, but the true residual cannot reach
    1e-14 |g| in FP64 (its floor is about eps |A| |u| / |g|), so after its
    restarts the level ends with TSFCDE_EACCEPT, the iterate and the stats
    set, and the plan at the next level.  Without the flag the same level is
    accepted on its backward error."""
    import paper_1603_00279_amd as P
    banner("strict residual n=2^14")
    prob = W.config_large(n=1 << 14, M=2)
    with P.TimeLevelSolver.from_problem(prob, rtol=1e-14, flags=P.TSFCDE_FLAG_STRICT_RESIDUAL) as s:
        F = sources(s, prob)
        st = s.step(F[0], raise_on_error=False)
        assert s.level == 1
        u1 = host(s.history()[1])
    print(f"[strict] {st}", flush=True)
    assert st["code"] == P.TSFCDE_EACCEPT, st
    assert st["status"] == P.TSFCDE_EACCEPT and st["restarts"] >= 1
    assert st["relres_true"] > 1e-14 and st["backward_err"] >= 0
    assert np.all(np.isfinite(u1)) and np.max(np.abs(u1)) > 0
    with P.TimeLevelSolver.from_problem(prob, rtol=1e-14) as s:
        st2 = s.step(F[0], raise_on_error=False)
    assert st2["code"] == P.TSFCDE_OK and 0 <= st2["backward_err"] <= 1e-13, st2


def test_batch_strict_residual_reports_eaccept():
    """The batch's acceptance test under TSFCDE_FLAG_STRICT_RESIDUAL: members
    whose true residual stays above rtol |g| report TSFCDE_EACCEPT, and the
    batch step returns that code."""
    import paper_1603_00279_amd as P
    banner("batch strict residual")
    probs = W.batched_instances(count=3, M=2, nmin=1 << 13, nmax=1 << 14, seed=7)
    with P.BatchSolver(probs, rtol=1e-15, flags=P.TSFCDE_FLAG_STRICT_RESIDUAL, callbacks=True) as bs:
        code, stats = bs.step(None, raise_on_error=False)
    print(f"[batch strict] code {code}, {[(x['status'], x['restarts'], x['relres_true']) for x in stats]}",
          flush=True)
    assert code == P.TSFCDE_EACCEPT
    assert any(x["status"] == P.TSFCDE_EACCEPT for x in stats)
    for x in stats:
        assert x["status"] in (P.TSFCDE_OK, P.TSFCDE_EACCEPT, P.TSFCDE_ENOCONV), x
        if x["status"] == P.TSFCDE_OK:
            assert x["relres_true"] <= 1e-15
