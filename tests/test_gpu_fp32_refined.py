"""GPU parity of the FP32-refined form (TSFCDE_FP32_REFINED): FP64 iterative
refinement, whose stopping test is the true residual |g - A u| <= rtol |g|,
around an inner CGS that stores its vectors, transform buffers and spectra in
FP32.  Levels outside the rounding-error model's envelope, or whose
refinement stalls, finish with the FP64 CGS; either way the level's answer
meets the FP64 parity bar against the oracle."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import banner, host, need_gpu, relerr, sources, t64

pytestmark = pytest.mark.gpu
EPS = 2.2e-16


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1603_00279_amd as P
    P.lib()


def test_refined_small_config_every_level_fp32():
    """alpha = 0.5, beta = 1.5, n = 64, M = 64: every level refines in FP32
    down to a true residual of 1e-13 and matches the oracle to 1e-10."""
    import paper_1603_00279_amd as P
    banner("fp32 refined n=64")
    prob = W.config_small()
    Uref = O.march(prob)
    with P.TimeLevelSolver.from_problem(prob, rtol=1e-13, precision=P.TSFCDE_FP32_REFINED) as s:
        code, stats = s.solve(sources(s, prob))
        U = host(s.history())
    assert code == 0
    assert all(st["precision_used"] == P.TSFCDE_FP32_REFINED for st in stats)
    assert all(st["relres"] <= 1e-13 and st["relres_true"] == st["relres"] for st in stats)
    assert max(st["outer_iters"] for st in stats) >= 2
    for j in range(1, prob.M + 1):
        assert relerr(U[j], Uref[j]) < 1e-10, j


@pytest.mark.parametrize("n,alpha,beta", [(100, 0.5, 1.5), (256, 0.7, 1.8), (1000, 0.3, 1.2), (1024, 0.5, 1.5)])
def test_refined_matches_oracle(n, alpha, beta):
    """At rtol = 1e-13 larger grids meet the FP64 matvec's own rounding floor
    (about eps |A| / eta) before the true residual gets there: such levels
    must fall back to the FP64 CGS, and every level meets the parity bound."""
    import paper_1603_00279_amd as P
    banner(f"fp32 refined parity n={n}")
    prob = W.config_large(n=n, M=8, alpha=alpha, beta=beta)
    Uref = O.march(prob)
    with P.TimeLevelSolver.from_problem(prob, rtol=1e-13, precision=P.TSFCDE_FP32_REFINED) as s:
        code, stats = s.solve(sources(s, prob))
        U = host(s.history())
    assert code == 0
    used = {st["precision_used"] for st in stats}
    assert used <= {P.TSFCDE_FP32_REFINED, P.TSFCDE_FP32_REFINED_FELL_BACK, P.TSFCDE_FP64}
    for j in range(1, prob.M + 1):
        bound = max(1e-10, 8 * EPS * np.linalg.cond(O.level_A(prob, j - 1), 1))
        assert relerr(U[j], Uref[j]) < bound, (j, relerr(U[j], Uref[j]), bound)


@pytest.mark.parametrize("n", [256, 1000, 1024])
def test_refined_default_tolerance_stays_fp32(n):
    """At the default rtol = 1e-10 the same grids refine in FP32 at every
    level; the forward error is bounded by cond_1(A) times the true relative
    residual plus the FP64 rounding term."""
    import paper_1603_00279_amd as P
    banner(f"fp32 refined rtol 1e-10 n={n}")
    prob = W.config_small(n=n, M=8)
    Uref = O.march(prob)
    with P.TimeLevelSolver.from_problem(prob, rtol=1e-10, precision=P.TSFCDE_FP32_REFINED) as s:
        code, stats = s.solve(sources(s, prob))
        U = host(s.history())
    assert code == 0
    assert all(st["precision_used"] == P.TSFCDE_FP32_REFINED for st in stats), [st["precision_used"] for st in stats]
    for j in range(1, prob.M + 1):
        st = stats[j - 1]
        assert st["relres"] <= 1e-10
        c1 = np.linalg.cond(O.level_A(prob, j - 1), 1)
        bound = 2 * c1 * st["relres"] + 8 * EPS * c1
        assert relerr(U[j], Uref[j]) < bound, (j, relerr(U[j], Uref[j]), bound)


def test_refined_forced_outside_envelope_falls_back():
    """Forced at every level where the model predicts failure (C1 parameters,
    n = 2^14: 2^-24 log2(L) |A|/eta is well above 0.1), the refinement stalls,
    the level finishes with the FP64 CGS, and the answer agrees with the plain
    FP64 path to the rounding level of the operator (|A|/eta ~ 1e6)."""
    import paper_1603_00279_amd as P
    banner("fp32 refined forced n=2^14")
    prob = W.config_large(n=1 << 14, M=3)
    with P.TimeLevelSolver.from_problem(prob, rtol=1e-10) as s:
        F = sources(s, prob)
        s.solve(F)
        U64 = host(s.history())
    with P.TimeLevelSolver.from_problem(prob, rtol=1e-10, precision=P.TSFCDE_FP32_REFINED,
                                        flags=P.TSFCDE_FLAG_FORCE_FP32) as s:
        code, stats = s.solve(F)
        U32 = host(s.history())
    assert code == 0
    assert all(st["precision_used"] in (P.TSFCDE_FP32_REFINED, P.TSFCDE_FP32_REFINED_FELL_BACK) for st in stats)
    for j in range(1, prob.M + 1):
        assert relerr(U32[j], U64[j]) < 1e-6, (j, relerr(U32[j], U64[j]))


def test_refined_policy_keeps_fp64_at_large_kappa():
    """Without the force flag the rounding-error model sends C1-like levels
    at n = 2^14 to the FP64 CGS."""
    import paper_1603_00279_amd as P
    banner("fp32 refined policy n=2^14")
    prob = W.config_large(n=1 << 14, M=2)
    with P.TimeLevelSolver.from_problem(prob, rtol=1e-10, precision=P.TSFCDE_FP32_REFINED) as s:
        code, stats = s.solve(sources(s, prob))
    assert code == 0
    assert all(st["precision_used"] == P.TSFCDE_FP64 for st in stats)


def test_batch_refuses_fp32_members():
    import paper_1603_00279_amd as P
    probs = W.batched_instances(count=2, M=2, nmin=100, nmax=200, seed=1)
    with pytest.raises(P.TsfcdeError):
        P.BatchSolver(probs, precision=P.TSFCDE_FP32_REFINED)
