"""GPU parity of the fast history (tsfcde_problem.history_tol > 0: the
L2-1sigma weights of Lemma 1 as a fitted sum of exponentials plus a cubic,
advanced by recursions) against the oracle's exact history.  The tolerance
model: each level's history term may move by at most
kappa tol sum_m c_m |u^{j-m+1} - u^{j-m}| (elementwise), and the level's
solution by at most that divided by eta_j (|A^-1|_2 <= 1/eta_j, the
coercivity pin), accumulated over the levels.  With tol = 1e-12 the march
must meet the method's 1e-10 bar."""
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


@pytest.mark.parametrize("n,M,alpha,beta", [(64, 64, 0.5, 1.5), (256, 300, 0.3, 1.7), (1000, 40, 0.8, 1.4)])
def test_fast_history_march_matches_exact_oracle(n, M, alpha, beta):
    import paper_1603_00279_amd as P
    banner(f"fast history n={n} M={M}")
    prob = W.config_large(n=n, M=M, alpha=alpha, beta=beta)
    Uref = O.march(prob)
    with P.TimeLevelSolver.from_problem(prob, rtol=1e-13, history_tol=1e-12) as s:
        code, stats = s.solve(sources(s, prob))
        U = host(s.history())
    assert code == 0, stats
    worst = 0.0
    for j in range(1, M + 1):
        e_norm = relerr(U[j], Uref[j])
        e_elem = float(np.max(np.abs(U[j] - Uref[j])) / np.max(np.abs(Uref[j])))
        worst = max(worst, e_norm, e_elem)
        assert e_norm < 1e-10 and e_elem < 1e-10, (j, e_norm, e_elem)
    print(f"[fast history n={n} M={M}] worst per-level error vs the exact oracle {worst:.2e}", flush=True)


def test_loose_fast_history_within_its_tolerance_model():
    """tol = 1e-6: the march moves away from the exact one (the fit is really
    in use), and by no more than the accumulated model bound (with a factor
    4 for the propagation through B and for rounding)."""
    import paper_1603_00279_amd as P
    banner("fast history tol 1e-6")
    prob = W.config_large(n=256, M=200, alpha=0.4, beta=1.6)
    tol = 1e-6
    runs = {}
    for ht in (0.0, tol):
        with P.TimeLevelSolver.from_problem(prob, rtol=1e-13, history_tol=ht) as s:
            code, stats = s.solve(sources(s, prob))
            assert code == 0, stats
            runs[ht] = host(s.history())
    Ue, Uf = runs[0.0], runs[tol]
    acc = 0.0
    moved = 0.0
    for j in range(prob.M):
        eta = O.level_scalars(prob, j)[0]
        acc += float(np.linalg.norm(O.history_perturbation_bound(prob, Ue, j, tol))) / eta
        d = float(np.linalg.norm(Uf[j + 1] - Ue[j + 1]))
        moved = max(moved, d)
        assert d <= 4.0 * acc + 1e-13 * np.linalg.norm(Ue[j + 1]), (j + 1, d, acc)
    print(f"[fast history tol=1e-6] largest level difference {moved:.2e}, final model bound {acc:.2e}", flush=True)
    assert moved > 0.0


def test_fast_history_resume_and_rhs_out_of_order():
    """A resumed march rebuilds the recursions from the stored levels and
    continues bit for bit; right-hand sides asked out of order match the
    oracle's exact ones within the model."""
    import paper_1603_00279_amd as P
    banner("fast history resume")
    prob = W.config_large(n=128, M=30, alpha=0.6, beta=1.8)
    with P.TimeLevelSolver.from_problem(prob, rtol=1e-13, history_tol=1e-12) as s:
        F = sources(s, prob)
        s.solve(F)
        U1 = host(s.history())
        Fh = host(F)
        for j in (25, 7, 18, 18, 2):
            g = host(s.rhs(j, F[j]))
            ref = O.rhs(prob, U1, j, Fh[j])
            slack = float(np.linalg.norm(O.history_perturbation_bound(prob, U1, j, 1e-12)))
            assert np.linalg.norm(g - ref) <= 1e-12 * np.linalg.norm(ref) + 2 * slack, j
    with P.TimeLevelSolver.from_problem(prob, rtol=1e-13, history_tol=1e-12) as s:
        s.set_state(12, t64(U1[:13]))
        s.solve(F)
        U2 = host(s.history())
    assert np.array_equal(U1, U2)
