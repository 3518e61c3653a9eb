"""GPU parity of the other Krylov method and the other circulant
preconditioner (tsfcde_problem.krylov = TSFCDE_KRYLOV_BICGSTAB,
tsfcde_problem.preconditioner = TSFCDE_PREC_TCHAN) against the oracle: the
T. Chan preconditioner solve against its dense matrix (backward error), whole
marches against the dense-LU march (1e-10 per level, or 8 eps cond_1(A)
where larger, normwise and elementwise), the headline size on sampled rows,
and the batch against single plans."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import banner, batch_sources, host, need_gpu, relerr, row_scale, sample_rows, sources, t64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1603_00279_amd as P
    P.lib()


@pytest.mark.parametrize("n", [64, 100, 1000, 1024])
def test_tchan_preconditioner_solve(n):
    import paper_1603_00279_amd as P
    banner(f"tchan Pinv n={n}")
    prob = W.config_large(n=n, M=8, alpha=0.6, beta=1.7)
    x = np.random.default_rng(n + 3).standard_normal(n)
    with P.TimeLevelSolver.from_problem(prob, preconditioner=P.TSFCDE_PREC_TCHAN) as s:
        for j in (0, 6):
            y = host(s.apply(P.TSFCDE_OP_PINV, j, t64(x)))
            Pm = O.preconditioner_matrix(prob, j, "tchan")
            berr = np.linalg.norm(Pm @ y - x) / (np.linalg.norm(Pm, 2) * np.linalg.norm(y))
            assert berr < 64 * 2.2e-16, (j, berr)


CASES = [("bicgstab", "strang"), ("bicgstab", "tchan"), ("cgs", "tchan")]


@pytest.mark.parametrize("krylov,prec", CASES)
@pytest.mark.parametrize("n,M", [(256, 12), (1000, 8), (64, 16)])
def test_march_parity(krylov, prec, n, M):
    import paper_1603_00279_amd as P
    banner(f"{krylov}+{prec} march n={n}")
    prob = W.config_large(n=n, M=M, alpha=0.55, beta=1.75)
    Uref = O.march(prob)
    kw = dict(krylov=P.TSFCDE_KRYLOV_BICGSTAB if krylov == "bicgstab" else P.TSFCDE_KRYLOV_CGS,
              preconditioner=P.TSFCDE_PREC_TCHAN if prec == "tchan" else P.TSFCDE_PREC_STRANG)
    with P.TimeLevelSolver.from_problem(prob, rtol=1e-13, **kw) as s:
        code, stats = s.solve(sources(s, prob))
        U = host(s.history())
    assert code == 0, stats
    want = P.TSFCDE_METHOD_PBICGSTAB if krylov == "bicgstab" else P.TSFCDE_METHOD_PCGS
    assert all(st["method"] == want for st in stats)
    worst = 0.0
    for j in range(1, M + 1):
        bound = max(1e-10, 8 * 2.2e-16 * np.linalg.cond(O.level_A(prob, j - 1), 1))
        e_norm = relerr(U[j], Uref[j])
        e_elem = float(np.max(np.abs(U[j] - Uref[j])) / np.max(np.abs(Uref[j])))
        worst = max(worst, e_norm, e_elem)
        assert e_norm < bound and e_elem < bound, (j, e_norm, e_elem, bound)
    its = [st["iters"] for st in stats]
    print(f"[{krylov}+{prec} n={n}] worst {worst:.2e}, iterations {min(its)}..{max(its)}", flush=True)
    assert max(its) <= 40


def test_bicgstab_headline_size():
    """Three levels of the n = 2^20 march by BiCGSTAB: accepted by the
    library's test, and the oracle's rows of g - A u (its own sampling) are
    rounding-sized against the row scale."""
    import paper_1603_00279_amd as P
    banner("bicgstab n=2^20")
    prob = W.config_large(n=1 << 20, M=512)
    rows = sample_rows(prob.n, 41)
    F = [O.source_level(prob, j) for j in range(3)]
    with P.TimeLevelSolver.from_problem(prob, rtol=1e-10, krylov=P.TSFCDE_KRYLOV_BICGSTAB) as s:
        Fd = sources(s, prob, 3)
        stats = [s.step(Fd[j]) for j in range(3)]
        U = host(s.history()[:4])
    for j in range(3):
        st = stats[j]
        assert st["code"] == 0 and st["method"] == P.TSFCDE_METHOD_PBICGSTAB and 0 <= st["backward_err"] <= 1e-13, st
        r = O.rhs_rows(prob, U, j, F[j], rows) - O.apply_A_rows(prob, j, U[j + 1], rows, "A")
        S = row_scale(prob, j, U[j + 1])
        assert np.abs(r).max() <= 1e-12 * S, (j, np.abs(r).max() / S)


def test_batch_tchan_equals_single_plans():
    """The batched form with T. Chan's preconditioner gives each instance's
    single-plan march bit for bit (n not a power of two: the same kernel
    path), and the oracle's to 1e-10."""
    import paper_1603_00279_amd as P
    banner("batch tchan")
    probs = W.batched_instances(count=5, M=5, nmin=50, nmax=1500, seed=17)
    with P.BatchSolver(probs, rtol=1e-13, preconditioner=P.TSFCDE_PREC_TCHAN, flags=P.TSFCDE_FLAG_NO_TUNE) as bs:
        Fs = batch_sources(bs, probs)
        for j in range(probs[0].M):
            code, stats = bs.step([F[j] for F in Fs])
            assert code == 0, stats
        Ub = [host(bs.history(i)) for i in range(len(probs))]
    for i, prob in enumerate(probs):
        Uref = O.march(prob)
        for j in range(1, prob.M + 1):
            assert relerr(Ub[i][j], Uref[j]) < 1e-10, (i, j)
        if prob.n & (prob.n - 1):
            with P.TimeLevelSolver.from_problem(prob, rtol=1e-13, preconditioner=P.TSFCDE_PREC_TCHAN) as s:
                s.solve(Fs[i])
                assert np.array_equal(host(s.history()), Ub[i]), i
