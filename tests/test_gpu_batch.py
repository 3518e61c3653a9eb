"""GPU parity of the batched form: grouped launches over instances of uneven
size and parameters give, instance by instance, the single-instance results
(bitwise where both take the same kernel path) and the oracle's levels."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_util import banner, batch_sources, host, need_gpu, relerr, t64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1603_00279_amd as P
    P.lib()


def _instances(count, M, nmin, nmax, seed):
    return W.batched_instances(count=count, M=M, nmin=nmin, nmax=nmax, seed=seed)


@pytest.mark.parametrize("warm", [0, 2])
def test_batch_matches_single_and_oracle(warm):
    import paper_1603_00279_amd as P
    banner(f"batch vs single, warm={warm}")
    probs = _instances(12, 6, 40, 3000, seed=11)
    assert len({p.n for p in probs}) > 6
    # the default values per lane (the single plans' own) for the bitwise check
    with P.BatchSolver(probs, rtol=1e-13, warm_start=warm, flags=P.TSFCDE_FLAG_NO_TUNE) as bs:
        Fs = batch_sources(bs, probs)
        for j in range(probs[0].M):
            code, stats = bs.step([F[j] for F in Fs])
            assert code == 0, stats
        Ub = [host(bs.history(i)) for i in range(len(probs))]
    for i, prob in enumerate(probs):
        Uref = O.march(prob)
        for j in range(1, prob.M + 1):
            assert relerr(Ub[i][j], Uref[j]) < 1e-10, (i, prob.n, j, relerr(Ub[i][j], Uref[j]))
        # the single-instance plan runs the same kernel bodies when n is not a power of two
        if prob.n & (prob.n - 1):
            with P.TimeLevelSolver.from_problem(prob, rtol=1e-13, warm_start=warm) as s:
                s.solve(Fs[i])
                Us = host(s.history())
            assert np.array_equal(Us, Ub[i]), (i, prob.n)


def test_batch_uneven_convergence_and_zero_source():
    """Instances converge at different iteration counts; an instance with f = 0
    and u0 = 0 stays exactly zero while the others advance."""
    import paper_1603_00279_amd as P
    banner("batch uneven")
    probs = _instances(6, 4, 100, 2000, seed=5)
    with P.BatchSolver(probs, rtol=1e-12) as bs:
        Fs = batch_sources(bs, probs)
        bs.reset([torch.zeros(p.n, dtype=torch.float64, device="cuda") for p in probs])
        its = []
        for j in range(probs[0].M):
            fs = [None] + [F[j] for F in Fs[1:]]
            code, stats = bs.step(fs)
            its.append([st["iters"] for st in stats])
        U0 = host(bs.history(0))
    assert np.all(U0 == 0.0)
    assert all(row[0] == 0 for row in its)
    assert len({it for row in its for it in row[1:]}) > 1


def test_batch_crosses_history_blocks():
    """19 levels: the history sums of the batch run in blocks of 8 levels
    (sweeps at levels 1, 9 and 17, catch-ups in between); every level
    matches the oracle's march."""
    import paper_1603_00279_amd as P
    banner("batch, 19 levels")
    probs = _instances(4, 19, 40, 300, seed=23)
    with P.BatchSolver(probs, rtol=1e-13) as bs:
        Fs = batch_sources(bs, probs)
        for j in range(probs[0].M):
            code, stats = bs.step([F[j] for F in Fs])
            assert code == 0, stats
        Ub = [host(bs.history(i)) for i in range(len(probs))]
    for i, prob in enumerate(probs):
        Uref = O.march(prob)
        for j in range(1, prob.M + 1):
            assert relerr(Ub[i][j], Uref[j]) < 1e-10, (i, prob.n, j, relerr(Ub[i][j], Uref[j]))


def test_batch_folded_finishing_is_bitwise_unfolded():
    """The batch with the finishing steps folded into later passes gives the
    same levels bit for bit as with separate finishing kernels
    (TSFCDE_FLAG_NO_FOLD), over chunks long enough to use every variant."""
    import paper_1603_00279_amd as P
    banner("batch fold vs no fold")
    probs = _instances(6, 10, 60, 2500, seed=29)
    runs = []
    Fs = None
    for flags in (0, P.TSFCDE_FLAG_NO_FOLD):
        its = []
        with P.BatchSolver(probs, rtol=1e-12, flags=flags) as bs:
            Fs = batch_sources(bs, probs) if Fs is None else Fs
            for j in range(probs[0].M):
                code, stats = bs.step([F[j] for F in Fs])
                assert code == 0, stats
                its.append([st["iters"] for st in stats])
            runs.append(([host(bs.history(i)) for i in range(len(probs))], its))
    assert runs[0][1] == runs[1][1]
    for a, b in zip(runs[0][0], runs[1][0]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("warm", [0, 2])
def test_batch_graph_replay_is_bitwise_direct(warm):
    """CGS chunks replayed from captured HIP graphs (TSFCDE_FLAG_GRAPHS) give
    the same levels and iteration counts bit for bit as direct launches.
    Every level re-stages its descriptors, runs history and right-hand-side
    kernels eagerly and polls the host between replays, and each chunk
    length is captured once and replayed at many levels."""
    import paper_1603_00279_amd as P
    banner(f"batch graphs warm={warm}")
    probs = _instances(7, 12, 60, 5000, seed=31)
    runs = []
    Fs = None
    for flags in (0, P.TSFCDE_FLAG_GRAPHS):
        its = []
        with P.BatchSolver(probs, rtol=1e-12, flags=flags, warm_start=warm) as bs:
            Fs = batch_sources(bs, probs) if Fs is None else Fs
            for j in range(probs[0].M):
                code, stats = bs.step([F[j] for F in Fs])
                assert code == 0, stats
                its.append([st["iters"] for st in stats])
            runs.append(([host(bs.history(i)) for i in range(len(probs))], its))
    assert runs[0][1] == runs[1][1]
    for a, b in zip(runs[0][0], runs[1][0]):
        assert np.array_equal(a, b)


def test_autotuned_batch_matches_oracle():
    """The autotuner picks 4 or 8 values per lane for each group's middle
    passes (TSFCDE_FLAG_NO_TUNE keeps 8 everywhere); the tuned batch matches
    the oracle to 1e-10 per level and the untuned one to FFT rounding."""
    import paper_1603_00279_amd as P
    banner("batch autotuner")
    probs = _instances(10, 5, 500, 6000, seed=41)
    runs = {}
    for flags in (0, P.TSFCDE_FLAG_NO_TUNE):
        with P.BatchSolver(probs, rtol=1e-13, flags=flags) as bs:
            groups = bs.groups()
            Fs = batch_sources(bs, probs)
            for j in range(probs[0].M):
                code, stats = bs.step([F[j] for F in Fs])
                assert code == 0, stats
            runs[flags] = ([host(bs.history(i)) for i in range(len(probs))], groups)
    print(f"[autotuner] groups (L, members, values per lane): {runs[0][1]}", flush=True)
    assert sum(m for _, m, _ in runs[0][1]) == len(probs)
    assert all(e in (4, 8) for _, _, e in runs[0][1])
    assert all(e == 8 for _, _, e in runs[P.TSFCDE_FLAG_NO_TUNE][1])
    for i, prob in enumerate(probs):
        Uref = O.march(prob)
        for j in range(1, prob.M + 1):
            # 1e-10, or the forward error a backward-stable solve can promise
            bound = max(1e-10, 8 * 2.2e-16 * np.linalg.cond(O.level_A(prob, j - 1), 1))
            assert relerr(runs[0][0][i][j], Uref[j]) < bound, (i, prob.n, j, bound)
            assert relerr(runs[0][0][i][j], runs[P.TSFCDE_FLAG_NO_TUNE][0][i][j]) < bound, (i, j)


def test_batch_large_members_sampled_rows():
    """Members with n in (4096, 2^16], the largest groups of the 512-instance
    workload (embedding lengths up to 2^17): every level is accepted (true
    residual within the tolerance or backward error at most 1e-13), and the
    oracle's rows of g - A u^{j+1} (its own sampling
    of f, its own history sum) are rounding-sized against the row scale
    (a componentwise backward error, as at the headline size)."""
    import paper_1603_00279_amd as P
    from gpu_util import row_scale, sample_rows
    banner("batch large members")
    probs = _instances(5, 3, 5000, 1 << 16, seed=53)
    probs += W.batched_instances(count=1, M=3, nmin=60000, nmax=65536, seed=59)
    with P.BatchSolver(probs, rtol=1e-10) as bs:
        groups = bs.groups()
        Fs = batch_sources(bs, probs)
        all_stats = []
        for j in range(probs[0].M):
            code, stats = bs.step([F[j] for F in Fs])
            assert code == 0, stats
            all_stats.append(stats)
        Ub = [host(bs.history(i)) for i in range(len(probs))]
    print(f"[batch large] n = {[p.n for p in probs]}, groups {groups}", flush=True)
    assert max(L for L, _, _ in groups) >= 1 << 16
    for i, prob in enumerate(probs):
        rows = sample_rows(prob.n, 60 + i, k=16, width=64)
        for j in range(prob.M):
            st = all_stats[j][i]
            assert st["iters"] > 0 and (st["relres_true"] <= 1e-10 or 0.0 <= st["backward_err"] <= 1e-13), (i, j, st)
            f = O.source_level(prob, j)
            r = O.rhs_rows(prob, Ub[i], j, f, rows) - O.apply_A_rows(prob, j, Ub[i][j + 1], rows, "A")
            S = row_scale(prob, j, Ub[i][j + 1])
            assert np.abs(r).max() <= 1e-12 * S, (i, prob.n, j, np.abs(r).max() / S)


@pytest.mark.parametrize("warm", [0, 2])
def test_batch_solve_equals_level_steps(warm):
    """tsfcde_batch_solve (instances advance through the levels on their own)
    gives bitwise the levels and iteration counts of tsfcde_batch_step called
    level by level, with stats instance-major; one instance takes its f from
    the callback."""
    import paper_1603_00279_amd as P
    banner(f"batch solve vs steps, warm={warm}")
    probs = _instances(10, 7, 40, 5000, seed=71)
    flags = P.TSFCDE_FLAG_NO_TUNE
    with P.BatchSolver(probs, rtol=1e-12, warm_start=warm, flags=flags) as bs:
        Fs = batch_sources(bs, probs)
        its_step = []
        for j in range(probs[0].M):
            code, stats = bs.step([F[j] for F in Fs])
            assert code == 0, stats
            its_step.append([st["iters"] for st in stats])
        U1 = [host(bs.history(i)) for i in range(len(probs))]
    with P.BatchSolver(probs, rtol=1e-12, warm_start=warm, flags=flags, callbacks=True) as bs:
        Fs2 = list(batch_sources(bs, probs))
        Fs2[3] = None  # the callback samples f itself
        code, st = bs.solve(Fs2)
        assert code == 0
        U2 = [host(bs.history(i)) for i in range(len(probs))]
        assert int(bs._level()) == probs[0].M
        code, _ = bs.solve(Fs2, raise_on_error=False)
        assert code == P.TSFCDE_EDONE
    assert st.shape == (len(probs), probs[0].M)
    assert np.array_equal(st["iters"].T, np.array(its_step)), (st["iters"].T, its_step)
    assert np.all(st["status"] == 0)
    assert np.all((st["backward_err"] >= 0) & ((st["backward_err"] <= 1e-13) | (st["relres_true"] <= 1e-12)))
    for i in range(len(probs)):
        if i == 3:  # f sampled by the callback on the host: the same values up to rounding
            assert relerr(U2[i], U1[i]) < 1e-10, relerr(U2[i], U1[i])
        else:
            assert np.array_equal(U1[i], U2[i]), (i, probs[i].n)
