"""GPU parity of the two-dimensional solver (include/tsfcde2d.h) against the
2D oracle: the operators A, B and P^{-1} on random arrays, whole marches
against the dense direct solves, sampled points at 1024^2 and 2048^2, exchange of
the axes, the f callback and the zero problem."""
import numpy as np
import pytest
import torch

import oracle.ids2d_oracle as O2
import workloads as W
from gpu_util import banner, host, need_gpu, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1603_00279_amd as P
    P.lib()


def solver(prob, **kw):
    import paper_1603_00279_amd as P
    return P.TimeLevelSolver2D.from_problem(prob, **kw)


def box_solution(theta, a, b):
    """theta(t) (x-a)^2 (b-x)^2: the manufactured profile on [a, b] (double
    roots at both ends, as the closed-form fractional derivatives need)."""
    L = b - a
    return W.ManufacturedSolution(theta, np.array([0.0, 0.0, L * L, -2.0 * L, 1.0]), a, b)


def sources(s, prob):
    x, y = s.nodes()
    return W.device_sources_2d(prob, x, y, s.level_times(), torch.device("cuda"))


@pytest.mark.parametrize("nx,ny", [(16, 16), (32, 64), (128, 32), (256, 256), (2048, 16), (16, 2048), (512, 64)])
def test_operators_match_oracle(nx, ny):
    import paper_1603_00279_amd as P
    banner(f"2d operators {nx}x{ny}")
    prob = W.problem_2d(nx, ny, 6, beta_x=1.8, beta_y=1.3)
    rng = np.random.default_rng(nx + 7 * ny)
    X = rng.standard_normal((nx, ny))
    with solver(prob) as s:
        for j in (0, 5):
            S = O2.anorm2(prob, j) * np.max(np.abs(X))
            for op, which in ((P.TSFCDE_OP_A, "A"), (P.TSFCDE_OP_B, "B")):
                got = host(s.apply(op, j, torch.as_tensor(X, device="cuda")))
                d = np.max(np.abs(got - O2.product2(prob, j, X, which)))
                print(f"[2d {nx}x{ny}] j={j} {which}: max|diff|/S = {d / S:.2e}", flush=True)
                assert d <= 1e-13 * S, (j, which, d / S)
            Y = host(s.apply(P.TSFCDE_OP_PINV, j, torch.as_tensor(X, device="cuda")))
            eig = O2.bccb_eigenvalues(prob, j)
            back = np.fft.ifft2(np.fft.fft2(Y) * eig).real  # P Y by the oracle's eigenvalues
            SY = np.max(np.abs(eig)) * np.max(np.abs(Y))
            d = np.max(np.abs(back - X))
            print(f"[2d {nx}x{ny}] j={j} P^-1: max|P y - x| / S = {d / SY:.2e}", flush=True)
            assert d <= 1e-13 * SY, (j, d / SY)


@pytest.mark.parametrize("nx,ny,M", [(16, 16, 8), (32, 16, 5), (16, 64, 4)])
def test_march_matches_dense_oracle(nx, ny, M):
    """Every level against the oracle's dense direct solves (its own sampling
    of f and its own history sum); the levels are accepted."""
    banner(f"2d march {nx}x{ny} M={M}")
    prob = W.problem_2d(nx, ny, M, alpha=0.7, beta_x=1.8, beta_y=1.5)
    with solver(prob, rtol=1e-12) as s:
        code, stats = s.solve(sources(s, prob))
        U = host(s.history())
    assert code == 0, stats
    Uref = O2.march2(prob)
    for j in range(1, M + 1):
        e = relerr(U[j], Uref[j])
        ee = np.max(np.abs(U[j] - Uref[j])) / np.max(np.abs(Uref[j]))
        assert e < 1e-10 and ee < 1e-10, (j, e, ee)
    print(f"[2d march {nx}x{ny}] worst rel err {max(relerr(U[j], Uref[j]) for j in range(1, M + 1)):.2e}, "
          f"iterations {[st['iters'] for st in stats]}", flush=True)
    for st in stats:
        assert st["relres_true"] <= 1e-12 or 0.0 <= st["backward_err"] <= 1e-13, st


def test_axes_exchanged_give_the_transpose():
    banner("2d axis exchange")
    prob = W.problem_2d(64, 32, 3, beta_x=1.3, beta_y=1.9)
    with solver(prob, rtol=1e-13) as s:
        s.solve(sources(s, prob))
        U = host(s.history())
    ps = prob.swapped()
    with solver(ps, rtol=1e-13) as s:
        s.solve(sources(s, ps))
        Us = host(s.history())
    assert Us.shape == (4, 32, 64)
    assert np.max(np.abs(Us - np.transpose(U, (0, 2, 1)))) <= 1e-10 * np.max(np.abs(U))


def test_callback_source_and_zero_problem():
    banner("2d callback and zero problem")
    prob = W.problem_2d(32, 32, 3)
    with solver(prob, rtol=1e-12) as s:
        s.solve(sources(s, prob))
        U1 = host(s.history())
    with solver(prob, rtol=1e-12, f=lambda x, y, t: float(prob.f(np.array([x]), np.array([y]), t)[0, 0])) as s:
        s.solve(None)
        U2 = host(s.history())
    assert relerr(U2, U1) < 1e-12
    z = W.problem_2d(16, 32, 3)
    with solver(z, with_phi=False) as s:
        code, stats = s.solve(torch.zeros(3, 16, 32, dtype=torch.float64, device="cuda"))
        U = host(s.history())
    assert code == 0 and np.all(U == 0.0) and all(st["iters"] == 0 for st in stats)


@pytest.mark.parametrize("n", [1024, 2048])
def test_large_sampled_points(n):
    """n x n (2^20 and 2^22 unknowns; 2048 points per axis runs the 4096-point
    Toeplitz transforms), two levels: acceptance and the oracle's point
    residuals g - A u^{j+1} (its own sampling of f) against the row scale
    |A| max|u|."""
    banner(f"2d {n}x{n}")
    prob = W.problem_2d(n, n, 8)
    rng = np.random.default_rng(5)
    pts = [(0, 0), (n - 1, n - 1), (0, n - 1), (n - 1, 0), (n // 2 - 1, n // 2)]
    pts += [tuple(v) for v in rng.integers(0, n, (11, 2))]
    with solver(prob) as s:
        F = sources(s, prob)
        stats = [s.step(F[j]) for j in range(2)]
        U = host(s.history()[:3])
    for j in range(2):
        st = stats[j]
        print(f"[2d {n}x{n}] j={j} iters {st['iters']} relres_true {st['relres_true']:.2e} "
              f"backward_err {st['backward_err']:.2e}", flush=True)
        assert st["code"] == 0 and st["iters"] > 0, st
        assert st["relres_true"] <= 1e-10 or 0.0 <= st["backward_err"] <= 1e-13, st
        f = O2.source_level(prob, j)
        r = O2.rhs2_points(prob, U, j, f, pts) - O2.apply_A2_points(prob, j, U[j + 1], pts, "A")
        S = O2.anorm2(prob, j) * np.max(np.abs(U[j + 1]))
        assert np.max(np.abs(r)) <= 1e-12 * S, (j, np.max(np.abs(r)) / S)


@pytest.mark.parametrize("warm", ["prev", "extrap"])
def test_warm_started_march_matches_dense_oracle(warm):
    """The previous-level and extrapolated initial guesses: every level against
    the oracle's dense direct solves (the converged level does not depend on
    the guess); the extrapolation takes fewer CGS iterations in total than the
    zero guess."""
    import paper_1603_00279_amd as P
    ws = P.TSFCDE_WS_PREV if warm == "prev" else P.TSFCDE_WS_EXTRAP
    banner(f"2d warm march {warm}")
    prob = W.problem_2d(32, 16, 8, alpha=0.7, beta_x=1.8, beta_y=1.5)
    with solver(prob, rtol=1e-12) as s:
        code0, st0 = s.solve(sources(s, prob))
    with solver(prob, rtol=1e-12, warm_start=ws) as s:
        code, stats = s.solve(sources(s, prob))
        U = host(s.history())
    assert code == 0 and code0 == 0, stats
    Uref = O2.march2(prob)
    worst = max(np.max(np.abs(U[j] - Uref[j])) / np.max(np.abs(Uref[j])) for j in range(1, prob.M + 1))
    its, its0 = [st["iters"] for st in stats], [st["iters"] for st in st0]
    print(f"[2d warm {warm}] worst rel err {worst:.2e}, iterations {its} (zero guess {its0}), "
          f"guesses {[st['guess'] for st in stats]}", flush=True)
    assert worst < 1e-10
    # the previous level saves little with tau = 1/8; the extrapolation must save iterations
    assert sum(its) < sum(its0) if warm == "extrap" else sum(its) <= sum(its0) + prob.M
    want = [ws if warm == "prev" else (P.TSFCDE_WS_EXTRAP if j >= 2 else P.TSFCDE_WS_PREV if j == 1
                                         else P.TSFCDE_WS_ZERO) for j in range(prob.M)]
    assert [st["guess"] for st in stats] == want


def test_edge_orders_and_box():
    """alpha = 1 (Crank-Nicolson in time), beta_x = 2 and beta_y near 1, a box
    other than the unit square and T != 1: every level against the dense
    oracle (both take the same problem statement and sample it themselves)."""
    import dataclasses
    banner("2d edge orders and box")
    base = W.problem_2d(16, 32, 4, alpha=1.0, beta_x=2.0, beta_y=1.02)
    prob = dataclasses.replace(base, a=-1.0, b=2.0, c=0.5, d=1.5, T=0.5,
                               sol_x=box_solution(base.sol_x.theta_terms, -1.0, 2.0),
                               sol_y=box_solution([(1.0, 0.0)], 0.5, 1.5))
    with solver(prob, rtol=1e-13) as s:
        code, stats = s.solve(sources(s, prob))
        U = host(s.history())
    assert code == 0, stats
    Uref = O2.march2(prob)
    worst = max(np.max(np.abs(U[j] - Uref[j])) / np.max(np.abs(Uref[j])) for j in range(1, prob.M + 1))
    print(f"[2d edge] worst rel err {worst:.2e}, iterations {[st['iters'] for st in stats]}", flush=True)
    assert worst < 1e-10


def test_determinism_resume_and_errors():
    """Two runs are bitwise equal (fixed-order reductions); a plan resumed from
    level 3 by set_state continues bitwise as the uninterrupted march; a tiny
    maxit gives TSFCDE_ENOCONV; bad calls are refused without side effects."""
    import paper_1603_00279_amd as P
    banner("2d determinism, resume, errors")
    prob = W.problem_2d(64, 32, 6)
    runs = []
    for _ in range(2):
        with solver(prob) as s:
            F = sources(s, prob)
            s.solve(F)
            runs.append(host(s.history()))
    assert np.array_equal(runs[0], runs[1])
    with solver(prob) as s:
        s.set_state(3, torch.as_tensor(runs[0][:4], device="cuda"))
        code, _ = s.solve(F)
        assert code == 0
        assert np.array_equal(host(s.history()), runs[0])
        assert s.step(F[0], raise_on_error=False)["code"] == P.TSFCDE_EDONE
    with solver(prob, maxit=3) as s:
        st = s.step(F[0], raise_on_error=False)
        assert st["code"] == P.TSFCDE_ENOCONV and st["iters"] == 3, st
        x = torch.zeros(64 * 32, dtype=torch.float64, device="cuda")
        L = P.lib()
        assert L.tsfcde2d_apply(s._plan, P.TSFCDE_OP_A, 0, x.data_ptr(), x.data_ptr()) == P.TSFCDE_EINVAL
        assert L.tsfcde2d_apply(s._plan, 7, 0, x.data_ptr(), x.data_ptr() + 8) == P.TSFCDE_EINVAL
        assert L.tsfcde2d_apply(s._plan, P.TSFCDE_OP_A, prob.M, x.data_ptr(), x.data_ptr() + 8) == P.TSFCDE_EINVAL
        assert L.tsfcde2d_set_state(s._plan, prob.M, x.data_ptr()) == P.TSFCDE_EINVAL
        assert L.tsfcde2d_solve(s._plan, x.data_ptr(), 5, None, None) == P.TSFCDE_EINVAL
        assert s.level == 1


def test_history_blocks_and_mid_block_resume():
    """A march of 20 levels (history sums in blocks of 8: levels 1-8, 9-16,
    17-20) against the dense oracle; a plan resumed at level 13, inside the
    second block, continues bitwise as the uninterrupted march."""
    banner("2d history blocks")
    prob = W.problem_2d(16, 16, 20, alpha=0.3, beta_x=1.6, beta_y=1.9)
    with solver(prob, rtol=1e-13) as s:
        F = sources(s, prob)
        code, stats = s.solve(F)
        U = host(s.history())
    assert code == 0, stats
    Uref = O2.march2(prob)
    worst = max(np.max(np.abs(U[j] - Uref[j])) / np.max(np.abs(Uref[j])) for j in range(1, prob.M + 1))
    print(f"[2d history blocks] worst rel err {worst:.2e}", flush=True)
    assert worst < 1e-10
    with solver(prob, rtol=1e-13) as s:
        s.set_state(13, torch.as_tensor(U[:14], device="cuda"))
        code, _ = s.solve(F)
        assert code == 0 and np.array_equal(host(s.history()), U)


def test_level_symbols_follow_the_level():
    """The axis symbols are tabulated once per level: A and P^{-1} applied at
    levels 5, 0, 5, 3 in turn match the oracle at each, and a march run after
    an apply at another level is bitwise the march of a fresh plan."""
    import paper_1603_00279_amd as P
    banner("2d level symbol tables")
    prob = W.problem_2d(32, 64, 6, beta_x=1.6, beta_y=1.3)
    X = np.random.default_rng(21).standard_normal((32, 64))
    with solver(prob, rtol=1e-12) as s:
        F = sources(s, prob)
        for j in (5, 0, 5, 3):
            S = O2.anorm2(prob, j) * np.max(np.abs(X))
            got = host(s.apply(P.TSFCDE_OP_A, j, torch.as_tensor(X, device="cuda")))
            assert np.max(np.abs(got - O2.product2(prob, j, X, "A"))) <= 1e-13 * S, j
            Y = host(s.apply(P.TSFCDE_OP_PINV, j, torch.as_tensor(X, device="cuda")))
            eig = O2.bccb_eigenvalues(prob, j)
            back = np.fft.ifft2(np.fft.fft2(Y) * eig).real
            assert np.max(np.abs(back - X)) <= 1e-13 * np.max(np.abs(eig)) * np.max(np.abs(Y)), j
        code, _ = s.solve(F)
        U1 = host(s.history())
    assert code == 0
    with solver(prob, rtol=1e-12) as s:
        code, _ = s.solve(F)
        assert code == 0 and np.array_equal(host(s.history()), U1)
