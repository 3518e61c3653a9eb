"""GPU parity of the three-dimensional solver (include/tsfcde3d.h) against the
3D oracle: the operators A, B and P^{-1} on random arrays, whole marches
against the dense direct solves and (larger grids) the oracle's FFT-route
PCGS, sampled points at 256^3, permutations of the axes, the f callback and
the zero problem."""
import numpy as np
import pytest
import torch

import oracle.ids3d_oracle as O3
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
    return P.TimeLevelSolver3D.from_problem(prob, **kw)


def box_solution(theta, a, b):
    """theta(t) (x-a)^2 (b-x)^2: the manufactured profile on [a, b]."""
    L = b - a
    return W.ManufacturedSolution(theta, np.array([0.0, 0.0, L * L, -2.0 * L, 1.0]), a, b)


def sources(s, prob):
    x, y, z = s.nodes()
    return W.device_sources_3d(prob, x, y, z, s.level_times(), torch.device("cuda"))


@pytest.mark.parametrize("ns", [(16, 16, 16), (16, 32, 64), (64, 16, 32), (128, 64, 128), (2048, 16, 32), (16, 32, 2048),
                                (512, 16, 32), (16, 512, 32), (1024, 16, 16)])
def test_operators_match_oracle(ns):
    import paper_1603_00279_amd as P
    banner(f"3d operators {ns}")
    prob = W.problem_3d(*ns, 6, betas=(1.8, 1.3, 1.55))
    rng = np.random.default_rng(sum(ns))
    X = rng.standard_normal(ns)
    with solver(prob) as s:
        for j in (0, 5):
            S = O3.anorm3(prob, j) * np.max(np.abs(X))
            for op, which in ((P.TSFCDE_OP_A, "A"), (P.TSFCDE_OP_B, "B")):
                got = host(s.apply(op, j, torch.as_tensor(X, device="cuda")))
                d = np.max(np.abs(got - O3.product3(prob, j, X, which)))
                print(f"[3d {ns}] j={j} {which}: max|diff|/S = {d / S:.2e}", flush=True)
                assert d <= 1e-13 * S, (j, which, d / S)
            Y = host(s.apply(P.TSFCDE_OP_PINV, j, torch.as_tensor(X, device="cuda")))
            eig = O3.bccb3_eigenvalues(prob, j)
            back = np.fft.ifftn(np.fft.fftn(Y) * eig).real  # P Y by the oracle's eigenvalues
            SY = np.max(np.abs(eig)) * np.max(np.abs(Y))
            d = np.max(np.abs(back - X))
            print(f"[3d {ns}] j={j} P^-1: max|P y - x| / S = {d / SY:.2e}", flush=True)
            assert d <= 1e-13 * SY, (j, d / SY)


def test_march_matches_dense_oracle():
    """Every level of a 16^3 march against the oracle's dense direct solves
    (its own sampling of f and its own history sum); the levels are accepted."""
    banner("3d march 16^3 dense")
    prob = W.problem_3d(16, 16, 16, 4, alpha=0.7, betas=(1.8, 1.5, 1.25))
    with solver(prob, rtol=1e-12) as s:
        code, stats = s.solve(sources(s, prob))
        U = host(s.history())
    assert code == 0, stats
    Uref = O3.march3(prob)
    for j in range(1, prob.M + 1):
        e = relerr(U[j], Uref[j])
        ee = np.max(np.abs(U[j] - Uref[j])) / np.max(np.abs(Uref[j]))
        assert e < 1e-10 and ee < 1e-10, (j, e, ee)
    print(f"[3d march 16^3] worst rel err {max(relerr(U[j], Uref[j]) for j in range(1, prob.M + 1)):.2e}, "
          f"iterations {[st['iters'] for st in stats]}", flush=True)
    for st in stats:
        assert st["relres_true"] <= 1e-12 or 0.0 <= st["backward_err"] <= 1e-13, st


@pytest.mark.parametrize("ns,M", [((32, 16, 64), 3), ((16, 128, 32), 2), ((512, 16, 16), 2)])
def test_march_matches_fft_oracle(ns, M):
    """Larger grids against the oracle's FFT-route PCGS march (pinned against
    the dense route), both solved to 1e-13."""
    banner(f"3d march {ns} fft oracle")
    prob = W.problem_3d(*ns, M, alpha=0.4, betas=(1.35, 1.9, 1.6))
    with solver(prob, rtol=1e-13) as s:
        code, stats = s.solve(sources(s, prob))
        U = host(s.history())
    assert code == 0, stats
    Uref, its = O3.march_pcgs3(prob, rtol=1e-13)
    worst = max(np.max(np.abs(U[j] - Uref[j])) / np.max(np.abs(Uref[j])) for j in range(1, M + 1))
    print(f"[3d march {ns}] worst rel err {worst:.2e}, iterations {[st['iters'] for st in stats]} "
          f"(oracle {its})", flush=True)
    assert worst < 1e-10


def test_permuted_axes_give_the_transpose():
    banner("3d axis permutation")
    prob = W.problem_3d(64, 16, 32, 3, betas=(1.3, 1.9, 1.6))
    with solver(prob, rtol=1e-13) as s:
        s.solve(sources(s, prob))
        U = host(s.history())
    perm = (2, 0, 1)
    pp = prob.permuted(perm)
    with solver(pp, rtol=1e-13) as s:
        s.solve(sources(s, pp))
        Up = host(s.history())
    ref = np.transpose(U, (0, 3, 1, 2))
    assert Up.shape == ref.shape
    assert np.max(np.abs(Up - ref)) <= 1e-10 * np.max(np.abs(U))


def test_callback_source_and_zero_problem():
    banner("3d callback and zero problem")
    prob = W.problem_3d(16, 32, 16, 3)
    with solver(prob, rtol=1e-12) as s:
        s.solve(sources(s, prob))
        U1 = host(s.history())
    f = lambda x, y, z, t: float(prob.f(np.array([x]), np.array([y]), np.array([z]), t)[0, 0, 0])  # noqa: E731
    with solver(prob, rtol=1e-12, f=f) as s:
        s.solve(None)
        U2 = host(s.history())
    assert relerr(U2, U1) < 1e-12
    z = W.problem_3d(16, 16, 32, 3)
    with solver(z, with_phi=False) as s:
        code, stats = s.solve(torch.zeros(3, 16, 16, 32, dtype=torch.float64, device="cuda"))
        U = host(s.history())
    assert code == 0 and np.all(U == 0.0) and all(st["iters"] == 0 for st in stats)


def test_large_sampled_points():
    """256^3 (2^24 unknowns), two levels: acceptance and the oracle's point
    residuals g - A u^{j+1} (its own sampling of f) against the row scale
    |A| max|u|."""
    banner("3d 256^3")
    n = 256
    prob = W.problem_3d(n, n, n, 8)
    rng = np.random.default_rng(6)
    pts = [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 0), (n - 1, 0, n - 1), (127, 128, 129)]
    pts += [tuple(v) for v in rng.integers(0, n, (11, 3))]
    with solver(prob) as s:
        F = sources(s, prob)
        stats = [s.step(F[j]) for j in range(2)]
        del F
        U = host(s.history()[:3])
    for j in range(2):
        st = stats[j]
        print(f"[3d 256^3] j={j} iters {st['iters']} relres_true {st['relres_true']:.2e} "
              f"backward_err {st['backward_err']:.2e}", flush=True)
        assert st["code"] == 0 and st["iters"] > 0, st
        assert st["relres_true"] <= 1e-10 or 0.0 <= st["backward_err"] <= 1e-13, st
        f = O3.source_level(prob, j)
        r = O3.rhs3_points(prob, U, j, f, pts) - O3.apply_A3_points(prob, j, U[j + 1], pts, "A")
        S = O3.anorm3(prob, j) * np.max(np.abs(U[j + 1]))
        assert np.max(np.abs(r)) <= 1e-12 * S, (j, np.max(np.abs(r)) / S)


def test_extrapolated_march_matches_dense_oracle():
    """The extrapolated initial guess on a 16^3 march: every level against the
    oracle's dense direct solves, fewer CGS iterations than the zero guess."""
    import paper_1603_00279_amd as P
    banner("3d warm march extrap")
    prob = W.problem_3d(16, 16, 16, 5, alpha=0.7, betas=(1.8, 1.5, 1.25))
    with solver(prob, rtol=1e-12) as s:
        code0, st0 = s.solve(sources(s, prob))
    with solver(prob, rtol=1e-12, warm_start=P.TSFCDE_WS_EXTRAP) as s:
        code, stats = s.solve(sources(s, prob))
        U = host(s.history())
    assert code == 0 and code0 == 0, stats
    Uref = O3.march3(prob)
    worst = max(np.max(np.abs(U[j] - Uref[j])) / np.max(np.abs(Uref[j])) for j in range(1, prob.M + 1))
    its, its0 = [st["iters"] for st in stats], [st["iters"] for st in st0]
    print(f"[3d warm] worst rel err {worst:.2e}, iterations {its} (zero guess {its0})", flush=True)
    assert worst < 1e-10
    assert sum(its) < sum(its0)


def test_edge_orders_box_and_resume():
    """alpha = 1, one beta = 2 and one near 1, a box other than the unit cube
    and T != 1 against the dense oracle; then a plan resumed from level 2
    continues bitwise as the uninterrupted march."""
    import dataclasses
    banner("3d edge orders, box, resume")
    base = W.problem_3d(16, 16, 16, 4, alpha=1.0, betas=(2.0, 1.02, 1.5))
    lo, hi = (-1.0, 0.0, 0.5), (1.0, 3.0, 1.0)
    sols = tuple(box_solution(base.sols[k].theta_terms, lo[k], hi[k]) for k in range(3))
    prob = dataclasses.replace(base, lo=lo, hi=hi, T=0.5, sols=sols)
    with solver(prob, rtol=1e-13) as s:
        F = sources(s, prob)
        code, stats = s.solve(F)
        U = host(s.history())
    assert code == 0, stats
    Uref = O3.march3(prob)
    worst = max(np.max(np.abs(U[j] - Uref[j])) / np.max(np.abs(Uref[j])) for j in range(1, prob.M + 1))
    print(f"[3d edge] worst rel err {worst:.2e}, iterations {[st['iters'] for st in stats]}", flush=True)
    assert worst < 1e-10
    with solver(prob, rtol=1e-13) as s:
        s.set_state(2, torch.as_tensor(U[:3], device="cuda"))
        code, _ = s.solve(F)
        assert code == 0 and np.array_equal(host(s.history()), U)


def test_history_blocks():
    """19 levels at 16 x 16 x 32 (history sums in blocks of 8) against the
    oracle's FFT-route march, both to 1e-13."""
    banner("3d history blocks")
    prob = W.problem_3d(16, 16, 32, 19, alpha=0.3, betas=(1.6, 1.9, 1.2))
    with solver(prob, rtol=1e-13) as s:
        code, stats = s.solve(sources(s, prob))
        U = host(s.history())
    assert code == 0, stats
    Uref, _ = O3.march_pcgs3(prob, rtol=1e-13)
    worst = max(np.max(np.abs(U[j] - Uref[j])) / np.max(np.abs(Uref[j])) for j in range(1, prob.M + 1))
    print(f"[3d history blocks] worst rel err {worst:.2e}", flush=True)
    assert worst < 1e-10


def test_level_symbols_follow_the_level():
    """The axis symbols are tabulated once per level: A and P^{-1} applied at
    levels 4, 0, 4, 2 in turn match the oracle at each, and a march run after
    an apply at another level is bitwise the march of a fresh plan."""
    import paper_1603_00279_amd as P
    banner("3d level symbol tables")
    prob = W.problem_3d(16, 32, 16, 5, betas=(1.6, 1.3, 1.9))
    X = np.random.default_rng(22).standard_normal(prob.ns)
    with solver(prob, rtol=1e-12) as s:
        F = sources(s, prob)
        for j in (4, 0, 4, 2):
            S = O3.anorm3(prob, j) * np.max(np.abs(X))
            got = host(s.apply(P.TSFCDE_OP_A, j, torch.as_tensor(X, device="cuda")))
            assert np.max(np.abs(got - O3.product3(prob, j, X, "A"))) <= 1e-13 * S, j
            Y = host(s.apply(P.TSFCDE_OP_PINV, j, torch.as_tensor(X, device="cuda")))
            eig = O3.bccb3_eigenvalues(prob, j)
            back = np.fft.ifftn(np.fft.fftn(Y) * eig).real
            assert np.max(np.abs(back - X)) <= 1e-13 * np.max(np.abs(eig)) * np.max(np.abs(Y)), j
        code, _ = s.solve(F)
        U1 = host(s.history())
    assert code == 0
    with solver(prob, rtol=1e-12) as s:
        code, _ = s.solve(F)
        assert code == 0 and np.array_equal(host(s.history()), U1)


class _PointSource:
    """f at t_{j+sigma} evaluated one node at a time, indexed like the full
    (nx, ny, nz) array (the point checks read only the sampled nodes)."""

    def __init__(self, prob, j):
        self.prob, self.t, self.xyz = prob, O3.t_sigma(prob, j), O3.nodes(prob)

    def __getitem__(self, idx):
        i, k, l = idx
        x, y, z = self.xyz
        return float(self.prob.f(x[i:i + 1], y[k:k + 1], z[l:l + 1], self.t)[0, 0, 0])


def test_maximum_size_sampled_points():
    """2048 x 256 x 512 = 2^28 unknowns (2 GiB per vector: offsets of the
    plan's vectors and levels pass 2^31 elements), the longest axis at the
    largest supported length: two levels accepted and the oracle's point
    residuals g - A u^{j+1} within 1e-12 of |A| max|u|."""
    banner("3d 2048x256x512 (2^28 unknowns)")
    ns = (2048, 256, 512)
    prob = W.problem_3d(*ns, 2, betas=(1.5, 1.8, 1.3))
    rng = np.random.default_rng(28)
    pts = [(0, 0, 0), (2047, 255, 511), (2047, 0, 511), (0, 255, 0), (1024, 128, 256), (1500, 7, 400)]
    pts += [tuple(int(v) for v in (rng.integers(0, ns[0]), rng.integers(0, ns[1]), rng.integers(0, ns[2])))
            for _ in range(6)]
    with solver(prob) as s:
        F = sources(s, prob)
        stats = [s.step(F[j]) for j in range(2)]
        del F
        U = host(s.history())
    for j in range(2):
        st = stats[j]
        print(f"[3d 2^28] j={j} iters {st['iters']} relres_true {st['relres_true']:.2e} "
              f"backward_err {st['backward_err']:.2e}", flush=True)
        assert st["code"] == 0 and st["iters"] > 0, st
        assert st["relres_true"] <= 1e-10 or 0.0 <= st["backward_err"] <= 1e-13, st
        r = (O3.rhs3_points(prob, U, j, _PointSource(prob, j), pts)
             - O3.apply_A3_points(prob, j, U[j + 1], pts, "A"))
        S = O3.anorm3(prob, j) * np.max(np.abs(U[j + 1]))
        print(f"[3d 2^28] j={j} max point residual / (|A| max|u|) = {np.max(np.abs(r)) / S:.2e}", flush=True)
        assert np.max(np.abs(r)) <= 1e-12 * S, (j, np.max(np.abs(r)) / S)
