"""GPU parity of the constant-coefficient path (TSFCDE_FLAG_CONSTANT_GSF:
Algorithm 3, with A^-1 applied by the Gohberg-Semencul formula, Algorithm 1)
against the oracle's dense-LU march (Algorithm 2), on Example 1 and the grids
of Tables 3 and 4 (h = tau = 1/N, n = N - 1), plus a power-of-two grid.  The
bar is the method's 1e-10 per level, normwise and elementwise against
max|u|, with the Krylov tolerance of level 0 and of the solves (3.4) at
1e-13.  Every level j >= 1 must be accepted on the formula's own result
(no CGS iterations after it), which is the formula's stability check."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import banner, host, need_gpu, relerr, sources

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1603_00279_amd as P
    P.lib()


@pytest.mark.parametrize("alpha,beta,N,levels", [
    (0.9, 1.2, 32, None), (0.9, 1.5, 64, None), (0.9, 1.8, 256, None),   # Table 3's alpha, its betas
    (0.1, 1.8, 64, None), (0.5, 1.8, 128, None),                         # Table 4's beta, its alphas
    (0.9, 1.8, 1024, 12), (0.5, 1.8, 1025, 8),                           # h = 2^-10; n = 1024 (power of two)
])
def test_gsf_march_matches_oracle(alpha, beta, N, levels):
    import paper_1603_00279_amd as P
    banner(f"gsf example1 alpha={alpha} beta={beta} N={N}")
    prob = W.example1(alpha, beta, N)
    L = prob.M if levels is None else levels
    Uref = O.march(prob, levels=L)
    with P.TimeLevelSolver.from_problem(prob, rtol=1e-13, flags=P.TSFCDE_FLAG_CONSTANT_GSF) as s:
        F = sources(s, prob, L)
        stats = [s.step(F[j]) for j in range(L)]
        U = host(s.history()[: L + 1])
    assert stats[0]["method"] == P.TSFCDE_METHOD_PCGS
    assert all(st["method"] == P.TSFCDE_METHOD_GSF for st in stats[1:])
    if L > 1:
        assert stats[1]["iters"] > 0  # the two solves (3.4)
    worst = 0.0
    for j in range(1, L + 1):
        e_norm = relerr(U[j], Uref[j])
        e_elem = float(np.max(np.abs(U[j] - Uref[j])) / np.max(np.abs(Uref[j])))
        worst = max(worst, e_norm, e_elem)
        assert e_norm < 1e-10 and e_elem < 1e-10, (j, e_norm, e_elem, stats[j - 1])
    cont = [st["iters"] for st in stats[2:]]
    print(f"[gsf N={N}] worst per-level error {worst:.2e}; solves (3.4): {stats[1]['iters'] if L > 1 else 0} "
          f"iterations; CGS after the formula: {sum(cont)}", flush=True)
    assert all(st["backward_err"] <= 1e-13 for st in stats[1:])
    assert sum(cont) == 0, cont


def test_gsf_equals_pcgs_path_and_refuses_varying_coefficients():
    """The formula and the plain PCGS path give the same march to the Krylov
    tolerance's reach; a problem whose coefficients vary in t is refused."""
    import paper_1603_00279_amd as P
    banner("gsf vs pcgs")
    prob = W.example1(0.7, 1.6, 300)
    runs = {}
    for flags in (0, P.TSFCDE_FLAG_CONSTANT_GSF):
        with P.TimeLevelSolver.from_problem(prob, rtol=1e-13, flags=flags) as s:
            s.solve(sources(s, prob))
            runs[flags] = host(s.history())
    assert relerr(runs[P.TSFCDE_FLAG_CONSTANT_GSF], runs[0]) < 1e-10
    with pytest.raises(P.TsfcdeError):
        P.TimeLevelSolver.from_problem(W.example2(0.5, 1.5, 32), flags=P.TSFCDE_FLAG_CONSTANT_GSF)
