"""tsfcde_apply_noalloc (the allocation-free variant of tsfcde_apply, for
callers that cannot allocate) against tsfcde_plan + tsfcde_apply, through the
C ABI: the same kernels on the same inputs, so the outputs agree bit for bit.
Two calls in a row on the shared static scratch array, the second with a
smaller input, for each operator; then sizes beyond the limit are refused."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from gpu_util import banner, host, need_gpu, t64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1603_00279_amd as P
    P.lib()


def _noalloc(P, solver, op, j, x):
    """y from tsfcde_apply_noalloc with the solver's own problem struct."""
    from paper_1603_00279_amd import _native as N
    y = torch.full_like(x, float("nan"))
    rc = P.lib().tsfcde_apply_noalloc(ctypes.byref(solver.problem), op, j, ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(solver.stream.cuda_stream))
    N.check(rc, "tsfcde_apply_noalloc")
    return y


@pytest.mark.parametrize("sizes", [(32768, 4096), (30000, 1000), (4096, 100)])
def test_noalloc_matches_planned_apply(sizes):
    import paper_1603_00279_amd as P
    for n in sizes:  # the second call has the smaller input
        banner(f"noalloc n={n}")
        prob = W.config_large(n=n, M=9, alpha=0.6, beta=1.7)
        x = t64(np.random.default_rng(n).standard_normal(n))
        with P.TimeLevelSolver.from_problem(prob) as s:
            for op in (P.TSFCDE_OP_A, P.TSFCDE_OP_B, P.TSFCDE_OP_PINV):
                for j in (0, 8):
                    ref = host(s.apply(op, j, x))
                    got = host(_noalloc(P, s, op, j, x))
                    assert np.array_equal(got, ref), (n, op, j, float(np.max(np.abs(got - ref))))


def test_noalloc_refuses_beyond_limit():
    import paper_1603_00279_amd as P
    from paper_1603_00279_amd import _native as N
    prob = W.config_large(n=N.TSFCDE_NOALLOC_NMAX * 2, M=2)
    with P.TimeLevelSolver.from_problem(prob) as s:
        x = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
        y = torch.zeros_like(x)
        rc = P.lib().tsfcde_apply_noalloc(ctypes.byref(s.problem), P.TSFCDE_OP_A, 0, ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(y.data_ptr()), None)
    assert rc == P.TSFCDE_EUNSUPPORTED
