"""GPU parity above the headline size:
- n = 2^22 with M = 256, the larger single-instance case.  Its product
  transform is 2048 x 2048 and its preconditioner transform 1024 x 2048.
- n = 2^24, the largest power of two the library takes (4096 x 4096 and
  2048 x 4096).
- n = 2^23 - 1, the largest other n.  Its preconditioner's inverse circulant
  comes from Bluestein's transform of length 2^25.

The checks and tolerances are those of the n = 2^20 tests.  Each sampled row
is compared with the oracle's direct sum against the row scale
  S = (eta + sigma (|gamma|/h + (d+ + d-) h^-beta sum|omega|)) max|x|,
with a bar of 1e-12 S.  An FFT product of length L carries about
eps log2(L) S, which is 6e-15 S at L = 2^25.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import banner, host, need_gpu, row_scale, sample_rows, sources, t64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1603_00279_amd as P  # noqa: F401  (fails loudly if the library is missing)
    P.lib()


def make(prob, **kw):
    import paper_1603_00279_amd as P
    return P.TimeLevelSolver.from_problem(prob, **kw)


@pytest.mark.parametrize("n,width", [(1 << 22, 2048), (1 << 24, 4096), ((1 << 23) - 1, 4096)])
def test_products_and_preconditioner_large(n, width):
    """A x and B x on sampled rows.  For y = P^-1 x, the oracle's rows of
    P y give back x: a backward-error check that does not depend on cond(P)."""
    import paper_1603_00279_amd as P
    banner(f"apply A/B/Pinv n={n}")
    prob = W.config_large(n=n, M=4)
    rng = np.random.default_rng(n % 1000 + 40)
    x = rng.standard_normal(n)
    rows = sample_rows(n, 7, k=12, width=width)
    with make(prob) as s:
        for j in (0, 3):
            yA = host(s.apply(P.TSFCDE_OP_A, j, t64(x)))
            yB = host(s.apply(P.TSFCDE_OP_B, j, t64(x)))
            y = host(s.apply(P.TSFCDE_OP_PINV, j, t64(x)))
            S = row_scale(prob, j, x)
            dA = np.abs(yA[rows] - O.apply_A_rows(prob, j, x, rows, "A"))
            dB = np.abs(yB[rows] - O.apply_A_rows(prob, j, x, rows, "B"))
            assert dA.max() <= 1e-12 * S, (j, dA.max() / S)
            assert dB.max() <= 1e-12 * S, (j, dB.max() / S)
            Sy = row_scale(prob, j, y)
            dP = np.abs(O.apply_P_rows(prob, j, y, rows) - x[rows])
            assert dP.max() <= 1e-12 * Sy, (j, dP.max() / Sy)


def test_spectra_n_2p22():
    """Both stored spectra at n = 2^22 against the library FFT of the
    oracle's columns, at every frequency."""
    import paper_1603_00279_amd as P
    banner("spectra n=2^22")
    prob = W.config_large(n=1 << 22, M=2)
    with make(prob) as s:
        L = s.embedding_length
        emb = host(s.spectrum(P.TSFCDE_SPEC_EMBED))
        strang = host(s.spectrum(P.TSFCDE_SPEC_STRANG))
    n, beta = prob.n, prob.beta
    ref_emb = np.fft.fft(O.embedding_column(beta, n, L))[: L // 2 + 1]
    w = O.wsgd_weights(beta, n + 1)
    col = O.strang_column(lambda m: w[m + 1] if m >= -1 else 0.0, n)
    ref_str = O.circulant_eigenvalues(col)[: n // 2 + 1]
    assert np.max(np.abs(emb - ref_emb)) <= 1e-13 * np.max(np.abs(ref_emb))
    assert np.max(np.abs(strang - ref_str)) <= 1e-13 * np.max(np.abs(ref_str))


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_levels_n_2p22(precision):
    """The first three levels of the n = 2^22, M = 256 march (alpha = 0.7,
    beta = 1.8), in FP64 and with TSFCDE_FP32_REFINED requested.  At this
    size the refined form's rounding-error model (2^-24 log2(L) |A|/eta far
    above 0.1) keeps every level in FP64, which the stats must say.
    Acceptance is as in the n = 2^20 level test.  The oracle's rows of
    g - A u^{j+1} (its own sampling of f) must be rounding-sized against the
    row scale (a componentwise backward error).  Level 1 starts a history
    block; levels 2 and 3 catch up within it."""
    import paper_1603_00279_amd as P
    banner(f"levels n=2^22 M=256 {precision}")
    prob = W.config_large(n=1 << 22, M=256)
    rows = sample_rows(prob.n, 9, k=24, width=2048)
    F = [O.source_level(prob, j) for j in range(3)]
    prec = P.TSFCDE_FP64 if precision == "fp64" else P.TSFCDE_FP32_REFINED
    with make(prob, rtol=1e-10, flags=P.TSFCDE_FLAG_VERIFY, precision=prec) as s:
        Fd = sources(s, prob, 3)
        stats = [s.step(Fd[j]) for j in range(3)]
        U = host(s.history()[:4])
    for j in range(3):
        st = stats[j]
        assert st["code"] == P.TSFCDE_OK and st["iters"] > 0, st
        assert st["precision_used"] == P.TSFCDE_FP64, st
        assert st["relres_true"] <= 1e-10 or 0.0 <= st["backward_err"] <= 1e-13, st
        r = O.rhs_rows(prob, U, j, F[j], rows) - O.apply_A_rows(prob, j, U[j + 1], rows, "A")
        S = row_scale(prob, j, U[j + 1])
        assert np.abs(r).max() <= 1e-12 * S, (j, np.abs(r).max() / S)


def test_levels_n_2p24():
    """The first two levels at n = 2^24 (alpha = 0.7, beta = 1.8): every pass
    of the CGS iteration at sixteen values per lane (product columns of 4096,
    preconditioner columns of 2048), whose four-step twiddles come from
    running products.  Acceptance and the oracle's sampled rows of
    g - A u^{j+1} as in the n = 2^22 test."""
    import paper_1603_00279_amd as P
    banner("levels n=2^24 M=4")
    prob = W.config_large(n=1 << 24, M=4)
    rows = sample_rows(prob.n, 11, k=16, width=4096)
    F = [O.source_level(prob, j) for j in range(2)]
    with make(prob, rtol=1e-10, flags=P.TSFCDE_FLAG_VERIFY) as s:
        Fd = sources(s, prob, 2)
        stats = [s.step(Fd[j]) for j in range(2)]
        U = host(s.history()[:3])
    for j in range(2):
        st = stats[j]
        print(f"[levels n=2^24] j={j} iters {st['iters']} relres_true {st['relres_true']:.2e} "
              f"backward_err {st['backward_err']:.2e}", flush=True)
        assert st["code"] == P.TSFCDE_OK and st["iters"] > 0, st
        assert st["relres_true"] <= 1e-10 or 0.0 <= st["backward_err"] <= 1e-13, st
        r = O.rhs_rows(prob, U, j, F[j], rows) - O.apply_A_rows(prob, j, U[j + 1], rows, "A")
        S = row_scale(prob, j, U[j + 1])
        assert np.abs(r).max() <= 1e-12 * S, (j, np.abs(r).max() / S)
