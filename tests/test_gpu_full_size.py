"""GPU parity at the full size of the headline march, n = 2^20 (product
transform 1024 x 1024, preconditioner transform 512 x 1024: the launch
geometry bench.py times), on outputs the oracle evaluates one by one, and
size-independent properties of whole levels.

Tolerances are absolute, per sampled row, against the row's scale
  S = (eta + sigma (|gamma|/h + (d+ + d-) h^-beta sum|omega|)) * max|x|,
an upper bound of sum_k |A_ik x_k|.  An FFT product of length L in FP64
carries errors of order eps * log2(L) * S (about 5e-15 S here); the bar is
1e-12 S.  A misplaced twiddle or permutation gives errors of order S.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import banner, host, need_gpu, row_scale, sample_rows, sources, t64

pytestmark = pytest.mark.gpu

N_FULL = 1 << 20
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "pcgs_headline_levels.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    import paper_1603_00279_amd as P  # noqa: F401  (fails loudly if the library is missing)
    P.lib()


def make(prob, **kw):
    import paper_1603_00279_amd as P
    return P.TimeLevelSolver.from_problem(prob, **kw)


def test_spectra_full_size():
    """Both stored spectra against the library FFT of the oracle's columns
    (every frequency)."""
    import paper_1603_00279_amd as P
    banner("spectra n=2^20")
    prob = W.config_large(n=N_FULL, M=4)
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


def test_products_full_size():
    import paper_1603_00279_amd as P
    banner("apply A/B n=2^20")
    prob = W.config_large(n=N_FULL, M=8)
    rng = np.random.default_rng(20)
    x = rng.standard_normal(prob.n)
    rows = sample_rows(prob.n, 1)
    with make(prob) as s:
        for j in (0, 5):
            yA = host(s.apply(P.TSFCDE_OP_A, j, t64(x)))
            yB = host(s.apply(P.TSFCDE_OP_B, j, t64(x)))
            S = row_scale(prob, j, x)
            dA = np.abs(yA[rows] - O.apply_A_rows(prob, j, x, rows, "A"))
            dB = np.abs(yB[rows] - O.apply_A_rows(prob, j, x, rows, "B"))
            assert dA.max() <= 1e-12 * S, (j, dA.max() / S)
            assert dB.max() <= 1e-12 * S, (j, dB.max() / S)


def test_preconditioner_solve_full_size():
    """y = P^-1 x through the FFT solve; the oracle's rows of P y give back x
    (a backward-error check, which does not depend on cond(P))."""
    import paper_1603_00279_amd as P
    banner("apply Pinv n=2^20")
    prob = W.config_large(n=N_FULL, M=8)
    x = np.random.default_rng(21).standard_normal(prob.n)
    rows = sample_rows(prob.n, 2, k=24)
    with make(prob) as s:
        for j in (0, 7):
            y = host(s.apply(P.TSFCDE_OP_PINV, j, t64(x)))
            d = np.abs(O.apply_P_rows(prob, j, y, rows) - x[rows])
            assert d.max() <= 1e-12 * row_scale(prob, j, y), (j, d.max() / row_scale(prob, j, y))


@pytest.mark.parametrize("j", [1, 3, 9])
def test_rhs_full_size(j):
    """Right-hand side with a random stored history: level 1 and 9 start a
    history block (one sweep), level 3 adds a catch-up to its block's sum."""
    banner(f"rhs n=2^20 j={j}")
    prob = W.config_large(n=N_FULL, M=12, alpha=0.4)
    rng = np.random.default_rng(100 + j)
    U = rng.standard_normal((j + 1, prob.n))
    f = rng.standard_normal(prob.n)
    rows = sample_rows(prob.n, 3 + j)
    with make(prob) as s:
        s.set_state(j, t64(U))
        g = host(s.rhs(j, t64(f)))
    ref = O.rhs_rows(prob, U, j, f, rows)
    # history: kappa sum_s |c_{j-s}| |u^{s+1} - u^s| <= kappa * sum|c| * 2 max|U|
    c = O.l21s_c(prob.alpha, j)
    hist = O.l21s_kappa(prob.alpha, O.time_step(prob)) * float(np.sum(np.abs(c))) * 2.0 * float(np.max(np.abs(U)))
    S = row_scale(prob, j, U[j]) + hist + float(np.max(np.abs(f)))
    d = np.abs(g[rows] - ref)
    assert d.max() <= 1e-12 * S, d.max() / S


def test_levels_full_size():
    """The first four levels of the headline march (n = 2^20, M = 512) with
    the true-residual check.  A level is accepted when its true relative
    residual is within the Krylov tolerance or, where FP64 cannot reach that
    (an FFT product carries errors of order eps |A| |x|, and |A| ~ h^-beta ~
    1e11 here), when its normwise backward error is at most 1e-13.  The
    oracle's rows of g - A u^{j+1} must then be rounding-sized against the
    row scale S (a componentwise backward-error check)."""
    import paper_1603_00279_amd as P
    banner("levels n=2^20 M=512")
    prob = W.config_large(n=N_FULL, M=512)
    rows = sample_rows(prob.n, 5)
    F = [O.source_level(prob, j) for j in range(4)]  # the oracle's own sampling, for its rows of g
    with make(prob, rtol=1e-10, flags=P.TSFCDE_FLAG_VERIFY) as s:
        Fd = sources(s, prob, 4)  # the plan's
        stats = [s.step(Fd[j]) for j in range(4)]
        U = host(s.history()[:5])
    for j in range(4):
        st = stats[j]
        assert st["code"] == P.TSFCDE_OK and st["iters"] > 0, st
        assert st["relres_true"] <= 1e-10 or 0.0 <= st["backward_err"] <= 1e-13, st
        r = O.rhs_rows(prob, U, j, F[j], rows) - O.apply_A_rows(prob, j, U[j + 1], rows, "A")
        S = row_scale(prob, j, U[j + 1])
        assert np.abs(r).max() <= 1e-12 * S, (j, np.abs(r).max() / S)


def test_general_n_full_size():
    """n = 1000003 (odd, not a power of two): products through the length
    2^21 embedding and the preconditioner solve through the per-level
    inverse Strang circulant built by Bluestein's transform, on sampled rows."""
    import paper_1603_00279_amd as P
    n = 1000003
    banner(f"general n={n}")
    prob = W.config_large(n=n, M=6)
    rng = np.random.default_rng(31)
    x = rng.standard_normal(n)
    fixed = np.array([0, 1, 2, 1023, 1024, n // 2, n - 3, n - 2, n - 1])
    rows = np.unique(np.concatenate([fixed, rng.integers(0, n, size=24)]))
    with make(prob) as s:
        for j in (0, 4):
            yA = host(s.apply(P.TSFCDE_OP_A, j, t64(x)))
            S = row_scale(prob, j, x)
            dA = np.abs(yA[rows] - O.apply_A_rows(prob, j, x, rows, "A"))
            assert dA.max() <= 1e-12 * S, (j, dA.max() / S)
            y = host(s.apply(P.TSFCDE_OP_PINV, j, t64(x)))
            d = np.abs(O.apply_P_rows(prob, j, y, rows) - x[rows])
            assert d.max() <= 1e-12 * row_scale(prob, j, y), (j, d.max() / row_scale(prob, j, y))


def product_rounding(prob, j, L, unorm):
    """2 log2(L) eps S_A |u|_2: first-order bound on the rounding of A u
    computed through FFTs of length L (forward, scale by eigenvalues of
    modulus <= S_A, inverse), S_A = the row scale of a unit vector."""
    return 2.0 * np.log2(L) * np.finfo(np.float64).eps * row_scale(prob, j, np.ones(1)) * unorm


def test_levels_against_fft_pcgs_golden():
    """u^1 and u^2 of the headline march (n = 2^20, M = 512) against the
    oracle's FFT-PCGS solutions stored on 2055 rows.  Both sides solve
    A u = g for the same g (level 2 starts from the oracle's u^1, recomputed
    here), so u_gpu - u_ref = A^-1 (r_gpu - r_ref) with r the exact residuals,
    and |A^-1|_2 <= 1/eta_j because the symmetric part of A is at least
    eta_j I.  Each exact residual is bounded by its computed norm plus the
    rounding of the product that computed it (phi); level 2 adds a phi for
    g, formed from a u^1 that may differ from the stored run's in its last
    bits, and one for the GPU's own g.  The 2-norm bound covers every row.
    It certifies a few per cent of max|u| (|A| |u| / eta is large at this
    h), so it catches structural mistakes (a wrong sign, a dropped history
    or source term changes u by order one); the componentwise
    backward-error test above is the sharp one."""
    import paper_1603_00279_amd as P
    banner("levels vs FFT-PCGS golden n=2^20")
    with open(GOLDEN) as fh:
        gold = json.load(fh)
    prob = W.config_large(n=N_FULL, M=512)
    assert (gold["n"], gold["M"], gold["alpha"], gold["beta"]) == (prob.n, prob.M, prob.alpha, prob.beta)
    rows = np.array(gold["rows"])
    u0 = O.initial_level(prob)
    u1_ref, _ = O.level_solve_pcgs(prob, u0[None, :], 0, O.source_level(prob, 0), rtol=1e-12)
    with make(prob, rtol=1e-10, flags=P.TSFCDE_FLAG_VERIFY) as s:
        L = s.embedding_length
        F = sources(s, prob, 2)
        st1 = s.step(F[0])
        u1 = host(s.history()[1])
        s.set_state(1, t64(np.stack([u0, u1_ref])))
        st2 = s.step(F[1])
        u2 = host(s.history()[2])
    for j, (st, u, extra) in enumerate(((st1, u1, 0), (st2, u2, 2))):
        lev = gold["levels"][j]
        assert lev["j"] == j + 1 and st["code"] == P.TSFCDE_OK, st
        eta = O.level_scalars(prob, j)[0]
        phi = product_rounding(prob, j, L, max(lev["u_norm"], float(np.linalg.norm(u))))
        r_gpu = st["relres_true"] * lev["g_norm"]
        tol = (r_gpu + lev["residual_norm"] + (2 + extra) * phi) / eta
        d = float(np.max(np.abs(u[rows] - np.array(lev["values"]))))
        print(f"u^{j + 1}: max row diff {d:.3e} = {d / lev['max_abs']:.2e} max|u|, bound {tol:.3e}", flush=True)
        assert d <= tol, (j + 1, d, tol)
