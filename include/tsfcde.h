/*
 * tsfcde.h -- C ABI of the MI355X (gfx950) time-level solver for the
 * time-space fractional convection-diffusion equation (TSFCDE)
 *
 *   D_t^alpha u = gamma(t) u_x + d_+(t) aD_x^beta u + d_-(t) xD_b^beta u + f,
 *   u(x,0) = phi(x),  u(a,t) = u(b,t) = 0,                       problem (1.1)
 *
 * of Gu, Huang, Ji, Carpentieri and Alikhanov, arXiv:1603.00279.
 *
 * Each call to tsfcde_step advances the implicit difference scheme (IDS) by
 * one time level (Algorithm 2): it assembles the right-hand side
 * g = B^(j+sigma) u^j - delta u^(j) + f^(j+sigma) of (3.3), including the
 * L2-1sigma history sum over all earlier levels (Lemma 1), and solves the
 * nonsymmetric Toeplitz system A^(j+sigma) u^(j+1) = g by CGS with the Strang
 * circulant preconditioner (3.7) (Sec. 3.2).  Every Toeplitz product is an
 * FFT over a circulant embedding of length 2n; every preconditioner solve is
 * an n-point circulant FFT solve.  All of it runs in the library's own HIP
 * kernels on the stream given to tsfcde_plan.
 *
 * Conventions
 *  - n is the number of interior unknowns, h = (b-a)/(n+1); the paper's N
 *    (number of subintervals) is n+1.  M is the number of time steps,
 *    tau = T/M.  gamma, d_+, d_- and f are sampled at t_{j+sigma},
 *    sigma = 1 - alpha/2 (Lemma 1, Sec. 2.1).
 *  - All device pointers are plain HIP device addresses (e.g. the data
 *    pointer of a torch tensor on the same device).  Vectors are contiguous
 *    FP64 arrays of n values ordered x_1..x_n.
 *  - Every call returns a status: TSFCDE_OK (0) or a negative TSFCDE_E*
 *    code; tsfcde_strerror names it.  Invalid arguments are rejected on the
 *    host before any device work.
 *  - A plan is bound to one device and one stream and is not thread-safe.
 *    Device work is asynchronous on that stream except where a call is
 *    documented to synchronize (tsfcde_step/tsfcde_solve synchronize on the
 *    convergence flag between Krylov chunks).
 */
#ifndef TSFCDE_H
#define TSFCDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------- */
#define TSFCDE_OK 0
#define TSFCDE_EINVAL (-1)       /* argument out of range (see tsfcde_plan) */
#define TSFCDE_ENOMEM (-2)       /* workspace too small                      */
#define TSFCDE_EDEVICE (-3)      /* a HIP runtime call failed                */
#define TSFCDE_ENOCONV (-4)      /* maxit reached; solution/stats still set  */
#define TSFCDE_EBREAKDOWN (-5)   /* CGS breakdown (rho or r~'v = 0)          */
#define TSFCDE_ENONFINITE (-6)   /* NaN/Inf met in the iteration             */
#define TSFCDE_EDONE (-7)        /* all M levels already computed            */
#define TSFCDE_EUNSUPPORTED (-8) /* valid problem outside the supported sizes or forms */
#define TSFCDE_EACCEPT (-9)      /* the level's iterate failed the acceptance test
                                    (true residual <= rtol |g| or backward error
                                    <= 1e-13; the first alone under
                                    TSFCDE_FLAG_STRICT_RESIDUAL) after every
                                    restart; solution/stats still set        */

/* ---- options -------------------------------------------------------- */
#define TSFCDE_FP64 0            /* every step in FP64                       */
#define TSFCDE_FP32_REFINED 1    /* FP64 iterative refinement around an inner
                                    CGS whose vectors, transform buffers and
                                    spectra are stored in FP32 (the right-hand
                                    side, the history, the refinement residual
                                    and all Krylov scalars stay FP64).  Used at
                                    a level only while 2^-24 log2(L) |A|/eta
                                    < 0.1, with |A|/eta bounded through Remark
                                    3.1; other levels, and levels whose
                                    refinement stalls, run the FP64 CGS.  The
                                    stopping test is the true FP64 residual
                                    |g - A u| <= rtol |g|.                    */
#define TSFCDE_FP32_REFINED_FELL_BACK 2 /* stats only: refinement started, then
                                    the level finished with the FP64 CGS     */
#define TSFCDE_WS_ZERO 0         /* Krylov initial guess 0 (as in Sec. 4)    */
#define TSFCDE_WS_PREV 1         /* initial guess u^j (previous level)       */
#define TSFCDE_WS_EXTRAP 2       /* 3u^j - 3u^{j-1} + u^{j-2} (quadratic in t; u^j
                                    for j = 1, 0 for j = 0)                  */
#define TSFCDE_WS_NET 3          /* learned guess (tsfcde_plan_set_net) from
                                    level 2 on, u^j for j = 1, 0 for j = 0;
                                    the previous-level guess replaces it when
                                    its true residual |g - A x0| is not below
                                    that of u^j                              */
#define TSFCDE_FLAG_TRUE_RESIDUAL 1 /* also compute |g - A u|/|g| per level  */
#define TSFCDE_FLAG_VERIFY 2     /* on recursive convergence, recompute r = g - A x
                                    and restart CGS from x while the true residual
                                    is above rtol |g| and still falling (at most 3
                                    restarts), even when the backward error
                                    already passes; also restarts once per
                                    breakdown                                */
#define TSFCDE_FLAG_FORCE_FP32 4 /* FP32_REFINED at every level, whatever the
                                    rounding-error model predicts (to measure
                                    where the refinement stops converging)   */
#define TSFCDE_FLAG_NO_FOLD 8    /* launch the Krylov reductions' finishing
                                    kernels separately instead of folding them
                                    into the passes that follow (diagnostic:
                                    the results are bitwise the same)        */
#define TSFCDE_FLAG_STRICT_RESIDUAL 16 /* accept a level only at a true residual
                                    |g - A u| <= rtol |g| (not at backward
                                    error 1e-13); otherwise TSFCDE_EACCEPT   */
#define TSFCDE_FLAG_CONSTANT_GSF 32 /* constant gamma, d_+- (every sample equal,
                                    else tsfcde_plan returns TSFCDE_EINVAL;
                                    FP64 single plans only): Algorithm 3.
                                    Level 0 by PCGS; before level 1, A x = e_1
                                    and A y = e_n (3.4) by PCGS to 1e-13 (or
                                    rtol if tighter); every level j >= 1 then
                                    applies A^-1 by the Gohberg-Semencul
                                    formula (Algorithm 1: four triangular
                                    Toeplitz products through the length-2n
                                    embedding) and checks the result like a
                                    converged CGS solve (CGS continues from
                                    it if the check fails).  xi_0 = 0 or a
                                    failed solve (3.4) ends level 1 with
                                    TSFCDE_EBREAKDOWN or that solve's code  */

/* Krylov methods (tsfcde_problem.krylov).  Both are right-preconditioned
 * (the monitored residual is the unpreconditioned one), run on
 * device-resident scalars and meet the same stopping and acceptance tests;
 * each iteration makes two products with A and two preconditioner solves.
 * The FP32 inner solve of TSFCDE_FP32_REFINED is always CGS; the batched
 * form runs CGS only. */
#define TSFCDE_KRYLOV_CGS 0      /* conjugate gradient squared (Sec. 3.2)    */
#define TSFCDE_KRYLOV_BICGSTAB 1 /* BiCGSTAB (van der Vorst 1992), the smooth-
                                    residual alternative the paper's outlook
                                    (Sec. 5) points to among Krylov solvers  */

/* circulant preconditioners (tsfcde_problem.preconditioner), each assembled
 * like (3.7) from the circulants of Q, W_beta and W_beta^T */
#define TSFCDE_PREC_STRANG 0     /* Strang's circulant s(.) of (3.7)         */
#define TSFCDE_PREC_TCHAN 1      /* T. Chan's optimal circulant (the circulant
                                    nearest in the Frobenius norm):
                                    c_k = ((n-k) t_k + k t_{k-n}) / n        */

#define TSFCDE_FLAG_GRAPHS 64   /* batched form: replay each chunk of CGS
                                    iterations (every group's launches) from
                                    a HIP graph captured the first time that
                                    chunk length is needed (kernels only; the
                                    level's descriptors are re-staged at the
                                    same device addresses); the results are
                                    bitwise those of direct launches          */

#define TSFCDE_FLAG_NO_TUNE 128 /* batched form: keep the default values per
                                    lane (8) in every group's middle passes
                                    instead of timing 4 and 8 at plan time   */

/* solution methods reported in tsfcde_stats.method */
#define TSFCDE_METHOD_PCGS 0     /* Strang-preconditioned CGS (Algorithm 2)  */
#define TSFCDE_METHOD_GSF 1      /* Gohberg-Semencul formula (Algorithm 1)   */
#define TSFCDE_METHOD_PBICGSTAB 2 /* preconditioned BiCGSTAB                 */

/* operators for tsfcde_apply */
#define TSFCDE_OP_A 0            /* y = A^(j+sigma) x      (3.3)            */
#define TSFCDE_OP_B 1            /* y = B^(j+sigma) x      (3.3)            */
#define TSFCDE_OP_PINV 2         /* y = (P^(j+sigma))^{-1} x   (3.7)        */

/* spectra for tsfcde_spectrum */
#define TSFCDE_SPEC_EMBED 0      /* DFT of the length-2n circulant embedding of W_beta */
#define TSFCDE_SPEC_STRANG 1     /* DFT of the n-point Strang circulant s(W_beta)      */

/* gamma(t), d_+(t), d_-(t) of problem (1.1) */
typedef double (*tsfcde_coef_fn)(double t, void *user);
/* phi(x), the initial condition of problem (1.1) */
typedef double (*tsfcde_ic_fn)(double x, void *user);
/* f(x, t), the source term of problem (1.1) */
typedef double (*tsfcde_src_fn)(double x, double t, void *user);

/* Problem statement (1.1) plus solver options.  The caller owns it; the
 * plan copies what it needs during tsfcde_plan. */
typedef struct tsfcde_problem {
    double alpha;      /* time order, 0 < alpha <= 1                        */
    double beta;       /* space order, 1 < beta <= 2                        */
    double a, b;       /* space interval, a < b                             */
    double T;          /* final time, T > 0                                 */
    int64_t n;         /* interior unknowns, 4 <= n <= 2^24 (2^23 unless a
                          power of two); powers of two >= 16 take the
                          fastest path                                     */
    int64_t M;         /* time steps, M >= 1                                */
    /* gamma(t), d_+(t), d_-(t): either callbacks (called on the host during
     * tsfcde_plan at t_{j+sigma}, j = 0..M-1) or, when a callback is NULL,
     * host arrays of those M samples.  d_+- must be >= 0 (problem (1.1);
     * Theorem 3.1 needs it for the preconditioner to be invertible). */
    tsfcde_coef_fn gamma, dplus, dminus;
    void *coef_user;
    const double *gamma_at, *dplus_at, *dminus_at;
    /* phi(x): callback on the host at x_1..x_n during tsfcde_plan; NULL means
     * u^0 = 0 unless tsfcde_set_state provides it. */
    tsfcde_ic_fn phi;
    void *phi_user;
    double rtol;       /* Krylov stop: |r_k|_2 <= rtol |g|_2 (<= 0: 1e-10)   */
    int32_t maxit;     /* CGS iterations per level (<= 0: 500)              */
    int32_t precision; /* TSFCDE_FP64 or TSFCDE_FP32_REFINED                */
    int32_t warm_start;/* TSFCDE_WS_ZERO, _PREV, _EXTRAP or _NET            */
    int32_t flags;     /* TSFCDE_FLAG_*                                     */
    /* f(x, t): callback on the host, evaluated at x_1..x_n and t_{j+sigma}
     * by tsfcde_step / tsfcde_solve / tsfcde_batch_step for every level whose
     * device source pointer is NULL; NULL here means f = 0 at such levels. */
    tsfcde_src_fn f;
    void *f_user;
    int32_t krylov;         /* TSFCDE_KRYLOV_CGS (0, the paper's PCGS) or
                               TSFCDE_KRYLOV_BICGSTAB                        */
    int32_t preconditioner; /* TSFCDE_PREC_STRANG (0, (3.7)) or
                               TSFCDE_PREC_TCHAN                             */
    double history_tol;     /* 0: the history sum of (3.3) over all earlier
                               levels exactly (Lemma 1's weights).  In
                               (0, 1e-2]: the fast history -- the weights c_m,
                               m >= 2, replaced by a sum of exponentials plus
                               a cubic in m, fitted at plan time to relative
                               error <= history_tol for every m the march
                               uses (TSFCDE_EUNSUPPORTED if the fit cannot),
                               so that each level costs K + 4 vector
                               recursions (K ~ 30-90) instead of a sum over
                               j levels; the result then differs from the
                               exact scheme by at most kappa history_tol
                               sum_m c_m |u^{j-m+1} - u^{j-m}| per level in
                               the history term.  Single plans only.       */
} tsfcde_problem;

typedef struct tsfcde_stats {
    int32_t iters;        /* CGS iterations of this level (inner FP32 ones
                             plus any FP64 ones)                             */
    int32_t outer_iters;  /* refinement residuals computed (1 for FP64)      */
    int32_t restarts;     /* CGS restarts (breakdown or true-residual gap)   */
    int32_t status;       /* TSFCDE_OK or the level's error code             */
    double relres;        /* |r|_2 / |g|_2 at exit (the true residual once the
                             level's answer has been checked)                */
    double relres_true;   /* |g - A u|_2/|g|_2 of the returned u             */
    double backward_err;  /* |g - A u|_2 / (|A|_2 |u|_2 + |g|_2), with |A|_2
                             bounded above by eta + sigma(|gamma|/h +
                             (d_+ + d_-) h^-beta sum_k |omega_k|).  A level
                             whose CGS stops on its recursive residual is
                             accepted when this is <= 1e-13 (or its true
                             residual meets rtol); otherwise CGS restarts
                             from u, at most 3 times, and the level ends
                             with TSFCDE_EACCEPT                            */
    double seconds;       /* host wall time of the level                     */
    int32_t precision_used; /* TSFCDE_FP64, TSFCDE_FP32_REFINED, or
                             TSFCDE_FP32_REFINED_FELL_BACK                   */
    int32_t guess;        /* initial guess used: TSFCDE_WS_ZERO, _PREV,
                             _EXTRAP or _NET                                 */
    int32_t method;       /* TSFCDE_METHOD_*; the first TSFCDE_METHOD_GSF
                             level's iters and restarts include those of the
                             two solves (3.4)                                */
    int32_t pad;
} tsfcde_stats;

typedef struct tsfcde_plan_s *tsfcde_plan_t;

/* Device workspace needed by a plan for this problem, in bytes.  Returns
 * TSFCDE_EINVAL / TSFCDE_EUNSUPPORTED for a problem tsfcde_plan would refuse. */
int tsfcde_workspace_bytes(const tsfcde_problem *prob, size_t *bytes);

/* Validate the problem, sample the coefficients, build the L2-1sigma tables
 * (Lemma 1), the WSGD weights (Lemma 2) and the two circulant spectra
 * (Sec. 3.2) on the device.  d_workspace: caller-owned device memory of at
 * least tsfcde_workspace_bytes bytes, 256-byte aligned, kept alive until
 * tsfcde_destroy.  stream: a hipStream_t (NULL = default stream).  On success
 * *out is a plan at level 0 with u^0 = phi(x_i). */
int tsfcde_plan(const tsfcde_problem *prob, void *d_workspace, size_t bytes, void *stream,
                tsfcde_plan_t *out);

/* Set the stored levels u^0..u^level from d_U ((level+1) x n, row-major,
 * device) and make `level` the current level (checkpoint resume; test
 * inputs).  0 <= level <= M. */
int tsfcde_set_state(tsfcde_plan_t plan, int64_t level, const double *d_U);

/* Advance one level j -> j+1 (Algorithm 2, one pass of its loop).
 * d_f: f(x_i, t_{j+sigma}) on the device (n values, any 8-byte alignment), or
 * NULL: then the problem's f callback is evaluated on the host at the plan's
 * nodes x_1..x_n and t_{j+sigma} and copied to the device (f = 0 when the
 * problem has no f callback).
 * d_u_out: optional device copy of u^{j+1} (n values) or NULL.
 * st: optional per-level statistics.  Returns TSFCDE_ENOCONV /
 * TSFCDE_EBREAKDOWN / TSFCDE_ENONFINITE / TSFCDE_EACCEPT with u^{j+1} set to
 * the last iterate and the level counted as done; TSFCDE_EDONE when all M
 * levels are done. */
int tsfcde_step(tsfcde_plan_t plan, const double *d_f, double *d_u_out, tsfcde_stats *st);

/* The time march of Algorithm 2 (its loop over j = level..M-1, each pass a
 * tsfcde_step): u^{j+1} from (3.3) for every remaining level.  d_F: device
 * array whose row j (stride ldF doubles, ldF >= n) holds f at t_{j+sigma} for
 * absolute level j, or NULL to take f from the problem's f callback (f = 0
 * without one).  d_U_out: optional device copy of U ((M+1) x n, row-major).
 * per_level: optional host array of M stats (entries of already-computed
 * levels are left untouched).  Stops after the first level that fails and
 * returns its code. */
int tsfcde_solve(tsfcde_plan_t plan, const double *d_F, int64_t ldF, double *d_U_out,
                 tsfcde_stats *per_level);

/* y = op x at level j (0 <= j < M) for op in TSFCDE_OP_*; device vectors of
 * n values, 16-byte aligned; d_x and d_y must not overlap the plan's
 * workspace. */
int tsfcde_apply(tsfcde_plan_t plan, int32_t op, int64_t j, const double *d_x, double *d_y);

/* Right-hand side g of (3.3) for level j from the stored levels u^0..u^j
 * (requires j <= current level) and f (device, or NULL for 0). */
int tsfcde_rhs(tsfcde_plan_t plan, int64_t j, const double *d_f, double *d_g);

/* WSGD weights omega_0..omega_n (Lemma 2) into d_w (n+1 doubles, device). */
int tsfcde_weights(tsfcde_plan_t plan, double *d_w);

/* Circulant spectra in natural frequency order as interleaved complex FP64:
 * TSFCDE_SPEC_EMBED: DFT_L of the embedding column of W_beta, L =
 *   tsfcde_embedding_length (the power of two >= 2n), k = 0..L/2 (L/2+1
 *   complex values);
 * TSFCDE_SPEC_STRANG: DFT_n of the Strang column of W_beta, k = 0..floor(n/2)
 *   (floor(n/2)+1 complex values).
 * DFT sign: lambda_k = sum_m c_m e^{-2 pi i mk/L}. */
int tsfcde_spectrum(tsfcde_plan_t plan, int32_t which, double *d_out);

/* Device pointer to the stored levels U, owned by the plan and valid until
 * tsfcde_destroy: M+1 rows of n values, row j = u^j, rows
 * tsfcde_history_ld(plan) doubles apart (n rounded up to even). */
const double *tsfcde_history(tsfcde_plan_t plan);
int64_t tsfcde_history_ld(tsfcde_plan_t plan);

/* t_{j+sigma} = (j + 1 - alpha/2) tau, the instant at which level j samples
 * gamma, d_+-, f (Lemma 1, Sec. 2.1); NaN for a NULL plan or j outside
 * 0..M-1. */
double tsfcde_level_time(tsfcde_plan_t plan, int64_t j);

/* The plan's interior nodes x_i = a + i h, i = 1..n, h = (b-a)/(n+1)
 * (Sec. 2.1), into the host array h_x of n doubles. */
int tsfcde_nodes(tsfcde_plan_t plan, double *h_x);

/* The fast history's fit (host only, no device work): for time order alpha,
 * M levels and relative tolerance tol, *terms = K exponentials rho_k (ratios)
 * with weights w_k and the cubic's coefficients poly[0..3], such that
 * c_m ~ sum_k w_k rho_k^m + sum_p poly[p] m^p for 2 <= m <= M-2 (the weights
 * of Lemma 1); *max_rel_err is the largest relative error met over those m
 * (against c_m from its integral form by Gauss-Legendre quadrature).  rho
 * and w (nullable) are written when K <= capacity.  Returns TSFCDE_OK when
 * the error is within tol, TSFCDE_EUNSUPPORTED otherwise, TSFCDE_EINVAL for
 * alpha outside (0, 1], M < 1 or tol <= 0. */
int tsfcde_history_soe_fit(double alpha, int64_t M, double tol, int32_t capacity, int32_t *terms, double *rho,
                           double *w, double *poly, double *max_rel_err);

/* Length L of the circulant embedding used for the Toeplitz products. */
int64_t tsfcde_embedding_length(tsfcde_plan_t plan);

/* Current level j (u^0..u^j are stored). */
int64_t tsfcde_level(tsfcde_plan_t plan);

/* Per-kernel timing with HIP events recorded on the plan's stream around
 * every launch of one kernel class: 0 = history sum, 1 = FFT column passes,
 * 2 = middle passes of the Toeplitz products (row FFTs with the embedding
 * symbol multiply), 3 = whole Krylov iteration chunks, 4 = middle passes of
 * the preconditioner solves (row FFTs with the Strang symbol divide), 5 =
 * fused column passes (preconditioner inverse + product forward).
 * enable > 0 starts recording and clears the totals: the events ride on every
 * enable-th launch of the class (1 = every launch; a launch that carries
 * events costs the stream a few microseconds of idle time, so a sample keeps
 * throughput measurements honest).  enable = 0 stops; enable < 0 is
 * TSFCDE_EINVAL.  tsfcde_profile_read synchronizes the stream and returns the
 * number of recorded (sampled) launches and their summed duration in
 * milliseconds; tsfcde_profile_issued returns how many launches of the class
 * were issued, sampled or not, since recording started. */
int tsfcde_profile(tsfcde_plan_t plan, int32_t kernel_class, int32_t enable);
int tsfcde_profile_read(tsfcde_plan_t plan, int32_t kernel_class, int64_t *launches,
                        double *milliseconds);
int tsfcde_profile_issued(tsfcde_plan_t plan, int32_t kernel_class, int64_t *issued);

/* Release the plan (host state only; the caller frees the workspace). */
int tsfcde_destroy(tsfcde_plan_t plan);

/* ---- allocation-free operator application ----------------------------
 * For callers that cannot allocate device or pinned memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * y = op x at level j of `prob`, exactly what tsfcde_plan(prob) followed by
 * tsfcde_apply(plan, op, j, d_x, d_y) gives, with no plan and no workspace.
 * Every device buffer (twiddles, weights, spectra, transform buffers) lives
 * in one static device array of TSFCDE_NOALLOC_SCRATCH_BYTES bytes inside
 * the library, which each device holds from the first call on it until the
 * process ends; the call makes no hipMalloc, hipFree, hipHostMalloc or
 * hipMemset.  d_x, d_y: device vectors of n values, 16-byte aligned,
 * caller-owned.  stream: a hipStream_t (NULL = default stream); the work is
 * queued on it and the call returns without waiting (y is ready when the
 * stream reaches that point).  All calls on one device share the array:
 * calls that overlap on a device (other streams, other threads) race, and
 * each call overwrites what the last one left.  Errors: TSFCDE_EINVAL as in
 * tsfcde_plan / tsfcde_apply; TSFCDE_EUNSUPPORTED for n >
 * TSFCDE_NOALLOC_NMAX; TSFCDE_EDEVICE when the array's address cannot be
 * found. */
#define TSFCDE_NOALLOC_NMAX 32768
#define TSFCDE_NOALLOC_SCRATCH_BYTES 16777216
int tsfcde_apply_noalloc(const tsfcde_problem *prob, int32_t op, int64_t j, const double *d_x, double *d_y,
                         void *stream);

/* ---- batched form ----------------------------------------------------
 * Many independent instances of (1.1) (any n, alpha, beta, coefficients,
 * same M) advanced together.  Work runs as grouped launches: instances with
 * the same embedding length share each kernel launch (one workgroup row per
 * listed instance); each instance follows Algorithm 2 with its own CGS
 * recurrence, stops on its own convergence flag and then drops out of its
 * group's launches.  All instances use the general-n preconditioner path.
 * Results equal those of single-instance plans of the same problems. */
typedef struct tsfcde_batch_s *tsfcde_batch_t;

/* Workspace for `count` instances (all with the same M). */
int tsfcde_batch_workspace_bytes(const tsfcde_problem *probs, int32_t count, size_t *bytes);

/* Plan `count` independent instances of problem (1.1) (each one what
 * tsfcde_plan would make of it: Lemma 1 tables, Lemma 2 weights, the spectra
 * of Sec. 3.2) in one caller-owned, 256-byte aligned device workspace of at
 * least tsfcde_batch_workspace_bytes bytes, kept alive until
 * tsfcde_batch_destroy.  Solver options are taken per instance for rtol and
 * from probs[0] for maxit, warm_start and flags.  Every instance must have
 * precision TSFCDE_FP64 (TSFCDE_EUNSUPPORTED otherwise) and the same M
 * (TSFCDE_EINVAL). */
int tsfcde_plan_batch(const tsfcde_problem *probs, int32_t count, void *d_workspace, size_t bytes, void *stream,
                      tsfcde_batch_t *out);

/* Member i as a plan handle, for tsfcde_set_state / tsfcde_history /
 * tsfcde_apply; step the batch only with tsfcde_batch_step or
 * tsfcde_batch_solve (after tsfcde_set_state on every member,
 * tsfcde_batch_set_level re-synchronises). */
tsfcde_plan_t tsfcde_batch_member(tsfcde_batch_t batch, int32_t i);
int tsfcde_batch_set_level(tsfcde_batch_t batch, int64_t level);

/* Advance every instance one level (one pass of Algorithm 2's loop each).
 * d_f: host array of `count` device pointers (f at t_{j+sigma} of each
 * instance); an entry or the array may be NULL, and that instance's f then
 * comes from its f callback, as in tsfcde_step.  stats: `count` entries or
 * NULL.  Returns the first failing instance's code (all instances still
 * advance). */
int tsfcde_batch_step(tsfcde_batch_t batch, const double *const *d_f, tsfcde_stats *stats);

/* Every remaining level of every instance (Algorithm 2's loop to j = M - 1),
 * in one call.  Instances advance on their own: one whose level has passed
 * its acceptance check starts its next level while others still iterate, so
 * the slowest instance of a level delays none of the others.  The numbers are
 * those of calling tsfcde_batch_step level by level.
 * d_F: host array of `count` device pointers, entry i holding f of instance
 * i at level j (at t_{j+sigma}) in row j, at d_F[i] + j * ldF[i] for
 * j = 0..M-1 (rows before the batch's current level are not read); ldF:
 * host array of `count` row strides (>= that instance's n).  An entry, or
 * d_F itself, may be NULL: that instance's f then comes from its f callback.
 * stats: count * (M - level) entries, instance-major (entry
 * i * (M - level) + (j - level)), or NULL.  Returns TSFCDE_EDONE when no
 * level is left, TSFCDE_EINVAL for a missing ldF or a stride below n, and
 * otherwise the first failure of any instance and level (all levels of all
 * instances are still computed). */
int tsfcde_batch_solve(tsfcde_batch_t batch, const double *const *d_F, const int64_t *ldF, tsfcde_stats *stats);

int tsfcde_batch_destroy(tsfcde_batch_t batch);

/* Autotuned launch geometry.  Instances with the same embedding length L form
 * a group that shares every launch.  Unless probs[0].flags has
 * TSFCDE_FLAG_NO_TUNE, tsfcde_plan_batch times each group's middle pass (the
 * row FFTs of the products and preconditioner solves, Sec. 3.2) at 4 and at 8
 * values per lane on the group's own buffers and keeps the faster; choices
 * are cached for the process by (row length, rows, instances) and, when the
 * environment variable TSFCDE_TUNE_CACHE names a file, in that file, which a
 * later process reads before tuning.  Different values per lane change the
 * FFT's rounding, not its result beyond it.
 * tsfcde_batch_group_count: number of groups (or TSFCDE_EINVAL).
 * tsfcde_batch_group_info: group g's L, member count and chosen values per
 * lane (each output nullable). */
int tsfcde_batch_group_count(tsfcde_batch_t batch);
int tsfcde_batch_group_info(tsfcde_batch_t batch, int32_t g, int64_t *L, int32_t *members, int32_t *values_per_lane);

/* ---- learned warm start ----------------------------------------------
 * A four-layer 1-D convolutional network (7 -> 32 -> 32 -> 32 -> 1 channels,
 * width 5, zero padding, tanh after the first three) predicts level j+1 from
 * levels j, j-1, j-2 as a correction to quadratic extrapolation in t:
 *   x0 = 3(u^j - u^{j-1}) + u^{j-2} + y * e2
 * (smooth, and zero where u is fixed in time, as at the Dirichlet boundary),
 * with y the network output for the channels (e1/s, e2/s, alpha, beta,
 * asinh q_gamma, log1p q_+, log1p q_-), e1 = u^j - u^{j-1},
 * e2 = u^j - 2u^{j-1} + u^{j-2}, s = RMS(e2) (1 if e2 = 0), and the level
 * coefficients q_gamma = sigma gamma_j / (h eta_j),
 * q_+- = sigma D_+-,j h^-beta / eta_j (the terms of sigma L_j in (3.3)
 * relative to eta_j).  Weights are bfloat16 (rounded from FP32 master
 * weights), everything else FP32; s and x0 are FP64.  Parameters form one
 * FP32 vector, layer by layer W[c_out][c_in][5] then b[c_out]. */
typedef struct tsfcde_net_s *tsfcde_net_t;

typedef struct tsfcde_net_sample {
    const double *u_next;   /* u^{j+1} on the device (training target) or NULL */
    const double *u0, *u1, *u2; /* u^j, u^{j-1}, u^{j-2} on the device       */
    float feat[5];          /* alpha, beta, asinh q_gamma, log1p q_+, log1p q_- */
    float pad;
} tsfcde_net_sample;

/* Number of FP32 parameters (11617). */
int32_t tsfcde_net_param_count(void);

/* Device workspace of a network able to take batches of up to max_batch
 * samples of up to max_points = batch * n grid points in all. */
int tsfcde_net_workspace_bytes(int64_t max_points, int32_t max_batch, size_t *bytes);

/* Network in a caller-owned, 256-byte aligned device workspace, all
 * parameters zero (so that, before training, x0 is the extrapolation). */
int tsfcde_net_create(void *d_workspace, size_t bytes, int64_t max_points, int32_t max_batch, void *stream,
                      tsfcde_net_t *out);

/* Copy the FP32 master parameters in (host array of
 * tsfcde_net_param_count() floats; resets the optimiser) or out. */
int tsfcde_net_set_params(tsfcde_net_t net, const float *h_params);
int tsfcde_net_get_params(tsfcde_net_t net, float *h_params);

/* Channels 2..6 of level j of a plan (the values a plan with TSFCDE_WS_NET
 * uses, so that training samples and inference agree). */
int tsfcde_level_features(tsfcde_plan_t plan, int64_t j, float *h_feat5);

/* One training step on `count` samples of n points (every u_next set):
 * loss = mean over samples of the relative error of the correction,
 * sum_p (y_p e2_p - d_p)^2 / (sum_p d_p^2 + n 1e-12 s^2), with
 * d = u^{j+1} - 3(u^j - u^{j-1}) - u^{j-2} (zero correction scores 1), its
 * gradient by the network's backward kernels, then one Adam update (lr; beta1 = 0.9,
 * beta2 = 0.999, eps = 1e-8, bias-corrected).  h_samples: host array.
 * loss_out (host, nullable) receives the loss before the update.
 * h_grad_out (host, nullable; param_count floats) receives the gradient; with
 * lr == 0 no update is made.  Synchronises the stream. */
int tsfcde_net_train_step(tsfcde_net_t net, const tsfcde_net_sample *h_samples, int32_t count, int64_t n, float lr,
                          double *loss_out, float *h_grad_out);

/* Prediction x0 (device, n doubles) for one sample (u_next ignored). */
int tsfcde_net_predict(tsfcde_net_t net, const tsfcde_net_sample *h_sample, int64_t n, double *d_x0);

/* Use `net` for TSFCDE_WS_NET guesses of this plan (n <= the net's
 * max_points; the net must outlive its use and run on the plan's stream).
 * NULL detaches it (levels then take the previous-level guess). */
int tsfcde_plan_set_net(tsfcde_plan_t plan, tsfcde_net_t net);

int tsfcde_net_destroy(tsfcde_net_t net);

/* Static description of a status code. */
const char *tsfcde_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* TSFCDE_H */
