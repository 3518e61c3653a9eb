/*
 * tsfcde3d.h -- C ABI of the MI355X (gfx950) time-level solver for the
 * time-space fractional convection-diffusion equation in three space
 * dimensions, the other extension that Sec. 5 of Gu, Huang, Ji, Carpentieri
 * and Alikhanov (arXiv:1603.00279) names as future work:
 *
 *   D_t^alpha u = sum over the axes s in {x, y, z} of
 *                 [ g_s(t) u_s + dp_s(t) D_{lo_s+}^{beta_s} u + dm_s(t) D_{hi_s-}^{beta_s} u ]
 *                 + f(x, y, z, t)
 *   on the box [lo_x, hi_x] x [lo_y, hi_y] x [lo_z, hi_z], u = 0 on its
 *   boundary, u(x, y, z, 0) = phi(x, y, z).
 *
 * The scheme is the two-dimensional one of tsfcde2d.h with a third axis:
 * L2-1sigma in time (Lemma 1, (3.1)) with gamma, d and f sampled at
 * t_{j+sigma}; in space the Kronecker sum of the three one-dimensional
 * operators of (3.2)-(3.3) (WSGD differences, Lemma 2, and central convection
 * differences), so each level solves
 *   (eta_j I - sigma L) u^{j+1} = (eta_j I + (1-sigma) L) u^j - history + f,
 * a system with three-level block-Toeplitz structure, by CGS right-
 * preconditioned with the three-level circulant analogue of (3.7),
 *   P = eta_j I - sigma (s(L_x) (x) I (x) I + I (x) s(L_y) (x) I + I (x) I (x) s(L_z)),
 * applied through three-dimensional FFTs; each product with L runs along each
 * axis through a length-2n circulant embedding (Sec. 3.2).
 *
 * Layout: a level is an nx x ny x nz array of FP64 values,
 * u[(i*ny + k)*nz + l] = u(x_{i+1}, y_{k+1}, z_{l+1}) (z fastest), with
 * h_s = (hi_s - lo_s)/(n_s + 1).  Status codes, operator codes (TSFCDE_OP_*),
 * the coefficient callback type and tsfcde_stats are those of tsfcde.h.
 * Device pointers are plain HIP device addresses; a plan is bound to one
 * device and one stream and is not thread-safe.
 */
#ifndef TSFCDE3D_H
#define TSFCDE3D_H

#include "tsfcde.h"

#ifdef __cplusplus
extern "C" {
#endif

/* phi(x, y, z) and f(x, y, z, t) of the three-dimensional problem */
typedef double (*tsfcde3d_ic_fn)(double x, double y, double z, void *user);
typedef double (*tsfcde3d_src_fn)(double x, double y, double z, double t, void *user);

/* Problem statement plus solver options; per-axis entries in the order
 * x, y, z.  The caller owns it; the plan copies what it needs during
 * tsfcde3d_plan. */
typedef struct tsfcde3d_problem {
    double alpha;           /* time order, 0 < alpha <= 1                      */
    double beta[3];         /* space orders, 1 < beta <= 2                     */
    double lo[3], hi[3];    /* the box, lo < hi on every axis                  */
    double T;               /* final time, T > 0                               */
    int64_t n[3];           /* interior unknowns per axis: powers of two in
                               [16, 2048], N at most 2^30 (TSFCDE_EUNSUPPORTED
                               otherwise)                                      */
    int64_t M;              /* time steps, M >= 1                              */
    /* gamma_s, d+_s, d-_s at t: host callbacks, called during tsfcde3d_plan
     * at t_{j+sigma}, j = 0..M-1; none may be NULL; the d's must be >= 0 */
    tsfcde_coef_fn gamma[3], dplus[3], dminus[3];
    void *coef_user;
    tsfcde3d_ic_fn phi;     /* u^0 at the nodes during tsfcde3d_plan; NULL: 0   */
    void *phi_user;
    tsfcde3d_src_fn f;      /* f at the nodes and t_{j+sigma} for levels whose
                               device source is NULL; NULL: f = 0 there        */
    void *f_user;
    double rtol;            /* CGS stop |r| <= rtol |g| (<= 0: 1e-10)          */
    int32_t maxit;          /* CGS iterations per level (<= 0: 500)            */
    int32_t warm_start;     /* CGS initial guess, as in tsfcde2d_problem:
                               TSFCDE_WS_ZERO, _PREV or _EXTRAP              */
} tsfcde3d_problem;

typedef struct tsfcde3d_plan_s *tsfcde3d_plan_t;

/* Device workspace a plan needs, in bytes (about (M + 23) N doubles for
 * N = nx ny nz).  TSFCDE_EINVAL / TSFCDE_EUNSUPPORTED for a problem
 * tsfcde3d_plan would refuse. */
int tsfcde3d_workspace_bytes(const tsfcde3d_problem *prob, size_t *bytes);

/* Validate, sample the coefficients at t_{j+sigma}, build the L2-1sigma
 * tables (Lemma 1), the WSGD weights of the three axes (Lemma 2) and the
 * spectra of their circulant embeddings and Strang circulants (Sec. 3.2) on
 * the device.  d_workspace: caller-owned, 256-byte aligned, at least
 * tsfcde3d_workspace_bytes bytes, alive until tsfcde3d_destroy.  stream: a
 * hipStream_t (NULL = default).  On success *out is a plan at level 0 with
 * u^0 = phi at the nodes.  Errors: TSFCDE_EINVAL (bad argument, NULL
 * coefficient callback, negative or non-finite coefficient),
 * TSFCDE_EUNSUPPORTED (sizes), TSFCDE_ENOMEM (workspace too small),
 * TSFCDE_EDEVICE. */
int tsfcde3d_plan(const tsfcde3d_problem *prob, void *d_workspace, size_t bytes, void *stream,
                  tsfcde3d_plan_t *out);

/* Levels u^0..u^level from d_U ((level+1) x N, device); the next step
 * computes level+1.  TSFCDE_EINVAL for level outside [0, M-1]. */
int tsfcde3d_set_state(tsfcde3d_plan_t plan, int64_t level, const double *d_U);

/* One level (Algorithm 2's loop body): g = B u^j - history + f, then PCGS
 * on A u^{j+1} = g from the initial guess (warm_start), accepted as in tsfcde2d_step (true
 * residual within rtol |g| or normwise backward error at most 1e-13, |A|
 * bounded above by eta + sigma sum over the three axes of |gamma|/h +
 * (d+ + d-) h^-beta sum_k |omega_k|, at most 3 restarts).  d_f: f at
 * t_{j+sigma} on the nodes (N values, device) or NULL (the f callback).
 * d_u_out: device copy of u^{j+1} (may be NULL).  stats may be NULL.  Returns
 * TSFCDE_OK, TSFCDE_ENOCONV, TSFCDE_EBREAKDOWN, TSFCDE_ENONFINITE,
 * TSFCDE_EACCEPT (u^{j+1} and stats still set), TSFCDE_EDONE after level M,
 * TSFCDE_EDEVICE. */
int tsfcde3d_step(tsfcde3d_plan_t plan, const double *d_f, double *d_u_out, tsfcde_stats *stats);

/* Every remaining level.  d_F: device rows of N values, row j at
 * d_F + j*ldF for levels j = 0..M-1 (or NULL: the f callback), ldF >= N;
 * d_U_out: optional device array of (M+1) x N for the history; stats:
 * M - level entries or NULL.  Returns the first failing level's code. */
int tsfcde3d_solve(tsfcde3d_plan_t plan, const double *d_F, int64_t ldF, double *d_U_out, tsfcde_stats *stats);

/* y = op x at level j: TSFCDE_OP_A (eta I - sigma L), TSFCDE_OP_B
 * (eta I + (1-sigma) L) or TSFCDE_OP_PINV (P^{-1} of the three-level
 * circulant Strang preconditioner).  d_x, d_y: N device values (distinct).
 * Queued on the plan's stream without waiting. */
int tsfcde3d_apply(tsfcde3d_plan_t plan, int32_t op, int64_t j, const double *d_x, double *d_y);

/* Host copies of the interior nodes of each axis (any pointer may be NULL). */
int tsfcde3d_nodes(tsfcde3d_plan_t plan, double *h_x, double *h_y, double *h_z);
/* t_{j+sigma} = (j + sigma) tau (NaN for a NULL plan or j outside [0, M-1]). */
double tsfcde3d_level_time(tsfcde3d_plan_t plan, int64_t j);
/* The next level to compute (0..M), or -1 for a NULL plan. */
int64_t tsfcde3d_level(tsfcde3d_plan_t plan);
/* Device address of the stored levels, (M+1) x N (plan-owned). */
const double *tsfcde3d_history(tsfcde3d_plan_t plan);

int tsfcde3d_destroy(tsfcde3d_plan_t plan);

#ifdef __cplusplus
}
#endif
#endif
