/*
 * tsfcde2d.h -- C ABI of the MI355X (gfx950) time-level solver for the
 * time-space fractional convection-diffusion equation in two space
 * dimensions, the extension that Sec. 5 of Gu, Huang, Ji, Carpentieri and
 * Alikhanov (arXiv:1603.00279) names as future work:
 *
 *   D_t^alpha u = gx(t) u_x + gy(t) u_y
 *               + dxp(t) aD_x^bx u + dxm(t) xD_b^bx u
 *               + dyp(t) cD_y^by u + dym(t) yD_d^by u + f(x, y, t)
 *   on [a,b] x [c,d],  u = 0 on the boundary,  u(x, y, 0) = phi(x, y).
 *
 * The scheme is the paper's, one axis at a time: L2-1sigma in time (Lemma 1,
 * (3.1)) with gamma, d and f sampled at t_{j+sigma}; in space the Kronecker
 * sum L = L_x (x) I + I (x) L_y of the one-dimensional operators of
 * (3.2)-(3.3) (WSGD differences, Lemma 2, and central convection
 * differences), so each level solves
 *   (eta_j I - sigma L) u^{j+1} = (eta_j I + (1-sigma) L) u^j - history + f,
 * a system with block-Toeplitz-Toeplitz-block structure.  It is solved by
 * CGS (Barrett et al., Templates) right-preconditioned by the
 * block-circulant-with-circulant-blocks analogue of (3.7),
 *   P = eta_j I - sigma (s(L_x) (x) I + I (x) s(L_y))
 * with Strang's circulants s(.), applied through two-dimensional FFTs; each
 * product with L runs along each axis through a length-2n circulant
 * embedding (Sec. 3.2).
 *
 * Layout: a level is an nx x ny array of FP64 values, u[i*ny + k] =
 * u(x_{i+1}, y_{k+1}) (x along the slow index), with hx = (b-a)/(nx+1),
 * hy = (d-c)/(ny+1).  Status codes, operator codes (TSFCDE_OP_*), the
 * coefficient callback type and tsfcde_stats are those of tsfcde.h.  Device
 * pointers are plain HIP device addresses; a plan is bound to one device and
 * one stream and is not thread-safe.
 */
#ifndef TSFCDE2D_H
#define TSFCDE2D_H

#include "tsfcde.h"

#ifdef __cplusplus
extern "C" {
#endif

/* phi(x, y) and f(x, y, t) of the two-dimensional problem */
typedef double (*tsfcde2d_ic_fn)(double x, double y, void *user);
typedef double (*tsfcde2d_src_fn)(double x, double y, double t, void *user);

/* Problem statement plus solver options.  The caller owns it; the plan
 * copies what it needs during tsfcde2d_plan. */
typedef struct tsfcde2d_problem {
    double alpha;          /* time order, 0 < alpha <= 1                      */
    double beta_x, beta_y; /* space orders, 1 < beta <= 2                     */
    double a, b, c, d;     /* [a,b] x [c,d], a < b, c < d                     */
    double T;              /* final time, T > 0                               */
    int64_t nx, ny;        /* interior unknowns per axis: powers of two in
                              [16, 2048] (TSFCDE_EUNSUPPORTED otherwise)       */
    int64_t M;             /* time steps, M >= 1                              */
    /* gx, gy, dxp, dxm, dyp, dym at t: host callbacks, called during
     * tsfcde2d_plan at t_{j+sigma}, j = 0..M-1; none may be NULL; the d's
     * must be >= 0 */
    tsfcde_coef_fn gamma_x, gamma_y, dplus_x, dminus_x, dplus_y, dminus_y;
    void *coef_user;
    tsfcde2d_ic_fn phi;    /* u^0 at the nodes during tsfcde2d_plan; NULL: 0   */
    void *phi_user;
    tsfcde2d_src_fn f;     /* f at the nodes and t_{j+sigma} for levels whose
                              device source is NULL; NULL: f = 0 there        */
    void *f_user;
    double rtol;           /* CGS stop |r| <= rtol |g| (<= 0: 1e-10)          */
    int32_t maxit;         /* CGS iterations per level (<= 0: 500)            */
    int32_t warm_start;    /* CGS initial guess of each level: TSFCDE_WS_ZERO
                              (as in Sec. 4), TSFCDE_WS_PREV (u^j) or
                              TSFCDE_WS_EXTRAP (3u^j - 3u^{j-1} + u^{j-2};
                              u^j at level 1, 0 at level 0); a nonzero guess
                              goes through the acceptance test first and CGS
                              restarts from it when it fails (EINVAL for
                              other values)                                   */
} tsfcde2d_problem;

typedef struct tsfcde2d_plan_s *tsfcde2d_plan_t;

/* Device workspace a plan needs, in bytes (about (M + 23) nx ny doubles).
 * TSFCDE_EINVAL / TSFCDE_EUNSUPPORTED for a problem tsfcde2d_plan would
 * refuse. */
int tsfcde2d_workspace_bytes(const tsfcde2d_problem *prob, size_t *bytes);

/* Validate, sample the coefficients at t_{j+sigma}, build the L2-1sigma
 * tables (Lemma 1), the WSGD weights of both axes (Lemma 2) and the spectra
 * of their circulant embeddings and Strang circulants (Sec. 3.2) on the
 * device.  d_workspace: caller-owned, 256-byte aligned, at least
 * tsfcde2d_workspace_bytes bytes, alive until tsfcde2d_destroy.  stream: a
 * hipStream_t (NULL = default).  On success *out is a plan at level 0 with
 * u^0 = phi at the nodes.  Errors: TSFCDE_EINVAL (bad argument, NULL
 * coefficient callback, negative or non-finite coefficient),
 * TSFCDE_EUNSUPPORTED (sizes), TSFCDE_ENOMEM (workspace too small),
 * TSFCDE_EDEVICE. */
int tsfcde2d_plan(const tsfcde2d_problem *prob, void *d_workspace, size_t bytes, void *stream,
                  tsfcde2d_plan_t *out);

/* Levels u^0..u^level from d_U ((level+1) x nx*ny, device); the next step
 * computes level+1.  TSFCDE_EINVAL for level outside [0, M-1]. */
int tsfcde2d_set_state(tsfcde2d_plan_t plan, int64_t level, const double *d_U);

/* One level (Algorithm 2's loop body): g = B u^j - history + f, then PCGS
 * on A u^{j+1} = g from the initial guess (warm_start); the level is accepted when the true
 * residual is within rtol |g| or the normwise backward error
 * |g - A u| / (|A| |u| + |g|) is at most 1e-13 (|A| bounded above by
 * eta + sigma sum over the axes of |gamma|/h + (d+ + d-) h^-beta
 * sum_k |omega_k|), after at most 3 restarts of CGS from u.
 * d_f: f at t_{j+sigma} on the nodes (nx*ny, device) or NULL (the f
 * callback).  d_u_out: device copy of u^{j+1} (may be NULL).  stats may be
 * NULL.  Returns TSFCDE_OK, TSFCDE_ENOCONV, TSFCDE_EBREAKDOWN,
 * TSFCDE_ENONFINITE, TSFCDE_EACCEPT (u^{j+1} and stats still set),
 * TSFCDE_EDONE after level M, TSFCDE_EDEVICE. */
int tsfcde2d_step(tsfcde2d_plan_t plan, const double *d_f, double *d_u_out, tsfcde_stats *stats);

/* Every remaining level.  d_F: device rows of nx*ny values, row j at
 * d_F + j*ldF for levels j = 0..M-1 (or NULL: the f callback), ldF >= nx*ny;
 * d_U_out: optional device array of (M+1) x nx*ny for the history; stats:
 * M - level entries or NULL.  Returns the first failing level's code. */
int tsfcde2d_solve(tsfcde2d_plan_t plan, const double *d_F, int64_t ldF, double *d_U_out, tsfcde_stats *stats);

/* y = op x at level j: TSFCDE_OP_A (eta I - sigma L), TSFCDE_OP_B
 * (eta I + (1-sigma) L) or TSFCDE_OP_PINV (P^{-1} of the BCCB Strang
 * preconditioner).  d_x, d_y: nx*ny device values (distinct).  Queued on the
 * plan's stream without waiting. */
int tsfcde2d_apply(tsfcde2d_plan_t plan, int32_t op, int64_t j, const double *d_x, double *d_y);

/* Host copies of the interior nodes x_1..x_nx and y_1..y_ny. */
int tsfcde2d_nodes(tsfcde2d_plan_t plan, double *h_x, double *h_y);
/* t_{j+sigma} = (j + sigma) tau, where level j samples the coefficients and f
 * (NaN for a NULL plan or j outside [0, M-1]). */
double tsfcde2d_level_time(tsfcde2d_plan_t plan, int64_t j);
/* The next level to compute (0..M), or -1 for a NULL plan. */
int64_t tsfcde2d_level(tsfcde2d_plan_t plan);
/* Device address of the stored levels, (M+1) x nx*ny (plan-owned). */
const double *tsfcde2d_history(tsfcde2d_plan_t plan);

int tsfcde2d_destroy(tsfcde2d_plan_t plan);

#ifdef __cplusplus
}
#endif
#endif
