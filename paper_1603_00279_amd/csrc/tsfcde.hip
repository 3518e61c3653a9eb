// tsfcde.hip -- host runtime and C ABI of the TSFCDE time-level solver.
//
// One time level (Algorithm 2 of Gu et al., arXiv:1603.00279):
//   1. history H = kappa * sum_{s<j} c_{j-s}^(j) (u^{s+1} - u^s)   (Lemma 1, (3.3))
//   2. y = A u^j through the circulant embedding, fused with
//      g = (eta/sigma) u^j - ((1-sigma)/sigma) y - H + f  (= B u^j - H + f),
//      r0 = g - A x0, rt = r0                                  ((3.1), (3.3))
//   3. preconditioned CGS on A u^{j+1} = g with the Strang circulant P (3.7),
//      12 kernels per iteration, device-resident scalars, convergence flag
//      polled between chunks of iterations.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/tsfcde.h"
#include "kernels.hpp"
#include "warmnet.hpp"

using namespace tsf;

namespace {

constexpr int PMAX_LOG2 = 12;  // longest in-LDS transform: 4096
constexpr int64_t NMAX = int64_t(1) << 24;
constexpr int64_t PARTIAL_SLOTS = 16384;  // doubles per reduction site
constexpr int NSITES = 4;
constexpr int NPROF = 6;  // profiling classes, see tsfcde_profile
// CGS's recursive residual can drift far from the true one after a
// near-breakdown (a tiny rt . vhat in an early step), so a converged level is
// accepted only when its normwise backward error is at most BW_TOL; otherwise
// CGS restarts from x.
constexpr double BW_TOL = 1e-13;

struct RT {  // real transform of length L = 2N as an R x C complex transform
    int64_t L = 0, N = 0, R = 0, C = 0;
    Tw2 tw{};
    double2 *lo = nullptr, *hi = nullptr;
    int64_t nlo = 0, nhi = 0;
    int shift = 0;
};

int ilog2(int64_t v) {
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

// L = 2N real values as an R x C complex transform.
void rt_init(RT &rt, int64_t L, int64_t R) {
    rt.L = L;
    rt.N = L / 2;
    rt.R = R;
    rt.C = rt.N / R;
    rt.shift = (ilog2(L) + 1) / 2;
    rt.nlo = int64_t(1) << rt.shift;
    rt.nhi = (L >> rt.shift) + 1;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// Toeplitz products: L = next power of two >= 2n (a circulant embedding of
// any length >= 2n is exact, and its W^T part has the conjugate spectrum),
// N = L/2 = R_A x C with R_A = 2^floor(log2(N)/2).
// Power-of-two n >= 16: the Strang preconditioner is an n-point real
// transform, N = n/2 = R_P x C with R_P = R_A/2 and the same C, so its inverse
// column pass and the next product's forward column pass share columns
// (k_fuse).  Any other n: the preconditioner's inverse circulant is built per
// level with Bluestein's chirp-z DFT (complex transform B of length L) and
// applied as a Toeplitz product through the same embedding as A.
bool rt_setup(RT &A, RT &P, RT &B, int64_t n, bool force_general = false) {
    const int64_t L = int64_t(1) << ilog2(2 * n);
    const int64_t NA = L / 2;
    const int64_t RA = int64_t(1) << (ilog2(NA) / 2);
    rt_init(A, L, RA);
    const bool p2 = is_pow2(n) && n >= 16 && !force_general;
    if (p2) {
        rt_init(P, n, RA / 2);
    } else {
        const int64_t NB = L;
        rt_init(B, 2 * NB, int64_t(1) << (ilog2(NB) / 2));
    }
    return p2;
}

struct Layout {
    size_t off_U, off_vec, off_v32, off_tmp, off_w, off_g0, off_cbase, off_buf, off_bufP, off_specA, off_specP, off_tw, off_tw2A,
        off_tw2P, off_part, off_sc, off_bufB, off_Bhat, off_chirp, off_Ls, off_wv, off_Wt, off_specPj, off_tw2B,
        off_buf32, off_bufP32, off_specA32, off_specP32, off_specPj32, off_gsf, off_soe, total;
};

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int NVEC = 11 + HB;  // H g r rt u p q phat vhat uhat fbuf, then the HB block sums Hq
constexpr int NV32 = 9;   // FP32 inner solve: r rt u p q phat vhat uhat d

// internal row stride: n rounded up to even, so every row starts 16-byte aligned
int64_t ld_of(int64_t n) { return n + (n & 1); }

Layout layout_for(int64_t n, int64_t M, const RT &A, const RT &P, const RT &B, bool p2, bool fp32,
                  bool gsf = false, int soe_terms = -1) {
    const int64_t ld = ld_of(n);
    Layout l{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = al(o + bytes);
        return at;
    };
    l.off_U = take(sizeof(double) * (size_t)(M + 1) * ld);
    l.off_vec = take(sizeof(double) * (size_t)NVEC * ld);
    l.off_v32 = take(sizeof(float) * (size_t)(fp32 ? NV32 * ld : 0));
    l.off_tmp = take(sizeof(double) * (size_t)std::max<int64_t>(A.L, n));
    l.off_w = take(sizeof(double) * (size_t)(n + 2));
    l.off_g0 = take(sizeof(double) * (size_t)(n + 2));
    l.off_cbase = take(sizeof(double) * (size_t)(M + 2));
    l.off_buf = take(sizeof(double2) * (size_t)A.N);
    l.off_bufP = take(sizeof(double2) * (size_t)(p2 ? P.N : 0));
    l.off_specA = take(sizeof(double2) * (size_t)A.N);
    l.off_specP = take(sizeof(double2) * (size_t)(p2 ? P.N : 0));
    l.off_tw = take(sizeof(double2) * (size_t)((int64_t(1) << (PMAX_LOG2 + 1)) - 2));
    l.off_tw2A = take(sizeof(double2) * (size_t)(A.nlo + A.nhi));
    l.off_tw2P = take(sizeof(double2) * (size_t)(p2 ? P.nlo + P.nhi : 0));
    l.off_part = take(sizeof(double) * (size_t)PARTIAL_SLOTS * NSITES);
    l.off_sc = take(sizeof(DevScalars));
    const size_t nb = p2 ? 0 : (size_t)B.N, nn = p2 ? 0 : (size_t)n;
    l.off_bufB = take(sizeof(double2) * nb);
    l.off_Bhat = take(sizeof(double2) * nb);
    l.off_chirp = take(sizeof(double2) * nn);
    l.off_Ls = take(sizeof(double2) * nn);
    l.off_wv = take(sizeof(double2) * nn);
    l.off_Wt = take(sizeof(double2) * nn);
    l.off_specPj = take(sizeof(double2) * (p2 ? 0 : (size_t)A.N));
    l.off_tw2B = take(sizeof(double2) * (p2 ? 0 : (size_t)(B.nlo + B.nhi)));
    // FP32 copies of the inner solve's transform buffers and spectra
    const size_t f = fp32 ? 1 : 0;
    l.off_buf32 = take(sizeof(float2) * f * (size_t)A.N);
    l.off_bufP32 = take(sizeof(float2) * f * (size_t)(p2 ? P.N : 0));
    l.off_specA32 = take(sizeof(float2) * f * (size_t)A.N);
    l.off_specP32 = take(sizeof(float2) * f * (size_t)(p2 ? P.N : 0));
    l.off_specPj32 = take(sizeof(float2) * f * (size_t)(p2 ? 0 : A.N));
    // Gohberg-Semencul path: x = A^-1 e_1, y = A^-1 e_n and the spectra of
    // the four triangular factors
    l.off_gsf = take(gsf ? 2 * sizeof(double) * (size_t)ld + 4 * al(sizeof(double2) * (size_t)A.N) : 0);
    // fast history: K + 4 recursion vectors, then the K weights and K ratios
    l.off_soe = take(soe_terms >= 0 ? sizeof(double) * ((size_t)(soe_terms + 4) * ld + 2 * (size_t)soe_terms) : 0);
    l.total = o;
    return l;
}

int validate(const tsfcde_problem *p) {
    if (!p) return TSFCDE_EINVAL;
    if (!(p->alpha > 0.0 && p->alpha <= 1.0)) return TSFCDE_EINVAL;
    if (!(p->beta > 1.0 && p->beta <= 2.0)) return TSFCDE_EINVAL;
    if (!(p->b > p->a) || !std::isfinite(p->a) || !std::isfinite(p->b)) return TSFCDE_EINVAL;
    if (!(p->T > 0.0) || !std::isfinite(p->T)) return TSFCDE_EINVAL;
    if (p->n < 2 || p->M < 1) return TSFCDE_EINVAL;
    if ((!p->gamma && !p->gamma_at) || (!p->dplus && !p->dplus_at) || (!p->dminus && !p->dminus_at))
        return TSFCDE_EINVAL;
    if (p->precision != TSFCDE_FP64 && p->precision != TSFCDE_FP32_REFINED) return TSFCDE_EINVAL;
    if (p->warm_start != TSFCDE_WS_ZERO && p->warm_start != TSFCDE_WS_PREV && p->warm_start != TSFCDE_WS_EXTRAP &&
        p->warm_start != TSFCDE_WS_NET)
        return TSFCDE_EINVAL;
    if (!std::isfinite(p->rtol)) return TSFCDE_EINVAL;
    if (p->n < 4 || p->n > (is_pow2(p->n) ? NMAX : NMAX / 2)) return TSFCDE_EUNSUPPORTED;
    if (p->krylov != TSFCDE_KRYLOV_CGS && p->krylov != TSFCDE_KRYLOV_BICGSTAB) return TSFCDE_EINVAL;
    if (!(p->history_tol >= 0.0 && p->history_tol <= 1e-2)) return TSFCDE_EINVAL;
    if (p->preconditioner != TSFCDE_PREC_STRANG && p->preconditioner != TSFCDE_PREC_TCHAN) return TSFCDE_EINVAL;
    if ((p->flags & TSFCDE_FLAG_CONSTANT_GSF) && p->precision != TSFCDE_FP64) return TSFCDE_EUNSUPPORTED;
    return TSFCDE_OK;
}

struct ProfRec {
    bool on = false;
    int64_t period = 1;  // events ride on every period-th launch of the class
    int64_t issued = 0;  // launches of the class since profiling was switched on
    int64_t launches = 0;
    double ms = 0.0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

}  // namespace

struct tsfcde_plan_s {
    int device = 0;
    hipStream_t stream = nullptr;
    double alpha, beta, a, b, T, h, tau, sigma, kappa, hb;
    int64_t n, M, ldn, level = 0;
    bool p2 = true;      // power-of-two fast path (fused preconditioner)
    int64_t pj_level = -1;  // level whose inverse-Strang spectrum specPj holds
    double rtol;
    int maxit, warm, flags;
    std::vector<double> gam, dp, dm, eta, cbase, clast;
    RT A, P, B;
    Layout lay;
    char *ws;
    double *U, *H, *g, *r, *rt, *u, *p, *q, *phat, *vhat, *uhat, *fbuf, *tmp, *w, *g0, *cb, *part, *Hq;
    // history partial sums: Hq holds the HB block sums Q of block hist_block
    // (the first level's complete), H the catch-up P of a later level; the
    // next block's sweep runs on the side stream `hs` while the last level of
    // the current block is solved
    hipStream_t hs = nullptr;
    hipEvent_t ev_main = nullptr, ev_hist = nullptr;
    int64_t hist_block = -1;    // block whose sums Hq holds (or is being summed into on hs)
    bool hist_pending = false;  // that sweep was queued on hs and not yet waited for
    double2 *buf, *bufP, *specA, *specP, *tw_all;
    double2 *bufB, *Bhat, *chirp, *Ls, *wv, *Wt, *specPj;
    DevScalars *sc;
    DevScalars *h_sc = nullptr;  // pinned mirror for polling
    int last_iters = 8;
    // FP32-refined form: FP32-stored inner CGS inside an FP64 refinement loop
    bool fp32 = false;
    std::vector<double> kbound;  // per level: bound on |A| / eta (Remark 3.1)
    std::vector<double> anorm;   // per level: upper bound on |A|_2 (backward error)
    float *r32, *rt32, *u32, *p32, *q32, *phat32, *vhat32, *uhat32, *d32;
    float2 *buf32, *bufP32, *specA32, *specP32, *specPj32;
    int last_inner = 8;
    tsfcde_net_s *net = nullptr;  // learned warm start (TSFCDE_WS_NET)
    tsfcde_src_fn fcb = nullptr;  // f(x, t) for levels stepped without a device source
    void *fuser = nullptr;
    double *h_f = nullptr;        // pinned staging of those f values (n doubles)
    // a plan made for one level only (tsfcde_apply_noalloc): that level's
    // scalars stand in for the per-level tables
    bool one_level = false;
    double one_eta = 0.0, one_gam = 0.0, one_dp = 0.0, one_dm = 0.0;
    // constant coefficients (TSFCDE_FLAG_CONSTANT_GSF): levels j >= 1 apply
    // A^-1 by the Gohberg-Semencul formula from x = A^-1 e_1, y = A^-1 e_n
    int krylov = TSFCDE_KRYLOV_CGS;  // Krylov method of the FP64 solves
    int prec = TSFCDE_PREC_STRANG;   // circulant preconditioner
    double qfac = 1.0;  // eigenvalues of the preconditioner's circulant of Q over 2i sin(2 pi k/n)
    // fast history (history_tol > 0): P_j from K + 4 recursions (soe_fit)
    bool soe = false;
    int soe_K = 0;
    int64_t soe_level = -1;  // the level whose history the recursions hold (-1: none)
    double *soe_S = nullptr, *soe_rho = nullptr, *soe_w = nullptr;
    SoePoly soe_poly{{0, 0, 0, 0}};
    double soe_err = 0.0;
    bool gsf = false, gsf_ready = false;
    double *gx = nullptr, *gy = nullptr;
    double2 *gspec[4] = {nullptr, nullptr, nullptr, nullptr};  // L_p, R_p, L0_p, R0_p
    double gsf_inv_xi0 = 0.0;
    ProfRec prof[NPROF];
    std::vector<hipEvent_t> event_pool;
};


// ===========================================================================
// Learned warm start: network state, training step and prediction.
// ===========================================================================
namespace {

struct NetLayer {
    int ci, co;
};
constexpr NetLayer NET_LAYERS[net::NLAYER] = {
    {net::CIN, net::WIDTH}, {net::WIDTH, net::WIDTH}, {net::WIDTH, net::WIDTH}, {net::WIDTH, 1}};
constexpr int net_param_count() {
    int t = 0;
    for (int l = 0; l < net::NLAYER; ++l) t += NET_LAYERS[l].co * NET_LAYERS[l].ci * net::KS + NET_LAYERS[l].co;
    return t;
}
constexpr int64_t net_layer_off(int l) {
    int64_t o = 0;
    for (int i = 0; i < l; ++i) o += NET_LAYERS[i].co * NET_LAYERS[i].ci * net::KS + NET_LAYERS[i].co;
    return o;
}
constexpr int NET_P = net_param_count();
static_assert(NET_P == 11617, "parameter count");
constexpr int NET_WG_MAX = 1024;  // workgroups of a weight-gradient pass
constexpr int NET_NE_MAX = net::WIDTH * net::WIDTH * net::KS + net::WIDTH;
constexpr int NET_LOSS_WG = 256;
constexpr int NET_SCALE_PARTS = 64;  // workgroups per sample of the scale reduction
// bfloat16 weights of the three 32-output layers in the matrix-core order
// (k = tap * CIP + ci, input channels padded to CIP = 8 or 32)
constexpr int NET_CIP0 = 8;
constexpr int NET_WM_OFF[3] = {0, 32 * net::KS * NET_CIP0, 32 * net::KS * NET_CIP0 + 32 * net::KS * net::WIDTH};
constexpr int NET_WM_TOTAL = NET_WM_OFF[2] + 32 * net::KS * net::WIDTH;
static_assert(sizeof(tsfcde_net_sample) == sizeof(net::Sample), "sample layout");

struct NetLayout {
    size_t theta, m, v, grad, wbf, wt, wb, wm, X, act, y, ystar, dy, dz0, dz1, part, s, den, lpart, smp, total;
};

NetLayout net_layout(int64_t mp, int32_t mb) {
    NetLayout l{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = al(o + bytes);
        return at;
    };
    l.theta = take(4 * (size_t)NET_P);
    l.m = take(4 * (size_t)NET_P);
    l.v = take(4 * (size_t)NET_P);
    l.grad = take(4 * (size_t)NET_P);
    l.wbf = take(2 * (size_t)NET_P);
    l.wt = take(4 * (size_t)NET_P);
    l.wb = take(4 * (size_t)NET_P);
    l.wm = take(2 * (size_t)NET_WM_TOTAL);
    l.X = take(4 * (size_t)net::CIN * mp);
    l.act = take(4 * (size_t)3 * net::WIDTH * mp);
    l.y = take(4 * (size_t)mp);
    l.ystar = take(4 * (size_t)mp);
    l.dy = take(4 * (size_t)mp);
    l.dz0 = take(4 * (size_t)net::WIDTH * mp);
    l.dz1 = take(4 * (size_t)net::WIDTH * mp);
    l.part = take(4 * (size_t)NET_WG_MAX * NET_NE_MAX);
    l.s = take(8 * (size_t)mb * NET_SCALE_PARTS);
    l.den = take(8 * (size_t)mb);
    l.lpart = take(8 * (size_t)NET_LOSS_WG);
    l.smp = take(sizeof(net::Sample) * (size_t)mb);
    l.total = o;
    return l;
}

}  // namespace

struct tsfcde_net_s {
    hipStream_t stream = nullptr;
    int64_t max_points = 0;
    int32_t max_batch = 0;
    float *theta, *m, *v, *grad, *wt, *wb, *X, *act, *y, *ystar, *dy, *dz0, *dz1, *part;
    uint16_t *wbf, *wm;
    double *s, *den, *lpart;
    net::Sample *smp;
    bool widened = false;
    int64_t step = 0;
};

namespace {

#define NCHK(x)                                      \
    do {                                             \
        if ((x) != hipSuccess) return TSFCDE_EDEVICE; \
    } while (0)

// bfloat16 weights -> the FP32 orders the convolutions read
int net_widen(tsfcde_net_s *nt) {
    if (nt->widened) return TSFCDE_OK;
    for (int l = 0; l < net::NLAYER; ++l) {
        const NetLayer &L = NET_LAYERS[l];
        const int64_t off = net_layer_off(l);
        hipLaunchKernelGGL(net::k_net_widen, dim3(32), dim3(256), 0, nt->stream, nt->wbf + off, L.ci, L.co,
                           nt->wt + off, l > 0 ? nt->wb + off : (float *)nullptr);
        if (l == 1 || l == 2)
            hipLaunchKernelGGL(net::k_net_widen_mfma, dim3(32), dim3(256), 0, nt->stream, nt->wbf + off, L.ci,
                               net::WIDTH, nt->wm + NET_WM_OFF[l]);
    }
    NCHK(hipGetLastError());
    nt->widened = true;
    return TSFCDE_OK;
}

// Inputs (and targets) of `count` samples already in nt->smp; then the
// forward pass.  Activations: act + l * WIDTH * count * n for layers 1..3.
int net_forward(tsfcde_net_s *nt, int count, int64_t n, bool targets, const net::Sample *one = nullptr) {
    int rc = net_widen(nt);
    if (rc) return rc;
    const net::Sample *smp = one ? nullptr : nt->smp;
    const net::Sample none = one ? *one : net::Sample{};
    const int sx = (int)std::max<int64_t>(1, std::min<int64_t>(NET_SCALE_PARTS, (n + 255) / 256));
    hipLaunchKernelGGL(net::k_net_scale<256>, dim3(sx, count), dim3(256), 0, nt->stream, smp, none, n, nt->s);
    const unsigned gx = (unsigned)std::min<int64_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(net::k_net_inputs, dim3(gx, count), dim3(256), 0, nt->stream, smp, none, n, nt->s, sx, nt->X,
                       targets ? nt->ystar : (float *)nullptr);
    const size_t A = (size_t)net::WIDTH * count * n;
    float *a1 = nt->act, *a2 = nt->act + A, *a3 = nt->act + 2 * A;
    auto grid = [&](int tx) { return dim3((unsigned)((n + tx - 1) / tx), (unsigned)count); };
    using G3 = net::ConvGeo<net::WIDTH, 1>;
    const int64_t o0 = net_layer_off(0), o1 = net_layer_off(1), o2 = net_layer_off(2), o3 = net_layer_off(3);
    // input layer in FP32, the two hidden layers on the matrix cores
    using G0 = net::ConvGeo<net::CIN, net::WIDTH>;
    hipLaunchKernelGGL((net::k_conv<net::CIN, net::WIDTH, 0>), grid(G0::TX), dim3(G0::NT), 0, nt->stream, nt->X,
                       nt->wt + o0, nt->theta + o0 + net::WIDTH * net::CIN * net::KS, (const float *)nullptr, a1, n);
    constexpr int MT = 32 * net::MFMA_WAVES;
    hipLaunchKernelGGL((net::k_conv_mfma<net::WIDTH, net::WIDTH>), grid(MT), dim3(64 * net::MFMA_WAVES), 0, nt->stream, a1,
                       nt->wm + NET_WM_OFF[1], nt->theta + o1 + net::WIDTH * net::WIDTH * net::KS, a2, n);
    hipLaunchKernelGGL((net::k_conv_mfma<net::WIDTH, net::WIDTH>), grid(MT), dim3(64 * net::MFMA_WAVES), 0, nt->stream, a2,
                       nt->wm + NET_WM_OFF[2], nt->theta + o2 + net::WIDTH * net::WIDTH * net::KS, a3, n);
    hipLaunchKernelGGL((net::k_conv<net::WIDTH, 1, 1>), grid(G3::TX), dim3(G3::NT), 0, nt->stream, a3, nt->wt + o3,
                       nt->theta + o3 + net::WIDTH * net::KS, (const float *)nullptr, nt->y, n);
    NCHK(hipGetLastError());
    return TSFCDE_OK;
}

template <int CI, int CO, bool ROUND>
int net_wgrad(tsfcde_net_s *nt, const float *dz, const float *a, int count, int64_t n, int64_t off) {
    using G = net::WgradGeo<CI, CO>;
    const int64_t tiles = (n + G::TX - 1) / G::TX;
    const int gx = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, NET_WG_MAX / count));
    hipLaunchKernelGGL((net::k_net_wgrad<CI, CO, ROUND>), dim3(gx, count), dim3(G::NT), 0, nt->stream, dz, a, n, nt->part);
    hipLaunchKernelGGL(net::k_net_wgrad_reduce, dim3((G::NE + 255) / 256), dim3(256), 0, nt->stream, nt->part,
                       gx * count, G::NE, nt->grad + off);
    NCHK(hipGetLastError());
    return TSFCDE_OK;
}

// Loss partials and the gradient of the loss in nt->grad (after net_forward
// with targets).
int net_backward(tsfcde_net_s *nt, int count, int64_t n) {
    hipLaunchKernelGGL(net::k_net_den<256>, dim3(count), dim3(256), 0, nt->stream, nt->ystar, n, nt->den);
    hipLaunchKernelGGL(net::k_net_loss<256>, dim3(NET_LOSS_WG), dim3(256), 0, nt->stream, nt->y, nt->ystar, nt->X,
                       nt->den, count, n, nt->dy, nt->lpart);
    const size_t A = (size_t)net::WIDTH * count * n;
    float *a1 = nt->act, *a2 = nt->act + A, *a3 = nt->act + 2 * A;
    auto grid = [&](int tx) { return dim3((unsigned)((n + tx - 1) / tx), (unsigned)count); };
    using GB3 = net::ConvGeo<1, net::WIDTH>;
    using GB = net::ConvGeo<net::WIDTH, net::WIDTH>;
    const int64_t o0 = net_layer_off(0), o1 = net_layer_off(1), o2 = net_layer_off(2), o3 = net_layer_off(3);
    int rc;
    // layer 3 (32 -> 1, linear): dZ3 = dy
    if ((rc = net_wgrad<net::WIDTH, 1, false>(nt, nt->dy, a3, count, n, o3))) return rc;
    hipLaunchKernelGGL((net::k_conv<1, net::WIDTH, 2>), grid(GB3::TX), dim3(GB3::NT), 0, nt->stream, nt->dy,
                       nt->wb + o3, (const float *)nullptr, a3, nt->dz0, n);
    // layer 2 (32 -> 32): dZ = dz0
    if ((rc = net_wgrad<net::WIDTH, net::WIDTH, true>(nt, nt->dz0, a2, count, n, o2))) return rc;
    hipLaunchKernelGGL((net::k_conv<net::WIDTH, net::WIDTH, 2>), grid(GB::TX), dim3(GB::NT), 0, nt->stream, nt->dz0,
                       nt->wb + o2, (const float *)nullptr, a2, nt->dz1, n);
    // layer 1 (32 -> 32): dZ = dz1
    if ((rc = net_wgrad<net::WIDTH, net::WIDTH, true>(nt, nt->dz1, a1, count, n, o1))) return rc;
    hipLaunchKernelGGL((net::k_conv<net::WIDTH, net::WIDTH, 2>), grid(GB::TX), dim3(GB::NT), 0, nt->stream, nt->dz1,
                       nt->wb + o1, (const float *)nullptr, a1, nt->dz0, n);
    // layer 0 (7 -> 32): dZ = dz0, inputs X
    if ((rc = net_wgrad<net::CIN, net::WIDTH, false>(nt, nt->dz0, nt->X, count, n, o0))) return rc;
    NCHK(hipGetLastError());
    return TSFCDE_OK;
}

int net_upload(tsfcde_net_s *nt, const tsfcde_net_sample *h, int count) {
    NCHK(hipMemcpyAsync(nt->smp, h, sizeof(net::Sample) * (size_t)count, hipMemcpyHostToDevice, nt->stream));
    // the host array must stay valid until the copy is done
    NCHK(hipStreamSynchronize(nt->stream));
    return TSFCDE_OK;
}

// x0 for one sample into d_x0 (on the network's stream; the sample goes to
// the kernels by value, so nothing waits on the host).
int net_predict(tsfcde_net_s *nt, const tsfcde_net_sample &smp, int64_t n, double *d_x0) {
    if (n > nt->max_points) return TSFCDE_EINVAL;
    net::Sample S;
    std::memcpy(&S, &smp, sizeof(S));
    int rc = net_forward(nt, 1, n, false, &S);
    if (rc) return rc;
    hipLaunchKernelGGL(net::k_net_output, dim3((unsigned)std::min<int64_t>(1024, (n + 255) / 256)), dim3(256), 0,
                       nt->stream, S, n, nt->y, d_x0);
    NCHK(hipGetLastError());
    return TSFCDE_OK;
}

// Channels 2..6 of level j (alpha, beta and the level's coefficients of
// sigma L_j relative to eta_j).
void level_features(const tsfcde_plan_s *pl, int64_t j, float *f) {
    const double e = pl->eta[j];
    const double qg = pl->sigma * pl->gam[j] / (pl->h * e);
    const double qp = pl->sigma * pl->dp[j] * pl->hb / e;
    const double qm = pl->sigma * pl->dm[j] * pl->hb / e;
    f[0] = (float)pl->alpha;
    f[1] = (float)pl->beta;
    f[2] = (float)std::asinh(qg);
    f[3] = (float)std::log1p(qp);
    f[4] = (float)std::log1p(qm);
}

}  // namespace

namespace {

#define HIPCHK(x)                                           \
    do {                                                    \
        hipError_t e_ = (x);                                \
        if (e_ != hipSuccess) return TSFCDE_EDEVICE;        \
    } while (0)

hipEvent_t get_event(tsfcde_plan_s *pl) {
    if (!pl->event_pool.empty()) {
        hipEvent_t e = pl->event_pool.back();
        pl->event_pool.pop_back();
        return e;
    }
    // no system-scope fence: the timing marker must not flush L2 around the
    // kernel it brackets
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

struct ProfScope {
    tsfcde_plan_s *pl;
    int cls;
    hipEvent_t e0 = nullptr;
    ProfScope(tsfcde_plan_s *p, int c) : pl(p), cls(c) {
        if (pl->prof[cls].on) {
            e0 = get_event(pl);
            if (e0) (void)hipEventRecord(e0, pl->stream);
        }
    }
    ~ProfScope() {
        if (e0) {
            hipEvent_t e1 = get_event(pl);
            if (e1) {
                (void)hipEventRecord(e1, pl->stream);
                pl->prof[cls].pending.emplace_back(e0, e1);
            } else {
                pl->event_pool.push_back(e0);
            }
        }
    }
};

// Called after the stream is known to be idle.
void harvest(tsfcde_plan_s *pl) {
    for (auto &pr : pl->prof) {
        std::vector<std::pair<hipEvent_t, hipEvent_t>> keep;
        for (auto &ev : pr.pending) {
            if (hipEventQuery(ev.second) == hipErrorNotReady) {  // still running on another stream
                keep.push_back(ev);
                continue;
            }
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev.first, ev.second) == hipSuccess) {
                pr.ms += ms;
                pr.launches += 1;
            }
            pl->event_pool.push_back(ev.first);
            pl->event_pool.push_back(ev.second);
        }
        pr.pending.swap(keep);
    }
}

// ---- kernel launch dispatch by transform size ------------------------------

#define TSF_SIZES(X) X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

// Launch on the plan's stream; while profiling class `cls` is on, the start
// and end events ride on every period-th dispatch of the class itself
// (hipExtLaunchKernelGGL), so the measured interval is the kernel's own run.
// A dispatch that carries events is separated from its neighbours by a few
// microseconds of idle time; sampling keeps that cost off most launches.
template <typename K, typename... Args>
void launch_timed_on(tsfcde_plan_s *pl, hipStream_t st, int cls, K kernel, dim3 grid, dim3 block, Args... args) {
    ProfRec &pr = pl->prof[cls];
    if (pr.on && pr.issued++ % pr.period == 0) {
        hipEvent_t e0 = get_event(pl), e1 = e0 ? get_event(pl) : nullptr;
        if (e0 && e1) {
            hipExtLaunchKernelGGL(kernel, grid, block, 0, st, e0, e1, 0, args...);
            pr.pending.emplace_back(e0, e1);
            return;
        }
        if (e0) pl->event_pool.push_back(e0);
    }
    hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
}

template <typename K, typename... Args>
void launch_timed(tsfcde_plan_s *pl, int cls, K kernel, dim3 grid, dim3 block, Args... args) {
    launch_timed_on(pl, pl->stream, cls, kernel, grid, block, args...);
}

// finish = false leaves a reducing pass's finishing kernel to the caller
// (a later pass folds it in, or it is launched with launch_final).
// Values per lane of a single plan's column pass of length R.
template <int R> constexpr int col_e() {
    return R == 512    ? TSF_E_COL_512
           : R == 1024 ? TSF_E_COL_1024
           : R == 2048 ? TSF_E_COL_2048
           : R == 4096 ? TSF_E_COL_4096
                       : TSF_E_COL;
}

template <int R, int DIR, class In, class Out>
hipError_t launch_col_t(tsfcde_plan_s *pl, int64_t C, const In &in, const Out &out, int pred, bool finish) {
    using G = ColGeo<R, col_e<R>()>;
    const int64_t grid = (C + G::B - 1) / G::B;
    launch_timed(pl, 1, k_col<R, col_e<R>(), DIR, In, Out>, dim3((unsigned)grid), dim3(G::NT), C, in, out,
                 (const double2 *)pl->tw_all, pl->sc, pred);
    if constexpr (Out::NACC > 0) {
        if (finish)
            hipLaunchKernelGGL((k_final<G::NT, Out>), dim3(1), dim3(G::NT), 0, pl->stream, out, (int)grid, pl->sc,
                               pred);
    }
    return hipGetLastError();
}

// Finishing kernel of a column pass of `rt` launched without its own.
template <int R, class Out>
hipError_t launch_final_t(tsfcde_plan_s *pl, int64_t C, const Out &out, int pred) {
    using G = ColGeo<R, col_e<R>()>;
    hipLaunchKernelGGL((k_final<G::NT, Out>), dim3(1), dim3(G::NT), 0, pl->stream, out, (int)((C + G::B - 1) / G::B),
                       pl->sc, pred);
    return hipGetLastError();
}

template <int DIR, class In, class Out>
hipError_t launch_col(tsfcde_plan_s *pl, const RT &rt, const In &in, const Out &out, int pred, bool finish = true) {
    switch (rt.R) {
#define TSF_CASE(P) \
    case P: return launch_col_t<P, DIR>(pl, rt.C, in, out, pred, finish);
        TSF_SIZES(TSF_CASE)
#undef TSF_CASE
        default: return hipErrorInvalidValue;
    }
}

template <class Out>
hipError_t launch_final(tsfcde_plan_s *pl, const RT &rt, const Out &out, int pred) {
    switch (rt.R) {
#define TSF_CASE(P) \
    case P: return launch_final_t<P>(pl, rt.C, out, pred);
        TSF_SIZES(TSF_CASE)
#undef TSF_CASE
        default: return hipErrorInvalidValue;
    }
}

// Workgroups of a column pass of `rt` (the partials its reduction leaves).
int col_grid(const RT &rt) {
    switch (rt.R) {
#define TSF_CASE(P) \
    case P: return (int)((rt.C + ColGeo<P, col_e<P>()>::B - 1) / ColGeo<P, col_e<P>()>::B);
        TSF_SIZES(TSF_CASE)
#undef TSF_CASE
        default: return 0;
    }
}

// The product transform's reducing passes leave one partial per workgroup and
// accumulator (at most two) in a site of PARTIAL_SLOTS doubles.
bool partials_fit(const RT &A) {
    const int g = col_grid(A);
    return g > 0 && 2 * (int64_t)g <= PARTIAL_SLOTS;
}

template <int RP, class Op, class CS>
hipError_t launch_fuse_t(tsfcde_plan_s *pl, const Op &op, const CS *bufP, CS *bufA, int pred) {
    if constexpr (RP > 2048) {
        return hipErrorInvalidValue;
    } else {
        constexpr int EF = RP == 2048 ? TSF_E_FUSE_4096 : (RP == 1024 ? TSF_E_FUSE_2048 : TSF_E_FUSE);
        using G = FuseGeo<RP, EF>;
        const int64_t C = pl->A.C;
        const int64_t grid = (C + G::B - 1) / G::B;
        launch_timed(pl, 5, k_fuse<RP, EF, Op, CS>, dim3((unsigned)grid), dim3(G::NT), C, bufP, pl->P.tw,
                     bufA, pl->A.tw, op, (const double2 *)pl->tw_all, pl->sc, pred);
        return hipGetLastError();
    }
}

// preconditioner inverse column pass fused with the next product's forward one
template <class Op, class CS>
hipError_t launch_fuse(tsfcde_plan_s *pl, const Op &op, const CS *bufP, CS *bufA, int pred) {
    switch (pl->P.R) {
#define TSF_CASE(P) \
    case P: return launch_fuse_t<P>(pl, op, bufP, bufA, pred);
        TSF_SIZES(TSF_CASE)
#undef TSF_CASE
        default: return hipErrorInvalidValue;
    }
}

template <int C_, int MODE, class CS>
hipError_t launch_mid_t(tsfcde_plan_s *pl, const RT &rt, CS *Y, const CS *spec, double2 *spec_out,
                        const SymParams &sp, int pred) {
    // rows of 2048 at four values per lane need 1024-thread workgroups: 14% slower
    constexpr int EM = C_ >= 4096   ? TSF_E_MID_4096
                       : C_ == 2048 ? TSF_E_MID_2048
                                    : (MODE == 1 && C_ <= 1024 ? TSF_E_MID_SOLVE : TSF_E_MID);
    using G = MidGeo<C_, EM>;
    // Rows of 2048 fill the LDS with one pair, so one workgroup runs per CU;
    // two pairs per workgroup then overlap one pair's memory traffic with the
    // other's transform (4.3% faster at n = 2^22).  On shorter rows two
    // workgroups per CU already run side by side, and the two-pair form,
    // with half the waves, made the product's middle pass 29% slower at
    // n = 2^20 (measured).
    if constexpr (MODE != 2 && C_ == 2048) {
        if (TSF_MID_PAIRS == 2 && rt.R / 4 >= 256) {
            launch_timed(pl, MODE == 1 ? 4 : 2, k_mid<C_, EM, MODE, CS, 2>, dim3((unsigned)(rt.R / 4)),
                         dim3(G::NT), rt.R, Y, spec, spec_out, rt.tw, sp, (const double2 *)pl->tw_all, pl->sc, pred);
            return hipGetLastError();
        }
    }
    launch_timed(pl, MODE == 1 ? 4 : 2, k_mid<C_, EM, MODE, CS>, dim3((unsigned)(rt.R / 2)), dim3(G::NT), rt.R,
                 Y, spec, spec_out, rt.tw, sp, (const double2 *)pl->tw_all, pl->sc, pred);
    return hipGetLastError();
}

template <int MODE, class CS>
hipError_t launch_mid(tsfcde_plan_s *pl, const RT &rt, CS *Y, const CS *spec, double2 *spec_out,
                      const SymParams &sp, int pred) {
    switch (rt.C) {
#define TSF_CASE(P) \
    case P: return launch_mid_t<P, MODE, CS>(pl, rt, Y, spec, spec_out, sp, pred);
        TSF_SIZES(TSF_CASE)
#undef TSF_CASE
        default: return hipErrorInvalidValue;
    }
}

template <int C_, int MODE>
hipError_t launch_row_t(tsfcde_plan_s *pl, double2 *Y, const double2 *spec, double2 *spec_out) {
    using G = RowGeo<C_, TSF_E_MID>;
    hipLaunchKernelGGL((k_row<C_, TSF_E_MID, MODE>), dim3((unsigned)pl->B.R), dim3(G::NT), 0, pl->stream, Y, spec,
                       spec_out, pl->tw_all);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_row(tsfcde_plan_s *pl, double2 *Y, const double2 *spec, double2 *spec_out) {
    switch (pl->B.C) {
#define TSF_CASE(P) \
    case P: return launch_row_t<P, MODE>(pl, Y, spec, spec_out);
        TSF_SIZES(TSF_CASE)
#undef TSF_CASE
        default: return hipErrorInvalidValue;
    }
}

// ---- per-level symbols -------------------------------------------------------

// s = -sigma for A and P, (1 - sigma) for B.  Product scale 1/(4N); solve scale 4N.
SymParams symbol(const tsfcde_plan_s *pl, int64_t j, double s, const RT &rt, bool solve) {
    const bool o = pl->one_level;
    const double eta = o ? pl->one_eta : pl->eta[j], gam = o ? pl->one_gam : pl->gam[j];
    const double dp = o ? pl->one_dp : pl->dp[j], dm = o ? pl->one_dm : pl->dm[j];
    SymParams sp;
    sp.s0 = eta;
    sp.cre = s * (dp + dm) * pl->hb;
    sp.cim = s * (dp - dm) * pl->hb;
    sp.cq = s * gam / pl->h;
    if (solve) sp.cq *= pl->qfac;
    sp.scale = solve ? 4.0 * (double)rt.N : 1.0 / (4.0 * (double)rt.N);
    return sp;
}

template <class Out>
Out with_red(Out o, tsfcde_plan_s *pl, int site) {
    o.partials = pl->part + (size_t)site * PARTIAL_SLOTS;
    return o;
}

double2 *buf_of(tsfcde_plan_s *pl, const RT &rt) { return &rt == &pl->P ? pl->bufP : pl->buf; }

OutSpec out_spec(tsfcde_plan_s *pl, const RT &rt) {
    OutSpec o{buf_of(pl, rt), rt.tw, rt.C};
    o.partials = nullptr;
    return o;
}

InSpec in_spec(tsfcde_plan_s *pl, const RT &rt) { return InSpec{buf_of(pl, rt), rt.tw, rt.C}; }

template <class CS> OutSpecT<CS> out_spec_on(CS *buf, const RT &rt) {
    OutSpecT<CS> o{buf, rt.tw, rt.C};
    o.partials = nullptr;
    return o;
}
template <class CS> InSpecT<CS> in_spec_on(const CS *buf, const RT &rt) { return InSpecT<CS>{buf, rt.tw, rt.C}; }

// run_op on an explicit transform buffer (any storage type)
template <int MODE, class CS, class In, class Out>
hipError_t run_op_on(tsfcde_plan_s *pl, const RT &rt, CS *buf, const CS *spec, const SymParams &sp, const In &in,
                     const Out &out, int pred, bool finish = true) {
    hipError_t e = launch_col<-1>(pl, rt, in, out_spec_on(buf, rt), pred);
    if (e != hipSuccess) return e;
    e = launch_mid<MODE>(pl, rt, buf, spec, (double2 *)nullptr, sp, pred);
    if (e != hipSuccess) return e;
    return launch_col<1>(pl, rt, in_spec_on<CS>(buf, rt), out, pred, finish);
}

// y-side of an operator: pass A with loader `in`, middle, pass C with store `out`.
template <int MODE, class In, class Out>
hipError_t run_op(tsfcde_plan_s *pl, const RT &rt, const double2 *spec, const SymParams &sp, const In &in,
                  const Out &out, int pred) {
    hipError_t e = launch_col<-1>(pl, rt, in, out_spec(pl, rt), pred);
    if (e != hipSuccess) return e;
    e = launch_mid<MODE>(pl, rt, buf_of(pl, rt), spec, (double2 *)nullptr, sp, pred);
    if (e != hipSuccess) return e;
    return launch_col<1>(pl, rt, in_spec(pl, rt), out, pred);
}

// dst[k] = sum_{m<n} src_m exp(-2 pi i m k / n), k < n, for any n (Bluestein):
// src times conj(chirp), circular convolution of length L with the chirp
// (spectrum Bhat, 1/L folded in), times conj(chirp).
hipError_t bluestein(tsfcde_plan_s *pl, const double2 *zc, const double *zr, double2 *dst) {
    const RT &B = pl->B;
    OutSpec o{pl->bufB, B.tw, B.C};
    o.partials = nullptr;
    hipError_t e = launch_col<-1>(pl, B, InCplx{zc, zr, pl->chirp, pl->n, B.C}, o, 0);
    if (e != hipSuccess) return e;
    if ((e = launch_row<3>(pl, pl->bufB, pl->Bhat, nullptr)) != hipSuccess) return e;
    OutCplx oc{dst, pl->chirp, pl->n, B.C};
    oc.partials = nullptr;
    return launch_col<1>(pl, B, InSpec{pl->bufB, B.tw, B.C}, oc, 0);
}

// Symbol of level j's preconditioner for k_pc_column: that of A with the
// circulant of Q in place of Q (the stored spectrum Ls is that of the
// preconditioner's circulant of W_beta).
SymParams precond_symbol(const tsfcde_plan_s *pl, int64_t j) {
    SymParams sp = symbol(pl, j, -pl->sigma, pl->A, false);
    sp.cq *= pl->qfac;
    return sp;
}

// Inverse Strang circulant of level j (general n): p = IDFT_n(1/lambda_P) and
// the DFT of its length-L embedding, in the product transform's native order.
hipError_t precond_level(tsfcde_plan_s *pl, int64_t j) {
    if (pl->p2 || pl->pj_level == j) return hipSuccess;
    if (pl->gsf && j >= 1 && pl->pj_level >= 1) return hipSuccess;  // constant coefficients: one P for j >= 1
    const int64_t n = pl->n;
    const SymParams sp = precond_symbol(pl, j);
    hipLaunchKernelGGL(k_pc_column, dim3(256), dim3(256), 0, pl->stream, pl->Ls, n, sp, pl->wv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = bluestein(pl, pl->wv, nullptr, pl->Wt)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_pc_embed, dim3(256), dim3(256), 0, pl->stream, pl->Wt, n, pl->A.L, pl->tmp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_col<-1>(pl, pl->A, InReal{pl->tmp, pl->A.L, pl->A.C}, out_spec(pl, pl->A), 0)) != hipSuccess)
        return e;
    SymParams none{};
    if ((e = launch_mid<2>(pl, pl->A, pl->buf, (const double2 *)nullptr, pl->specPj, none, 0)) != hipSuccess)
        return e;
    if (pl->fp32) {
        hipLaunchKernelGGL(k_to_f32, dim3(512), dim3(256), 0, pl->stream, pl->specPj, pl->specPj32, pl->A.N);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    pl->pj_level = j;
    return hipSuccess;
}

// Symbol that multiplies by a stored spectrum as it is.
SymParams unit_symbol(const RT &rt) { return SymParams{0.0, 1.0, 1.0, 0.0, 1.0 / (4.0 * (double)rt.N)}; }

int poll(tsfcde_plan_s *pl) {
    HIPCHK(hipMemcpyAsync(pl->h_sc, pl->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, pl->stream));
    HIPCHK(hipStreamSynchronize(pl->stream));
    harvest(pl);
    return TSFCDE_OK;
}

// Vectors and transform buffers of one CGS solve: the FP64 ones of the plan, or
// the FP32-stored ones of the inner solve of the refinement loop.
template <class S, class CS> struct Bufs {
    S *r, *rt, *u, *p, *q, *phat, *vhat, *uhat;
    CS *buf, *bufP;
    const CS *specA, *specP, *specPj;
};

Bufs<double, double2> bufs64(tsfcde_plan_s *pl) {
    return {pl->r, pl->rt, pl->u, pl->p, pl->q, pl->phat, pl->vhat, pl->uhat,
            pl->buf, pl->bufP, pl->specA, pl->specP, pl->specPj};
}

Bufs<float, float2> bufs32(tsfcde_plan_s *pl) {
    return {pl->r32, pl->rt32, pl->u32, pl->p32, pl->q32, pl->phat32, pl->vhat32, pl->uhat32,
            pl->buf32, pl->bufP32, pl->specA32, pl->specP32, pl->specPj32};
}

// One CGS iteration (Templates-style preconditioned CGS, Sec. 3.2 "PCGS"),
// ten kernels (plus the two finishing kernels of the reductions):
//  u = r + beta q ; p = u + beta (q + beta p)      [K1 prologue]
//  phat = P^{-1} p ; vhat = A phat               [K1, K2, K3 (fused), K4, K5]
//  alpha = rho / (rt . vhat)                     [K5 epilogue]
//  q = u - alpha vhat ; uhat = P^{-1} (u + q)     [K6 prologue, K7]
//  x += alpha uhat ; r -= alpha A uhat            [K8 (fused), K9, K10], rho' = rt . r
// One CGS iteration (power-of-two n).  With fold, the finishing steps of the
// two reducing passes are folded into the passes that follow them: the
// rt.vhat sum into this iteration's q pass, the residual sums into the next
// iteration's u,p pass (ci >= 1, its index in the chunk).  The caller then
// ends the chunk with finish_chunk.
template <class S, class CS>
hipError_t cgs_iteration(tsfcde_plan_s *pl, int64_t j, const Bufs<S, CS> &b, S *x, int ci = 0, bool fold = false) {
    const int64_t n = pl->n;
    const SymParams sP = symbol(pl, j, -pl->sigma, pl->P, true);
    const SymParams sA = symbol(pl, j, -pl->sigma, pl->A, false);
    hipError_t e;
    InCgsUPT<S> k1{b.r, b.u, b.p, b.q, n, pl->P.C, 0.0, false};
    if (fold && ci >= 1) {
        k1.fpart = pl->part + (size_t)1 * PARTIAL_SLOTS;
        k1.fnparts = col_grid(pl->A);
        k1.ci = ci;
    }
    if ((e = launch_col<-1>(pl, pl->P, k1, out_spec_on(b.bufP, pl->P), 1)) != hipSuccess) return e;
    if ((e = launch_mid<1>(pl, pl->P, b.bufP, b.specP, (double2 *)nullptr, sP, 1)) != hipSuccess) return e;
    if ((e = launch_fuse(pl, OpIdent{}, b.bufP, b.buf, 1)) != hipSuccess) return e;
    if ((e = launch_mid<0>(pl, pl->A, b.buf, b.specA, (double2 *)nullptr, sA, 1)) != hipSuccess) return e;
    OutCgsDotT<S> k5 = with_red(OutCgsDotT<S>{b.vhat, b.rt, n, pl->A.C}, pl, 0);
    if ((e = launch_col<1>(pl, pl->A, in_spec_on<CS>(b.buf, pl->A), k5, 1, !fold)) != hipSuccess) return e;
    InCgsQT<S> k6{b.u, b.vhat, b.q, n, pl->P.C, 0.0};
    if (fold) {
        k6.fpart = pl->part;  // site 0
        k6.fnparts = col_grid(pl->A);
        k6.ci = ci;
    }
    if ((e = launch_col<-1>(pl, pl->P, k6, out_spec_on(b.bufP, pl->P), 1)) != hipSuccess) return e;
    if ((e = launch_mid<1>(pl, pl->P, b.bufP, b.specP, (double2 *)nullptr, sP, 1)) != hipSuccess) return e;
    if ((e = launch_fuse(pl, OpCgsXT<S>{x, pl->A.C, 0.0}, b.bufP, b.buf, 1)) != hipSuccess) return e;
    if ((e = launch_mid<0>(pl, pl->A, b.buf, b.specA, (double2 *)nullptr, sA, 1)) != hipSuccess) return e;
    OutCgsRT<S> k10 = with_red(OutCgsRT<S>{b.r, b.rt, n, pl->A.C, 0.0}, pl, 1);
    return launch_col<1>(pl, pl->A, in_spec_on<CS>(b.buf, pl->A), k10, 1, !fold);
}

// End of a folded chunk of `len` iterations: the finishing kernel of the last
// residual pass, which no later pass folds in.
template <class S, class CS>
hipError_t finish_chunk(tsfcde_plan_s *pl, const Bufs<S, CS> &b, int len) {
    OutCgsRT<S> k10 = with_red(OutCgsRT<S>{b.r, b.rt, pl->n, pl->A.C, 0.0}, pl, 1);
    k10.ci = len - 1;
    return launch_final(pl, pl->A, k10, 1);
}

// The same iteration for general n: the preconditioner solve is a Toeplitz
// product with the level's inverse-Strang spectrum (12 kernels).
// One CGS iteration for any n (every transform on the product geometry), with
// the finishing steps folded as in cgs_iteration when fold is set.
template <class S, class CS>
hipError_t cgs_iteration_general(tsfcde_plan_s *pl, int64_t j, const Bufs<S, CS> &b, S *x, int ci = 0,
                                 bool fold = false) {
    const int64_t n = pl->n;
    const SymParams sA = symbol(pl, j, -pl->sigma, pl->A, false);
    const SymParams sI = unit_symbol(pl->A);
    const int64_t C = pl->A.C;
    hipError_t e;
    OutRealT<S> o1{b.phat, n, C};
    o1.partials = nullptr;
    InCgsUPT<S> i1{b.r, b.u, b.p, b.q, n, C, 0.0, false};
    if (fold && ci >= 1) {
        i1.fpart = pl->part + (size_t)1 * PARTIAL_SLOTS;
        i1.fnparts = col_grid(pl->A);
        i1.ci = ci;
    }
    if ((e = run_op_on<0>(pl, pl->A, b.buf, b.specPj, sI, i1, o1, 1))) return e;
    OutCgsDotT<S> o2 = with_red(OutCgsDotT<S>{b.vhat, b.rt, n, C}, pl, 0);
    if ((e = run_op_on<0>(pl, pl->A, b.buf, b.specA, sA, InRealT<S>{b.phat, n, C}, o2, 1, !fold))) return e;
    OutRealT<S> o3{b.uhat, n, C};
    o3.partials = nullptr;
    InCgsQT<S> i3{b.u, b.vhat, b.q, n, C, 0.0};
    if (fold) {
        i3.fpart = pl->part;  // site 0
        i3.fnparts = col_grid(pl->A);
        i3.ci = ci;
    }
    if ((e = run_op_on<0>(pl, pl->A, b.buf, b.specPj, sI, i3, o3, 1))) return e;
    OutCgsRT<S> o4 = with_red(OutCgsRT<S>{b.r, b.rt, n, C, 0.0}, pl, 1);
    return run_op_on<0>(pl, pl->A, b.buf, b.specA, sA, InCgsXT<S>{b.uhat, x, n, C, 0.0}, o4, 1, !fold);
}

// One BiCGSTAB iteration in FP64 (any n): two preconditioner solves, two
// products with A, one update pass; the vectors p, v, s, t, phat, shat sit in
// the plan's p, vhat, q, u, phat, uhat.
hipError_t bicg_iteration(tsfcde_plan_s *pl, int64_t j, double *x) {
    const int64_t n = pl->n;
    const RT &A = pl->A;
    const RT &R = pl->p2 ? pl->P : pl->A;  // geometry of the preconditioner solve
    const SymParams sA = symbol(pl, j, -pl->sigma, A, false);
    const SymParams sP = symbol(pl, j, -pl->sigma, pl->P, true);
    auto psolve = [&](const auto &in, double *out) {
        OutReal o{out, n, R.C};
        o.partials = nullptr;
        return pl->p2 ? run_op_on<1>(pl, pl->P, pl->bufP, (const double2 *)pl->specP, sP, in, o, 1)
                      : run_op_on<0>(pl, pl->A, pl->buf, (const double2 *)pl->specPj, unit_symbol(pl->A), in, o, 1);
    };
    hipError_t e;
    if ((e = psolve(InBiP{pl->r, pl->vhat, pl->p, n, R.C}, pl->phat)) != hipSuccess) return e;
    OutBiV ov = with_red(OutBiV{pl->vhat, pl->rt, n, A.C}, pl, 0);
    if ((e = run_op_on<0>(pl, A, pl->buf, (const double2 *)pl->specA, sA, InReal{pl->phat, n, A.C}, ov, 1)) !=
        hipSuccess)
        return e;
    if ((e = psolve(InBiS{pl->r, pl->vhat, pl->q, n, R.C}, pl->uhat)) != hipSuccess) return e;
    OutBiT ot = with_red(OutBiT{pl->u, pl->q, n, A.C}, pl, 1);
    if ((e = run_op_on<0>(pl, A, pl->buf, (const double2 *)pl->specA, sA, InReal{pl->uhat, n, A.C}, ot, 1)) !=
        hipSuccess)
        return e;
    const int grid = (int)std::min<int64_t>(1024, (n + 255) / 256);
    double *part = pl->part + (size_t)2 * PARTIAL_SLOTS;
    hipLaunchKernelGGL(k_bicg_update, dim3(grid), dim3(256), 0, pl->stream, x, pl->r, (const double *)pl->rt,
                       (const double *)pl->phat, (const double *)pl->uhat, (const double *)pl->q,
                       (const double *)pl->u, n, (const DevScalars *)pl->sc, part, 1);
    hipLaunchKernelGGL(k_bicg_final, dim3(1), dim3(256), 0, pl->stream, (const double *)part, grid, pl->sc, 1);
    return hipGetLastError();
}

template <class S, class CS>
hipError_t cgs_iter(tsfcde_plan_s *pl, int64_t j, const Bufs<S, CS> &b, S *x) {
    return pl->p2 ? cgs_iteration(pl, j, b, x) : cgs_iteration_general(pl, j, b, x);
}

// `len` CGS iterations with their finishing steps folded (two launches fewer
// per iteration), the same arithmetic bit for bit: the partial sums reduce
// in an order that does not depend on the reducing workgroup's size.
template <class S, class CS>
hipError_t cgs_chunk(tsfcde_plan_s *pl, int64_t j, const Bufs<S, CS> &b, S *x, int len) {
    hipError_t e = hipSuccess;
    if (pl->flags & TSFCDE_FLAG_NO_FOLD) {
        for (int k = 0; k < len && e == hipSuccess; ++k) e = cgs_iter(pl, j, b, x);
        return e;
    }
    for (int k = 0; k < len; ++k) {
        e = pl->p2 ? cgs_iteration(pl, j, b, x, k, true) : cgs_iteration_general(pl, j, b, x, k, true);
        if (e != hipSuccess) return e;
    }
    return len > 0 ? finish_chunk(pl, b, len) : hipSuccess;
}

// kappa c_1^(j): the weight of u^j in the history sum of level j (j >= 1)
double hist_c1(const tsfcde_plan_s *pl, int64_t j) { return pl->kappa * (j == 1 ? pl->clast[1] : pl->cbase[1]); }

// First level of the history block of level L >= 1 (blocks of HB levels from level 1).
int64_t hist_block_of(int64_t L) { return 1 + HB * ((L - 1) / HB); }

HistBlock hist_block_params(const tsfcde_plan_s *pl, int64_t b) {
    HistBlock hb{};
    hb.b = (int)b;
    hb.nl = (int)std::min<int64_t>(HB, pl->M - b);
    for (int l = 0; l < hb.nl; ++l) hb.clast[l] = pl->clast[b + l];
    hb.c1b = b == 1 ? pl->clast[1] : pl->cbase[1];
    return hb;
}

// Where the right-hand side of level j >= 1 finds P_j.
const double *hist_src(const tsfcde_plan_s *pl, int64_t j) {
    if (pl->soe && j >= 2) return pl->H;
    return j == hist_block_of(j) ? pl->Hq : pl->H;
}

// Fast history: one pass of k_hist_soe at level L (writing P_L into H when
// write_p, advancing the recursions to level L + 1).
hipError_t launch_soe(tsfcde_plan_s *pl, int64_t L, bool write_p) {
    const int64_t n = pl->n;
    const unsigned grid = (unsigned)std::min<int64_t>(2048, (n + 255) / 256);
    const double cL = pl->clast[L], c1 = pl->cbase[1];
    launch_timed(pl, 0, k_hist_soe, dim3(grid), dim3(256), (const double *)pl->U, n, pl->ldn, (int)L, pl->soe_S,
                 pl->soe_K, (const double *)pl->soe_rho, (const double *)pl->soe_w, pl->soe_poly, pl->kappa, c1, cL,
                 pl->H, write_p ? 1 : 0, 1);
    return hipGetLastError();
}

// The recursions for level j >= 2 rebuilt from the stored levels (after a
// resume, or a right-hand side asked out of order): zero, then advanced
// through levels 2..j-1.
int soe_rebuild(tsfcde_plan_s *pl, int64_t j) {
    const size_t cnt = (size_t)(pl->soe_K + 4) * pl->ldn;
    hipLaunchKernelGGL(k_fill<double>, dim3(1024), dim3(256), 0, pl->stream, pl->soe_S, 0.0, (int64_t)cnt);
    HIPCHK(hipGetLastError());
    for (int64_t L = 2; L < j; ++L) HIPCHK(launch_soe(pl, L, false));
    pl->soe_level = j;
    return TSFCDE_OK;
}

#ifndef TSF_HIST_SIDE_WG
#define TSF_HIST_SIDE_WG 256
#endif
// On the main stream the sweep takes the whole chip; on the side stream it
// runs beside the solve on a small grid (TSF_HIST_SIDE_WG workgroups).
hipError_t launch_sweep(tsfcde_plan_s *pl, hipStream_t st, int64_t b) {
    const int64_t n = pl->n, threads = (n + 1) / 2;
    int64_t wg = (threads + 255) / 256;
    if (st != pl->stream) wg = std::min<int64_t>(wg, TSF_HIST_SIDE_WG);
    launch_timed_on(pl, st, 0, k_hist_sweep, dim3((unsigned)wg), dim3(256), (const double *)pl->U, n, pl->ldn,
                    (const double *)pl->cb, hist_block_params(pl, b), pl->kappa, pl->Hq);
    return hipGetLastError();
}

hipError_t launch_catch(tsfcde_plan_s *pl, int64_t L) {
    const int64_t n = pl->n, threads = (n + 1) / 2, b = hist_block_of(L);
    const int64_t wg = (threads + 255) / 256;
    launch_timed(pl, 0, k_hist_catch, dim3((unsigned)wg), dim3(256), (const double *)pl->U, n, pl->ldn,
                 (const double *)pl->cb, (int)b, (int)L, pl->clast[L], L == 1 ? pl->clast[1] : pl->cbase[1],
                 pl->kappa, (const double *)(pl->Hq + (size_t)(L - b) * pl->ldn), pl->H);
    return hipGetLastError();
}

// The side stream is idle and holds no block sums (before anything other
// than a level step touches U or the history buffers).
int history_quiesce(tsfcde_plan_s *pl) {
    if (pl->hs) HIPCHK(hipStreamSynchronize(pl->hs));
    pl->hist_pending = false;
    pl->hist_block = -1;
    return TSFCDE_OK;
}

// P_j ready for the right-hand side of level j: the block's sums (waited for
// if the side stream summed them, else summed now from u^0..u^{b-1}, which
// are final), then the catch-up of a level past the block's first.
int history_for(tsfcde_plan_s *pl, int64_t j) {
    if (j < 1) return TSFCDE_OK;
    if (pl->soe && j >= 2) {
        if (pl->soe_level != j) {
            if (int rc = soe_rebuild(pl, j)) return rc;
        }
        HIPCHK(launch_soe(pl, j, true));
        pl->soe_level = j + 1;
        return TSFCDE_OK;
    }
    const int64_t b = hist_block_of(j);
    if (pl->hist_pending) {  // whatever the side stream queued is finished before the buffers are used
        HIPCHK(hipStreamWaitEvent(pl->stream, pl->ev_hist, 0));
        pl->hist_pending = false;
    }
    if (pl->hist_block != b) {
        HIPCHK(launch_sweep(pl, pl->stream, b));
        pl->hist_block = b;
    }
    if (j > b) HIPCHK(launch_catch(pl, j));
    return TSFCDE_OK;
}

// After the right-hand side of level j is queued: when level j + 1 starts a
// block, its sweep (u^0..u^j, all final) goes to the side stream, behind
// everything the main stream has queued, including the right-hand side and
// catch-up that last read the block buffers it overwrites.
int history_next(tsfcde_plan_s *pl, int64_t j) {
    if (pl->soe) return TSFCDE_OK;  // no block sweeps: levels from 2 on use the recursions
    const int64_t b = j + 1;
    if (b >= pl->M || hist_block_of(b) != b || pl->hist_block == b) return TSFCDE_OK;
    if (!pl->hs) {
        HIPCHK(hipStreamCreateWithFlags(&pl->hs, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&pl->ev_main, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&pl->ev_hist, hipEventDisableTiming));
    }
    HIPCHK(hipEventRecord(pl->ev_main, pl->stream));
    HIPCHK(hipStreamWaitEvent(pl->hs, pl->ev_main, 0));
    HIPCHK(launch_sweep(pl, pl->hs, b));
    HIPCHK(hipEventRecord(pl->ev_hist, pl->hs));
    pl->hist_block = b;
    pl->hist_pending = true;
    return TSFCDE_OK;
}

int level_rhs(tsfcde_plan_s *pl, int64_t j, const double *d_f, double *x, int warm) {
    const int64_t n = pl->n, ld = pl->ldn;
    int rc = history_for(pl, j);
    if (rc) return rc;
    if (d_f && (reinterpret_cast<uintptr_t>(d_f) & 15)) {  // pairs are read as 16-byte loads
        hipLaunchKernelGGL(k_copy, dim3(256), dim3(256), 0, pl->stream, d_f, pl->fbuf, n);
        HIPCHK(hipGetLastError());
        d_f = pl->fbuf;
    }
    const SymParams sA = symbol(pl, j, -pl->sigma, pl->A, false);
    InReal in{pl->U + (size_t)j * ld, n, pl->A.C};
    OutRhs out{pl->U + (size_t)j * ld, j >= 1 ? hist_src(pl, j) : nullptr, d_f, pl->g, pl->r, pl->rt, x, n,
               pl->A.C,
               pl->eta[j] / pl->sigma - (j >= 1 ? hist_c1(pl, j) : 0.0), (1.0 - pl->sigma) / pl->sigma, warm,
               j >= 1 ? 1 : 0,
               j >= 2 ? pl->U + (size_t)(j - 1) * ld : nullptr, j >= 2 ? pl->U + (size_t)(j - 2) * ld : nullptr};
    out = with_red(out, pl, 2);
    HIPCHK(run_op<0>(pl, pl->A, pl->specA, sA, in, out, 0));
    return history_next(pl, j);
}

int status_code(int st) {
    if (st == ST_BREAKDOWN) return TSFCDE_EBREAKDOWN;
    if (st == ST_NONFINITE) return TSFCDE_ENONFINITE;
    return TSFCDE_OK;
}

constexpr int MAX_RESTARTS = 3;

// y = A x and r = g - y, rt = r (restart from the current iterate); queued
// on the stream, no synchronisation.
// r = g - A x, rt = r and a fresh CGS state; x itself is accepted when it
// meets rtol or, with bwtol > 0, the backward-error test.
int restart_launch(tsfcde_plan_s *pl, int64_t j, const double *x, double bwtol, int pred = 0, bool check = false) {
    const SymParams sA = symbol(pl, j, -pl->sigma, pl->A, false);
    InReal in{x, pl->n, pl->A.C};
    OutRestart out =
        with_red(OutRestart{pl->g, x, pl->r, pl->rt, pl->n, pl->A.C, pl->anorm[j], bwtol}, pl, 3);
    out.check = check ? 1 : 0;
    HIPCHK(run_op<0>(pl, pl->A, pl->specA, sA, in, out, pred));
    return TSFCDE_OK;
}

int restart_from_x(tsfcde_plan_s *pl, int64_t j, const double *x, double bwtol) {
    int rc = restart_launch(pl, j, x, bwtol);
    return rc ? rc : poll(pl);
}

// FP64 CGS on A x = g from the state the device scalars describe (after the
// right-hand side or a restart): chunks of iterations between polls, then
// breakdown recovery and, with TSFCDE_FLAG_VERIFY, true-residual checks.
struct SolveOut {
    int code = TSFCDE_OK, restarts = 0, iters = 0;
    double relres_true = -1.0, backward_err = -1.0;
};

// Normwise backward error |g - A x| / (|A| |x| + |g|) from the last restart
// pass (aux0 = |g - A x|^2, aux1 = |x|^2), with |A|_2 bounded from above.
double backward_error(const tsfcde_plan_s *pl, int64_t j) {
    const DevScalars &h = *pl->h_sc;
    const double den = pl->anorm[j] * std::sqrt(h.aux1) + std::sqrt(h.gnorm2);
    return den > 0 ? std::sqrt(h.aux0) / den : 0.0;
}


int fp64_cgs(tsfcde_plan_s *pl, int64_t j, double *x, SolveOut &so) {
    const bool verify = (pl->flags & TSFCDE_FLAG_VERIFY) != 0;
    const bool strict = (pl->flags & TSFCDE_FLAG_STRICT_RESIDUAL) != 0;
    // the device accepts x at backward error BW_TOL; with TSFCDE_FLAG_VERIFY
    // (restarts while the true residual falls) or TSFCDE_FLAG_STRICT_RESIDUAL
    // only at a true residual within rtol |g|
    const double bwtol = (verify || strict) ? 0.0 : BW_TOL;
    const Bufs<double, double2> b64 = bufs64(pl);
    int rc, iters_seen = 0, checks_seen = 0;
    double last_true2 = HUGE_VAL;
    int chunk = std::max(2, pl->last_iters);
    // set where the device's acceptance check (true residual within rtol |g|,
    // or backward error within bwtol) passed x; a level that leaves the loop
    // any other way with no error of its own is TSFCDE_EACCEPT
    bool accepted = false;
    for (;;) {
        // a chunk of CGS, then the acceptance check, which the device runs
        // only when the chunk ended the solve (one poll serves both): restart
        // from x recovers from a breakdown and checks a converged level,
        // continuing CGS from x when the check fails
        const int todo = std::min(chunk, pl->maxit - iters_seen);
        if (todo > 0) {
            if (pl->krylov == TSFCDE_KRYLOV_BICGSTAB) {
                for (int k = 0; k < todo; ++k) HIPCHK(bicg_iteration(pl, j, x));
            } else {
                HIPCHK(cgs_chunk(pl, j, b64, x, todo));
            }
        }
        if ((rc = restart_launch(pl, j, x, bwtol, 3, true))) return rc;
        if ((rc = poll(pl))) return rc;
        const DevScalars &h = *pl->h_sc;
        iters_seen = h.iter;
        const bool ran = h.nchecks > checks_seen;
        checks_seen = h.nchecks;
        if (!ran) {
            if (h.done) {  // the level's first residual already met the tolerance
                so.relres_true = h.gnorm2 > 0 ? std::sqrt(h.aux0 / h.gnorm2) : 0.0;
                so.backward_err = backward_error(pl, j);
                so.code = status_code(h.status);
                accepted = so.code == TSFCDE_OK;
                break;
            }
            if (todo <= 0) {
                so.code = TSFCDE_ENOCONV;
                break;
            }
            chunk = 2;
            continue;
        }
        so.relres_true = h.gnorm2 > 0 ? std::sqrt(h.aux0 / h.gnorm2) : 0.0;
        so.backward_err = backward_error(pl, j);
        if (h.done) {  // accepted, or non-finite
            so.code = status_code(h.status);
            accepted = so.code == TSFCDE_OK;
            break;
        }
        const int stat = h.prestat;  // how CGS stopped
        if (stat == ST_BREAKDOWN && so.restarts >= MAX_RESTARTS) {
            so.code = TSFCDE_EBREAKDOWN;
            break;
        }
        if (stat == ST_OK) {
            if (verify) {
                // true residual above tolerance: continue while it keeps falling
                if (so.restarts >= MAX_RESTARTS || !(h.aux0 < 0.25 * last_true2)) break;
                last_true2 = h.aux0;
            } else if (so.restarts >= MAX_RESTARTS) {
                break;  // x stays as it is
            }
        }
        ++so.restarts;
        if (iters_seen >= pl->maxit) {
            so.code = TSFCDE_ENOCONV;
            break;
        }
        chunk = std::max(2, pl->last_iters / 2);
    }
    // with TSFCDE_FLAG_VERIFY alone, a level whose true residual stopped
    // falling above rtol |g| is still accepted at backward error BW_TOL
    if (!accepted && verify && !strict && so.backward_err >= 0.0 && so.backward_err <= BW_TOL) accepted = true;
    if (so.code == TSFCDE_OK && !accepted) so.code = TSFCDE_EACCEPT;
    so.iters = pl->h_sc->iter;
    pl->last_iters = std::max(1, so.iters / (so.restarts + 1));
    return TSFCDE_OK;
}

// FP32-refined form.  The level's rounding-error model: an FP32-stored
// transform of a vector v errs by about eps32 * log2(L) * |v| in every
// frequency, and A multiplies that error by up to |A| while a smooth
// correction d has |A d| near eta |d|, so the inner products are useful only
// while eps32 * log2(L) * |A| / eta is well below one.  |A| / eta is bounded
// by Remark 3.1 (|lambda(W)| <= 2 |omega_1|) and |eig(Q)| <= 2.
constexpr double EPS32 = 5.9604644775390625e-08;  // 2^-24
constexpr double IR_MODEL_LIMIT = 0.1;
constexpr int IR_MAX_OUTER = 30;
constexpr int IR_INNER_MAXIT = 64;

bool level_uses_fp32(const tsfcde_plan_s *pl, int64_t j) {
    if (!pl->fp32) return false;
    if (pl->flags & TSFCDE_FLAG_FORCE_FP32) return true;
    return EPS32 * (double)ilog2(pl->A.L) * pl->kbound[j] < IR_MODEL_LIMIT;
}

// Inner tolerance: what the FP32-stored operator can resolve, at least 1e-5.
double ir_inner_rtol(const tsfcde_plan_s *pl, int64_t j) {
    return std::min(0.5, std::max(1e-5, 8.0 * EPS32 * pl->kbound[j]));
}

// Iterative refinement: r = g - A x in FP64 (x += d folded into the same
// pass), then the FP32-stored inner CGS solves A d = r to the inner
// tolerance, and again until |g - A x| <= rtol |g|.  The stopping test is the
// true FP64 residual.  On a non-finite inner result, or when a sweep no longer
// halves the residual, the level continues with the FP64 CGS from x.
int ir_solve(tsfcde_plan_s *pl, int64_t j, double *x, SolveOut &so, int &outer, bool &fell_back) {
    const int64_t n = pl->n;
    const SymParams sA = symbol(pl, j, -pl->sigma, pl->A, false);
    const double irtol = ir_inner_rtol(pl, j);
    const Bufs<float, float2> b32 = bufs32(pl);
    int rc, inner_total = 0, slow = 0;
    double prev2 = HUGE_VAL;
    outer = 0;
    fell_back = false;
    // no correction is pending when a level starts
    hipLaunchKernelGGL(k_fill<float>, dim3(256), dim3(256), 0, pl->stream, pl->d32, 0.0f, n);
    HIPCHK(hipGetLastError());
    for (;;) {
        // outer residual, then at once the first chunk of the inner solve: the
        // residual pass sets `done` when the level has converged, which
        // predicates the inner kernels off, so one poll serves both
        InIR in{x, pl->d32, n, pl->A.C};
        OutIR out = with_red(OutIR{pl->g, x, pl->r32, pl->rt32, pl->d32, n, pl->A.C, irtol * irtol}, pl, 2);
        HIPCHK(run_op<0>(pl, pl->A, pl->specA, sA, in, out, 0));
        const int budget = std::min(IR_INNER_MAXIT, pl->maxit - inner_total);
        int chunk = std::min(std::max(2, pl->last_inner), std::max(0, budget));
        HIPCHK(cgs_chunk(pl, j, b32, pl->d32, chunk));
        if ((rc = poll(pl))) return rc;
        ++outer;
        const double res2 = pl->h_sc->aux1;
        so.relres_true = pl->h_sc->gnorm2 > 0 ? std::sqrt(res2 / pl->h_sc->gnorm2) : 0.0;
        {
            const double den = pl->anorm[j] * std::sqrt(pl->h_sc->aux0) + std::sqrt(pl->h_sc->gnorm2);
            so.backward_err = den > 0 ? std::sqrt(res2) / den : 0.0;
        }
        if (!std::isfinite(res2)) {
            so.code = TSFCDE_ENONFINITE;
            break;
        }
        if (res2 <= pl->h_sc->rtol2 * pl->h_sc->gnorm2) break;  // converged; the inner chunk did not run
        slow = res2 > 0.25 * prev2 ? slow + 1 : 0;
        prev2 = res2;
        if (slow >= 2 || outer > IR_MAX_OUTER || inner_total >= pl->maxit) {
            fell_back = true;
            break;
        }
        // the inner FP32-stored CGS on A d = r continues until its tolerance
        // or the sweep's iteration budget
        int seen = pl->h_sc->iter;
        while (!pl->h_sc->done && seen < budget) {
            const int todo = std::min(2, budget - seen);
            HIPCHK(cgs_chunk(pl, j, b32, pl->d32, todo));
            if ((rc = poll(pl))) return rc;
            seen = pl->h_sc->iter;
        }
        inner_total += seen;
        pl->last_inner = std::max(2, seen);
        if (pl->h_sc->status == ST_NONFINITE) {
            fell_back = true;
            break;
        }
    }
    so.iters = inner_total;
    if (fell_back && so.code == TSFCDE_OK) {
        // continue in FP64 from x (the pending correction d is dropped)
        const bool no_bw = (pl->flags & (TSFCDE_FLAG_VERIFY | TSFCDE_FLAG_STRICT_RESIDUAL)) != 0;
        if ((rc = restart_from_x(pl, j, x, no_bw ? 0.0 : BW_TOL))) return rc;
        if (!pl->h_sc->done) {
            const int base = pl->h_sc->iter;  // the restart keeps the inner count
            SolveOut f;
            if ((rc = fp64_cgs(pl, j, x, f))) return rc;
            so.code = f.code;
            so.restarts = f.restarts;
            so.iters += f.iters - base;
            so.relres_true = f.relres_true;
            so.backward_err = f.backward_err;
        } else {
            so.code = status_code(pl->h_sc->status);
        }
    }
    return TSFCDE_OK;
}

// ---- constant coefficients: Algorithm 3 with the Gohberg-Semencul formula
// (Sec. 3.1).  Every level j >= 1 has the same matrix A, whose inverse is
// applied from x = A^-1 e_1 and y = A^-1 e_n (3.4), solved once by the FP64
// PCGS, as four triangular Toeplitz products through the product transform
// (Algorithm 1).

// Tolerance of the two solves (3.4): tighter than the levels' own, since the
// formula's products carry their error into every later level.
constexpr double GSF_GEN_RTOL = 1e-13;

// The solves (3.4) for the matrix of levels j >= 1 and the spectra of the
// four factors.  Uses g, r, rt and the device scalars as scratch (before the
// level's right-hand side).  so accumulates the solves' iterations.
int gsf_prepare(tsfcde_plan_s *pl, SolveOut &so) {
    const int64_t n = pl->n, j = 1;
    HIPCHK(precond_level(pl, j));
    const double tol = std::min(pl->rtol, GSF_GEN_RTOL);
    double *outs[2] = {pl->gx, pl->gy};
    const int64_t pos[2] = {0, n - 1};
    for (int k = 0; k < 2; ++k) {
        hipLaunchKernelGGL(k_unit_rhs, dim3(256), dim3(256), 0, pl->stream, pl->g, outs[k], pl->r, pl->rt, pl->ldn,
                           pos[k], tol, pl->sc);
        HIPCHK(hipGetLastError());
        SolveOut one;
        if (int rc = fp64_cgs(pl, j, outs[k], one)) return rc;
        so.iters += one.iters;
        so.restarts += one.restarts;
        if (one.code != TSFCDE_OK) return one.code;
    }
    double xi0 = 0.0;
    HIPCHK(hipMemcpyAsync(&xi0, pl->gx, sizeof(double), hipMemcpyDeviceToHost, pl->stream));
    HIPCHK(hipStreamSynchronize(pl->stream));
    if (!(std::isfinite(xi0) && xi0 != 0.0)) return TSFCDE_EBREAKDOWN;  // the formula needs xi_0 != 0
    pl->gsf_inv_xi0 = 1.0 / xi0;
    for (int w = 0; w < 4; ++w) {
        hipLaunchKernelGGL(k_gsf_column, dim3(512), dim3(256), 0, pl->stream, (const double *)pl->gx,
                           (const double *)pl->gy, n, pl->A.L, w, pl->tmp);
        HIPCHK(hipGetLastError());
        HIPCHK(launch_col<-1>(pl, pl->A, InReal{pl->tmp, pl->A.L, pl->A.C}, out_spec(pl, pl->A), 0));
        HIPCHK(launch_mid<2>(pl, pl->A, pl->buf, (const double2 *)nullptr, pl->gspec[w], SymParams{}, 0));
    }
    pl->gsf_ready = true;
    return TSFCDE_OK;
}

// x = A^-1 g by Algorithm 1: z2 = R_p g, z1 = R0_p g, z4 = L_p z2, and the
// pass that forms z3 = L0_p z1 stores x = (z4 - z3) / xi_0.
int gsf_apply(tsfcde_plan_s *pl, double *x) {
    const int64_t n = pl->n, C = pl->A.C;
    const SymParams sI = unit_symbol(pl->A);
    double *z1 = pl->phat, *z2 = pl->vhat, *z4 = pl->uhat;
    OutReal o{z2, n, C};
    o.partials = nullptr;
    HIPCHK(run_op<0>(pl, pl->A, pl->gspec[1], sI, InReal{pl->g, n, C}, o, 0));
    o.x = z1;
    HIPCHK(run_op<0>(pl, pl->A, pl->gspec[3], sI, InReal{pl->g, n, C}, o, 0));
    o.x = z4;
    HIPCHK(run_op<0>(pl, pl->A, pl->gspec[0], sI, InReal{z2, n, C}, o, 0));
    OutGsfCombine oc{z4, x, n, C, pl->gsf_inv_xi0};
    oc.partials = nullptr;
    HIPCHK(run_op<0>(pl, pl->A, pl->gspec[2], sI, InReal{z1, n, C}, oc, 0));
    return TSFCDE_OK;
}

// ---- fast history: a sum of exponentials for the L2-1sigma weights --------
// For m >= 2 the weights c_m = a_m + b_{m+1} - b_m of Lemma 1 are integrals
// of the kernels x^-alpha and x^-alpha-1 over unit intervals:
//   a_m = (1-alpha) int_0^1 g(m-1+sigma+t) dt,                  g(x) = x^-alpha,
//   b_m = alpha(1-alpha)/2 int_0^1 t(1-t) h(m-1+sigma+t) dt,     h(x) = x^-alpha-1
// (the second is the trapezoid rule's error for x^(1-alpha) on the interval).
// Each kernel has the integral form x^-b = (1/Gamma(b)) int e^(b y - x e^y) dy;
// its trapezoid sum with step D on the grid y_k = y0 + k D is spectrally
// accurate in D.  Grid points with y_k >= y0 give exponentials e^(-s_k x),
// s_k = e^(y_k); those below y0, where s x <= e^y0 x_max = 1e-3, are summed
// as a geometric series of the Taylor terms of e^(-s x), a cubic in x.  The
// t-integrals of exponentials and cubics are closed form, so
//   c_m ~ sum_k W_k rho_k^m + sum_{p<=3} C_p m^p,   rho_k = e^(-s_k),
// and the history sum over m = 2..j-1 runs as K + 4 recursions, one vector
// each, updated once per level.  The fit is checked against c_m for every m
// the march uses, c_m evaluated from its integral form by Gauss-Legendre
// quadrature (the closed form's differences of powers lose about m^(2-alpha)
// ulps to cancellation, more than the fit's tolerance at large m).
struct SoeFit {
    std::vector<double> rho, w;  // exponentials
    double poly[4] = {0, 0, 0, 0};  // cubic in m
    double max_rel_err = 0.0;
};

// int_0^1 e^{-s t} dt and int_0^1 t (1-t) e^{-s t} dt, stable for small s.
double int_e(double s) { return s < 1e-4 ? 1.0 - s / 2 + s * s / 6 : -std::expm1(-s) / s; }
double int_tt_e(double s) {
    if (s < 1e-2) return 1.0 / 6 - s / 12 + s * s / 40 - s * s * s / 180;
    return ((s - 2.0) + (s + 2.0) * std::exp(-s)) / (s * s * s);
}

// c_m of Lemma 1 for m >= 2 from the integral forms above by 24-point
// Gauss-Legendre quadrature on [0, 1] (smooth integrands), free of the
// cancellation the closed form's differences of powers suffer at large m:
// c_m = (1-alpha) int_0^1 g(m-1+sg+t) dt
//       + alpha(1-alpha)/2 int_0^1 t(1-t) [h(m+sg+t) - h(m-1+sg+t)] dt.
struct GaussLegendre {
    double x[24], w[24];
    GaussLegendre() {
        const int n = 24;
        for (int i = 0; i < n; ++i) {  // Newton on P_n from the Chebyshev guess
            double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 1.0;
            for (int it = 0; it < 100; ++it) {
                double p1 = 1.0, p2 = 0.0;
                for (int k = 1; k <= n; ++k) {
                    const double p3 = p2;
                    p2 = p1;
                    p1 = ((2.0 * k - 1.0) * z * p2 - (k - 1.0) * p3) / k;
                }
                pp = n * (z * p1 - p2) / (z * z - 1.0);
                const double dz = p1 / pp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) break;
            }
            x[i] = 0.5 * (1.0 - z);
            w[i] = 1.0 / ((1.0 - z * z) * pp * pp);  // 2/((1-z^2)P'^2), halved for [0, 1]
        }
    }
};

double l21s_cbase_accurate(double al, double sg, int64_t m) {
    static const GaussLegendre gl;
    double a = 0.0, db = 0.0;
    for (int q = 0; q < 24; ++q) {
        const double t = gl.x[q], x0 = (double)m - 1.0 + sg + t;
        a += gl.w[q] * std::pow(x0, -al);
        // h(x0 + 1) - h(x0) = x0^-(al+1) ((1 + 1/x0)^-(al+1) - 1), the bracket by expm1/log1p
        db += gl.w[q] * t * (1.0 - t) * std::pow(x0, -al - 1.0) * std::expm1(-(al + 1.0) * std::log1p(1.0 / x0));
    }
    return (1.0 - al) * a + al * (1.0 - al) / 2.0 * db;
}

int soe_fit(double al, int64_t M, double tol, SoeFit &fit) {
    const double sg = 1.0 - al / 2.0;
    if (M < 4) return TSFCDE_OK;  // no m in 2..M-2 ever used: nothing to fit
    const double xmin = 1.0 + sg, xmax = (double)M + sg;
    // the trapezoid sum's relative error is about 4 e^(-pi^2 / D)
    const double D = std::min(0.6, M_PI * M_PI / std::log(40.0 / tol));
    const double y0 = std::log(1e-3 / xmax), y1 = std::log(40.0 / xmin);
    const double ga = std::tgamma(al), gh = std::tgamma(al + 1.0);
    const double k1 = 1.0 - al, k2 = al * (1.0 - al) / 2.0;
    fit.rho.clear();
    fit.w.clear();
    for (double y = y0; y <= y1 + 1e-12; y += D) {
        const double sk = std::exp(y);
        const double pg = D * std::exp(al * y) / ga, ph = D * std::exp((al + 1.0) * y) / gh;
        // a_m: k1 pg e^{-s(m-1+sg)} int_e(s); b_{m+1} - b_m: k2 ph int_tt_e(s) e^{-s(m-1+sg)} (e^{-s} - 1)
        const double base = std::exp(-sk * (sg - 1.0));
        const double wk = base * (k1 * pg * int_e(sk) + k2 * ph * int_tt_e(sk) * std::expm1(-sk));
        fit.rho.push_back(std::exp(-sk));
        fit.w.push_back(wk);
    }
    // tails below y0: x^-b ~ sum_p tau_p x^p, tau_p = (-1)^p/p! D sum_{k<0} e^{(b+p) y_k} / Gamma(b)
    auto tail = [&](double b, double gb, int p) {
        const double fact[4] = {1, 1, 2, 6};
        const double geo = std::exp((b + p) * (y0 - D)) / (-std::expm1(-(b + p) * D));
        return ((p & 1) ? -1.0 : 1.0) / fact[p] * D * geo / gb;
    };
    // the cubic part of c_m: each tail sum_p tau_p x^p at x = m + c(t),
    // expanded in powers of m (binomially) and integrated over t by 3-point
    // Gauss-Legendre (exact for the degree-5 integrands); the coefficients come
    // out directly, with no extrapolation from small m
    const double gx[3] = {0.5 - 0.5 * std::sqrt(0.6), 0.5, 0.5 + 0.5 * std::sqrt(0.6)};
    const double gw[3] = {5.0 / 18, 8.0 / 18, 5.0 / 18};
    const double binom[4][4] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
    for (int p = 0; p < 4; ++p) {
        const double tg = tail(al, ga, p), th = tail(al + 1.0, gh, p);
        for (int q = 0; q <= p; ++q) {
            double acc = 0.0;
            for (int i = 0; i < 3; ++i) {
                const double t = gx[i], c0 = sg - 1.0 + t, c1 = sg + t;
                const double e = (double)(p - q);
                acc += gw[i] * (k1 * tg * std::pow(c0, e) + k2 * th * t * (1.0 - t) * (std::pow(c1, e) - std::pow(c0, e)));
            }
            fit.poly[q] += binom[p][q] * acc;
        }
    }
    // check against the exact weights for every m the recursion serves
    double worst = 0.0;
    for (int64_t m = 2; m <= M - 2; ++m) {
        double v = fit.poly[0] + m * (fit.poly[1] + m * (fit.poly[2] + m * fit.poly[3]));
        for (size_t k = 0; k < fit.rho.size(); ++k) v += fit.w[k] * std::pow(fit.rho[k], (double)m);
        const double c = l21s_cbase_accurate(al, sg, m);
        worst = std::max(worst, std::fabs(v - c) / std::fabs(c));
    }
    fit.max_rel_err = worst;
    return worst <= tol ? TSFCDE_OK : TSFCDE_EUNSUPPORTED;
}

// eta_j = kappa c_0^(j): kappa a_0 at level 0, kappa (a_0 + b_1) after
// (Lemma 1; the diagonal of A and B in (3.3)).
double eta_level(double alpha, double sigma, double kappa, int64_t j) {
    const double al = alpha, sg = sigma;
    const double a0 = std::pow(sg, 1.0 - al);
    if (j == 0) return kappa * a0;
    const double b1 = (std::pow(1.0 + sg, 2.0 - al) - std::pow(sg, 2.0 - al)) / (2.0 - al) -
                      0.5 * (std::pow(1.0 + sg, 1.0 - al) + std::pow(sg, 1.0 - al));
    return kappa * (a0 + b1);
}

// t_{j+sigma} = (j + sigma) tau (Lemma 1)
double level_time(const tsfcde_plan_s *pl, int64_t j) { return ((double)j + pl->sigma) * pl->tau; }

// x_i = a + i h, i = 1..n (Sec. 2.1)
double node(const tsfcde_plan_s *pl, int64_t i) { return pl->a + (double)i * pl->h; }

// f(x_i, t_{j+sigma}) from the problem's callback into the plan's f buffer
// (through a pinned staging array), for a level stepped without a device
// source; *d_f stays NULL (f = 0) when there is no callback.
int callback_source(tsfcde_plan_s *pl, int64_t j, const double **d_f) {
    *d_f = nullptr;
    if (!pl->fcb) return TSFCDE_OK;
    if (!pl->h_f && hipHostMalloc(reinterpret_cast<void **>(&pl->h_f), sizeof(double) * (size_t)pl->n) != hipSuccess) {
        pl->h_f = nullptr;
        return TSFCDE_EDEVICE;
    }
    HIPCHK(hipStreamSynchronize(pl->stream));  // the last copy out of h_f has finished
    const double t = level_time(pl, j);
    for (int64_t i = 0; i < pl->n; ++i) pl->h_f[i] = pl->fcb(node(pl, i + 1), t, pl->fuser);
    HIPCHK(hipMemcpyAsync(pl->fbuf, pl->h_f, sizeof(double) * (size_t)pl->n, hipMemcpyHostToDevice, pl->stream));
    *d_f = pl->fbuf;
    return TSFCDE_OK;
}

int level_step(tsfcde_plan_s *pl, const double *d_f, double *d_u_out, tsfcde_stats *st) {
    if (pl->level >= pl->M) return TSFCDE_EDONE;
    auto t0 = std::chrono::steady_clock::now();
    const int64_t j = pl->level, n = pl->n;
    if (!d_f) {
        if (int rc = callback_source(pl, j, &d_f)) return rc;
    }
    double *x = pl->U + (size_t)(j + 1) * pl->ldn;
    // Gohberg-Semencul levels (constant coefficients, j >= 1): the two solves
    // (3.4) before the first such level's right-hand side
    const bool gsf_level = pl->gsf && j >= 1;
    SolveOut gprep;
    if (gsf_level && !pl->gsf_ready) {
        if (int rc = gsf_prepare(pl, gprep)) return rc;
    }
    // initial guess: 0, u^j, or quadratic extrapolation (u^j below level 2)
    int warm = 0;
    if (pl->warm == TSFCDE_WS_PREV) warm = 1;
    if (pl->warm == TSFCDE_WS_EXTRAP) warm = j >= 2 ? 2 : (j >= 1 ? 1 : 0);
    const bool use_net = pl->warm == TSFCDE_WS_NET && pl->net && j >= 2 && !gsf_level;
    if (pl->warm == TSFCDE_WS_NET) warm = j >= 1 ? 1 : 0;
    if (gsf_level) warm = 0;
    int rc = level_rhs(pl, j, d_f, x, warm);
    if (rc) return rc;
    int guess = warm == 2 ? TSFCDE_WS_EXTRAP : (warm == 1 ? TSFCDE_WS_PREV : TSFCDE_WS_ZERO);
    if (use_net) {
        // the network's guess, kept only if its true residual is below that of
        // u^j (which the right-hand side pass left in r0sq); decided on the
        // device: the restart pass records the comparison, k_keep_better puts
        // u^j back when the network lost, and a second restart pass sets the
        // CGS state for whichever guess stayed
        const double *Uj = pl->U + (size_t)j * pl->ldn;
        tsfcde_net_sample smp{nullptr, Uj, Uj - pl->ldn, Uj - 2 * pl->ldn, {0, 0, 0, 0, 0}, 0.0f};
        level_features(pl, j, smp.feat);
        if ((rc = net_predict(pl->net, smp, n, x))) return rc;
        if ((rc = restart_launch(pl, j, x, 0.0))) return rc;
        hipLaunchKernelGGL(k_keep_better, dim3((unsigned)std::min<int64_t>(1024, (n + 255) / 256)), dim3(256), 0,
                           pl->stream, x, Uj, n, pl->sc);
        HIPCHK(hipGetLastError());
        if ((rc = restart_launch(pl, j, x, 0.0, 2))) return rc;  // only when u^j was put back
        guess = TSFCDE_WS_NET;  // replaced below by what the device decided
        warm = 2;  // the CGS state is set by a restart pass, as for extrapolation
    }
    HIPCHK(precond_level(pl, j));
    SolveOut so;
    int outer = 1;
    bool fp32 = !gsf_level && level_uses_fp32(pl, j), fell_back = false;
    {
        ProfScope ps(pl, 3);
        if (gsf_level) {
            // x = A^-1 g by the formula, then the acceptance check as after a
            // CGS solve; CGS continues from x only if the check fails
            if ((rc = gsf_apply(pl, x))) return rc;
            const bool no_bw = (pl->flags & (TSFCDE_FLAG_VERIFY | TSFCDE_FLAG_STRICT_RESIDUAL)) != 0;
            if ((rc = restart_launch(pl, j, x, no_bw ? 0.0 : BW_TOL))) return rc;
            if ((rc = fp64_cgs(pl, j, x, so))) return rc;
            guess = TSFCDE_WS_ZERO;
        } else if (fp32) {
            if ((rc = ir_solve(pl, j, x, so, outer, fell_back))) return rc;
        } else {
            if (warm == 2 && !use_net && (rc = restart_launch(pl, j, x, 0.0))) return rc;  // r0 = g - A x0
            if ((rc = fp64_cgs(pl, j, x, so))) return rc;
        }
    }
    const DevScalars hs = *pl->h_sc;
    double relres_true = so.relres_true;
    if (relres_true < 0 && (pl->flags & TSFCDE_FLAG_TRUE_RESIDUAL)) {
        const SymParams sA = symbol(pl, j, -pl->sigma, pl->A, false);
        InReal in{x, n, pl->A.C};
        OutTrueRes out = with_red(OutTrueRes{pl->g, n, pl->A.C}, pl, 3);
        HIPCHK(run_op<0>(pl, pl->A, pl->specA, sA, in, out, 0));
        if ((rc = poll(pl))) return rc;
        relres_true = pl->h_sc->gnorm2 > 0 ? std::sqrt(pl->h_sc->aux0 / pl->h_sc->gnorm2) : 0.0;
    }
    if (d_u_out) HIPCHK(hipMemcpyAsync(d_u_out, x, sizeof(double) * n, hipMemcpyDeviceToDevice, pl->stream));
    pl->level = j + 1;
    if (st) {
        st->iters = so.iters;
        st->outer_iters = fp32 ? outer : 1;
        st->restarts = so.restarts;
        st->status = so.code;
        st->relres = (fp32 && !fell_back) ? relres_true
                                           : (hs.gnorm2 > 0 ? std::sqrt(hs.rnorm2 / hs.gnorm2) : 0.0);
        st->relres_true = relres_true;
        st->backward_err = so.backward_err;
        st->precision_used = fp32 ? (fell_back ? TSFCDE_FP32_REFINED_FELL_BACK : TSFCDE_FP32_REFINED) : TSFCDE_FP64;
        st->guess = use_net ? (hs.netkept ? TSFCDE_WS_NET : TSFCDE_WS_PREV) : guess;
        st->method = gsf_level ? TSFCDE_METHOD_GSF
                               : (pl->krylov == TSFCDE_KRYLOV_BICGSTAB && !fp32 ? TSFCDE_METHOD_PBICGSTAB
                                                                               : TSFCDE_METHOD_PCGS);
        st->pad = 0;
        st->iters += gprep.iters;
        st->restarts += gprep.restarts;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return so.code;
}

// Pointers of every buffer of pl->lay inside the workspace ws.
void bind_workspace(tsfcde_plan_s *pl, char *ws) {
    pl->ws = ws;
    const Layout &L = pl->lay;
    pl->U = reinterpret_cast<double *>(ws + L.off_U);
    double *vec = reinterpret_cast<double *>(ws + L.off_vec);
    double **vp[11] = {&pl->H, &pl->g, &pl->r, &pl->rt, &pl->u, &pl->p, &pl->q, &pl->phat, &pl->vhat, &pl->uhat,
                       &pl->fbuf};
    for (int k = 0; k < 11; ++k) *vp[k] = vec + (size_t)k * pl->ldn;
    pl->Hq = vec + (size_t)11 * pl->ldn;
    pl->tmp = reinterpret_cast<double *>(ws + L.off_tmp);
    pl->w = reinterpret_cast<double *>(ws + L.off_w);
    pl->g0 = reinterpret_cast<double *>(ws + L.off_g0);
    pl->cb = reinterpret_cast<double *>(ws + L.off_cbase);
    pl->buf = reinterpret_cast<double2 *>(ws + L.off_buf);
    pl->bufP = reinterpret_cast<double2 *>(ws + L.off_bufP);
    pl->specA = reinterpret_cast<double2 *>(ws + L.off_specA);
    pl->specP = reinterpret_cast<double2 *>(ws + L.off_specP);
    pl->tw_all = reinterpret_cast<double2 *>(ws + L.off_tw);
    pl->A.lo = reinterpret_cast<double2 *>(ws + L.off_tw2A);
    pl->A.hi = pl->A.lo + pl->A.nlo;
    pl->P.lo = reinterpret_cast<double2 *>(ws + L.off_tw2P);
    pl->P.hi = pl->P.lo + pl->P.nlo;
    pl->A.tw = Tw2{pl->A.lo, pl->A.hi, pl->A.shift};
    pl->P.tw = Tw2{pl->P.lo, pl->P.hi, pl->P.shift};
    pl->bufB = reinterpret_cast<double2 *>(ws + L.off_bufB);
    pl->Bhat = reinterpret_cast<double2 *>(ws + L.off_Bhat);
    pl->chirp = reinterpret_cast<double2 *>(ws + L.off_chirp);
    pl->Ls = reinterpret_cast<double2 *>(ws + L.off_Ls);
    pl->wv = reinterpret_cast<double2 *>(ws + L.off_wv);
    pl->Wt = reinterpret_cast<double2 *>(ws + L.off_Wt);
    pl->specPj = reinterpret_cast<double2 *>(ws + L.off_specPj);
    pl->B.lo = reinterpret_cast<double2 *>(ws + L.off_tw2B);
    pl->B.hi = pl->B.lo + pl->B.nlo;
    pl->B.tw = Tw2{pl->B.lo, pl->B.hi, pl->B.shift};
    pl->part = reinterpret_cast<double *>(ws + L.off_part);
    pl->sc = reinterpret_cast<DevScalars *>(ws + L.off_sc);
    {
        float *v32 = reinterpret_cast<float *>(ws + L.off_v32);
        float **vq[NV32] = {&pl->r32, &pl->rt32, &pl->u32, &pl->p32, &pl->q32,
                            &pl->phat32, &pl->vhat32, &pl->uhat32, &pl->d32};
        for (int k = 0; k < NV32; ++k) *vq[k] = pl->fp32 ? v32 + (size_t)k * pl->ldn : nullptr;
        pl->buf32 = reinterpret_cast<float2 *>(ws + L.off_buf32);
        pl->bufP32 = reinterpret_cast<float2 *>(ws + L.off_bufP32);
        pl->specA32 = reinterpret_cast<float2 *>(ws + L.off_specA32);
        pl->specP32 = reinterpret_cast<float2 *>(ws + L.off_specP32);
        pl->specPj32 = reinterpret_cast<float2 *>(ws + L.off_specPj32);
    }
    if (pl->soe) {
        pl->soe_S = reinterpret_cast<double *>(ws + L.off_soe);
        pl->soe_rho = pl->soe_S + (size_t)(pl->soe_K + 4) * pl->ldn;
        pl->soe_w = pl->soe_rho + pl->soe_K;
    }
    if (pl->gsf) {
        char *g = ws + L.off_gsf;
        pl->gx = reinterpret_cast<double *>(g);
        pl->gy = pl->gx + pl->ldn;
        g += 2 * sizeof(double) * (size_t)pl->ldn;
        for (int w = 0; w < 4; ++w) pl->gspec[w] = reinterpret_cast<double2 *>(g + (size_t)w * al(sizeof(double2) * (size_t)pl->A.N));
    }
}

// Twiddle tables, the WSGD weights omega_0..omega_n and the two circulant
// spectra of W_beta (Sec. 3.2), queued on pl->stream into the bound workspace
// (everything a plan computes on the device before its first level).
hipError_t setup_spectra(tsfcde_plan_s *pl, double beta) {
    const int64_t n = pl->n;
    // twiddle tables
    hipLaunchKernelGGL(k_twiddle_packed, dim3(32), dim3(256), 0, pl->stream, pl->tw_all, PMAX_LOG2);
    for (RT *rt : {&pl->A, pl->p2 ? &pl->P : &pl->B})
        hipLaunchKernelGGL(k_twiddle_tw2, dim3(64), dim3(256), 0, pl->stream, rt->lo, rt->hi, rt->L, rt->shift,
                           rt->nhi);
    // WSGD weights omega_0..omega_n (Lemma 2, Lemma 3 recurrence)
    hipLaunchKernelGGL(k_grunwald, dim3(1), dim3(1024), 0, pl->stream, beta, n, pl->g0);
    {
        const double b2 = beta * beta;
        const double l1 = (b2 + 3.0 * beta + 2.0) / 12.0, l0 = (4.0 - b2) / 6.0,
                     lm1 = (b2 - 3.0 * beta + 2.0) / 12.0;
        hipLaunchKernelGGL(k_wsgd, dim3(256), dim3(256), 0, pl->stream, pl->g0, n, l1, l0, lm1, pl->w);
    }
    if (hipError_t e = hipGetLastError()) return e;
    // spectra: embedding of W (length 2n) and Strang s(W) (length n)
    {
        hipLaunchKernelGGL(k_embed_column, dim3(512), dim3(256), 0, pl->stream, pl->w, n, pl->A.L, pl->tmp);
        InReal in{pl->tmp, pl->A.L, pl->A.C};
        if (launch_col<-1>(pl, pl->A, in, out_spec(pl, pl->A), 0) != hipSuccess) return hipErrorLaunchFailure;
        SymParams sp{};
        if (launch_mid<2>(pl, pl->A, pl->buf, (const double2 *)nullptr, pl->specA, sp, 0) != hipSuccess)
            return hipErrorLaunchFailure;
        if (pl->prec == TSFCDE_PREC_TCHAN)
            hipLaunchKernelGGL(k_tchan_column, dim3(512), dim3(256), 0, pl->stream, pl->w, n, pl->tmp);
        else
            hipLaunchKernelGGL(k_strang_column, dim3(512), dim3(256), 0, pl->stream, pl->w, n, pl->tmp);
        if (pl->p2) {
            InReal inP{pl->tmp, n, pl->P.C};
            if (launch_col<-1>(pl, pl->P, inP, out_spec(pl, pl->P), 0) != hipSuccess) return hipErrorLaunchFailure;
            if (launch_mid<2>(pl, pl->P, pl->bufP, (const double2 *)nullptr, pl->specP, sp, 0) != hipSuccess)
                return hipErrorLaunchFailure;
        } else {
            // Bluestein set-up: chirp, the spectrum of its circular arrangement
            // (with the 1/L of the inverse transform folded in), then the Strang
            // spectrum lambda = DFT_n(strang column).
            const RT &B = pl->B;
            hipLaunchKernelGGL(k_chirp, dim3(256), dim3(256), 0, pl->stream, pl->chirp, n);
            hipLaunchKernelGGL(k_chirp_embed, dim3(256), dim3(256), 0, pl->stream, pl->chirp, n, B.N,
                               1.0 / (double)B.N, pl->Bhat);
            OutSpec o{pl->bufB, B.tw, B.C};
            o.partials = nullptr;
            if (launch_col<-1>(pl, B, InCplx{pl->Bhat, nullptr, nullptr, B.N, B.C}, o, 0) != hipSuccess)
                return hipErrorLaunchFailure;
            if (launch_row<4>(pl, pl->bufB, nullptr, pl->Bhat) != hipSuccess) return hipErrorLaunchFailure;
            if (bluestein(pl, nullptr, pl->tmp, pl->Ls) != hipSuccess) return hipErrorLaunchFailure;
        }
    }
    return hipGetLastError();
}

double sample(tsfcde_coef_fn fn, const double *arr, void *user, int64_t j, double t) {
    return fn ? fn(t, user) : arr[j];
}

}  // namespace

extern "C" {

static int workspace_bytes_impl(const tsfcde_problem *prob, bool force_general, size_t *bytes) {
    int rc = validate(prob);
    if (rc) return rc;
    if (!bytes) return TSFCDE_EINVAL;
    RT A, P, B;
    const bool p2 = rt_setup(A, P, B, prob->n, force_general);
    if (!partials_fit(A)) return TSFCDE_EUNSUPPORTED;
    int soe_terms = -1;
    if (prob->history_tol > 0.0) {
        SoeFit fit;
        if ((rc = soe_fit(prob->alpha, prob->M, prob->history_tol, fit))) return rc;
        soe_terms = (int)fit.rho.size();
    }
    *bytes = layout_for(prob->n, prob->M, A, P, B, p2, prob->precision == TSFCDE_FP32_REFINED,
                        (prob->flags & TSFCDE_FLAG_CONSTANT_GSF) != 0, soe_terms)
                 .total;
    return TSFCDE_OK;
}

int tsfcde_workspace_bytes(const tsfcde_problem *prob, size_t *bytes) {
    return workspace_bytes_impl(prob, false, bytes);
}

static int plan_create(const tsfcde_problem *prob, void *d_workspace, size_t bytes, void *stream,
                       bool force_general, tsfcde_plan_t *out) {
    if (!out) return TSFCDE_EINVAL;
    *out = nullptr;
    int rc = validate(prob);
    if (rc) return rc;
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255)) return TSFCDE_EINVAL;
    {
        RT A, P, B;
        rt_setup(A, P, B, prob->n, force_general);
        if (!partials_fit(A)) return TSFCDE_EUNSUPPORTED;
    }
    const int64_t n = prob->n, M = prob->M;
    tsfcde_plan_s *pl = new (std::nothrow) tsfcde_plan_s();
    if (!pl) return TSFCDE_ENOMEM;
    pl->alpha = prob->alpha;
    pl->beta = prob->beta;
    pl->a = prob->a;
    pl->b = prob->b;
    pl->T = prob->T;
    pl->n = n;
    pl->M = M;
    pl->h = (prob->b - prob->a) / (double)(n + 1);
    pl->tau = prob->T / (double)M;
    pl->sigma = 1.0 - prob->alpha / 2.0;
    pl->kappa = std::pow(pl->tau, -prob->alpha) / std::tgamma(2.0 - prob->alpha);
    pl->hb = std::pow(pl->h, -prob->beta);
    pl->rtol = prob->rtol > 0 ? prob->rtol : 1e-10;
    pl->maxit = prob->maxit > 0 ? prob->maxit : 500;
    pl->warm = prob->warm_start;
    pl->flags = prob->flags;
    pl->fcb = prob->f;
    pl->fuser = prob->f_user;
    pl->krylov = prob->krylov;
    pl->prec = prob->preconditioner;
    pl->qfac = pl->prec == TSFCDE_PREC_TCHAN ? (double)(n - 1) / (double)n : 1.0;
    // coefficients at t_{j+sigma}
    pl->gam.resize(M);
    pl->dp.resize(M);
    pl->dm.resize(M);
    for (int64_t j = 0; j < M; ++j) {
        const double t = level_time(pl, j);
        pl->gam[j] = sample(prob->gamma, prob->gamma_at, prob->coef_user, j, t);
        pl->dp[j] = sample(prob->dplus, prob->dplus_at, prob->coef_user, j, t);
        pl->dm[j] = sample(prob->dminus, prob->dminus_at, prob->coef_user, j, t);
        if (!std::isfinite(pl->gam[j]) || !std::isfinite(pl->dp[j]) || !std::isfinite(pl->dm[j]) ||
            pl->dp[j] < 0.0 || pl->dm[j] < 0.0) {
            delete pl;
            return TSFCDE_EINVAL;
        }
    }
    // L2-1sigma tables (Lemma 1)
    {
        const double al = prob->alpha, sg = pl->sigma;
        std::vector<double> av(M + 2), bv(M + 2, 0.0);
        av[0] = std::pow(sg, 1.0 - al);
        for (int64_t l = 1; l <= M + 1; ++l) {
            av[l] = std::pow(l + sg, 1.0 - al) - std::pow(l - 1 + sg, 1.0 - al);
            bv[l] = (std::pow(l + sg, 2.0 - al) - std::pow(l - 1 + sg, 2.0 - al)) / (2.0 - al) -
                    0.5 * (std::pow(l + sg, 1.0 - al) + std::pow(l - 1 + sg, 1.0 - al));
        }
        pl->eta.resize(M);
        pl->cbase.assign(M + 2, 0.0);
        pl->clast.assign(M + 1, 0.0);
        for (int64_t j = 0; j < M; ++j) pl->eta[j] = eta_level(al, sg, pl->kappa, j);
        for (int64_t m = 1; m <= M; ++m) pl->cbase[m] = av[m] + bv[m + 1] - bv[m];
        for (int64_t j = 1; j <= M; ++j) pl->clast[j] = av[j] - bv[j];
    }
    pl->p2 = rt_setup(pl->A, pl->P, pl->B, n, force_general);
    pl->ldn = ld_of(n);
    // |A|_2 <= eta + sigma (|gamma|/h + (d+ + d-) h^-beta sum_k |omega_k|): A is
    // eta I - sigma L with |Q|_2 <= 2 and |W|_2 <= max(|W|_1, |W|_inf) <= sum |omega_k|
    {
        const double b = prob->beta;
        const double l1 = (b * b + 3.0 * b + 2.0) / 12.0, l0 = (4.0 - b * b) / 6.0, lm1 = (b * b - 3.0 * b + 2.0) / 12.0;
        double gkm2 = 0.0, gkm1 = 0.0, gk = 1.0, sabs = 0.0;  // g_{k-2}, g_{k-1}, g_k (Lemma 3 recurrence)
        for (int64_t k = 0; k <= n; ++k) {
            if (k > 0) {
                gkm2 = gkm1;
                gkm1 = gk;
                gk = (1.0 - (b + 1.0) / (double)k) * gkm1;
            }
            const double om = l1 * gk + (k >= 1 ? l0 * gkm1 : 0.0) + (k >= 2 ? lm1 * gkm2 : 0.0);
            sabs += std::fabs(om);
        }
        pl->anorm.resize(M);
        for (int64_t j = 0; j < M; ++j)
            pl->anorm[j] = pl->eta[j] + pl->sigma * (std::fabs(pl->gam[j]) / pl->h + (pl->dp[j] + pl->dm[j]) * pl->hb * sabs);
    }
    pl->fp32 = prob->precision == TSFCDE_FP32_REFINED;
    pl->gsf = (prob->flags & TSFCDE_FLAG_CONSTANT_GSF) != 0;
    if (pl->gsf) {  // Algorithm 3 needs gamma, d_+- constant in t
        for (int64_t j = 1; j < M; ++j)
            if (pl->gam[j] != pl->gam[0] || pl->dp[j] != pl->dp[0] || pl->dm[j] != pl->dm[0]) {
                delete pl;
                return TSFCDE_EINVAL;
            }
    }
    SoeFit fit;
    if (prob->history_tol > 0.0) {
        if ((rc = soe_fit(prob->alpha, M, prob->history_tol, fit))) {
            delete pl;
            return rc;
        }
        pl->soe = true;
        pl->soe_K = (int)fit.rho.size();
        for (int p = 0; p < 4; ++p) pl->soe_poly.c[p] = fit.poly[p];
        pl->soe_err = fit.max_rel_err;
    }
    pl->lay = layout_for(n, M, pl->A, pl->P, pl->B, pl->p2, pl->fp32, pl->gsf, pl->soe ? pl->soe_K : -1);
    if (pl->fp32) {
        // |A| / eta <= 1 + sigma (|gamma|/h + (d+ + d-) h^-beta 2|omega_1|) / eta  (Remark 3.1, eig(Q))
        const double b = prob->beta;
        const double om1 = std::fabs(-b * (b * b + 3.0 * b + 2.0) / 12.0 + (4.0 - b * b) / 6.0);
        pl->kbound.resize(M);
        for (int64_t j = 0; j < M; ++j)
            pl->kbound[j] = 1.0 + pl->sigma *
                                      (std::fabs(pl->gam[j]) / pl->h + (pl->dp[j] + pl->dm[j]) * pl->hb * 2.0 * om1) /
                                      pl->eta[j];
    }
    if (bytes < pl->lay.total) {
        delete pl;
        return TSFCDE_ENOMEM;
    }
    if (hipGetDevice(&pl->device) != hipSuccess) {
        delete pl;
        return TSFCDE_EDEVICE;
    }
    pl->stream = reinterpret_cast<hipStream_t>(stream);
    bind_workspace(pl, reinterpret_cast<char *>(d_workspace));
    const Layout &L = pl->lay;
    auto fail = [&](int code) {
        if (pl->h_sc) (void)hipHostFree(pl->h_sc);
        delete pl;
        return code;
    };
    if (hipHostMalloc(reinterpret_cast<void **>(&pl->h_sc), sizeof(DevScalars)) != hipSuccess)
        return fail(TSFCDE_EDEVICE);
    // scalars: zero, rtol^2
    std::memset(pl->h_sc, 0, sizeof(DevScalars));
    pl->h_sc->rtol2 = pl->rtol * pl->rtol;
    pl->h_sc->done = 1;
    if (hipMemcpyAsync(pl->sc, pl->h_sc, sizeof(DevScalars), hipMemcpyHostToDevice, pl->stream) != hipSuccess)
        return fail(TSFCDE_EDEVICE);
    // stored levels and vectors start at zero (the pad of an odd-length row stays zero)
    if (hipMemsetAsync(pl->ws + L.off_U, 0, L.off_tmp - L.off_U, pl->stream) != hipSuccess) return fail(TSFCDE_EDEVICE);
    if (hipMemcpyAsync(pl->cb, pl->cbase.data(), sizeof(double) * (M + 1), hipMemcpyHostToDevice, pl->stream) !=
        hipSuccess)
        return fail(TSFCDE_EDEVICE);
    if (setup_spectra(pl, prob->beta) != hipSuccess) return fail(TSFCDE_EDEVICE);
    if (pl->soe && pl->soe_K > 0) {
        if (hipMemcpyAsync(pl->soe_rho, fit.rho.data(), sizeof(double) * pl->soe_K, hipMemcpyHostToDevice,
                           pl->stream) != hipSuccess ||
            hipMemcpyAsync(pl->soe_w, fit.w.data(), sizeof(double) * pl->soe_K, hipMemcpyHostToDevice, pl->stream) !=
                hipSuccess)
            return fail(TSFCDE_EDEVICE);
    }
    // FP32 copies of the spectra for the inner solve of the FP32-refined form
    if (pl->fp32) {
        hipLaunchKernelGGL(k_to_f32, dim3(512), dim3(256), 0, pl->stream, pl->specA, pl->specA32, pl->A.N);
        if (pl->p2)
            hipLaunchKernelGGL(k_to_f32, dim3(512), dim3(256), 0, pl->stream, pl->specP, pl->specP32, pl->P.N);
        if (hipGetLastError() != hipSuccess) return fail(TSFCDE_EDEVICE);
    }
    // u^0 = phi(x_i)
    {
        std::vector<double> u0(n, 0.0);
        if (prob->phi)
            for (int64_t i = 0; i < n; ++i) u0[i] = prob->phi(node(pl, i + 1), prob->phi_user);
        if (hipMemcpyAsync(pl->U, u0.data(), sizeof(double) * n, hipMemcpyHostToDevice, pl->stream) != hipSuccess)
            return fail(TSFCDE_EDEVICE);
        if (hipGetLastError() != hipSuccess) return fail(TSFCDE_EDEVICE);
        if (hipStreamSynchronize(pl->stream) != hipSuccess) return fail(TSFCDE_EDEVICE);
    }
    pl->level = 0;
    *out = pl;
    return TSFCDE_OK;
}

int tsfcde_plan(const tsfcde_problem *prob, void *d_workspace, size_t bytes, void *stream, tsfcde_plan_t *out) {
    return plan_create(prob, d_workspace, bytes, stream, false, out);
}

int tsfcde_set_state(tsfcde_plan_t pl, int64_t level, const double *d_U) {
    if (!pl || !d_U || level < 0 || level > pl->M) return TSFCDE_EINVAL;
    if (int rc = history_quiesce(pl)) return rc;  // no partial sum reads U while it changes
    HIPCHK(hipMemcpy2DAsync(pl->U, sizeof(double) * pl->ldn, d_U, sizeof(double) * pl->n, sizeof(double) * pl->n,
                            (size_t)(level + 1), hipMemcpyDeviceToDevice, pl->stream));
    pl->level = level;
    pl->soe_level = -1;  // the recursions no longer match the stored levels
    return TSFCDE_OK;
}

int tsfcde_step(tsfcde_plan_t pl, const double *d_f, double *d_u_out, tsfcde_stats *st) {
    if (!pl) return TSFCDE_EINVAL;
    return level_step(pl, d_f, d_u_out, st);
}

int tsfcde_solve(tsfcde_plan_t pl, const double *d_F, int64_t ldF, double *d_U_out, tsfcde_stats *per_level) {
    if (!pl) return TSFCDE_EINVAL;
    if (d_F && ldF < pl->n) return TSFCDE_EINVAL;
    if (pl->level >= pl->M) return TSFCDE_EDONE;
    while (pl->level < pl->M) {
        const int64_t j = pl->level;
        int rc = level_step(pl, d_F ? d_F + (size_t)j * ldF : nullptr, nullptr, per_level ? per_level + j : nullptr);
        if (rc) return rc;
    }
    if (d_U_out)
        HIPCHK(hipMemcpy2DAsync(d_U_out, sizeof(double) * pl->n, pl->U, sizeof(double) * pl->ldn,
                                sizeof(double) * pl->n, (size_t)(pl->M + 1), hipMemcpyDeviceToDevice, pl->stream));
    return TSFCDE_OK;
}

static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// y = op x at level j, queued on the plan's stream (arguments checked by the caller).
static int apply_queue(tsfcde_plan_t pl, int32_t op, int64_t j, const double *d_x, double *d_y) {
    const int64_t n = pl->n;
    if (op == TSFCDE_OP_A || op == TSFCDE_OP_B) {
        const double s = op == TSFCDE_OP_A ? -pl->sigma : 1.0 - pl->sigma;
        InReal in{d_x, n, pl->A.C};
        OutReal out{d_y, n, pl->A.C};
        out.partials = nullptr;
        HIPCHK(run_op<0>(pl, pl->A, pl->specA, symbol(pl, j, s, pl->A, false), in, out, 0));
    } else if (op == TSFCDE_OP_PINV && pl->p2) {
        InReal in{d_x, n, pl->P.C};
        OutReal out{d_y, n, pl->P.C};
        out.partials = nullptr;
        HIPCHK(run_op<1>(pl, pl->P, pl->specP, symbol(pl, j, -pl->sigma, pl->P, true), in, out, 0));
    } else if (op == TSFCDE_OP_PINV) {
        HIPCHK(precond_level(pl, j));
        InReal in{d_x, n, pl->A.C};
        OutReal out{d_y, n, pl->A.C};
        out.partials = nullptr;
        HIPCHK(run_op<0>(pl, pl->A, pl->specPj, unit_symbol(pl->A), in, out, 0));
    } else {
        return TSFCDE_EINVAL;
    }
    return TSFCDE_OK;
}

int tsfcde_apply(tsfcde_plan_t pl, int32_t op, int64_t j, const double *d_x, double *d_y) {
    if (!pl || !d_x || !d_y || j < 0 || j >= pl->M || !aligned16(d_x) || !aligned16(d_y)) return TSFCDE_EINVAL;
    if (int rc = apply_queue(pl, op, j, d_x, d_y)) return rc;
    HIPCHK(hipStreamSynchronize(pl->stream));
    harvest(pl);
    return TSFCDE_OK;
}

// ---- tsfcde_apply_noalloc: the same product or solve with every device
// buffer in a static array of this library (no allocation of any kind) ----
static __device__ __align__(256) char scratch[TSFCDE_NOALLOC_SCRATCH_BYTES];
static constexpr int NOALLOC_MAX_DEVICES = 64;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES];  // device address of `scratch` on each device
static std::mutex g_scratch_mu;

// The address of `scratch` on device dev (current), looked up once per device.
static int scratch_address(int dev, char **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TSFCDE_EDEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<char *>(g_scratch_ptr[dev]);
    return TSFCDE_OK;
}

int tsfcde_apply_noalloc(const tsfcde_problem *prob, int32_t op, int64_t j, const double *d_x, double *d_y,
                         void *stream) {
    if (int rc = validate(prob)) return rc;
    if (!d_x || !d_y || j < 0 || j >= prob->M || !aligned16(d_x) || !aligned16(d_y)) return TSFCDE_EINVAL;
    if (op != TSFCDE_OP_A && op != TSFCDE_OP_B && op != TSFCDE_OP_PINV) return TSFCDE_EINVAL;
    if (prob->n > TSFCDE_NOALLOC_NMAX) return TSFCDE_EUNSUPPORTED;
    tsfcde_plan_s pl;  // host state only; every device buffer lies in `scratch`
    pl.alpha = prob->alpha;
    pl.beta = prob->beta;
    pl.a = prob->a;
    pl.b = prob->b;
    pl.T = prob->T;
    pl.n = prob->n;
    pl.M = prob->M;
    pl.h = (prob->b - prob->a) / (double)(prob->n + 1);
    pl.tau = prob->T / (double)prob->M;
    pl.sigma = 1.0 - prob->alpha / 2.0;
    pl.kappa = std::pow(pl.tau, -prob->alpha) / std::tgamma(2.0 - prob->alpha);
    pl.hb = std::pow(pl.h, -prob->beta);
    pl.prec = prob->preconditioner;
    pl.qfac = pl.prec == TSFCDE_PREC_TCHAN ? (double)(pl.n - 1) / (double)pl.n : 1.0;
    pl.one_level = true;
    {
        const double t = level_time(&pl, j);
        pl.one_gam = sample(prob->gamma, prob->gamma_at, prob->coef_user, j, t);
        pl.one_dp = sample(prob->dplus, prob->dplus_at, prob->coef_user, j, t);
        pl.one_dm = sample(prob->dminus, prob->dminus_at, prob->coef_user, j, t);
        if (!std::isfinite(pl.one_gam) || !std::isfinite(pl.one_dp) || !std::isfinite(pl.one_dm) ||
            pl.one_dp < 0.0 || pl.one_dm < 0.0)
            return TSFCDE_EINVAL;
        pl.one_eta = eta_level(pl.alpha, pl.sigma, pl.kappa, j);
    }
    pl.p2 = rt_setup(pl.A, pl.P, pl.B, pl.n, false);
    if (!partials_fit(pl.A)) return TSFCDE_EUNSUPPORTED;
    pl.ldn = ld_of(pl.n);
    pl.lay = layout_for(pl.n, 1, pl.A, pl.P, pl.B, pl.p2, false);
    if (pl.lay.total > TSFCDE_NOALLOC_SCRATCH_BYTES) return TSFCDE_EUNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return TSFCDE_EDEVICE;
    char *ws = nullptr;
    if (int rc = scratch_address(dev, &ws)) return rc;
    pl.device = dev;
    pl.stream = reinterpret_cast<hipStream_t>(stream);
    bind_workspace(&pl, ws);
    HIPCHK(setup_spectra(&pl, prob->beta));
    return apply_queue(&pl, op, j, d_x, d_y);
}

int tsfcde_rhs(tsfcde_plan_t pl, int64_t j, const double *d_f, double *d_g) {
    if (!pl || !d_g || j < 0 || j >= pl->M || j > pl->level || !aligned16(d_g)) return TSFCDE_EINVAL;
    int rc = level_rhs(pl, j, d_f, pl->uhat, 0);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(d_g, pl->g, sizeof(double) * pl->n, hipMemcpyDeviceToDevice, pl->stream));
    HIPCHK(hipStreamSynchronize(pl->stream));
    harvest(pl);
    return TSFCDE_OK;
}

int tsfcde_weights(tsfcde_plan_t pl, double *d_w) {
    if (!pl || !d_w) return TSFCDE_EINVAL;
    HIPCHK(hipMemcpyAsync(d_w, pl->w, sizeof(double) * (pl->n + 1), hipMemcpyDeviceToDevice, pl->stream));
    HIPCHK(hipStreamSynchronize(pl->stream));
    return TSFCDE_OK;
}

int tsfcde_spectrum(tsfcde_plan_t pl, int32_t which, double *d_out) {
    if (!pl || !d_out) return TSFCDE_EINVAL;
    if (which == TSFCDE_SPEC_EMBED) {
        hipLaunchKernelGGL(k_spec_export, dim3(256), dim3(256), 0, pl->stream, pl->specA, pl->A.R, pl->A.C,
                           reinterpret_cast<double2 *>(d_out));
    } else if (which == TSFCDE_SPEC_STRANG && pl->p2) {
        hipLaunchKernelGGL(k_spec_export, dim3(256), dim3(256), 0, pl->stream, pl->specP, pl->P.R, pl->P.C,
                           reinterpret_cast<double2 *>(d_out));
    } else if (which == TSFCDE_SPEC_STRANG) {
        HIPCHK(hipMemcpyAsync(d_out, pl->Ls, sizeof(double2) * (size_t)(pl->n / 2 + 1), hipMemcpyDeviceToDevice,
                              pl->stream));
    } else {
        return TSFCDE_EINVAL;
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(pl->stream));
    return TSFCDE_OK;
}

const double *tsfcde_history(tsfcde_plan_t pl) { return pl ? pl->U : nullptr; }

int64_t tsfcde_history_ld(tsfcde_plan_t pl) { return pl ? pl->ldn : -1; }

int64_t tsfcde_embedding_length(tsfcde_plan_t pl) { return pl ? pl->A.L : -1; }

int tsfcde_history_soe_fit(double alpha, int64_t M, double tol, int32_t capacity, int32_t *terms, double *rho,
                           double *w, double *poly, double *max_rel_err) {
    if (!(alpha > 0.0 && alpha <= 1.0) || M < 1 || !(tol > 0.0) || capacity < 0) return TSFCDE_EINVAL;
    SoeFit fit;
    const int rc = soe_fit(alpha, M, tol, fit);
    if (terms) *terms = (int32_t)fit.rho.size();
    if (max_rel_err) *max_rel_err = fit.max_rel_err;
    if ((int)fit.rho.size() <= capacity) {
        for (size_t k = 0; k < fit.rho.size(); ++k) {
            if (rho) rho[k] = fit.rho[k];
            if (w) w[k] = fit.w[k];
        }
    }
    if (poly)
        for (int p = 0; p < 4; ++p) poly[p] = fit.poly[p];
    return rc;
}

double tsfcde_level_time(tsfcde_plan_t pl, int64_t j) {
    if (!pl || j < 0 || j >= pl->M) return std::nan("");
    return level_time(pl, j);
}

int tsfcde_nodes(tsfcde_plan_t pl, double *h_x) {
    if (!pl || !h_x) return TSFCDE_EINVAL;
    for (int64_t i = 0; i < pl->n; ++i) h_x[i] = node(pl, i + 1);
    return TSFCDE_OK;
}

int64_t tsfcde_level(tsfcde_plan_t pl) { return pl ? pl->level : -1; }

int tsfcde_profile(tsfcde_plan_t pl, int32_t cls, int32_t enable) {
    if (!pl || cls < 0 || cls >= NPROF || enable < 0) return TSFCDE_EINVAL;
    HIPCHK(hipStreamSynchronize(pl->stream));
    harvest(pl);
    pl->prof[cls].on = enable != 0;
    pl->prof[cls].period = enable > 0 ? enable : 1;
    pl->prof[cls].issued = 0;
    pl->prof[cls].launches = 0;
    pl->prof[cls].ms = 0.0;
    return TSFCDE_OK;
}

int tsfcde_profile_read(tsfcde_plan_t pl, int32_t cls, int64_t *launches, double *ms) {
    if (!pl || cls < 0 || cls >= NPROF) return TSFCDE_EINVAL;
    HIPCHK(hipStreamSynchronize(pl->stream));
    harvest(pl);
    if (launches) *launches = pl->prof[cls].launches;
    if (ms) *ms = pl->prof[cls].ms;
    return TSFCDE_OK;
}

int tsfcde_profile_issued(tsfcde_plan_t pl, int32_t cls, int64_t *issued) {
    if (!pl || cls < 0 || cls >= NPROF || !issued) return TSFCDE_EINVAL;
    *issued = pl->prof[cls].issued;
    return TSFCDE_OK;
}


int32_t tsfcde_net_param_count(void) { return NET_P; }

int tsfcde_net_workspace_bytes(int64_t max_points, int32_t max_batch, size_t *bytes) {
    if (!bytes || max_points < 1 || max_batch < 1 || max_batch > NET_WG_MAX) return TSFCDE_EINVAL;
    *bytes = net_layout(max_points, max_batch).total;
    return TSFCDE_OK;
}

int tsfcde_net_create(void *d_workspace, size_t bytes, int64_t max_points, int32_t max_batch, void *stream,
                      tsfcde_net_t *out) {
    if (!out || !d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255)) return TSFCDE_EINVAL;
    *out = nullptr;
    if (max_points < 1 || max_batch < 1 || max_batch > NET_WG_MAX) return TSFCDE_EINVAL;
    const NetLayout L = net_layout(max_points, max_batch);
    if (bytes < L.total) return TSFCDE_ENOMEM;
    tsfcde_net_s *nt = new (std::nothrow) tsfcde_net_s();
    if (!nt) return TSFCDE_ENOMEM;
    char *ws = reinterpret_cast<char *>(d_workspace);
    nt->stream = reinterpret_cast<hipStream_t>(stream);
    nt->max_points = max_points;
    nt->max_batch = max_batch;
    nt->theta = reinterpret_cast<float *>(ws + L.theta);
    nt->m = reinterpret_cast<float *>(ws + L.m);
    nt->v = reinterpret_cast<float *>(ws + L.v);
    nt->grad = reinterpret_cast<float *>(ws + L.grad);
    nt->wbf = reinterpret_cast<uint16_t *>(ws + L.wbf);
    nt->wt = reinterpret_cast<float *>(ws + L.wt);
    nt->wb = reinterpret_cast<float *>(ws + L.wb);
    nt->wm = reinterpret_cast<uint16_t *>(ws + L.wm);
    nt->X = reinterpret_cast<float *>(ws + L.X);
    nt->act = reinterpret_cast<float *>(ws + L.act);
    nt->y = reinterpret_cast<float *>(ws + L.y);
    nt->ystar = reinterpret_cast<float *>(ws + L.ystar);
    nt->dy = reinterpret_cast<float *>(ws + L.dy);
    nt->dz0 = reinterpret_cast<float *>(ws + L.dz0);
    nt->dz1 = reinterpret_cast<float *>(ws + L.dz1);
    nt->part = reinterpret_cast<float *>(ws + L.part);
    nt->s = reinterpret_cast<double *>(ws + L.s);
    nt->den = reinterpret_cast<double *>(ws + L.den);
    nt->lpart = reinterpret_cast<double *>(ws + L.lpart);
    nt->smp = reinterpret_cast<net::Sample *>(ws + L.smp);
    // parameters, optimiser state and the bfloat16 copy start at zero
    if (hipMemsetAsync(ws, 0, L.X, nt->stream) != hipSuccess || hipStreamSynchronize(nt->stream) != hipSuccess) {
        delete nt;
        return TSFCDE_EDEVICE;
    }
    *out = nt;
    return TSFCDE_OK;
}

int tsfcde_net_set_params(tsfcde_net_t nt, const float *h) {
    if (!nt || !h) return TSFCDE_EINVAL;
    NCHK(hipMemcpyAsync(nt->theta, h, 4 * (size_t)NET_P, hipMemcpyHostToDevice, nt->stream));
    hipLaunchKernelGGL(net::k_net_round, dim3((NET_P + 255) / 256), dim3(256), 0, nt->stream, nt->theta, nt->wbf,
                       NET_P);
    hipLaunchKernelGGL(k_fill<float>, dim3(64), dim3(256), 0, nt->stream, nt->m, 0.0f, (int64_t)NET_P);
    hipLaunchKernelGGL(k_fill<float>, dim3(64), dim3(256), 0, nt->stream, nt->v, 0.0f, (int64_t)NET_P);
    NCHK(hipGetLastError());
    NCHK(hipStreamSynchronize(nt->stream));
    nt->widened = false;
    nt->step = 0;
    return TSFCDE_OK;
}

int tsfcde_net_get_params(tsfcde_net_t nt, float *h) {
    if (!nt || !h) return TSFCDE_EINVAL;
    NCHK(hipMemcpyAsync(h, nt->theta, 4 * (size_t)NET_P, hipMemcpyDeviceToHost, nt->stream));
    NCHK(hipStreamSynchronize(nt->stream));
    return TSFCDE_OK;
}

int tsfcde_level_features(tsfcde_plan_t pl, int64_t j, float *f) {
    if (!pl || !f || j < 0 || j >= pl->M) return TSFCDE_EINVAL;
    level_features(pl, j, f);
    return TSFCDE_OK;
}

int tsfcde_net_train_step(tsfcde_net_t nt, const tsfcde_net_sample *h, int32_t count, int64_t n, float lr,
                          double *loss_out, float *h_grad) {
    if (!nt || !h || count < 1 || count > nt->max_batch || n < 1 || (int64_t)count * n > nt->max_points)
        return TSFCDE_EINVAL;
    for (int i = 0; i < count; ++i)
        if (!h[i].u_next || !h[i].u0 || !h[i].u1 || !h[i].u2) return TSFCDE_EINVAL;
    int rc = net_upload(nt, h, count);
    if (rc) return rc;
    if ((rc = net_forward(nt, count, n, true))) return rc;
    if ((rc = net_backward(nt, count, n))) return rc;
    if (lr != 0.0f) {
        nt->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.0f - std::pow(b1, (float)nt->step), c2 = 1.0f - std::pow(b2, (float)nt->step);
        hipLaunchKernelGGL(net::k_net_adam, dim3((NET_P + 255) / 256), dim3(256), 0, nt->stream, nt->theta, nt->m,
                           nt->v, nt->grad, nt->wbf, NET_P, lr, b1, b2, 1e-8f, c1, c2);
        NCHK(hipGetLastError());
        nt->widened = false;
    }
    double lp[NET_LOSS_WG];
    NCHK(hipMemcpyAsync(lp, nt->lpart, sizeof(lp), hipMemcpyDeviceToHost, nt->stream));
    if (h_grad) NCHK(hipMemcpyAsync(h_grad, nt->grad, 4 * (size_t)NET_P, hipMemcpyDeviceToHost, nt->stream));
    NCHK(hipStreamSynchronize(nt->stream));
    if (loss_out) {
        double t = 0.0;
        for (double v : lp) t += v;
        *loss_out = t / (double)count;
    }
    return TSFCDE_OK;
}

int tsfcde_net_predict(tsfcde_net_t nt, const tsfcde_net_sample *h, int64_t n, double *d_x0) {
    if (!nt || !h || !d_x0 || !h->u0 || !h->u1 || !h->u2 || n < 1) return TSFCDE_EINVAL;
    return net_predict(nt, *h, n, d_x0);
}

int tsfcde_plan_set_net(tsfcde_plan_t pl, tsfcde_net_t nt) {
    if (!pl) return TSFCDE_EINVAL;
    if (nt && (pl->n > nt->max_points || nt->stream != pl->stream)) return TSFCDE_EINVAL;
    pl->net = nt;
    return TSFCDE_OK;
}

int tsfcde_net_destroy(tsfcde_net_t nt) {
    if (!nt) return TSFCDE_EINVAL;
    (void)hipStreamSynchronize(nt->stream);
    delete nt;
    return TSFCDE_OK;
}

int tsfcde_destroy(tsfcde_plan_t pl) {
    if (!pl) return TSFCDE_EINVAL;
    (void)hipStreamSynchronize(pl->stream);
    (void)history_quiesce(pl);
    harvest(pl);
    if (pl->hs) (void)hipStreamDestroy(pl->hs);
    for (hipEvent_t e : {pl->ev_main, pl->ev_hist})
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : pl->event_pool) (void)hipEventDestroy(e);
    if (pl->h_sc) (void)hipHostFree(pl->h_sc);
    if (pl->h_f) (void)hipHostFree(pl->h_f);
    delete pl;
    return TSFCDE_OK;
}

const char *tsfcde_strerror(int s) {
    switch (s) {
        case TSFCDE_OK: return "ok";
        case TSFCDE_EINVAL: return "invalid argument";
        case TSFCDE_ENOMEM: return "workspace too small";
        case TSFCDE_EDEVICE: return "HIP runtime error";
        case TSFCDE_ENOCONV: return "Krylov iteration did not converge within maxit";
        case TSFCDE_EBREAKDOWN: return "CGS breakdown";
        case TSFCDE_ENONFINITE: return "non-finite value in the iteration";
        case TSFCDE_EDONE: return "all time levels already computed";
        case TSFCDE_EUNSUPPORTED: return "valid problem outside the supported sizes or forms";
        case TSFCDE_EACCEPT: return "the level's iterate failed the acceptance test after every restart";
        default: return "unknown status";
    }
}

}  // extern "C"

// ===========================================================================
// Batched form: many independent instances advanced one level at a time with
// grouped launches.  Instances with the same embedding length L share a
// transform geometry and form a group; every kernel of the level runs once per
// group, blockIdx.y selecting the instance, whose vectors, spectra, symbol and
// CGS scalars come from device descriptors rebuilt once per level.  Each
// instance stops on its own convergence flag (its later launches exit at once).
// All instances take the general path (Bluestein-built inverse Strang
// preconditioner), so they run the same kernel sequence.
// ===========================================================================
struct DoneRec {
    int done, status, iter, checked, nchecks, pad;
    double rnorm2, gnorm2, aux0, aux1;
};

namespace tsf {
__global__ void k_gather_state(DevScalars *const *__restrict__ scs, int count, DoneRec *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        const DevScalars *s = scs[i];
        DoneRec r;
        r.done = s->done;
        r.status = s->status;
        r.iter = s->iter;
        r.checked = s->checked;
        r.nchecks = s->nchecks;
        r.pad = 0;
        r.rnorm2 = s->rnorm2;
        r.gnorm2 = s->gnorm2;
        r.aux0 = s->aux0;
        r.aux1 = s->aux1;
        out[i] = r;
    }
}

// Instances the host has stopped (restarts or iterations exhausted) are
// marked done and checked, so that no later launch of the level, predicated
// or not on a list, touches them again.
__global__ void k_retire(DevScalars *const *__restrict__ scs, const int *__restrict__ list, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) {
        DevScalars *s = scs[list[k]];
        s->done = 1;
        s->checked = 1;
    }
}
}  // namespace tsf

namespace {

struct ChunkGraph {
    hipGraphExec_t exec;
    const void *key;  // descriptor address the capture read
};

// The descriptors of one group for a level, staged for upload (pointers into
// the device staging area).
struct GroupDesc {
    ColDesc<InReal, OutSpec> *rhsA, *rstA, *r2cA, *s4;
    ColDesc<InSpec, OutRhs> *rhsC;
    ColDesc<InSpec, OutRestart> *rstC, *vfyC;
    MidDesc *midA, *midR2C, *midP;
    ColDesc<InCplx, OutSpec> *bsA;
    RowDesc *bsRow;
    ColDesc<InSpec, OutCplx> *bsC;
    // CGS passes.  Folded finishing steps read and write parity slots that
    // depend on the iteration's index ci in its chunk, so the two folding
    // passes and the chunk's closing finishing kernel come in variants:
    // s1[v]: v = 0 (ci = 0, no fold), 1 (ci = 1), 2 (even ci >= 2), 3 (odd ci >= 3);
    // s7[v], s12[v]: v = 0 (ci = 0), 1 (odd ci), 2 (even ci >= 2).
    ColDesc<InCgsUP, OutSpec> *s1[4];
    ColDesc<InSpec, OutReal> *s3, *s9;
    ColDesc<InSpec, OutCgsDot> *s6;
    ColDesc<InCgsQ, OutSpec> *s7[3], *s7_plain;
    ColDesc<InCgsX, OutSpec> *s10;
    ColDesc<InSpec, OutCgsR> *s12[3];
};

struct BatchGroup {
    int64_t L = 0;
    RT A, B;
    std::vector<int> members;
    int e_mid = TSF_E_MID;  // values per lane of the group's middle passes (autotuned)
    int slot = 0;           // the group's stream (the largest groups on different ones)
    GroupDesc fixed{};      // the descriptors that are the same at every level
};

// bump allocator mirroring a pinned host staging area onto a device area
struct Stage {
    char *host = nullptr, *dev = nullptr;
    size_t cap = 0, used = 0;
    template <class T> T *put(const std::vector<T> &v) {
        const size_t off = used;
        const size_t bytes = sizeof(T) * v.size();
        used = (used + bytes + 255) & ~size_t(255);
        if (used > cap) return nullptr;
        std::memcpy(host + off, v.data(), bytes);
        return reinterpret_cast<T *>(dev + off);
    }
};

}  // namespace

struct tsfcde_batch_s {
    hipStream_t stream = nullptr;
    int count = 0;
    int64_t M = 0, level = 0;
    int maxit = 500, warm = 0;
    std::vector<tsfcde_plan_s *> plans;
    std::vector<BatchGroup> groups;
    Stage st;
    size_t st_fixed = 0;   // end of the fixed descriptors in the staging area (its start)
    size_t st_levels = 0;  // end of the per-instance level slots (after the fixed ones)
    DevScalars **d_scs = nullptr;
    DoneRec *d_done = nullptr, *h_done = nullptr;
    bool fold = true;  // finishing steps folded into later passes (TSFCDE_FLAG_NO_FOLD clears it)
    bool strict = false;  // TSFCDE_FLAG_STRICT_RESIDUAL: accept only at a true residual within rtol |g|
    bool graphs = false;  // TSFCDE_FLAG_GRAPHS: CGS chunks replayed from captured HIP graphs
    hipStream_t cap_stream = nullptr;  // private stream the chunk graphs are captured on
    std::map<int, ChunkGraph> chunk_graphs;  // by chunk length
    // instance lists of a round (per group: starting, extrapolating and
    // iterating instances as group-local positions; then the instances to
    // retire), staged in pinned memory and copied to the device
    const int *act = nullptr;  // list the grouped launches read (null: every instance)
    int *h_act = nullptr, *d_act = nullptr;
    // streams the groups' set-up and rounds run on (none with chunk graphs),
    // and their joins with the batch stream; groups by size, largest first
    std::vector<hipStream_t> gstreams;
    std::vector<size_t> group_order;
    hipEvent_t ev_go = nullptr;
    std::vector<hipEvent_t> ev_done;
    // per instance: CGS iterations to its first stop and in all at the last
    // level (the estimates that size the next level's chunks before and after
    // a failed acceptance check)
    std::vector<int> conv_iters, final_iters;
    std::vector<char> conv_seen;
};

namespace {

template <int R, int DIR, class In, class Out>
hipError_t blaunch_col_t(tsfcde_batch_s *bt, int64_t C, const ColDesc<In, Out> *d, int cnt, int pred, bool finish) {
    using G = ColGeo<R, TSF_E_COL>;
    const int64_t grid = (C + G::B - 1) / G::B;
    hipLaunchKernelGGL((k_col_b<R, TSF_E_COL, DIR, In, Out>), dim3((unsigned)grid, cnt), dim3(G::NT), 0, bt->stream,
                       d, bt->act, bt->plans[0]->tw_all, pred);
    if constexpr (Out::NACC > 0) {
        if (finish)
            hipLaunchKernelGGL((k_final_b<G::NT, In, Out>), dim3(1, cnt), dim3(G::NT), 0, bt->stream, d, bt->act,
                               (int)grid, pred);
    }
    return hipGetLastError();
}

template <int R, class In, class Out>
hipError_t bfinal_t(tsfcde_batch_s *bt, int64_t C, const ColDesc<In, Out> *d, int cnt, int pred) {
    using G = ColGeo<R, TSF_E_COL>;
    hipLaunchKernelGGL((k_final_b<G::NT, In, Out>), dim3(1, cnt), dim3(G::NT), 0, bt->stream, d, bt->act,
                       (int)((C + G::B - 1) / G::B), pred);
    return hipGetLastError();
}

template <int DIR, class In, class Out>
hipError_t blaunch_col(tsfcde_batch_s *bt, const RT &rt, const ColDesc<In, Out> *d, int cnt, int pred,
                       bool finish = true) {
    if (!d) return hipErrorOutOfMemory;
    switch (rt.R) {
#define TSF_CASE(P) \
    case P: return blaunch_col_t<P, DIR>(bt, rt.C, d, cnt, pred, finish);
        TSF_SIZES(TSF_CASE)
#undef TSF_CASE
        default: return hipErrorInvalidValue;
    }
}

// Finishing kernel of a grouped column pass launched without its own.
template <class In, class Out>
hipError_t bfinal(tsfcde_batch_s *bt, const RT &rt, const ColDesc<In, Out> *d, int cnt, int pred) {
    if (!d) return hipErrorOutOfMemory;
    switch (rt.R) {
#define TSF_CASE(P) \
    case P: return bfinal_t<P>(bt, rt.C, d, cnt, pred);
        TSF_SIZES(TSF_CASE)
#undef TSF_CASE
        default: return hipErrorInvalidValue;
    }
}

template <int C_, int E, int MODE>
hipError_t blaunch_mid_e(tsfcde_batch_s *bt, const RT &rt, const MidDesc *d, int cnt, int pred) {
    using G = MidGeo<C_, E>;
    hipLaunchKernelGGL((k_mid_b<C_, E, MODE>), dim3((unsigned)(rt.R / 2), cnt), dim3(G::NT), 0, bt->stream, d,
                       bt->act, bt->plans[0]->tw_all, pred);
    return hipGetLastError();
}

// Values per lane the batch's middle passes can take (the tuner picks one
// per group): 4 or the default 8 on rows of 16..1024 points.
constexpr int TUNE_E_ALT = 4;
template <int C_, int MODE>
hipError_t blaunch_mid_t(tsfcde_batch_s *bt, const RT &rt, const MidDesc *d, int cnt, int pred, int e) {
    if constexpr (C_ >= 16 && C_ <= 1024) {
        if (e == TUNE_E_ALT) return blaunch_mid_e<C_, TUNE_E_ALT, MODE>(bt, rt, d, cnt, pred);
    }
    return blaunch_mid_e<C_, TSF_E_MID, MODE>(bt, rt, d, cnt, pred);
}

template <int MODE>
hipError_t blaunch_mid(tsfcde_batch_s *bt, const RT &rt, const MidDesc *d, int cnt, int pred, int e = TSF_E_MID) {
    if (!d) return hipErrorOutOfMemory;
    switch (rt.C) {
#define TSF_CASE(P) \
    case P: return blaunch_mid_t<P, MODE>(bt, rt, d, cnt, pred, e);
        TSF_SIZES(TSF_CASE)
#undef TSF_CASE
        default: return hipErrorInvalidValue;
    }
}

template <int C_>
hipError_t blaunch_row_t(tsfcde_batch_s *bt, const RT &rt, const RowDesc *d, int cnt) {
    using G = RowGeo<C_, TSF_E_MID>;
    hipLaunchKernelGGL((k_row_b<C_, TSF_E_MID, 3>), dim3((unsigned)rt.R, cnt), dim3(G::NT), 0, bt->stream, d,
                       bt->act, bt->plans[0]->tw_all);
    return hipGetLastError();
}

hipError_t blaunch_row(tsfcde_batch_s *bt, const RT &rt, const RowDesc *d, int cnt) {
    if (!d) return hipErrorOutOfMemory;
    switch (rt.C) {
#define TSF_CASE(P) \
    case P: return blaunch_row_t<P>(bt, rt, d, cnt);
        TSF_SIZES(TSF_CASE)
#undef TSF_CASE
        default: return hipErrorInvalidValue;
    }
}

template <class In, class Out> ColDesc<In, Out> cdesc(tsfcde_plan_s *pl, int64_t C, In in, Out out) {
    return ColDesc<In, Out>{C, in, out, pl->sc};
}

template <class Out> Out nored(Out o) {
    o.partials = nullptr;
    return o;
}


int s1_variant(int ci) { return ci <= 1 ? ci : 2 + (ci & 1); }
int s7_variant(int ci) { return ci == 0 ? 0 : ((ci & 1) ? 1 : 2); }

// Descriptors of one group that stay the same at every level (the CGS passes
// other than x's update, the preconditioner's construction and solve),
// staged once when the batch is planned.
bool stage_group_fixed(tsfcde_batch_s *bt, const BatchGroup &g, GroupDesc &D) {
    std::vector<ColDesc<InReal, OutSpec>> r2cA, s4;
    std::vector<MidDesc> midR2C, midP;
    std::vector<ColDesc<InCplx, OutSpec>> bsA;
    std::vector<RowDesc> bsRow;
    std::vector<ColDesc<InSpec, OutCplx>> bsC;
    std::vector<ColDesc<InCgsUP, OutSpec>> s1[4];
    std::vector<ColDesc<InSpec, OutReal>> s3, s9;
    std::vector<ColDesc<InSpec, OutCgsDot>> s6;
    std::vector<ColDesc<InCgsQ, OutSpec>> s7[3], s7_plain;
    std::vector<ColDesc<InSpec, OutCgsR>> s12[3];
    const int fnparts = col_grid(g.A);
    for (int idx : g.members) {
        tsfcde_plan_s *pl = bt->plans[idx];
        const int64_t n = pl->n, C = pl->A.C, CB = pl->B.C;
        const SymParams sI = unit_symbol(pl->A);
        OutSpec osA = out_spec(pl, pl->A);
        InSpec isA = in_spec(pl, pl->A);
        // inverse Strang circulant of a level: Bluestein DFT and embedding spectrum
        OutSpec osB{pl->bufB, pl->B.tw, CB};
        bsA.push_back(cdesc(pl, CB, InCplx{pl->wv, nullptr, pl->chirp, n, CB}, nored(osB)));
        bsRow.push_back(RowDesc{pl->bufB, pl->Bhat, nullptr});
        bsC.push_back(cdesc(pl, CB, InSpec{pl->bufB, pl->B.tw, CB}, nored(OutCplx{pl->Wt, pl->chirp, n, CB})));
        r2cA.push_back(cdesc(pl, C, InReal{pl->tmp, pl->A.L, C}, osA));
        midR2C.push_back(MidDesc{pl->A.R, pl->buf, nullptr, pl->specPj, pl->A.tw, SymParams{}, pl->sc});
        midP.push_back(MidDesc{pl->A.R, pl->buf, pl->specPj, nullptr, pl->A.tw, sI, pl->sc});
        // CGS iteration
        for (int v = 0; v < 4; ++v) {
            InCgsUP in{pl->r, pl->u, pl->p, pl->q, n, C, 0.0, false};
            if (v > 0) {  // representative chunk index of the variant: 1, 2, 3
                in.fpart = pl->part + (size_t)1 * PARTIAL_SLOTS;
                in.fnparts = fnparts;
                in.ci = v;
            }
            s1[v].push_back(cdesc(pl, C, in, osA));
        }
        s3.push_back(cdesc(pl, C, isA, nored(OutReal{pl->phat, n, C})));
        s4.push_back(cdesc(pl, C, InReal{pl->phat, n, C}, osA));
        s6.push_back(cdesc(pl, C, isA, with_red(OutCgsDot{pl->vhat, pl->rt, n, C}, pl, 0)));
        s7_plain.push_back(cdesc(pl, C, InCgsQ{pl->u, pl->vhat, pl->q, n, C, 0.0}, osA));
        for (int v = 0; v < 3; ++v) {
            InCgsQ in{pl->u, pl->vhat, pl->q, n, C, 0.0};
            in.fpart = pl->part;  // site 0
            in.fnparts = fnparts;
            in.ci = v;  // 0, 1 (odd), 2 (even >= 2)
            s7[v].push_back(cdesc(pl, C, in, osA));
            OutCgsR out = with_red(OutCgsR{pl->r, pl->rt, n, C, 0.0}, pl, 1);
            out.ci = v;
            s12[v].push_back(cdesc(pl, C, isA, out));
        }
        s9.push_back(cdesc(pl, C, isA, nored(OutReal{pl->uhat, n, C})));
    }
    Stage &S = bt->st;
    D.bsA = S.put(bsA);
    D.bsRow = S.put(bsRow);
    D.bsC = S.put(bsC);
    D.r2cA = S.put(r2cA);
    D.midR2C = S.put(midR2C);
    D.midP = S.put(midP);
    for (int v = 0; v < 4; ++v) D.s1[v] = S.put(s1[v]);
    D.s3 = S.put(s3);
    D.s4 = S.put(s4);
    D.s6 = S.put(s6);
    for (int v = 0; v < 3; ++v) {
        D.s7[v] = S.put(s7[v]);
        D.s12[v] = S.put(s12[v]);
    }
    D.s7_plain = S.put(s7_plain);
    D.s9 = S.put(s9);
    return S.used <= S.cap;
}

// Descriptors that depend on an instance's level (its right-hand side, the
// product's symbol, x = u^{j+1}, the acceptance check): one slot per
// instance in each of the group's arrays, reserved when the batch is planned
// and rewritten in the pinned staging copy whenever an instance starts a
// level, so that instances of one group may be at different levels.
bool reserve_group_levels(tsfcde_batch_s *bt, const BatchGroup &g, GroupDesc &D) {
    const size_t c = g.members.size();
    Stage &S = bt->st;
    D.rhsA = S.put(std::vector<ColDesc<InReal, OutSpec>>(c));
    D.rhsC = S.put(std::vector<ColDesc<InSpec, OutRhs>>(c));
    D.midA = S.put(std::vector<MidDesc>(c));
    D.rstA = S.put(std::vector<ColDesc<InReal, OutSpec>>(c));
    D.rstC = S.put(std::vector<ColDesc<InSpec, OutRestart>>(c));
    D.vfyC = S.put(std::vector<ColDesc<InSpec, OutRestart>>(c));
    D.s10 = S.put(std::vector<ColDesc<InCgsX, OutSpec>>(c));
    return S.used <= S.cap;
}

template <class T> T *host_slot(Stage &S, T *dev, size_t k) {
    return reinterpret_cast<T *>(S.host + (reinterpret_cast<char *>(dev) - S.dev)) + k;
}

// Writes the level-j descriptors of instance idx (position k in group g)
// into the pinned staging copy; f is its source at level j, warm its guess.
void stage_member_level(tsfcde_batch_s *bt, const GroupDesc &D, size_t k, int idx, int64_t j, const double *f,
                        int warm) {
    tsfcde_plan_s *pl = bt->plans[idx];
    Stage &S = bt->st;
    const int64_t n = pl->n, ld = pl->ldn, C = pl->A.C;
    double *x = pl->U + (size_t)(j + 1) * ld;
    const SymParams sA = symbol(pl, j, -pl->sigma, pl->A, false);
    OutSpec osA = out_spec(pl, pl->A);
    InSpec isA = in_spec(pl, pl->A);
    // right-hand side through A u^j
    *host_slot(S, D.rhsA, k) = cdesc(pl, C, InReal{pl->U + (size_t)j * ld, n, C}, osA);
    OutRhs orhs{pl->U + (size_t)j * ld, j >= 1 ? hist_src(pl, j) : nullptr, f, pl->g, pl->r, pl->rt, x, n, C,
                pl->eta[j] / pl->sigma - (j >= 1 ? hist_c1(pl, j) : 0.0), (1.0 - pl->sigma) / pl->sigma, warm,
                j >= 1 ? 1 : 0,
                j >= 2 ? pl->U + (size_t)(j - 1) * ld : nullptr, j >= 2 ? pl->U + (size_t)(j - 2) * ld : nullptr};
    *host_slot(S, D.rhsC, k) = cdesc(pl, C, isA, with_red(orhs, pl, 2));
    *host_slot(S, D.midA, k) = MidDesc{pl->A.R, pl->buf, pl->specA, nullptr, pl->A.tw, sA, pl->sc};
    // restart from an extrapolated guess
    *host_slot(S, D.rstA, k) = cdesc(pl, C, InReal{x, n, C}, osA);
    *host_slot(S, D.rstC, k) =
        cdesc(pl, C, isA, with_red(OutRestart{pl->g, x, pl->r, pl->rt, n, C, pl->anorm[j], 0.0}, pl, 3));
    // acceptance check of a converged instance (backward error)
    OutRestart ovfy =
        with_red(OutRestart{pl->g, x, pl->r, pl->rt, n, C, pl->anorm[j], bt->strict ? 0.0 : BW_TOL}, pl, 3);
    ovfy.check = 1;  // counted in nchecks: the host learns that the check ran
    *host_slot(S, D.vfyC, k) = cdesc(pl, C, isA, ovfy);
    // CGS: x += alpha uhat
    *host_slot(S, D.s10, k) = cdesc(pl, C, InCgsX{pl->uhat, x, n, C, 0.0}, osA);
}

#define BCHK(x)                                             \
    do {                                                    \
        hipError_t e_ = (x);                                \
        if (e_ != hipSuccess) return TSFCDE_EDEVICE;        \
    } while (0)

#define TSF_TRY(x)                             \
    do {                                       \
        if ((e = (x)) != hipSuccess) return e; \
    } while (0)

// Iteration k (0-based) of a chunk of CGS over one group's `c` instances (all
// of them, or the ones bt->act lists), as launches on bt->stream.  With
// folding, the two reductions' finishing steps run inside the next passes
// and the chunk ends with one finishing kernel (issue_group_close).
hipError_t issue_group_iteration(tsfcde_batch_s *bt, const BatchGroup &G, const GroupDesc &D, int c, int k) {
    const bool fold = bt->fold;
    hipError_t e = hipSuccess;
    TSF_TRY(blaunch_col<-1>(bt, G.A, D.s1[fold ? s1_variant(k) : 0], c, 1));
    TSF_TRY(blaunch_mid<0>(bt, G.A, D.midP, c, 1, G.e_mid));
    TSF_TRY(blaunch_col<1>(bt, G.A, D.s3, c, 1));
    TSF_TRY(blaunch_col<-1>(bt, G.A, D.s4, c, 1));
    TSF_TRY(blaunch_mid<0>(bt, G.A, D.midA, c, 1, G.e_mid));
    TSF_TRY(blaunch_col<1>(bt, G.A, D.s6, c, 1, !fold));
    if (fold) {
        TSF_TRY(blaunch_col<-1>(bt, G.A, D.s7[s7_variant(k)], c, 1));
    } else {
        TSF_TRY(blaunch_col<-1>(bt, G.A, D.s7_plain, c, 1));
    }
    TSF_TRY(blaunch_mid<0>(bt, G.A, D.midP, c, 1, G.e_mid));
    TSF_TRY(blaunch_col<1>(bt, G.A, D.s9, c, 1));
    TSF_TRY(blaunch_col<-1>(bt, G.A, D.s10, c, 1));
    TSF_TRY(blaunch_mid<0>(bt, G.A, D.midA, c, 1, G.e_mid));
    TSF_TRY(blaunch_col<1>(bt, G.A, D.s12[0], c, 1, !fold));
    return e;
}

// The finishing kernel that closes a folded chunk of `todo` iterations.
hipError_t issue_group_close(tsfcde_batch_s *bt, const BatchGroup &G, const GroupDesc &D, int c, int todo) {
    if (!bt->fold || todo <= 0) return hipSuccess;
    return bfinal(bt, G.A, D.s12[s7_variant(todo - 1)], c, 1);
}

// The acceptance check of one group's `c` instances, queued behind a chunk:
// y = A x, r = g - y and the backward-error test, run by the device only for
// instances the chunk stopped that no check has confirmed yet (pred 3).  One
// that fails restarts CGS from x.
hipError_t issue_group_check(tsfcde_batch_s *bt, const BatchGroup &G, const GroupDesc &D, int c) {
    hipError_t e = hipSuccess;
    TSF_TRY(blaunch_col<-1>(bt, G.A, D.rstA, c, 3));
    TSF_TRY(blaunch_mid<0>(bt, G.A, D.midA, c, 3, G.e_mid));
    TSF_TRY(blaunch_col<1>(bt, G.A, D.vfyC, c, 3));
    return e;
}

// `todo` CGS iterations of every group over all its instances (the form the
// chunk graphs capture).
hipError_t issue_chunk(tsfcde_batch_s *bt, const std::vector<GroupDesc> &gd, int todo) {
    hipError_t e = hipSuccess;
    for (int k = 0; k < todo; ++k)
        for (size_t g = 0; g < bt->groups.size(); ++g)
            TSF_TRY(issue_group_iteration(bt, bt->groups[g], gd[g], (int)bt->groups[g].members.size(), k));
    for (size_t g = 0; g < bt->groups.size(); ++g)
        TSF_TRY(issue_group_close(bt, bt->groups[g], gd[g], (int)bt->groups[g].members.size(), todo));
    return e;
}

// The chunk of `todo` iterations as an instantiated HIP graph, captured from
// issue_chunk the first time that length is needed.  Its kernels read every
// level-dependent value (symbols, scalars, vector addresses) from the staged
// descriptors and the device scalars, never from their launch arguments, so
// one capture serves every level while the descriptors sit at the same
// addresses (checked; a change recaptures).  Kernels only: no memset or copy
// nodes.  The capture runs on a private stream (the batch's own may be the
// null stream, which cannot capture); the graph is launched on the batch's.
int chunk_graph(tsfcde_batch_s *bt, const std::vector<GroupDesc> &gd, int todo, hipGraphExec_t *out) {
    const void *key = gd.empty() ? nullptr : (const void *)gd[0].s1[0];
    auto it = bt->chunk_graphs.find(todo);
    if (it != bt->chunk_graphs.end() && it->second.key == key) {
        *out = it->second.exec;
        return TSFCDE_OK;
    }
    if (it != bt->chunk_graphs.end()) {
        (void)hipGraphExecDestroy(it->second.exec);
        bt->chunk_graphs.erase(it);
    }
    if (!bt->cap_stream) BCHK(hipStreamCreateWithFlags(&bt->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    BCHK(hipStreamBeginCapture(bt->cap_stream, hipStreamCaptureModeThreadLocal));
    hipStream_t own = bt->stream;
    bt->stream = bt->cap_stream;  // issue_chunk launches on bt->stream
    const hipError_t e = issue_chunk(bt, gd, todo);
    bt->stream = own;
    const hipError_t ec = hipStreamEndCapture(bt->cap_stream, &graph);
    if (e != hipSuccess || ec != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();  // leave no sticky error behind
        return TSFCDE_EDEVICE;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess || !ex) return TSFCDE_EDEVICE;
    bt->chunk_graphs[todo] = ChunkGraph{ex, key};
    *out = ex;
    return TSFCDE_OK;
}

// ---- autotuner of the batch's middle passes ---------------------------------
// A group's middle passes (the row FFTs with the symbol, most of a product's
// time) can hold 4 or 8 values per lane; which is faster depends on the row
// length and on how many instances share the launch.  plan_batch times both
// on the group's own buffers and keeps the faster.  Choices are cached per
// process by (row length, rows, instances) and, when the environment variable
// TSFCDE_TUNE_CACHE names a file, in that file too (one line per choice:
// "mid <C> <R> <instances> <E> <us E=4> <us E=8>"), read before tuning.
struct TuneKey {
    int64_t C, R;
    int count;
    bool operator<(const TuneKey &o) const {
        return C != o.C ? C < o.C : (R != o.R ? R < o.R : count < o.count);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune_cache;
bool g_tune_file_read = false;

void tune_cache_read() {
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const char *path = std::getenv("TSFCDE_TUNE_CACHE");
    if (!path) return;
    FILE *fh = std::fopen(path, "r");
    if (!fh) return;
    char kind[16];
    long long c, r;
    int cnt, e;
    double t4, t8;
    while (std::fscanf(fh, "%15s %lld %lld %d %d %lf %lf", kind, &c, &r, &cnt, &e, &t4, &t8) == 7)
        if (std::strcmp(kind, "mid") == 0 && (e == TUNE_E_ALT || e == TSF_E_MID)) g_tune_cache[TuneKey{c, r, cnt}] = e;
    std::fclose(fh);
}

void tune_cache_append(const TuneKey &k, int e, double t4, double t8) {
    const char *path = std::getenv("TSFCDE_TUNE_CACHE");
    if (!path) return;
    if (FILE *fh = std::fopen(path, "a")) {
        std::fprintf(fh, "mid %lld %lld %d %d %.3f %.3f\n", (long long)k.C, (long long)k.R, k.count, e, t4, t8);
        std::fclose(fh);
    }
}

// Times the group's middle pass (product mode, unit symbol, on every
// member's own transform buffer) at each values-per-lane choice: one warm-up
// launch, then the mean of `reps` launches between events.
int tune_group(tsfcde_batch_s *bt, BatchGroup &G) {
    const int cnt = (int)G.members.size();
    const TuneKey key{G.A.C, G.A.R, cnt};
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_cache_read();
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
        G.e_mid = it->second;
        return TSFCDE_OK;
    }
    if (G.A.C < 16 || G.A.C > 1024) return TSFCDE_OK;  // one choice only
    std::vector<MidDesc> md;
    for (int idx : G.members) {
        tsfcde_plan_s *pl = bt->plans[idx];
        md.push_back(MidDesc{pl->A.R, pl->buf, pl->specA, nullptr, pl->A.tw, unit_symbol(pl->A), pl->sc});
    }
    bt->st.used = 0;
    MidDesc *d = bt->st.put(md);
    if (!d) return TSFCDE_ENOMEM;
    BCHK(hipMemcpyAsync(bt->st.dev, bt->st.host, bt->st.used, hipMemcpyHostToDevice, bt->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return TSFCDE_EDEVICE;
    }
    constexpr int reps = 4;
    double us[2] = {0.0, 0.0};
    const int cand[2] = {TUNE_E_ALT, TSF_E_MID};
    hipError_t err = hipSuccess;
    for (int c = 0; c < 2 && err == hipSuccess; ++c) {
        err = blaunch_mid<0>(bt, G.A, d, cnt, 0, cand[c]);
        if (err == hipSuccess) err = hipEventRecord(e0, bt->stream);
        for (int r = 0; r < reps && err == hipSuccess; ++r) err = blaunch_mid<0>(bt, G.A, d, cnt, 0, cand[c]);
        if (err == hipSuccess) err = hipEventRecord(e1, bt->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        us[c] = 1e3 * (double)ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    bt->st.used = 0;
    if (err != hipSuccess) return TSFCDE_EDEVICE;
    G.e_mid = us[0] < us[1] ? cand[0] : cand[1];
    g_tune_cache[key] = G.e_mid;
    tune_cache_append(key, G.e_mid, us[0], us[1]);
    return TSFCDE_OK;
}

int batch_poll(tsfcde_batch_s *bt) {
    hipLaunchKernelGGL(k_gather_state, dim3((bt->count + 255) / 256), dim3(256), 0, bt->stream, bt->d_scs, bt->count,
                       bt->d_done);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(bt->h_done, bt->d_done, sizeof(DoneRec) * bt->count, hipMemcpyDeviceToHost, bt->stream));
    HIPCHK(hipStreamSynchronize(bt->stream));
    return TSFCDE_OK;
}

// Sources of a batch run: f of instance i at level j, or null when the plan
// samples its own (the f callback) or f is zero.
struct BatchSources {
    const double *const *d_f = nullptr;  // one level: a vector per instance
    const double *const *d_F = nullptr;  // all levels: rows 0..M-1 per instance
    const int64_t *ldF = nullptr;
    const double *get(int i, int64_t j) const {
        if (d_F) return d_F[i] ? d_F[i] + (size_t)j * (size_t)ldF[i] : nullptr;
        return d_f ? d_f[i] : nullptr;
    }
};

// Progress of one instance in a batch run.
struct MemberRun {
    int64_t level = 0;    // the level being solved (the run's end once finished)
    bool active = false;  // takes CGS launches
    bool start = false;   // its level's set-up goes out in the next round
    int restarts = 0, seen_checks = 0, iter = 0;  // iter: CGS iterations of the level so far
    char accepted = 0, checked = 0;
    std::chrono::steady_clock::time_point t0;
};

// Per group, the instance lists of one round (group-local positions): the
// instances whose level starts (set-up), those of them restarting from an
// extrapolated guess, and those that iterate (including the starting ones).
struct RoundLists {
    std::vector<int> start, warm2, iter;
    int todo = 0;
};

// One round: for every group, the set-up of the levels its starting
// instances begin, then a chunk of CGS over the instances that iterate and
// the acceptance check behind it.  A group's chunk is sized so that about
// three quarters of its iterating instances are expected to stop within it,
// from the iterations each took at its last level (to its first stop, or in
// all once its check has failed at this level).  Groups run on up to four
// streams of their own, joined to the batch stream before and after; with
// chunk graphs everything runs on the batch stream and the chunk covers every
// instance (the graph's launches are fixed).  `retire` lists instances the
// host has stopped; they are marked done on the device first.
int batch_round(tsfcde_batch_s *bt, const std::vector<GroupDesc> &gd, std::vector<RoundLists> &rl,
                const std::vector<int> &retire, const std::vector<HistDesc> &hsweep,
                const std::vector<HistDesc> &hcatch, const std::vector<PcDesc> &pc,
                const std::vector<size_t> &pcoff, const std::vector<int> &pccnt, int64_t nmax) {
    const size_t ng = bt->groups.size();
    // staging: level slots are already in the pinned copy; the lists follow
    bt->st.used = bt->st_levels;
    HistDesc *dhs = hsweep.empty() ? nullptr : bt->st.put(hsweep);
    HistDesc *dhc = hcatch.empty() ? nullptr : bt->st.put(hcatch);
    PcDesc *dpc = pc.empty() ? nullptr : bt->st.put(pc);
    if ((!hsweep.empty() && !dhs) || (!hcatch.empty() && !dhc) || (!pc.empty() && !dpc) ||
        bt->st.used > bt->st.cap)
        return TSFCDE_ENOMEM;
    BCHK(hipMemcpyAsync(bt->st.dev + bt->st_fixed, bt->st.host + bt->st_fixed, bt->st.used - bt->st_fixed,
                        hipMemcpyHostToDevice, bt->stream));
    // index lists
    std::vector<size_t> o_start(ng), o_warm(ng), o_iter(ng);
    size_t used = 0;
    int longest = 0;
    for (size_t g = 0; g < ng; ++g) {
        o_start[g] = used;
        for (int k : rl[g].start) bt->h_act[used++] = k;
        o_warm[g] = used;
        for (int k : rl[g].warm2) bt->h_act[used++] = k;
        o_iter[g] = used;
        for (int k : rl[g].iter) bt->h_act[used++] = k;
        longest = std::max(longest, rl[g].todo);
    }
    const size_t roff = used;
    for (int i : retire) bt->h_act[used++] = i;
    if (used > 0)
        BCHK(hipMemcpyAsync(bt->d_act, bt->h_act, sizeof(int) * used, hipMemcpyHostToDevice, bt->stream));
    if (!retire.empty()) {
        hipLaunchKernelGGL(k_retire, dim3((unsigned)((retire.size() + 255) / 256)), dim3(256), 0, bt->stream,
                           bt->d_scs, bt->d_act + roff, (int)retire.size());
        BCHK(hipGetLastError());
    }
    // history sums of the starting levels (every group's, on the batch stream)
    const unsigned gx = (unsigned)std::min<int64_t>(1024, ((nmax + 1) / 2 + 255) / 256);
    if (dhs) {
        hipLaunchKernelGGL(k_hist_sweep_b, dim3(gx, (unsigned)hsweep.size()), dim3(256), 0, bt->stream, dhs);
        BCHK(hipGetLastError());
    }
    if (dhc) {
        hipLaunchKernelGGL(k_hist_catch_b, dim3(gx, (unsigned)hcatch.size()), dim3(256), 0, bt->stream, dhc);
        BCHK(hipGetLastError());
    }
    const bool split = !bt->gstreams.empty();
    const size_t ns = bt->gstreams.size();
    if (split) {
        BCHK(hipEventRecord(bt->ev_go, bt->stream));
        for (size_t k = 0; k < ns; ++k) BCHK(hipStreamWaitEvent(bt->gstreams[k], bt->ev_go, 0));
    }
    hipStream_t own = bt->stream;
    hipError_t e = hipSuccess;
    auto on = [&](size_t g, const size_t *o) {
        if (split) bt->stream = bt->gstreams[bt->groups[g].slot];
        bt->act = o ? bt->d_act + o[g] : nullptr;
    };
    // set-up of the starting levels: right-hand side and initial guess, then
    // the inverse Strang circulant (its column, Bluestein DFT, embedding and
    // spectrum)
    for (size_t g : bt->group_order) {
        const BatchGroup &G = bt->groups[g];
        const GroupDesc &D = gd[g];
        const int c = (int)rl[g].start.size();
        if (!c || e != hipSuccess) continue;
        on(g, o_start.data());
        e = blaunch_col<-1>(bt, G.A, D.rhsA, c, 0);
        if (e == hipSuccess) e = blaunch_mid<0>(bt, G.A, D.midA, c, 0, G.e_mid);
        if (e == hipSuccess) e = blaunch_col<1>(bt, G.A, D.rhsC, c, 0);
        const int c2 = (int)rl[g].warm2.size();
        if (c2 && e == hipSuccess) {
            on(g, o_warm.data());
            e = blaunch_col<-1>(bt, G.A, D.rstA, c2, 0);
            if (e == hipSuccess) e = blaunch_mid<0>(bt, G.A, D.midA, c2, 0, G.e_mid);
            if (e == hipSuccess) e = blaunch_col<1>(bt, G.A, D.rstC, c2, 0);
            on(g, o_start.data());
        }
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_pc_column_b, dim3((unsigned)std::min<int64_t>(256, (G.L / 2 + 255) / 256), pccnt[g]),
                           dim3(256), 0, bt->stream, dpc + pcoff[g]);
        e = hipGetLastError();
        if (e == hipSuccess) e = blaunch_col<-1>(bt, G.B, D.bsA, c, 0);
        if (e == hipSuccess) e = blaunch_row(bt, G.B, D.bsRow, c);
        if (e == hipSuccess) e = blaunch_col<1>(bt, G.B, D.bsC, c, 0);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_pc_embed_b, dim3((unsigned)std::min<int64_t>(256, (G.L + 255) / 256), pccnt[g]),
                               dim3(256), 0, bt->stream, dpc + pcoff[g]);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = blaunch_col<-1>(bt, G.A, D.r2cA, c, 0);
        if (e == hipSuccess) e = blaunch_mid<2>(bt, G.A, D.midR2C, c, 0, G.e_mid);
    }
    if (e == hipSuccess && longest > 0) {
        if (bt->graphs) {
            bt->stream = own;
            bt->act = nullptr;
            hipGraphExec_t ex = nullptr;
            if (int rc = chunk_graph(bt, gd, longest, &ex)) return rc;
            e = hipGraphLaunch(ex, bt->stream);
            for (size_t g = 0; g < ng && e == hipSuccess; ++g)
                e = issue_group_check(bt, bt->groups[g], gd[g], (int)bt->groups[g].members.size());
        } else {
            // launches go out iteration by iteration across the groups, so that
            // every stream has work queued within microseconds of the round's start
            for (int it = 0; it < longest && e == hipSuccess; ++it) {
                for (size_t g : bt->group_order) {
                    if (it >= rl[g].todo || e != hipSuccess) continue;
                    on(g, o_iter.data());
                    e = issue_group_iteration(bt, bt->groups[g], gd[g], (int)rl[g].iter.size(), it);
                }
            }
            for (size_t g : bt->group_order) {
                if (!rl[g].todo || e != hipSuccess) continue;
                on(g, o_iter.data());
                const int c = (int)rl[g].iter.size();
                e = issue_group_close(bt, bt->groups[g], gd[g], c, rl[g].todo);
                if (e == hipSuccess) e = issue_group_check(bt, bt->groups[g], gd[g], c);
            }
        }
    }
    bt->stream = own;
    bt->act = nullptr;
    for (size_t k = 0; k < ns && split; ++k) {
        if (e == hipSuccess) e = hipEventRecord(bt->ev_done[k], bt->gstreams[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(bt->stream, bt->ev_done[k], 0);
    }
    BCHK(e);
    return TSFCDE_OK;
}

// Levels [bt->level, jend) of every instance.  Instances advance on their own:
// one that has passed its acceptance check starts its next level in the next
// round while others still iterate, so a level's slowest instances hold up
// none of the rest.  stats (optional) gets one record per instance and level,
// instance-major: stats[i * (jend - j0) + (j - j0)].  Returns the first
// failure of any instance and level (every level is still computed).
int batch_run(tsfcde_batch_s *bt, int64_t jend, const BatchSources &src, tsfcde_stats *stats) {
    const int64_t j0 = bt->level;
    if (j0 >= bt->M) return TSFCDE_EDONE;
    jend = std::min(jend, bt->M);
    const int64_t nlev = jend - j0;
    const int cnt = bt->count;
    const size_t ng = bt->groups.size();
    std::vector<MemberRun> mr(cnt);
    for (int i = 0; i < cnt; ++i) {
        mr[i].level = j0;
        mr[i].start = true;
    }
    // position of every instance in its group
    std::vector<int> gof(cnt), pos(cnt);
    for (size_t g = 0; g < ng; ++g)
        for (size_t k = 0; k < bt->groups[g].members.size(); ++k) {
            gof[bt->groups[g].members[k]] = (int)g;
            pos[bt->groups[g].members[k]] = (int)k;
        }
    std::vector<GroupDesc> gd(ng);
    for (size_t g = 0; g < ng; ++g) gd[g] = bt->groups[g].fixed;
    int code = TSFCDE_OK;
    std::vector<int> retire;
    for (;;) {
        std::vector<RoundLists> rl(ng);
        std::vector<HistDesc> hsweep, hcatch;
        std::vector<PcDesc> pc;
        std::vector<size_t> pcoff(ng, 0);
        std::vector<int> pccnt(ng, 0);
        int64_t nmax = 0;
        bool any = false;
        // instances that start a level this round, group by group (each
        // group's preconditioner descriptors contiguous)
        for (size_t g = 0; g < ng; ++g) {
            pcoff[g] = pc.size();
            for (int i : bt->groups[g].members) {
                MemberRun &m = mr[i];
                if (!m.start) continue;
                tsfcde_plan_s *pl = bt->plans[i];
                const int64_t j = m.level;
                // sources that are not 16-byte aligned go through the plan's own buffer
                const double *f = src.get(i, j);
                if (f && (reinterpret_cast<uintptr_t>(f) & 15)) {
                    hipLaunchKernelGGL(k_copy, dim3(64), dim3(256), 0, bt->stream, f, pl->fbuf, pl->n);
                    BCHK(hipGetLastError());
                    f = pl->fbuf;
                }
                if (!f) {
                    if (int rc = callback_source(pl, j, &f)) return rc;
                }
                const int warm =
                    bt->warm == TSFCDE_WS_PREV ? 1 : (bt->warm == TSFCDE_WS_EXTRAP ? (j >= 2 ? 2 : (j >= 1)) : 0);
                // history: the block's sweep when the instance's block sums are
                // not those of its block, then the catch-up of a level past the
                // block's first
                if (j >= 1) {
                    if (pl->hist_pending) {
                        if (int rc = history_quiesce(pl)) return rc;
                    }
                    const int64_t hb0 = hist_block_of(j);
                    HistDesc d{pl->U, pl->n, pl->ldn, pl->cb, hist_block_params(pl, hb0), (int)j, pl->clast[j],
                               j == 1 ? pl->clast[1] : pl->cbase[1], pl->kappa, nullptr, nullptr};
                    if (pl->hist_block != hb0) {
                        d.out = pl->Hq;
                        hsweep.push_back(d);
                        pl->hist_block = hb0;
                    }
                    if (j > hb0) {
                        d.QL = pl->Hq + (size_t)(j - hb0) * pl->ldn;
                        d.out = pl->H;
                        hcatch.push_back(d);
                    }
                    nmax = std::max(nmax, pl->n);
                }
                stage_member_level(bt, gd[g], (size_t)pos[i], i, j, f, warm);
                pc.push_back(PcDesc{pl->Ls, pl->wv, pl->Wt, pl->tmp, pl->n, pl->A.L, precond_symbol(pl, j)});
                ++pccnt[g];
                rl[g].start.push_back(pos[i]);
                if (warm == 2) rl[g].warm2.push_back(pos[i]);
                m.start = false;
                m.active = true;
                m.restarts = m.seen_checks = m.iter = 0;
                m.accepted = m.checked = 0;
                m.t0 = std::chrono::steady_clock::now();
                bt->conv_seen[i] = 0;
            }
        }
        // the iterating instances and their chunk lengths
        for (size_t g = 0; g < ng; ++g) {
            std::vector<int> rem;
            int itmax = 0;
            for (int i : bt->groups[g].members) {
                if (!mr[i].active) continue;
                rl[g].iter.push_back(pos[i]);
                const int now = mr[i].iter;
                const int est = bt->conv_seen[i] ? bt->final_iters[i] : bt->conv_iters[i];
                rem.push_back(std::max(0, est - now));
                itmax = std::max(itmax, now);
            }
            if (rem.empty()) continue;
            any = true;
            std::sort(rem.begin(), rem.end());
            const int q = rem[(rem.size() - 1) * 3 / 4];
            rl[g].todo = std::max(1, std::min(std::max(2, q), bt->maxit - itmax));
        }
        if (!any) break;
        if (int rc = batch_round(bt, gd, rl, retire, hsweep, hcatch, pc, pcoff, pccnt, nmax)) return rc;
        retire.clear();
        if (int rc = batch_poll(bt)) return rc;
        for (int i = 0; i < cnt; ++i) {
            MemberRun &m = mr[i];
            if (!m.active) continue;
            tsfcde_plan_s *pl = bt->plans[i];
            const DoneRec &r = bt->h_done[i];
            m.iter = r.iter;
            const bool ran = r.nchecks > m.seen_checks;
            m.seen_checks = r.nchecks;
            if (ran) {
                m.checked = 1;
                m.accepted = r.done && r.status == ST_OK;
                if (!bt->conv_seen[i]) {  // iterations to the first stop, the next level's estimate
                    bt->conv_seen[i] = 1;
                    bt->conv_iters[i] = r.iter;
                }
                if (r.done) {
                    m.active = false;  // accepted, or non-finite
                } else if (m.restarts >= MAX_RESTARTS) {
                    m.active = false;  // x stays as it is (TSFCDE_EACCEPT)
                    retire.push_back(i);
                } else {
                    ++m.restarts;  // the device restarted CGS from x
                }
            } else if (r.done) {
                // stopped with no check of its own: the level's first residual
                // already met the tolerance
                m.accepted = r.status == ST_OK;
                m.active = false;
            }
            if (m.active && r.iter >= bt->maxit) {  // TSFCDE_ENOCONV (or EACCEPT after a failed check)
                m.active = false;
                if (!r.done) retire.push_back(i);
            }
            if (m.active) continue;
            // the instance's level is finished
            const int64_t j = m.level;
            int ci = status_code(r.status);
            if (ci == TSFCDE_OK && !m.accepted) ci = m.checked ? TSFCDE_EACCEPT : TSFCDE_ENOCONV;
            if (ci && !code) code = ci;
            if (!bt->conv_seen[i]) bt->conv_iters[i] = r.iter;
            bt->final_iters[i] = r.iter;
            pl->level = j + 1;
            pl->pj_level = j;
            if (stats) {
                tsfcde_stats &s = stats[(size_t)i * (size_t)nlev + (size_t)(j - j0)];
                s.iters = r.iter;
                s.outer_iters = 1;
                s.restarts = m.restarts;
                s.status = ci;
                s.relres = r.gnorm2 > 0 ? std::sqrt(r.rnorm2 / r.gnorm2) : 0.0;
                s.relres_true = m.checked ? (r.gnorm2 > 0 ? std::sqrt(r.aux0 / r.gnorm2) : 0.0) : -1.0;
                const double den = pl->anorm[j] * std::sqrt(r.aux1) + std::sqrt(r.gnorm2);
                s.backward_err = m.checked ? (den > 0 ? std::sqrt(r.aux0) / den : 0.0) : -1.0;
                s.precision_used = TSFCDE_FP64;
                s.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - m.t0).count();
                s.guess = bt->warm == TSFCDE_WS_EXTRAP
                              ? (j >= 2 ? TSFCDE_WS_EXTRAP : (j >= 1 ? TSFCDE_WS_PREV : TSFCDE_WS_ZERO))
                              : (bt->warm == TSFCDE_WS_PREV ? TSFCDE_WS_PREV : TSFCDE_WS_ZERO);
                s.method = TSFCDE_METHOD_PCGS;
                s.pad = 0;
            }
            m.level = j + 1;
            m.start = m.level < jend;
        }
    }
    bt->level = jend;
    return code;
}

int batch_step(tsfcde_batch_s *bt, const double *const *d_f, tsfcde_stats *stats) {
    BatchSources src;
    src.d_f = d_f;
    return batch_run(bt, bt->level + 1, src, stats);
}

}  // namespace

extern "C" {

// Bytes of the per-level descriptor staging area of a batch of `count`
// instances (the workspace size and the layout both use this).
size_t batch_staging_bytes(int32_t count) { return (size_t)count * 12288 + (1 << 20); }

int tsfcde_batch_workspace_bytes(const tsfcde_problem *probs, int32_t count, size_t *bytes) {
    if (!probs || count < 1 || !bytes) return TSFCDE_EINVAL;
    size_t tot = 0;
    for (int i = 0; i < count; ++i) {
        size_t b = 0;
        int rc = workspace_bytes_impl(&probs[i], true, &b);
        if (rc) return rc;
        if (probs[i].precision != TSFCDE_FP64) return TSFCDE_EUNSUPPORTED;  // the batch runs the FP64 form
        if (probs[i].flags & TSFCDE_FLAG_CONSTANT_GSF) return TSFCDE_EUNSUPPORTED;  // single plans only
        if (probs[i].krylov != TSFCDE_KRYLOV_CGS) return TSFCDE_EUNSUPPORTED;       // the batch runs CGS
        if (probs[i].history_tol > 0.0) return TSFCDE_EUNSUPPORTED;                // exact history only
        if (probs[i].M != probs[0].M) return TSFCDE_EINVAL;
        tot += al(b);
    }
    // descriptors (per level), scalar pointers, gathered states, instance lists
    tot += al(batch_staging_bytes(count)) + al(sizeof(void *) * count) + al(sizeof(DoneRec) * count) +
           al(sizeof(int) * 4 * (size_t)count);
    *bytes = tot;
    return TSFCDE_OK;
}

int tsfcde_plan_batch(const tsfcde_problem *probs, int32_t count, void *d_workspace, size_t bytes, void *stream,
                      tsfcde_batch_t *out) {
    if (!out) return TSFCDE_EINVAL;
    *out = nullptr;
    size_t need = 0;
    int rc = tsfcde_batch_workspace_bytes(probs, count, &need);
    if (rc) return rc;
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255)) return TSFCDE_EINVAL;
    if (bytes < need) return TSFCDE_ENOMEM;
    tsfcde_batch_s *bt = new (std::nothrow) tsfcde_batch_s();
    if (!bt) return TSFCDE_ENOMEM;
    bt->stream = reinterpret_cast<hipStream_t>(stream);
    bt->count = count;
    bt->M = probs[0].M;
    bt->maxit = probs[0].maxit > 0 ? probs[0].maxit : 500;
    bt->warm = probs[0].warm_start;
    bt->fold = (probs[0].flags & TSFCDE_FLAG_NO_FOLD) == 0;
    bt->strict = (probs[0].flags & TSFCDE_FLAG_STRICT_RESIDUAL) != 0;
    bt->graphs = (probs[0].flags & TSFCDE_FLAG_GRAPHS) != 0;
    char *ws = reinterpret_cast<char *>(d_workspace);
    size_t off = 0;
    auto fail = [&](int code) {
        for (tsfcde_plan_s *pl : bt->plans) tsfcde_destroy(pl);
        if (bt->st.host) (void)hipHostFree(bt->st.host);
        if (bt->h_done) (void)hipHostFree(bt->h_done);
        if (bt->h_act) (void)hipHostFree(bt->h_act);
        for (hipStream_t st : bt->gstreams) (void)hipStreamDestroy(st);
        for (hipEvent_t ev : bt->ev_done) (void)hipEventDestroy(ev);
        if (bt->ev_go) (void)hipEventDestroy(bt->ev_go);
        delete bt;
        return code;
    };
    for (int i = 0; i < count; ++i) {
        size_t b = 0;
        workspace_bytes_impl(&probs[i], true, &b);
        tsfcde_plan_t pl = nullptr;
        rc = plan_create(&probs[i], ws + off, b, stream, true, &pl);
        if (rc) return fail(rc);
        bt->plans.push_back(pl);
        off += al(b);
    }
    bt->st.cap = batch_staging_bytes(count);
    bt->st.dev = ws + off;
    off += al(bt->st.cap);
    bt->d_scs = reinterpret_cast<DevScalars **>(ws + off);
    off += al(sizeof(void *) * count);
    bt->d_done = reinterpret_cast<DoneRec *>(ws + off);
    off += al(sizeof(DoneRec) * count);
    bt->d_act = reinterpret_cast<int *>(ws + off);
    off += al(sizeof(int) * 4 * (size_t)count);
    if (off > need) return fail(TSFCDE_EINVAL);  // the layout outgrew tsfcde_batch_workspace_bytes
    bt->conv_iters.assign(count, 8);
    bt->final_iters.assign(count, 8);
    bt->conv_seen.assign(count, 0);
    if (hipHostMalloc(reinterpret_cast<void **>(&bt->h_act), sizeof(int) * 4 * (size_t)count) != hipSuccess)
        return fail(TSFCDE_EDEVICE);
    if (hipHostMalloc(reinterpret_cast<void **>(&bt->st.host), bt->st.cap) != hipSuccess) return fail(TSFCDE_EDEVICE);
    if (hipHostMalloc(reinterpret_cast<void **>(&bt->h_done), sizeof(DoneRec) * count) != hipSuccess)
        return fail(TSFCDE_EDEVICE);
    std::vector<DevScalars *> scs;
    for (tsfcde_plan_s *pl : bt->plans) scs.push_back(pl->sc);
    std::memcpy(bt->st.host, scs.data(), sizeof(void *) * count);
    if (hipMemcpyAsync(bt->d_scs, bt->st.host, sizeof(void *) * count, hipMemcpyHostToDevice, bt->stream) !=
        hipSuccess)
        return fail(TSFCDE_EDEVICE);
    if (hipStreamSynchronize(bt->stream) != hipSuccess) return fail(TSFCDE_EDEVICE);
    // groups by embedding length
    for (int i = 0; i < count; ++i) {
        tsfcde_plan_s *pl = bt->plans[i];
        auto it = std::find_if(bt->groups.begin(), bt->groups.end(),
                               [&](const BatchGroup &g) { return g.L == pl->A.L; });
        if (it == bt->groups.end()) {
            BatchGroup g;
            g.L = pl->A.L;
            g.A = pl->A;
            g.B = pl->B;
            bt->groups.push_back(g);
            it = bt->groups.end() - 1;
        }
        it->members.push_back(i);
    }
    if (!(probs[0].flags & TSFCDE_FLAG_NO_TUNE)) {
        for (BatchGroup &G : bt->groups)
            if ((rc = tune_group(bt, G))) return fail(rc);
    }
    // the descriptors that are the same at every level, staged once, and the
    // slots of those that depend on an instance's level
    bt->st.used = 0;
    for (BatchGroup &G : bt->groups)
        if (!stage_group_fixed(bt, G, G.fixed)) return fail(TSFCDE_ENOMEM);
    bt->st_fixed = bt->st.used;
    for (BatchGroup &G : bt->groups)
        if (!reserve_group_levels(bt, G, G.fixed)) return fail(TSFCDE_ENOMEM);
    bt->st_levels = bt->st.used;
    if (hipMemcpyAsync(bt->st.dev, bt->st.host, bt->st_levels, hipMemcpyHostToDevice, bt->stream) != hipSuccess ||
        hipStreamSynchronize(bt->stream) != hipSuccess)
        return fail(TSFCDE_EDEVICE);
    // groups by unknowns (embedding length times instances), largest first,
    // spread over up to four streams of their own
    for (size_t g = 0; g < bt->groups.size(); ++g) bt->group_order.push_back(g);
    std::sort(bt->group_order.begin(), bt->group_order.end(), [&](size_t a, size_t b) {
        const BatchGroup &A = bt->groups[a], &B = bt->groups[b];
        return A.L * (int64_t)A.members.size() > B.L * (int64_t)B.members.size();
    });
    if (!bt->graphs) {
        const size_t ns = std::min<size_t>(4, bt->groups.size());
        for (size_t k = 0; k < ns; ++k) {
            hipStream_t st = nullptr;
            hipEvent_t ev = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return fail(TSFCDE_EDEVICE);
            bt->gstreams.push_back(st);
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return fail(TSFCDE_EDEVICE);
            bt->ev_done.push_back(ev);
        }
        if (hipEventCreateWithFlags(&bt->ev_go, hipEventDisableTiming) != hipSuccess) return fail(TSFCDE_EDEVICE);
        // largest first, each to the stream with the least work so far
        std::vector<int64_t> load(ns, 0);
        for (size_t g : bt->group_order) {
            const size_t k = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
            bt->groups[g].slot = (int)k;
            load[k] += bt->groups[g].L * (int64_t)bt->groups[g].members.size();
        }
    }
    *out = bt;
    return TSFCDE_OK;
}

int tsfcde_batch_group_count(tsfcde_batch_t bt) { return bt ? (int)bt->groups.size() : TSFCDE_EINVAL; }

int tsfcde_batch_group_info(tsfcde_batch_t bt, int32_t g, int64_t *L, int32_t *members, int32_t *values_per_lane) {
    if (!bt || g < 0 || g >= (int)bt->groups.size()) return TSFCDE_EINVAL;
    const BatchGroup &G = bt->groups[g];
    if (L) *L = G.L;
    if (members) *members = (int32_t)G.members.size();
    if (values_per_lane) *values_per_lane = G.e_mid;
    return TSFCDE_OK;
}

tsfcde_plan_t tsfcde_batch_member(tsfcde_batch_t bt, int32_t i) {
    if (!bt || i < 0 || i >= bt->count) return nullptr;
    return bt->plans[i];
}

int tsfcde_batch_step(tsfcde_batch_t bt, const double *const *d_f, tsfcde_stats *stats) {
    if (!bt) return TSFCDE_EINVAL;
    for (tsfcde_plan_s *pl : bt->plans)
        if (pl->level != bt->level) return TSFCDE_EINVAL;
    return batch_step(bt, d_f, stats);
}

int tsfcde_batch_solve(tsfcde_batch_t bt, const double *const *d_F, const int64_t *ldF, tsfcde_stats *stats) {
    if (!bt) return TSFCDE_EINVAL;
    for (tsfcde_plan_s *pl : bt->plans)
        if (pl->level != bt->level) return TSFCDE_EINVAL;
    if (d_F) {
        if (!ldF) return TSFCDE_EINVAL;
        for (int i = 0; i < bt->count; ++i)
            if (d_F[i] && ldF[i] < bt->plans[i]->n) return TSFCDE_EINVAL;
    }
    BatchSources src;
    src.d_F = d_F;
    src.ldF = ldF;
    return batch_run(bt, bt->M, src, stats);
}

int tsfcde_batch_set_level(tsfcde_batch_t bt, int64_t level) {
    if (!bt || level < 0 || level > bt->M) return TSFCDE_EINVAL;
    for (tsfcde_plan_s *pl : bt->plans)
        if (pl->level != level) return TSFCDE_EINVAL;
    bt->level = level;
    return TSFCDE_OK;
}

int tsfcde_batch_destroy(tsfcde_batch_t bt) {
    if (!bt) return TSFCDE_EINVAL;
    (void)hipStreamSynchronize(bt->stream);
    for (hipStream_t st : bt->gstreams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (hipEvent_t ev : bt->ev_done) (void)hipEventDestroy(ev);
    if (bt->ev_go) (void)hipEventDestroy(bt->ev_go);
    for (auto &kv : bt->chunk_graphs) (void)hipGraphExecDestroy(kv.second.exec);
    if (bt->cap_stream) (void)hipStreamDestroy(bt->cap_stream);
    for (tsfcde_plan_s *pl : bt->plans) tsfcde_destroy(pl);
    if (bt->st.host) (void)hipHostFree(bt->st.host);
    if (bt->h_done) (void)hipHostFree(bt->h_done);
    if (bt->h_act) (void)hipHostFree(bt->h_act);
    delete bt;
    return TSFCDE_OK;
}

}  // extern "C"
