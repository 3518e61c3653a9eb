// tsfcde2d.hip -- the time-level solver in two space dimensions (tsfcde2d.h).
//
// One level solves (eta_j I - sigma L) u^{j+1} = g with L = L_x (x) I + I (x) L_y,
// the Kronecker sum of the one-dimensional operators of (3.2)-(3.3), by CGS
// right-preconditioned with the BCCB Strang preconditioner
// P = eta_j I - sigma (s(L_x) (x) I + I (x) s(L_y)).  Data are nx x ny arrays
// (x along the slow index).
//
// Kernels:
//  * k2_line: transforms along the lines of an array -- rows (contiguous,
//    along y) or columns (stride ny, along x), B lines per workgroup, each
//    line a length-P FFT held in registers with LDS exchanges (fft_core.hpp).
//    Its operation decides what happens around the transform:
//      ToepOp   -- L_axis v on every line through a length-2n circulant
//                  embedding (forward FFT, symbol, inverse FFT), with the
//                  second axis's pass combining y = a v + b (L_y v + L_x v);
//      RowFwdOp / ColDivOp / RowInvOp -- the three passes of P^{-1}: row
//                  FFTs, column FFTs with the division by the eigenvalues
//                  eta - sigma (mu_x + mu_y) and the inverse column FFTs,
//                  inverse row FFTs;
//      SpecOp   -- the forward FFT of one real column (plan-time spectra).
//  * vector kernels of the CGS recurrence with two-stage reductions in a
//    fixed order (reproducible results), the right-hand side, the history
//    sum and the acceptance check.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fft_core.hpp"
#include "tsfcde2d.h"

namespace tsf2d {

using tsf::cmul;
using tsf::fft;
using tsf::LdsSink;
using tsf::lpad;
using tsf::lpad_size;
using tsf::tw_offset;

constexpr int PMAX_LOG2 = 11;  // transforms up to 2048 points (embeddings of n = 1024)
constexpr int NT = 512;        // threads of a line workgroup
constexpr int RB = 256;        // threads of a vector workgroup
constexpr int RBLK = 1024;     // vector workgroups at most (partial sums)

// Device scalars of one plan's CGS recurrence.
struct Sc {
    double rho, rho_prev, alpha, beta, rnorm2, gnorm2, tol2, aux0, aux1;
    int iter, done, status, fresh, nchecks, pad;
};
enum : int { ST_OK = 0, ST_BREAKDOWN = 1, ST_NONFINITE = 2 };

// Packed tables tw_P[m] = exp(-2 pi i m / P) for P = 2, 4, ..., 2^pmax_log2.
__global__ void k2_twiddles(double2 *tw, int pmax_log2) {
    const int64_t total = (int64_t(1) << (pmax_log2 + 1)) - 2;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int lg = 1;
        while (((int64_t(1) << (lg + 1)) - 2) <= idx) ++lg;
        const int64_t P = int64_t(1) << lg;
        const int64_t m = idx - (P - 2);
        double s, c;
        sincospi(2.0 * (double)m / (double)P, &s, &c);
        tw[idx] = make_double2(c, -s);
    }
}

// ---------------------------------------------------------------------------
// Line transforms.
// ---------------------------------------------------------------------------
template <int P> struct LineGeo {
    static constexpr int E = 8;          // values per lane
    static constexpr int T = P / E;      // lanes per line
    static constexpr int B = NT / T;     // lines per workgroup
    static constexpr int LS = lpad_size(P);
    static_assert(P >= 16 && P <= (1 << PMAX_LOG2), "line length");
};

// Workgroups go to the eight XCDs round-robin; column tiles that share cache
// lines are given to one XCD in a contiguous run (identity otherwise).
__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t grid) {
    if (grid % 8) return bid;
    return (bid % 8) * (grid / 8) + bid / 8;
}

template <class Op> struct OpSink {
    const Op *op;
    int64_t line;
    __device__ __forceinline__ void operator()(int pos, double2 val, int) const { op->store(line, pos, val); }
};

template <int P, bool ROWS, class Op>
__global__ void __launch_bounds__(NT) k2_line(Op op, int64_t nlines, const double2 *__restrict__ tw_all,
                                              const Sc *sc) {
    if (op.pred && sc->done) return;
    using G = LineGeo<P>;
    constexpr int E = G::E, T = G::T, B = G::B, LS = G::LS;
    __shared__ double2 lds[B * LS];
    const int t = threadIdx.x;
    const int b = ROWS ? t / T : t % B;
    const int j = ROWS ? t % T : t / B;
    const int64_t tile = ROWS ? (int64_t)blockIdx.x : xcd_block(blockIdx.x, gridDim.x);
    const int64_t line = tile * B + b;
    const bool active = line < nlines;
    double2 *slab = ROWS ? lds + b * LS : lds + b;
    const int ls = ROWS ? 1 : B;
    double2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = active ? op.load(line, j + T * m) : make_double2(0.0, 0.0);
    OpSink<Op> sink{&op, line};
    if constexpr (Op::NFFT == 2) {
        LdsSink lsink{slab, ls};
        fft<P, E, -1>(v, j, active, tw_all, slab, ls, lsink);
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int k = j + T * m;
            v[m] = active ? op.spec(line, k, slab[lpad(k) * ls]) : make_double2(0.0, 0.0);
        }
        __syncthreads();
        fft<P, E, 1>(v, j, active, tw_all, slab, ls, sink);
    } else {
        fft<P, E, Op::DIR>(v, j, active, tw_all, slab, ls, sink);
    }
}

// L_axis v on every line, W and W^T through the embedding of length P = 2n:
// the line zero-padded to P, its DFT times the symbol
//   S(k) = cre Re Lam(k) + i (cim Im Lam(k) + cq sin(2 pi k / P)),
// (Lam the DFT of W's embedding column; cre = h^-b (d+ + d-), cim =
// h^-b (d+ - d-), cq = gamma/h, the last from Q's closed-form spectrum
// 2i sin(2 pi k/P)), the inverse DFT, the first n values.  epi 0 stores
// w = L v; epi 1 stores y = ca v + cb (w + L v).
struct ToepOp {
    static constexpr int NFFT = 2, DIR = 0;
    const double *v;
    int64_t n, sl, se;  // value p of line l at l*sl + p*se
    const double2 *lam, *twP;
    double cre, cim, cq, invP;
    int epi, pred;
    double *w_out;
    const double *w_in;
    double *y;
    double ca, cb;
    __device__ __forceinline__ double2 load(int64_t l, int p) const {
        return p < n ? make_double2(v[l * sl + p * se], 0.0) : make_double2(0.0, 0.0);
    }
    __device__ __forceinline__ double2 spec(int64_t, int k, double2 V) const {
        const double2 L = lam[k];
        const double s = -twP[k].y;  // sin(2 pi k / P)
        return cmul(V, make_double2(cre * L.x, fma(cim, L.y, cq * s)));
    }
    __device__ __forceinline__ void store(int64_t l, int p, double2 V) const {
        if (p >= n) return;
        const int64_t i = l * sl + p * se;
        const double Lv = V.x * invP;
        if (epi == 0) {
            w_out[i] = Lv;
        } else {
            y[i] = fma(ca, v[i], cb * (w_in[i] + Lv));
        }
    }
};

// P^{-1}, pass 1: the DFT of every row (length ny) of a real array into Z.
struct RowFwdOp {
    static constexpr int NFFT = 1, DIR = -1;
    const double *x;
    double2 *Z;
    int64_t ny;
    int pred;
    __device__ __forceinline__ double2 load(int64_t l, int p) const { return make_double2(x[l * ny + p], 0.0); }
    __device__ __forceinline__ void store(int64_t l, int p, double2 V) const { Z[l * ny + p] = V; }
};

// P^{-1}, pass 2: on every column of Z (frequency ky), the DFT along x, the
// division by eta - sigma (mu_x(kx) + mu_y(ky)), the inverse DFT.  mu(k) =
// cre Re lam_s(k) + i (cim Im lam_s(k) + cq sin(2 pi k / n)): the Strang
// circulants' eigenvalues (lam_s the DFT of W's Strang column; s(Q) has
// 2i sin(2 pi k/n), s(W^T) the conjugates of s(W)'s).
struct ColDivOp {
    static constexpr int NFFT = 2, DIR = 0;
    double2 *Z;
    int64_t ny;
    const double2 *lsx, *lsy, *twx, *twy;
    double eta, sigma, crex, cimx, cqx, crey, cimy, cqy;
    int pred;
    __device__ __forceinline__ double2 load(int64_t col, int p) const { return Z[p * ny + col]; }
    __device__ __forceinline__ double2 spec(int64_t col, int k, double2 V) const {
        const double2 Lx = lsx[k], Ly = lsy[col];
        const double sx = -twx[k].y, sy = -twy[col].y;
        const double mr = crex * Lx.x + crey * Ly.x;
        const double mi = fma(cimx, Lx.y, cqx * sx) + fma(cimy, Ly.y, cqy * sy);
        const double er = eta - sigma * mr, ei = -sigma * mi;
        const double q = 1.0 / fma(er, er, ei * ei);
        return make_double2(fma(V.x, er, V.y * ei) * q, fma(V.y, er, -V.x * ei) * q);
    }
    __device__ __forceinline__ void store(int64_t col, int p, double2 V) const { Z[p * ny + col] = V; }
};

// P^{-1}, pass 3: the inverse DFT of every row, scaled by 1/(nx ny), real part.
struct RowInvOp {
    static constexpr int NFFT = 1, DIR = 1;
    const double2 *Z;
    double *y;
    int64_t ny;
    double scale;
    int pred;
    __device__ __forceinline__ double2 load(int64_t l, int p) const { return Z[l * ny + p]; }
    __device__ __forceinline__ void store(int64_t l, int p, double2 V) const { y[l * ny + p] = V.x * scale; }
};

// Forward DFT of one real column of `len` values zero-padded to P (spectra).
struct SpecOp {
    static constexpr int NFFT = 1, DIR = -1;
    const double *col;
    double2 *out;
    int64_t len;
    int pred;
    __device__ __forceinline__ double2 load(int64_t, int p) const {
        return p < len ? make_double2(col[p], 0.0) : make_double2(0.0, 0.0);
    }
    __device__ __forceinline__ void store(int64_t, int p, double2 V) const { out[p] = V; }
};

// ---------------------------------------------------------------------------
// Vector kernels.  Sums: each workgroup reduces its lanes in a fixed tree and
// stores one partial per accumulator; a one-workgroup finishing kernel adds
// the partials in a fixed strided order.
// ---------------------------------------------------------------------------
template <int NA> __device__ __forceinline__ void block_sum(double (&acc)[NA], double *partials) {
    __shared__ double red[NA][RB];
    const int t = threadIdx.x;
#pragma unroll
    for (int a = 0; a < NA; ++a) red[a][t] = acc[a];
    __syncthreads();
    for (int s = RB / 2; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int a = 0; a < NA; ++a) red[a][t] += red[a][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
#pragma unroll
        for (int a = 0; a < NA; ++a) partials[(int64_t)blockIdx.x * NA + a] = red[a][0];
    }
}

template <int NA> __device__ __forceinline__ void final_sum(const double *partials, int nb, double (&tot)[NA]) {
    __shared__ double red[NA][RB];
    const int t = threadIdx.x;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        double s = 0.0;
        for (int i = t; i < nb; i += RB) s += partials[(int64_t)i * NA + a];
        red[a][t] = s;
    }
    __syncthreads();
    for (int s = RB / 2; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int a = 0; a < NA; ++a) red[a][t] += red[a][t + s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < NA; ++a) tot[a] = red[a][0];
}

__device__ __forceinline__ bool finite(double x) { return x - x == 0.0; }

#define TSF2_LOOP(i, N) for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < (N); i += (int64_t)gridDim.x * RB)

__global__ void __launch_bounds__(RB) k2_fill(double *x, int64_t N, double val) {
    TSF2_LOOP(i, N) x[i] = val;
}

// history of (3.1): H = kappa sum_{s<j} c_{j-s}^(j) (u^{s+1} - u^s), with
// c_j^(j) = clast[j] and c_m^(j) = cbase[m] for 1 <= m < j (Lemma 1)
__global__ void __launch_bounds__(RB) k2_hist(const double *__restrict__ U, int64_t N, int j,
                                              const double *__restrict__ cbase, double clast_j, double kappa,
                                              double *__restrict__ H) {
    TSF2_LOOP(i, N) {
        double acc = clast_j * (U[N + i] - U[i]);
        for (int s = 1; s < j; ++s) acc = fma(cbase[j - s], U[(int64_t)(s + 1) * N + i] - U[(int64_t)s * N + i], acc);
        H[i] = kappa * acc;
    }
}

// g = B u^j - H + f; r = rt = g (zero initial guess); partial |g|^2
__global__ void __launch_bounds__(RB) k2_rhs(const double *__restrict__ Bu, const double *__restrict__ H,
                                             const double *__restrict__ f, double *__restrict__ g,
                                             double *__restrict__ r, double *__restrict__ rt, int64_t N,
                                             double *partials) {
    double acc[1] = {0.0};
    TSF2_LOOP(i, N) {
        double v = Bu[i];
        if (H) v -= H[i];
        if (f) v += f[i];
        g[i] = v;
        r[i] = v;
        rt[i] = v;
        acc[0] = fma(v, v, acc[0]);
    }
    block_sum<1>(acc, partials);
}

__global__ void __launch_bounds__(RB) k2_fin_rhs(const double *partials, int nb, Sc *sc, double rtol) {
    double tot[1];
    final_sum<1>(partials, nb, tot);
    if (threadIdx.x == 0) {
        Sc s{};
        s.gnorm2 = tot[0];
        s.rnorm2 = tot[0];
        s.rho = tot[0];
        s.rho_prev = 1.0;
        s.tol2 = rtol * rtol * tot[0];
        s.aux0 = tot[0];
        s.fresh = 1;
        s.status = finite(tot[0]) ? ST_OK : ST_NONFINITE;
        s.done = (tot[0] == 0.0 || !finite(tot[0])) ? 1 : 0;
        *sc = s;
    }
}

// CGS (Barrett et al., Templates), right preconditioned:
//   u = r + beta q ; p = u + beta (q + beta p)   (u = p = r when fresh)
__global__ void __launch_bounds__(RB) k2_up(const Sc *sc, const double *__restrict__ r, const double *__restrict__ q,
                                            double *__restrict__ p, double *__restrict__ u, int64_t N) {
    if (sc->done) return;
    const bool fresh = sc->fresh != 0;
    const double beta = sc->beta;
    TSF2_LOOP(i, N) {
        const double ri = r[i];
        if (fresh) {
            u[i] = ri;
            p[i] = ri;
        } else {
            const double qi = q[i];
            const double ui = fma(beta, qi, ri);
            u[i] = ui;
            p[i] = fma(beta, fma(beta, p[i], qi), ui);
        }
    }
}

// partial rt . vhat
__global__ void __launch_bounds__(RB) k2_dot(const Sc *sc, const double *__restrict__ a, const double *__restrict__ b,
                                             int64_t N, double *partials) {
    if (sc->done) return;
    double acc[1] = {0.0};
    TSF2_LOOP(i, N) acc[0] = fma(a[i], b[i], acc[0]);
    block_sum<1>(acc, partials);
}

// alpha = rho / (rt . vhat)
__global__ void __launch_bounds__(RB) k2_fin_alpha(const double *partials, int nb, Sc *sc) {
    if (sc->done) return;
    double tot[1];
    final_sum<1>(partials, nb, tot);
    if (threadIdx.x == 0) {
        if (!finite(tot[0])) {
            sc->status = ST_NONFINITE;
            sc->done = 1;
        } else if (tot[0] == 0.0) {
            sc->status = ST_BREAKDOWN;
            sc->done = 1;
        } else {
            sc->alpha = sc->rho / tot[0];
        }
    }
}

// q = u - alpha vhat ; s = u + q
__global__ void __launch_bounds__(RB) k2_q(const Sc *sc, const double *__restrict__ u,
                                           const double *__restrict__ vhat, double *__restrict__ q,
                                           double *__restrict__ s, int64_t N) {
    if (sc->done) return;
    const double alpha = sc->alpha;
    TSF2_LOOP(i, N) {
        const double qi = fma(-alpha, vhat[i], u[i]);
        q[i] = qi;
        s[i] = u[i] + qi;
    }
}

// x += alpha uhat ; r -= alpha (A uhat); partial rt . r and r . r
__global__ void __launch_bounds__(RB) k2_xr(const Sc *sc, double *__restrict__ x, const double *__restrict__ uhat,
                                            double *__restrict__ r, const double *__restrict__ Au,
                                            const double *__restrict__ rt, int64_t N, double *partials) {
    if (sc->done) return;
    const double alpha = sc->alpha;
    double acc[2] = {0.0, 0.0};
    TSF2_LOOP(i, N) {
        x[i] = fma(alpha, uhat[i], x[i]);
        const double ri = fma(-alpha, Au[i], r[i]);
        r[i] = ri;
        acc[0] = fma(rt[i], ri, acc[0]);
        acc[1] = fma(ri, ri, acc[1]);
    }
    block_sum<2>(acc, partials);
}

// rho_prev = rho, rho = rt . r, beta = rho / rho_prev; stop at |r|^2 <= tol2
__global__ void __launch_bounds__(RB) k2_fin_rho(const double *partials, int nb, Sc *sc) {
    if (sc->done) return;
    double tot[2];
    final_sum<2>(partials, nb, tot);
    if (threadIdx.x == 0) {
        sc->iter += 1;
        sc->fresh = 0;
        sc->rho_prev = sc->rho;
        sc->rho = tot[0];
        sc->rnorm2 = tot[1];
        sc->beta = tot[0] / sc->rho_prev;
        if (!finite(tot[0]) || !finite(tot[1])) {
            sc->status = ST_NONFINITE;
            sc->done = 1;
        } else if (tot[1] <= sc->tol2) {
            sc->done = 1;
        } else if (tot[0] == 0.0) {
            sc->status = ST_BREAKDOWN;
            sc->done = 1;
        }
    }
}

// acceptance check of x: r = g - A x, rt = r; partial |r|^2, |x|^2
__global__ void __launch_bounds__(RB) k2_true(const double *__restrict__ g, const double *__restrict__ Ax,
                                              const double *__restrict__ x, double *__restrict__ r,
                                              double *__restrict__ rt, int64_t N, double *partials) {
    double acc[2] = {0.0, 0.0};
    TSF2_LOOP(i, N) {
        const double ri = g[i] - Ax[i];
        r[i] = ri;
        rt[i] = ri;
        acc[0] = fma(ri, ri, acc[0]);
        acc[1] = fma(x[i], x[i], acc[1]);
    }
    block_sum<2>(acc, partials);
}

// accept x at |r| <= rtol |g| or backward error |r| / (anorm |x| + |g|) <=
// bwtol; otherwise restart CGS from x (r = rt = g - A x)
__global__ void __launch_bounds__(RB) k2_fin_true(const double *partials, int nb, Sc *sc, double anorm,
                                                  double bwtol) {
    double tot[2];
    final_sum<2>(partials, nb, tot);
    if (threadIdx.x == 0) {
        sc->nchecks += 1;
        sc->aux0 = tot[0];
        sc->aux1 = tot[1];
        sc->rnorm2 = tot[0];
        sc->rho = tot[0];
        sc->rho_prev = 1.0;
        sc->beta = 0.0;
        sc->fresh = 1;
        sc->status = ST_OK;
        const double den = anorm * sqrt(tot[1]) + sqrt(sc->gnorm2);
        const bool ok = tot[0] <= sc->tol2 || (bwtol > 0.0 && sqrt(tot[0]) <= bwtol * den);
        sc->done = ok ? 1 : 0;
        if (!finite(tot[0]) || !finite(tot[1])) {
            sc->status = ST_NONFINITE;
            sc->done = 1;
        }
    }
}

#undef TSF2_LOOP

}  // namespace tsf2d

// ===========================================================================
// Host side.
// ===========================================================================
using namespace tsf2d;

struct tsfcde2d_plan_s {
    hipStream_t stream = nullptr;
    int64_t nx = 0, ny = 0, N = 0, M = 0, level = 0;
    double alpha = 0, bx = 0, by = 0, a = 0, b = 0, c = 0, d = 0, T = 0, hx = 0, hy = 0, tau = 0, sigma = 0,
           kappa = 0, rtol = 1e-10, hbx = 0, hby = 0;
    int maxit = 500, last_iters = 8;
    std::vector<double> eta, gx, gy, dxp, dxm, dyp, dym, anorm, cbase, clast;
    tsfcde2d_src_fn fcb = nullptr;
    void *fuser = nullptr;
    double *h_f = nullptr;  // pinned staging of callback sources
    Sc *h_sc = nullptr;     // pinned copy of the device scalars
    // device (inside the caller's workspace)
    double *U = nullptr, *g = nullptr, *r = nullptr, *rt = nullptr, *u = nullptr, *p = nullptr, *q = nullptr,
           *s = nullptr, *phat = nullptr, *uhat = nullptr, *vhat = nullptr, *t = nullptr, *w = nullptr,
           *H = nullptr, *fbuf = nullptr, *part = nullptr, *d_cbase = nullptr, *colx = nullptr, *coly = nullptr;
    double2 *Z = nullptr, *lamx = nullptr, *lamy = nullptr, *lsx = nullptr, *lsy = nullptr, *tw = nullptr;
    Sc *sc = nullptr;
};

namespace {

constexpr double BW_TOL2 = 1e-13;
constexpr int MAX_RESTARTS2 = 3;

bool pow2_in(int64_t v, int64_t lo, int64_t hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

size_t al2(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout2 {
    size_t U, vec, Z, lam, tw, part, sc, cb, cols, total;
};
constexpr int NVEC2 = 15;  // g r rt u p q s phat uhat vhat t w H fbuf (+1 spare)

Layout2 layout2(int64_t nx, int64_t ny, int64_t M) {
    const size_t N = (size_t)(nx * ny);
    Layout2 L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = al2(o + bytes);
        return at;
    };
    L.U = take(sizeof(double) * (size_t)(M + 1) * N);
    L.vec = take(sizeof(double) * NVEC2 * N);
    L.Z = take(sizeof(double2) * N);
    L.lam = take(sizeof(double2) * (size_t)(2 * nx + 2 * ny + nx + ny));
    L.tw = take(sizeof(double2) * (size_t)((int64_t(1) << (PMAX_LOG2 + 1)) - 2));
    L.part = take(sizeof(double) * 2 * RBLK);
    L.sc = take(sizeof(Sc));
    L.cb = take(sizeof(double) * (size_t)(M + 2));
    L.cols = take(sizeof(double) * (size_t)(2 * nx + 2 * ny + nx + ny));
    L.total = o;
    return L;
}

int validate2(const tsfcde2d_problem *p) {
    if (!p) return TSFCDE_EINVAL;
    if (!(p->alpha > 0.0 && p->alpha <= 1.0)) return TSFCDE_EINVAL;
    if (!(p->beta_x > 1.0 && p->beta_x <= 2.0) || !(p->beta_y > 1.0 && p->beta_y <= 2.0)) return TSFCDE_EINVAL;
    if (!(p->b > p->a) || !(p->d > p->c) || !(p->T > 0.0) || p->M < 1) return TSFCDE_EINVAL;
    if (!std::isfinite(p->a) || !std::isfinite(p->b) || !std::isfinite(p->c) || !std::isfinite(p->d) ||
        !std::isfinite(p->T))
        return TSFCDE_EINVAL;
    if (!p->gamma_x || !p->gamma_y || !p->dplus_x || !p->dminus_x || !p->dplus_y || !p->dminus_y)
        return TSFCDE_EINVAL;
    if (p->nx < 1 || p->ny < 1) return TSFCDE_EINVAL;
    if (!pow2_in(p->nx, 16, 1024) || !pow2_in(p->ny, 16, 1024)) return TSFCDE_EUNSUPPORTED;
    if (p->M > (int64_t(1) << 20)) return TSFCDE_EUNSUPPORTED;
    return TSFCDE_OK;
}

// WSGD weights omega_0..omega_K (Lemma 2, with the recurrence of Lemma 3 for
// the Grunwald coefficients)
std::vector<double> wsgd(double beta, int64_t K) {
    const double l1 = (beta * beta + 3.0 * beta + 2.0) / 12.0, l0 = (4.0 - beta * beta) / 6.0,
                 lm1 = (beta * beta - 3.0 * beta + 2.0) / 12.0;
    std::vector<double> gk(K + 1), w(K + 1);
    gk[0] = 1.0;
    for (int64_t k = 1; k <= K; ++k) gk[k] = (1.0 - (beta + 1.0) / (double)k) * gk[k - 1];
    for (int64_t k = 0; k <= K; ++k)
        w[k] = l1 * gk[k] + (k >= 1 ? l0 * gk[k - 1] : 0.0) + (k >= 2 ? lm1 * gk[k - 2] : 0.0);
    return w;
}

double level_time2(const tsfcde2d_plan_s *pl, int64_t j) { return ((double)j + pl->sigma) * pl->tau; }

int nblocks(int64_t N) { return (int)std::min<int64_t>(RBLK, (N + RB - 1) / RB); }

#define HIPCHK2(x)                                   \
    do {                                             \
        if ((x) != hipSuccess) return TSFCDE_EDEVICE; \
    } while (0)

template <int P, bool ROWS, class Op>
hipError_t line_t(tsfcde2d_plan_s *pl, const Op &op, int64_t nlines) {
    using G = LineGeo<P>;
    const int64_t grid = (nlines + G::B - 1) / G::B;
    hipLaunchKernelGGL((k2_line<P, ROWS, Op>), dim3((unsigned)grid), dim3(NT), 0, pl->stream, op, nlines,
                       (const double2 *)pl->tw, (const Sc *)pl->sc);
    return hipGetLastError();
}

template <bool ROWS, class Op> hipError_t line(tsfcde2d_plan_s *pl, int64_t P, const Op &op, int64_t nlines) {
    switch (P) {
        case 16: return line_t<16, ROWS>(pl, op, nlines);
        case 32: return line_t<32, ROWS>(pl, op, nlines);
        case 64: return line_t<64, ROWS>(pl, op, nlines);
        case 128: return line_t<128, ROWS>(pl, op, nlines);
        case 256: return line_t<256, ROWS>(pl, op, nlines);
        case 512: return line_t<512, ROWS>(pl, op, nlines);
        case 1024: return line_t<1024, ROWS>(pl, op, nlines);
        case 2048: return line_t<2048, ROWS>(pl, op, nlines);
        default: return hipErrorInvalidValue;
    }
}

// symbol coefficients of the level-j operator along one axis
void axis_coef(double hb, double h, double gam, double dp, double dm, double *cre, double *cim, double *cq) {
    *cre = hb * (dp + dm);
    *cim = hb * (dp - dm);
    *cq = gam / h;
}

// y = ca v + cb L v (L at level j): ca = eta, cb = -sigma for A; cb = 1 - sigma for B
hipError_t product2(tsfcde2d_plan_s *pl, int64_t j, const double *v, double *y, double ca, double cb, int pred) {
    const int64_t nx = pl->nx, ny = pl->ny;
    ToepOp oy{};
    oy.v = v;
    oy.n = ny;
    oy.sl = ny;
    oy.se = 1;
    oy.lam = pl->lamy;
    oy.twP = pl->tw + tw_offset((int)(2 * ny));
    axis_coef(pl->hby, pl->hy, pl->gy[j], pl->dyp[j], pl->dym[j], &oy.cre, &oy.cim, &oy.cq);
    oy.invP = 1.0 / (double)(2 * ny);
    oy.epi = 0;
    oy.pred = pred;
    oy.w_out = pl->w;
    hipError_t e = line<true>(pl, 2 * ny, oy, nx);
    if (e != hipSuccess) return e;
    ToepOp ox{};
    ox.v = v;
    ox.n = nx;
    ox.sl = 1;
    ox.se = ny;
    ox.lam = pl->lamx;
    ox.twP = pl->tw + tw_offset((int)(2 * nx));
    axis_coef(pl->hbx, pl->hx, pl->gx[j], pl->dxp[j], pl->dxm[j], &ox.cre, &ox.cim, &ox.cq);
    ox.invP = 1.0 / (double)(2 * nx);
    ox.epi = 1;
    ox.pred = pred;
    ox.w_in = pl->w;
    ox.y = y;
    ox.ca = ca;
    ox.cb = cb;
    return line<false>(pl, 2 * nx, ox, ny);
}

// y = P^{-1} v (BCCB Strang preconditioner of level j); y may equal v
hipError_t psolve2(tsfcde2d_plan_s *pl, int64_t j, const double *v, double *y, int pred) {
    const int64_t nx = pl->nx, ny = pl->ny;
    RowFwdOp o1{v, pl->Z, ny, pred};
    hipError_t e = line<true>(pl, ny, o1, nx);
    if (e != hipSuccess) return e;
    ColDivOp o2{};
    o2.Z = pl->Z;
    o2.ny = ny;
    o2.lsx = pl->lsx;
    o2.lsy = pl->lsy;
    o2.twx = pl->tw + tw_offset((int)nx);
    o2.twy = pl->tw + tw_offset((int)ny);
    o2.eta = pl->eta[j];
    o2.sigma = pl->sigma;
    axis_coef(pl->hbx, pl->hx, pl->gx[j], pl->dxp[j], pl->dxm[j], &o2.crex, &o2.cimx, &o2.cqx);
    axis_coef(pl->hby, pl->hy, pl->gy[j], pl->dyp[j], pl->dym[j], &o2.crey, &o2.cimy, &o2.cqy);
    o2.pred = pred;
    if ((e = line<false>(pl, nx, o2, ny)) != hipSuccess) return e;
    RowInvOp o3{pl->Z, y, ny, 1.0 / (double)(nx * ny), pred};
    return line<true>(pl, ny, o3, nx);
}

hipError_t cgs_iteration2(tsfcde2d_plan_s *pl, int64_t j, double *x) {
    const int64_t N = pl->N;
    const int nb = nblocks(N);
    const double eta = pl->eta[j], sg = pl->sigma;
    hipError_t e;
    hipLaunchKernelGGL(k2_up, dim3(nb), dim3(RB), 0, pl->stream, (const Sc *)pl->sc, pl->r, pl->q, pl->p, pl->u, N);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = psolve2(pl, j, pl->p, pl->phat, 1)) != hipSuccess) return e;
    if ((e = product2(pl, j, pl->phat, pl->vhat, eta, -sg, 1)) != hipSuccess) return e;
    hipLaunchKernelGGL(k2_dot, dim3(nb), dim3(RB), 0, pl->stream, (const Sc *)pl->sc, pl->rt, pl->vhat, N, pl->part);
    hipLaunchKernelGGL(k2_fin_alpha, dim3(1), dim3(RB), 0, pl->stream, pl->part, nb, pl->sc);
    hipLaunchKernelGGL(k2_q, dim3(nb), dim3(RB), 0, pl->stream, (const Sc *)pl->sc, pl->u, pl->vhat, pl->q, pl->s, N);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = psolve2(pl, j, pl->s, pl->uhat, 1)) != hipSuccess) return e;
    if ((e = product2(pl, j, pl->uhat, pl->t, eta, -sg, 1)) != hipSuccess) return e;
    hipLaunchKernelGGL(k2_xr, dim3(nb), dim3(RB), 0, pl->stream, (const Sc *)pl->sc, x, pl->uhat, pl->r, pl->t,
                       pl->rt, N, pl->part);
    hipLaunchKernelGGL(k2_fin_rho, dim3(1), dim3(RB), 0, pl->stream, pl->part, nb, pl->sc);
    return hipGetLastError();
}

int poll2(tsfcde2d_plan_s *pl) {
    HIPCHK2(hipMemcpyAsync(pl->h_sc, pl->sc, sizeof(Sc), hipMemcpyDeviceToHost, pl->stream));
    HIPCHK2(hipStreamSynchronize(pl->stream));
    return TSFCDE_OK;
}

int status_code2(int st) {
    if (st == ST_BREAKDOWN) return TSFCDE_EBREAKDOWN;
    if (st == ST_NONFINITE) return TSFCDE_ENONFINITE;
    return TSFCDE_OK;
}

int callback_source2(tsfcde2d_plan_s *pl, int64_t j, const double **d_f) {
    *d_f = nullptr;
    if (!pl->fcb) return TSFCDE_OK;
    if (!pl->h_f && hipHostMalloc(reinterpret_cast<void **>(&pl->h_f), sizeof(double) * (size_t)pl->N) != hipSuccess) {
        pl->h_f = nullptr;
        return TSFCDE_EDEVICE;
    }
    HIPCHK2(hipStreamSynchronize(pl->stream));  // the last copy out of h_f has finished
    const double t = level_time2(pl, j);
    for (int64_t i = 0; i < pl->nx; ++i) {
        const double x = pl->a + (double)(i + 1) * pl->hx;
        for (int64_t k = 0; k < pl->ny; ++k)
            pl->h_f[i * pl->ny + k] = pl->fcb(x, pl->c + (double)(k + 1) * pl->hy, t, pl->fuser);
    }
    HIPCHK2(hipMemcpyAsync(pl->fbuf, pl->h_f, sizeof(double) * (size_t)pl->N, hipMemcpyHostToDevice, pl->stream));
    *d_f = pl->fbuf;
    return TSFCDE_OK;
}

int level_step2(tsfcde2d_plan_s *pl, const double *d_f, double *d_u_out, tsfcde_stats *st) {
    if (pl->level >= pl->M) return TSFCDE_EDONE;
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t j = pl->level, N = pl->N;
    const int nb = nblocks(N);
    if (!d_f) {
        if (int rc = callback_source2(pl, j, &d_f)) return rc;
    }
    double *x = pl->U + (size_t)(j + 1) * N;
    // history sum and right-hand side g = B u^j - H + f
    if (j >= 1) {
        hipLaunchKernelGGL(k2_hist, dim3(nb), dim3(RB), 0, pl->stream, (const double *)pl->U, N, (int)j,
                           (const double *)pl->d_cbase, pl->clast[j], pl->kappa, pl->H);
        HIPCHK2(hipGetLastError());
    }
    HIPCHK2(product2(pl, j, pl->U + (size_t)j * N, pl->t, pl->eta[j], 1.0 - pl->sigma, 0));
    hipLaunchKernelGGL(k2_rhs, dim3(nb), dim3(RB), 0, pl->stream, (const double *)pl->t,
                       (const double *)(j >= 1 ? pl->H : nullptr), d_f, pl->g, pl->r, pl->rt, N, pl->part);
    hipLaunchKernelGGL(k2_fin_rhs, dim3(1), dim3(RB), 0, pl->stream, (const double *)pl->part, nb, pl->sc, pl->rtol);
    hipLaunchKernelGGL(k2_fill, dim3(nb), dim3(RB), 0, pl->stream, x, N, 0.0);
    HIPCHK2(hipGetLastError());
    // CGS in chunks between polls; a stopped solve is checked on its true
    // residual and backward error and restarted from x when it fails
    int restarts = 0, chunk = std::max(2, pl->last_iters), code = TSFCDE_OK;
    bool accepted = false, checked = false;
    pl->h_sc->iter = 0;  // the right-hand side's finishing step starts the count at 0
    for (;;) {
        const int todo = std::min(chunk, pl->maxit - pl->h_sc->iter);
        for (int k = 0; k < todo; ++k) HIPCHK2(cgs_iteration2(pl, j, x));
        if (int rc = poll2(pl)) return rc;
        const Sc &h = *pl->h_sc;
        if (!h.done) {
            if (h.iter >= pl->maxit || todo <= 0) {
                code = TSFCDE_ENOCONV;
                break;
            }
            chunk = 2;
            continue;
        }
        if (h.status == ST_NONFINITE) {
            code = TSFCDE_ENONFINITE;
            break;
        }
        // the check: r = g - A x and the acceptance test
        HIPCHK2(product2(pl, j, x, pl->t, pl->eta[j], -pl->sigma, 0));
        hipLaunchKernelGGL(k2_true, dim3(nb), dim3(RB), 0, pl->stream, (const double *)pl->g,
                           (const double *)pl->t, (const double *)x, pl->r, pl->rt, N, pl->part);
        hipLaunchKernelGGL(k2_fin_true, dim3(1), dim3(RB), 0, pl->stream, (const double *)pl->part, nb, pl->sc,
                           pl->anorm[j], BW_TOL2);
        HIPCHK2(hipGetLastError());
        if (int rc = poll2(pl)) return rc;
        checked = true;
        if (pl->h_sc->done) {
            code = status_code2(pl->h_sc->status);
            accepted = code == TSFCDE_OK;
            break;
        }
        if (restarts >= MAX_RESTARTS2 || pl->h_sc->iter >= pl->maxit) break;
        ++restarts;
        chunk = std::max(2, pl->last_iters / 2);
    }
    const Sc &h = *pl->h_sc;
    if (code == TSFCDE_OK && !accepted) code = checked ? TSFCDE_EACCEPT : TSFCDE_ENOCONV;
    pl->last_iters = std::max(1, h.iter / (restarts + 1));
    if (d_u_out) HIPCHK2(hipMemcpyAsync(d_u_out, x, sizeof(double) * (size_t)N, hipMemcpyDeviceToDevice, pl->stream));
    HIPCHK2(hipStreamSynchronize(pl->stream));
    if (st) {
        st->iters = h.iter;
        st->outer_iters = 1;
        st->restarts = restarts;
        st->status = code;
        st->relres = h.gnorm2 > 0 ? std::sqrt(h.rnorm2 / h.gnorm2) : 0.0;
        st->relres_true = checked ? (h.gnorm2 > 0 ? std::sqrt(h.aux0 / h.gnorm2) : 0.0) : -1.0;
        const double den = pl->anorm[j] * std::sqrt(h.aux1) + std::sqrt(h.gnorm2);
        st->backward_err = checked ? (den > 0 ? std::sqrt(h.aux0) / den : 0.0) : -1.0;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        st->precision_used = TSFCDE_FP64;
        st->guess = TSFCDE_WS_ZERO;
        st->method = 0;
        st->pad = 0;
    }
    pl->level = j + 1;
    return code;
}

}  // namespace

extern "C" {

int tsfcde2d_workspace_bytes(const tsfcde2d_problem *prob, size_t *bytes) {
    if (!bytes) return TSFCDE_EINVAL;
    if (int rc = validate2(prob)) return rc;
    *bytes = layout2(prob->nx, prob->ny, prob->M).total;
    return TSFCDE_OK;
}

int tsfcde2d_plan(const tsfcde2d_problem *prob, void *d_workspace, size_t bytes, void *stream, tsfcde2d_plan_t *out) {
    if (!out) return TSFCDE_EINVAL;
    *out = nullptr;
    if (int rc = validate2(prob)) return rc;
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255)) return TSFCDE_EINVAL;
    const Layout2 L = layout2(prob->nx, prob->ny, prob->M);
    if (bytes < L.total) return TSFCDE_ENOMEM;
    tsfcde2d_plan_s *pl = new (std::nothrow) tsfcde2d_plan_s();
    if (!pl) return TSFCDE_ENOMEM;
    auto fail = [&](int code) {
        if (pl->h_sc) (void)hipHostFree(pl->h_sc);
        if (pl->h_f) (void)hipHostFree(pl->h_f);
        delete pl;
        return code;
    };
    pl->stream = reinterpret_cast<hipStream_t>(stream);
    const int64_t nx = prob->nx, ny = prob->ny, M = prob->M, N = nx * ny;
    pl->nx = nx;
    pl->ny = ny;
    pl->N = N;
    pl->M = M;
    pl->alpha = prob->alpha;
    pl->bx = prob->beta_x;
    pl->by = prob->beta_y;
    pl->a = prob->a;
    pl->b = prob->b;
    pl->c = prob->c;
    pl->d = prob->d;
    pl->T = prob->T;
    pl->hx = (prob->b - prob->a) / (double)(nx + 1);
    pl->hy = (prob->d - prob->c) / (double)(ny + 1);
    pl->hbx = std::pow(pl->hx, -prob->beta_x);
    pl->hby = std::pow(pl->hy, -prob->beta_y);
    pl->tau = prob->T / (double)M;
    pl->sigma = 1.0 - prob->alpha / 2.0;
    pl->kappa = std::pow(pl->tau, -prob->alpha) / std::tgamma(2.0 - prob->alpha);
    pl->rtol = prob->rtol > 0 ? prob->rtol : 1e-10;
    pl->maxit = prob->maxit > 0 ? prob->maxit : 500;
    pl->fcb = prob->f;
    pl->fuser = prob->f_user;
    // coefficients at t_{j+sigma}
    pl->gx.resize(M);
    pl->gy.resize(M);
    pl->dxp.resize(M);
    pl->dxm.resize(M);
    pl->dyp.resize(M);
    pl->dym.resize(M);
    for (int64_t j = 0; j < M; ++j) {
        const double t = level_time2(pl, j);
        void *u = prob->coef_user;
        pl->gx[j] = prob->gamma_x(t, u);
        pl->gy[j] = prob->gamma_y(t, u);
        pl->dxp[j] = prob->dplus_x(t, u);
        pl->dxm[j] = prob->dminus_x(t, u);
        pl->dyp[j] = prob->dplus_y(t, u);
        pl->dym[j] = prob->dminus_y(t, u);
        const double all[6] = {pl->gx[j], pl->gy[j], pl->dxp[j], pl->dxm[j], pl->dyp[j], pl->dym[j]};
        for (double v : all)
            if (!std::isfinite(v)) return fail(TSFCDE_EINVAL);
        if (pl->dxp[j] < 0 || pl->dxm[j] < 0 || pl->dyp[j] < 0 || pl->dym[j] < 0) return fail(TSFCDE_EINVAL);
    }
    // L2-1sigma tables (Lemma 1): eta_j = kappa c_0^(j), c_m = a_m + b_{m+1} - b_m
    // (1 <= m < j), c_j = a_j - b_j
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
        for (int64_t j = 0; j < M; ++j) pl->eta[j] = pl->kappa * (j == 0 ? av[0] : av[0] + bv[1]);
        for (int64_t m = 1; m <= M; ++m) pl->cbase[m] = av[m] + bv[m + 1] - bv[m];
        for (int64_t j = 1; j <= M; ++j) pl->clast[j] = av[j] - bv[j];
    }
    // weights, embedding and Strang columns of both axes; |A| bound
    const std::vector<double> wx = wsgd(prob->beta_x, nx + 1), wy = wsgd(prob->beta_y, ny + 1);
    double sx = 0.0, sy = 0.0;
    for (double v : wx) sx += std::fabs(v);
    for (double v : wy) sy += std::fabs(v);
    pl->anorm.resize(M);
    for (int64_t j = 0; j < M; ++j)
        pl->anorm[j] = pl->eta[j] + pl->sigma * (std::fabs(pl->gx[j]) / pl->hx + (pl->dxp[j] + pl->dxm[j]) * pl->hbx * sx +
                                                 std::fabs(pl->gy[j]) / pl->hy + (pl->dyp[j] + pl->dym[j]) * pl->hby * sy);
    // embedding column of W (length 2n): c_m = omega_{m+1} (m < n), c_{2n-1} = omega_0;
    // Strang column (length n): c_k = omega_{k+1} (k <= n/2), c_{n-1} = omega_0, else 0
    std::vector<double> cols((size_t)(2 * nx + 2 * ny + nx + ny), 0.0);
    double *ex = cols.data(), *ey = ex + 2 * nx, *stx = ey + 2 * ny, *sty = stx + nx;
    for (int64_t m = 0; m < nx; ++m) ex[m] = wx[m + 1];
    ex[2 * nx - 1] = wx[0];
    for (int64_t m = 0; m < ny; ++m) ey[m] = wy[m + 1];
    ey[2 * ny - 1] = wy[0];
    for (int64_t k = 0; k <= nx / 2; ++k) stx[k] = wx[k + 1];
    stx[nx - 1] = wx[0];
    for (int64_t k = 0; k <= ny / 2; ++k) sty[k] = wy[k + 1];
    sty[ny - 1] = wy[0];
    // device buffers
    char *ws = reinterpret_cast<char *>(d_workspace);
    pl->U = reinterpret_cast<double *>(ws + L.U);
    double *vec = reinterpret_cast<double *>(ws + L.vec);
    double **bufs[NVEC2 - 1] = {&pl->g, &pl->r, &pl->rt, &pl->u, &pl->p, &pl->q, &pl->s,
                                &pl->phat, &pl->uhat, &pl->vhat, &pl->t, &pl->w, &pl->H, &pl->fbuf};
    for (int k = 0; k < NVEC2 - 1; ++k) *bufs[k] = vec + (size_t)k * N;
    pl->Z = reinterpret_cast<double2 *>(ws + L.Z);
    pl->lamx = reinterpret_cast<double2 *>(ws + L.lam);
    pl->lamy = pl->lamx + 2 * nx;
    pl->lsx = pl->lamy + 2 * ny;
    pl->lsy = pl->lsx + nx;
    pl->tw = reinterpret_cast<double2 *>(ws + L.tw);
    pl->part = reinterpret_cast<double *>(ws + L.part);
    pl->sc = reinterpret_cast<Sc *>(ws + L.sc);
    pl->d_cbase = reinterpret_cast<double *>(ws + L.cb);
    pl->colx = reinterpret_cast<double *>(ws + L.cols);
    if (hipHostMalloc(reinterpret_cast<void **>(&pl->h_sc), sizeof(Sc)) != hipSuccess) {
        pl->h_sc = nullptr;
        return fail(TSFCDE_EDEVICE);
    }
    std::memset(pl->h_sc, 0, sizeof(Sc));
    std::vector<double> h_cb(pl->cbase.begin(), pl->cbase.end());
    bool ok = hipMemcpyAsync(pl->d_cbase, h_cb.data(), sizeof(double) * (size_t)(M + 2), hipMemcpyHostToDevice,
                             pl->stream) == hipSuccess &&
              hipMemcpyAsync(pl->colx, cols.data(), sizeof(double) * cols.size(), hipMemcpyHostToDevice, pl->stream) ==
                  hipSuccess &&
              hipMemsetAsync(pl->sc, 0, sizeof(Sc), pl->stream) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(k2_twiddles, dim3(16), dim3(256), 0, pl->stream, pl->tw, PMAX_LOG2);
        ok = hipGetLastError() == hipSuccess;
    }
    // spectra: DFT of the embedding columns (2n points) and Strang columns (n points)
    const double *dex = pl->colx, *dey = dex + 2 * nx, *dsx = dey + 2 * ny, *dsy = dsx + nx;
    if (ok) ok = line<true>(pl, 2 * nx, SpecOp{dex, pl->lamx, 2 * nx, 0}, 1) == hipSuccess;
    if (ok) ok = line<true>(pl, 2 * ny, SpecOp{dey, pl->lamy, 2 * ny, 0}, 1) == hipSuccess;
    if (ok) ok = line<true>(pl, nx, SpecOp{dsx, pl->lsx, nx, 0}, 1) == hipSuccess;
    if (ok) ok = line<true>(pl, ny, SpecOp{dsy, pl->lsy, ny, 0}, 1) == hipSuccess;
    // u^0 = phi at the nodes (or 0)
    if (ok) {
        if (prob->phi) {
            std::vector<double> u0((size_t)N);
            for (int64_t i = 0; i < nx; ++i) {
                const double x = pl->a + (double)(i + 1) * pl->hx;
                for (int64_t k = 0; k < ny; ++k)
                    u0[(size_t)(i * ny + k)] = prob->phi(x, pl->c + (double)(k + 1) * pl->hy, prob->phi_user);
            }
            ok = hipMemcpyAsync(pl->U, u0.data(), sizeof(double) * (size_t)N, hipMemcpyHostToDevice, pl->stream) ==
                 hipSuccess;
            if (ok) ok = hipStreamSynchronize(pl->stream) == hipSuccess;
        } else {
            hipLaunchKernelGGL(k2_fill, dim3(nblocks(N)), dim3(RB), 0, pl->stream, pl->U, N, 0.0);
            ok = hipGetLastError() == hipSuccess;
        }
    }
    if (ok) ok = hipStreamSynchronize(pl->stream) == hipSuccess;
    if (!ok) return fail(TSFCDE_EDEVICE);
    *out = pl;
    return TSFCDE_OK;
}

int tsfcde2d_set_state(tsfcde2d_plan_t pl, int64_t level, const double *d_U) {
    if (!pl || !d_U || level < 0 || level >= pl->M) return TSFCDE_EINVAL;
    HIPCHK2(hipMemcpyAsync(pl->U, d_U, sizeof(double) * (size_t)((level + 1) * pl->N), hipMemcpyDeviceToDevice,
                           pl->stream));
    HIPCHK2(hipStreamSynchronize(pl->stream));
    pl->level = level;
    return TSFCDE_OK;
}

int tsfcde2d_step(tsfcde2d_plan_t pl, const double *d_f, double *d_u_out, tsfcde_stats *stats) {
    if (!pl) return TSFCDE_EINVAL;
    return level_step2(pl, d_f, d_u_out, stats);
}

int tsfcde2d_solve(tsfcde2d_plan_t pl, const double *d_F, int64_t ldF, double *d_U_out, tsfcde_stats *stats) {
    if (!pl) return TSFCDE_EINVAL;
    if (d_F && ldF < pl->N) return TSFCDE_EINVAL;
    if (pl->level >= pl->M) return TSFCDE_EDONE;
    int first = TSFCDE_OK;
    const int64_t j0 = pl->level;
    while (pl->level < pl->M) {
        const int64_t j = pl->level;
        const int rc = level_step2(pl, d_F ? d_F + (size_t)j * (size_t)ldF : nullptr, nullptr,
                                   stats ? stats + (j - j0) : nullptr);
        if (rc == TSFCDE_EDEVICE) return rc;
        if (rc && !first) first = rc;
    }
    if (d_U_out) {
        HIPCHK2(hipMemcpyAsync(d_U_out, pl->U, sizeof(double) * (size_t)((pl->M + 1) * pl->N), hipMemcpyDeviceToDevice,
                               pl->stream));
        HIPCHK2(hipStreamSynchronize(pl->stream));
    }
    return first;
}

int tsfcde2d_apply(tsfcde2d_plan_t pl, int32_t op, int64_t j, const double *d_x, double *d_y) {
    if (!pl || !d_x || !d_y || d_x == d_y || j < 0 || j >= pl->M) return TSFCDE_EINVAL;
    hipError_t e;
    if (op == TSFCDE_OP_A) {
        e = product2(pl, j, d_x, d_y, pl->eta[j], -pl->sigma, 0);
    } else if (op == TSFCDE_OP_B) {
        e = product2(pl, j, d_x, d_y, pl->eta[j], 1.0 - pl->sigma, 0);
    } else if (op == TSFCDE_OP_PINV) {
        e = psolve2(pl, j, d_x, d_y, 0);
    } else {
        return TSFCDE_EINVAL;
    }
    return e == hipSuccess ? TSFCDE_OK : TSFCDE_EDEVICE;
}

int tsfcde2d_nodes(tsfcde2d_plan_t pl, double *h_x, double *h_y) {
    if (!pl) return TSFCDE_EINVAL;
    if (h_x)
        for (int64_t i = 0; i < pl->nx; ++i) h_x[i] = pl->a + (double)(i + 1) * pl->hx;
    if (h_y)
        for (int64_t k = 0; k < pl->ny; ++k) h_y[k] = pl->c + (double)(k + 1) * pl->hy;
    return TSFCDE_OK;
}

double tsfcde2d_level_time(tsfcde2d_plan_t pl, int64_t j) {
    if (!pl || j < 0 || j >= pl->M) return std::nan("");
    return level_time2(pl, j);
}

int64_t tsfcde2d_level(tsfcde2d_plan_t pl) { return pl ? pl->level : -1; }

const double *tsfcde2d_history(tsfcde2d_plan_t pl) { return pl ? pl->U : nullptr; }

int tsfcde2d_destroy(tsfcde2d_plan_t pl) {
    if (!pl) return TSFCDE_EINVAL;
    (void)hipStreamSynchronize(pl->stream);
    if (pl->h_sc) (void)hipHostFree(pl->h_sc);
    if (pl->h_f) (void)hipHostFree(pl->h_f);
    delete pl;
    return TSFCDE_OK;
}

}  // extern "C"
