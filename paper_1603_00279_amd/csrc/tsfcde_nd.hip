// tsfcde_nd.hip -- the time-level solver in two and three space dimensions
// (tsfcde2d.h, tsfcde3d.h): one engine for d = 2 or 3 axes.
//
// One level solves (eta_j I - sigma L) u^{j+1} = g with L the Kronecker sum
// of the one-dimensional operators of (3.2)-(3.3), one per axis, by CGS
// right-preconditioned with the multi-level circulant Strang preconditioner
// P = eta_j I - sigma sum_axes s(L_axis) (the analogue of (3.7)).  Arrays
// are row-major with axis 0 (x) slowest and axis d-1 (the "fast" axis)
// contiguous.
//
// Every pass is a batch of one-dimensional transforms along one axis
// (k_line: B lines per workgroup, each a length-P FFT in registers with LDS
// exchanges, fft_core.hpp), with an operation around the transform:
//  * ToepOp: L_axis v on every line through the length-2n circulant
//    embedding (forward FFT, symbol, inverse FFT).  The embedding of a real
//    Toeplitz matrix is a real circulant, so one complex transform carries
//    two real lines (v_a + i v_b -> L v_a + i L v_b).  The fast axis stores
//    w = L v; a middle axis adds its product to w; the slow axis combines
//    y = a v + b (w + L v) with an epilogue: store y, or store y and reduce
//    rt.y, or (CGS) update x and r from y = A uhat and reduce rt.r, r.r.
//  * P^{-1} as a real-to-complex multi-dimensional FFT: the fast-axis pass
//    (HalfFwdOp) transforms two real rows per complex transform and unpacks
//    them into the half spectra k = 0..n/2 of both (W = n/2 + 1 values per
//    row); in 3D a pass along y (CplxOp) follows; the pass along x (DivOp)
//    transforms, divides by the eigenvalues eta - sigma sum mu_axis(k_axis)
//    and transforms back; then y back (3D), and the fast axis back
//    (HalfInvOp: the half spectra of two rows rebuilt into one complex
//    transform whose real and imaginary parts are the two rows).  In two
//    dimensions the half spectrum is stored transposed, written and read
//    through LDS by whole workgroups (HalfFwdOp<., true>, HalfInvTOp), so
//    that the division pass runs along contiguous rows.
//  * The history sum in blocks of HB levels (k_hist_sweep, k_hist_catch).
//  * The CGS vector updates run inside the passes: the u/p update in the
//    first pass of the first preconditioner solve of an iteration, the q/s
//    update in the first pass of the second, x and r in the last product's
//    epilogue.  Dot products are reduced per workgroup (fixed order) and
//    finished inside the pass that needs them, in the same fixed order in
//    every workgroup (reproducible results; a one-workgroup kernel only when
//    a pass has more than MAXPART workgroups, and at the end of a chunk).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fft_core.hpp"
#include "tsfcde2d.h"
#include "tsfcde3d.h"

namespace tsfnd {

using tsf::cmul;
using tsf::fft;
using tsf::LdsSink;
using tsf::lpad;
using tsf::lpad_size;
using tsf::tw_offset;

constexpr int PMAX_LOG2 = 12;  // transforms up to 4096 points (embeddings of n = 2048)
constexpr int NT = 512;        // threads of a strided line workgroup
constexpr int NT_MAX = 1024;   // threads of a line workgroup at most (strided 1024-point products)
constexpr int RB = 256;        // threads of a vector workgroup
constexpr int RBLK = 1024;     // vector workgroups at most (partial sums)
constexpr int MAXPART = 1024;  // partials a pass folds at most (more are summed first by k_squash)

// Device scalars of one plan's CGS recurrence.  rt.r at the start of
// iteration k sits in rho[k & 1], so a pass that finishes iteration k's
// reduction never overwrites the value the other workgroups still read.
struct Sc {
    double rho[2], alpha, rnorm2, gnorm2, tol2, aux0, aux1;
    int iter, done, status, nchecks;
};
enum : int { ST_OK = 0, ST_BREAKDOWN = 1, ST_NONFINITE = 2 };

__device__ __forceinline__ bool finite(double x) { return x - x == 0.0; }

// Packed tables tw_P[m] = exp(-2 pi i m / P) for P = 2, 4, ..., 2^pmax_log2.
__global__ void k_twiddles(double2 *tw, int pmax_log2) {
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
// Reductions: a workgroup sums its lanes (wave64 shuffles, then the waves in
// order) into one partial per accumulator; the partials are summed by
// reduce_partials in a 256-wide layout (thread t < 256 adds partials t,
// t + 256, ..., then the trees of waves 0..3), the same order in a
// one-workgroup finishing kernel and in a line pass of 512 threads.
// ---------------------------------------------------------------------------
template <int NA, int NTB = RB>  // NTB: the workgroup's threads at most
__device__ __forceinline__ void block_partial(const double (&acc)[NA], double *partials, int64_t slot) {
    __shared__ double red[NA][NTB / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwave = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        double v = acc[a];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[a][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            double s = 0.0;
            for (int w = 0; w < nwave; ++w) s += red[a][w];
            partials[slot * NA + a] = s;
        }
    }
}

constexpr int RED_WIDTH = 256;
template <int NA> __device__ __forceinline__ void reduce_partials(const double *partials, int np, double (&tot)[NA]) {
    __shared__ double red[NA][RED_WIDTH / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double loc[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) loc[a] = 0.0;
    if (threadIdx.x < RED_WIDTH) {
        for (int i = threadIdx.x; i < np; i += RED_WIDTH) {
#pragma unroll
            for (int a = 0; a < NA; ++a) loc[a] += partials[(int64_t)i * NA + a];
        }
    }
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        double v = loc[a];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0 && wave < RED_WIDTH / 64) red[a][wave] = v;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < RED_WIDTH / 64; ++w) s += red[a][w];
        tot[a] = s;
    }
}

// ---------------------------------------------------------------------------
// Line transforms.
// ---------------------------------------------------------------------------
template <int P, int NTL, int E_ = 8> struct LineGeo {
    static constexpr int E = E_;      // values per lane
    static constexpr int T = P / E;   // lanes per line
    static constexpr int B = NTL / T;  // lines per workgroup
    static constexpr int LS = lpad_size(P);
    static_assert(P >= 16 && P <= (1 << PMAX_LOG2) && NTL <= NT_MAX && B >= 1, "line geometry");
};

// Workgroups go to the eight XCDs round-robin; tiles of strided lines that
// share cache lines are given to one XCD in a contiguous run (identity when
// the tile count is not a multiple of eight).
__device__ __forceinline__ int64_t xcd_tile(int64_t t, int64_t ntiles) {
    if (ntiles % 8) return t;
    return (t % 8) * (ntiles / 8) + t / 8;
}

// Line l of an axis: element p at base(l) + p * s, base(l) = (l / s) * ns + l % s
// (s the axis's stride, ns = n s).
__device__ __forceinline__ int64_t line_base(int64_t l, int64_t s, int64_t ns) { return (l / s) * ns + (l % s); }

// Sink of a forward transform whose outputs stay in registers, multiplied by
// the operation's symbol (slot m of the lane holds frequency pos).
template <class Op, int E> struct SpecSink {
    const Op *op;
    const typename Op::Ctx *ctx;
    double2 *s;
    __device__ __forceinline__ void operator()(int pos, double2 val, int slot) const {
        s[slot] = op->spec(*ctx, pos, val);
    }
};

template <class Op> struct OpSink {
    const Op *op;
    const typename Op::Ctx *ctx;
    double *acc;
    __device__ __forceinline__ void operator()(int pos, double2 val, int) const { op->store(*ctx, pos, val, acc); }
};

// One launch: one tile of B lines per workgroup.  Op supplies
//   NFFT (1: one transform of direction DIR; 2: forward, spec(), inverse),
//   HALF (after a forward transform, unpack the half spectra of two real
//   rows), NRAW doubles fetched per position, NACC reductions, FOLD,
//   ctx(line), fetch/finish (loads, then the values the transform takes),
//   store (the sink of the last stage), fold (the previous pass's finishing
//   step; every thread calls it, and its result is uniform).
// (four waves per SIMD: the register budget that lets the LDS-bound number
// of workgroups per CU run together)
template <int P, bool ROWS, int NTL, class Op, int EV>
__global__ void __launch_bounds__(NTL, 4) k_line(Op op, int64_t nlines, const double2 *__restrict__ tw_all, Sc *sc) {
    if (op.pred && sc->done) return;
    using G = LineGeo<P, NTL, EV>;
    constexpr int E = G::E, T = G::T, B = G::B, LS = G::LS;
    __shared__ double2 lds[B * LS];
    const int t = threadIdx.x;
    const int b = ROWS ? t / T : t % B;
    const int j = ROWS ? t % T : t / B;
    Op o = op;
    o.prep(sc);
    double acc[Op::NACC > 0 ? Op::NACC : 1];
#pragma unroll
    for (int a = 0; a < (Op::NACC > 0 ? Op::NACC : 1); ++a) acc[a] = 0.0;
    const int64_t ntiles = (nlines + B - 1) / B;
    const int64_t tile = ROWS ? (int64_t)blockIdx.x : xcd_tile(blockIdx.x, ntiles);
    const int64_t line = tile * B + b;
    const bool active = line < nlines;
    double2 *slab = ROWS ? lds + b * LS : lds + b;
    const int ls = ROWS ? 1 : B;
    if constexpr (Op::IN_T) {  // transposed input staged in LDS by the whole workgroup
        o.stage_in(lds, LS, B, tile * B, nlines, t, NTL);
        __syncthreads();
    }
    typename Op::Ctx ctx{};
    if (active) ctx = o.ctx(line);
    if constexpr (Op::IN_T) ctx.slab = slab;
    double raw[E][Op::NRAW];
#pragma unroll
    for (int m = 0; m < E; ++m)
        if (active) o.fetch(ctx, j + T * m, raw[m]);
    if constexpr (Op::IN_T) __syncthreads();  // every staged value read: the slab is the transform's
    // a folded finishing step runs while the loads are in flight
    if constexpr (Op::FOLD) {
        if (o.fold(sc)) return;
    }
    double2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = active ? o.finish(ctx, j + T * m, raw[m]) : make_double2(0.0, 0.0);
    OpSink<Op> sink{&o, &ctx, acc};
    if constexpr (Op::NFFT == 2 && !(Op::NACC > 0 && (P == 128 || P == 4096))) {
        // the forward transform's last stage leaves slot m of lane j at
        // frequency j + T m, the layout the inverse transform starts from:
        // the symbol is applied there, in registers, with no round trip
        // through LDS (3.8% less time per CGS iteration at 1024^2, 1.7% at
        // 256^3).  The reducing passes of 128 and 4096 points, which spill
        // with the extra registers, keep the LDS form below.
        double2 s[E];
#pragma unroll
        for (int m = 0; m < E; ++m) s[m] = make_double2(0.0, 0.0);
        SpecSink<Op, E> ssink{&o, &ctx, s};
        fft<P, E, -1>(v, j, active, tw_all, slab, ls, ssink);
        fft<P, E, 1>(s, j, active, tw_all, slab, ls, sink);
    } else if constexpr (Op::NFFT == 2) {
        LdsSink lsink{slab, ls};
        fft<P, E, -1>(v, j, active, tw_all, slab, ls, lsink);
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int k = j + T * m;
            v[m] = active ? o.spec(ctx, k, slab[lpad(k) * ls]) : make_double2(0.0, 0.0);
        }
        __syncthreads();
        fft<P, E, 1>(v, j, active, tw_all, slab, ls, sink);
    } else if constexpr (Op::HALF) {
        // Z = DFT(a + i b) of two real rows: A_k = (Z_k + conj Z_{P-k}) / 2,
        // B_k = (Z_k - conj Z_{P-k}) / (2i), k = 0..P/2
        LdsSink lsink{slab, ls};
        fft<P, E, -1>(v, j, active, tw_all, slab, ls, lsink);
        __syncthreads();
        if (active) {
            for (int k = j; k <= P / 2; k += T) {
                const double2 Z = slab[lpad(k) * ls];
                const double2 Zc = slab[lpad((P - k) & (P - 1)) * ls];
                o.store_half(ctx, k, make_double2(0.5 * (Z.x + Zc.x), 0.5 * (Z.y - Zc.y)),
                             make_double2(0.5 * (Z.y + Zc.y), -0.5 * (Z.x - Zc.x)));
            }
        }
    } else if constexpr (Op::HALF_T) {
        // as HALF, the unpacked half spectra written transposed by the workgroup
        LdsSink lsink{slab, ls};
        fft<P, E, -1>(v, j, active, tw_all, slab, ls, lsink);
        __syncthreads();
        o.store_half_t(lds, LS, B, tile * B, nlines, t, NTL);
    } else {
        fft<P, E, Op::DIR>(v, j, active, tw_all, slab, ls, sink);
    }
    if constexpr (Op::NACC > 0) block_partial<Op::NACC, NTL>(acc, o.part, blockIdx.x);
}

// Symbol of the level's L_axis on the embedding (length P = 2n) or of its
// Strang circulant (length n): cre Re lam(k) + i (cim Im lam(k) + cq sin(2 pi k / P)),
// lam the DFT of W's column (embedding or Strang), cre = h^-b (d+ + d-),
// cim = h^-b (d+ - d-), cq = gamma/h (Q's spectrum is 2i sin(2 pi k / P)).
// A real shift c0 (the identity's symbol is 1) folds the a v term of the
// slow-axis pass into its transform, so that pass's epilogue needs no
// second read of v.
// The level's symbol values are tabulated once per level (k_symbols): one
// load per frequency in the passes instead of the spectrum and a twiddle.
struct Sym {
    const double2 *tab;  // the level's symbol at k = 0..P-1
    double c0 = 0.0;
    __device__ __forceinline__ double2 operator()(int64_t k) const {
        const double2 S = tab[k];
        return make_double2(S.x + c0, S.y);
    }
};

// The symbols of one level: for each of up to 6 tables (per axis, the
// embedding of length 2n and the Strang circulant of length n),
// out[k] = (cre Re lam(k), cim Im lam(k) + cq sin(2 pi k / P)).
struct SymTabs {
    const double2 *lam[6];
    const double2 *tw[6];  // the length-P twiddle tables
    double2 *out[6];
    int64_t P[6];
    double cre[6], cim[6], cq[6];
    int count;
};
__global__ void __launch_bounds__(256) k_symbols(SymTabs t) {
    const int e = blockIdx.y;
    if (e >= t.count) return;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < t.P[e]; k += (int64_t)gridDim.x * 256) {
        const double2 L = t.lam[e][k];
        t.out[e][k] = make_double2(t.cre[e] * L.x, fma(t.cim[e], L.y, -t.cq[e] * t.tw[e][k].y));
    }
}

enum : int { EPI_W = 0, EPI_WADD = 1, EPI_Y = 2, EPI_DOT = 3, EPI_XR = 4 };

// L_axis v on pairs of real lines (2c, 2c+1) of one axis.  EPI_W: w = L v;
// EPI_WADD: w += L v; otherwise y = cb (w + (ca/cb + L) v), the shift ca/cb
// in the symbol (Sym::c0), and
//   EPI_Y: store y;  EPI_DOT: store y, reduce rt.y;
//   EPI_XR: (y = A uhat) r -= alpha y, reduce rt.r and r.r (x += alpha uhat
//   is done where uhat is formed, HalfInvOp).
template <int EPI> struct ToepOp {
    static constexpr int NFFT = 2, DIR = 0, NRAW = 2, FOLD = 0;
    // the slow-axis products (y = cb (w + L v) and its CGS forms) take the
    // wide strided tile at 1024 points (line_t)
    static constexpr bool WIDE = EPI >= EPI_Y;
    static constexpr bool HALF = false, HALF_T = false, IN_T = false;
    static constexpr int NACC = EPI == EPI_DOT ? 1 : EPI == EPI_XR ? 2 : 0;
    struct Ctx {
        int64_t ia, ib;
    };
    const double *v;
    int64_t n, s, ns;
    Sym sym;
    double invP;
    double *w;
    double *y;
    double cb;
    const double *rt;
    double *r;
    double *part;
    double alpha;
    int pred;
    __device__ void prep(const Sc *sc) {
        if constexpr (EPI == EPI_XR) alpha = sc->alpha;
    }
    __device__ bool fold(Sc *) { return false; }
    __device__ __forceinline__ Ctx ctx(int64_t c) const {
        return Ctx{line_base(2 * c, s, ns), line_base(2 * c + 1, s, ns)};
    }
    __device__ __forceinline__ void fetch(const Ctx &cx, int p, double *raw) const {
        if (p < n) {
            raw[0] = v[cx.ia + p * s];
            raw[1] = v[cx.ib + p * s];
        }
    }
    __device__ __forceinline__ double2 finish(const Ctx &, int p, const double *raw) const {
        return p < n ? make_double2(raw[0], raw[1]) : make_double2(0.0, 0.0);
    }
    __device__ __forceinline__ double2 spec(const Ctx &, int k, double2 V) const { return cmul(V, sym(k)); }
    __device__ __forceinline__ void one(int64_t i, double Lv, double *acc) const {
        if constexpr (EPI == EPI_W) {
            w[i] = Lv;
        } else if constexpr (EPI == EPI_WADD) {
            w[i] += Lv;
        } else {
            const double yi = cb * (w[i] + Lv);
            if constexpr (EPI == EPI_Y) {
                y[i] = yi;
            } else if constexpr (EPI == EPI_DOT) {
                y[i] = yi;
                acc[0] = fma(rt[i], yi, acc[0]);
            } else {
                const double ri = fma(-alpha, yi, r[i]);
                r[i] = ri;
                acc[0] = fma(rt[i], ri, acc[0]);
                acc[1] = fma(ri, ri, acc[1]);
            }
        }
    }
    __device__ __forceinline__ void store(const Ctx &cx, int p, double2 V, double *acc) const {
        if (p >= n) return;
        one(cx.ia + p * s, V.x * invP, acc);
        one(cx.ib + p * s, V.y * invP, acc);
    }
    __device__ void store_half(const Ctx &, int, double2, double2) const {}
};

enum : int { PRE_X = 0, PRE_UP = 1, PRE_Q = 2 };

// P^{-1}, fast-axis forward pass: rows 2c and 2c+1 (length nf) of the input
// as one complex transform, unpacked into their half spectra (W = nf/2 + 1
// values per row in Z).  The input is
//   PRE_X: x;
//   PRE_UP: CGS's p after u = r + beta q, p = u + beta (q + beta p) (u and p
//     stored; u = p = r on a fresh start); beta from the folded reduction of
//     the previous iteration's rt.r and r.r, which also decides convergence;
//   PRE_Q: u + q after q = u - alpha vhat (q stored); alpha = rho / rt.vhat
//     from the folded reduction of rt.vhat.
template <int PRE, bool TR = false> struct HalfFwdOp {
    static constexpr int NFFT = 1, DIR = -1, FOLD = PRE != PRE_X, NACC = 0;
    // TR: the half spectra go to Z transposed (Z[k * nx + row], two dimensions),
    // written by the whole workgroup from LDS so that each k takes a run of
    // the tile's rows
    static constexpr bool HALF = !TR, HALF_T = TR, IN_T = false;
    static constexpr int NRAW = PRE == PRE_X ? 2 : PRE == PRE_UP ? 6 : 4;
    struct Ctx {
        int64_t ra, hb;
    };
    const double *x;        // PRE_X: input; PRE_UP: r; PRE_Q: u
    const double *q_in;     // PRE_UP: q; PRE_Q: vhat
    double *p_io, *u_out;   // PRE_UP
    double *q_out;          // PRE_Q
    double2 *Z;
    int64_t nf, W, nx;      // nx: rows of the array (TR)
    const double *fpart;    // partials folded here
    int fnp, k, fresh;
    double coef;            // beta (PRE_UP) or alpha (PRE_Q)
    double *part;           // unused (no reduction)
    int pred;
    __device__ void prep(const Sc *) {}
    __device__ bool fold(Sc *sc) {
        if constexpr (PRE == PRE_UP) {
            if (fresh) return false;
            double tot[2];
            reduce_partials<2>(fpart, fnp, tot);  // rt.r, r.r of r_k
            const double rho_old = sc->rho[(k - 1) & 1];
            int status = ST_OK, done = 0;
            if (!finite(tot[0]) || !finite(tot[1])) {
                status = ST_NONFINITE;
                done = 1;
            } else if (tot[1] <= sc->tol2) {
                done = 1;
            } else if (tot[0] == 0.0) {
                status = ST_BREAKDOWN;
                done = 1;
            }
            if (threadIdx.x == 0 && blockIdx.x == 0) {
                sc->rho[k & 1] = tot[0];
                sc->rnorm2 = tot[1];
                sc->iter = k;
                if (done) {
                    sc->status = status;
                    sc->done = 1;
                }
            }
            coef = tot[0] / rho_old;
            return done != 0;
        } else if constexpr (PRE == PRE_Q) {
            double tot[1];
            reduce_partials<1>(fpart, fnp, tot);  // rt.vhat
            const double a = sc->rho[k & 1] / tot[0];
            int status = ST_OK;
            if (tot[0] == 0.0) status = ST_BREAKDOWN;
            else if (!finite(a)) status = ST_NONFINITE;
            if (threadIdx.x == 0 && blockIdx.x == 0) {
                sc->alpha = a;
                if (status != ST_OK) {
                    sc->status = status;
                    sc->done = 1;
                }
            }
            coef = a;
            return status != ST_OK;
        } else {
            return false;
        }
    }
    __device__ __forceinline__ Ctx ctx(int64_t c) const { return Ctx{2 * c * nf, 2 * c * W}; }
    __device__ __forceinline__ void fetch(const Ctx &cx, int p, double *raw) const {
        const int64_t ia = cx.ra + p, ib = ia + nf;
        raw[0] = x[ia];
        raw[1] = x[ib];
        if constexpr (PRE == PRE_UP) {
            if (!fresh) {
                raw[2] = q_in[ia];
                raw[3] = q_in[ib];
                raw[4] = p_io[ia];
                raw[5] = p_io[ib];
            }
        } else if constexpr (PRE == PRE_Q) {
            raw[2] = q_in[ia];
            raw[3] = q_in[ib];
        }
    }
    __device__ __forceinline__ double2 finish(const Ctx &cx, int p, const double *raw) const {
        if constexpr (PRE == PRE_X) {
            return make_double2(raw[0], raw[1]);
        } else if constexpr (PRE == PRE_UP) {
            const int64_t ia = cx.ra + p, ib = ia + nf;
            double ua = raw[0], ub = raw[1], pa = raw[0], pb = raw[1];
            if (!fresh) {
                const double be = coef;
                ua = fma(be, raw[2], raw[0]);
                ub = fma(be, raw[3], raw[1]);
                pa = fma(be, fma(be, raw[4], raw[2]), ua);
                pb = fma(be, fma(be, raw[5], raw[3]), ub);
            }
            u_out[ia] = ua;
            u_out[ib] = ub;
            p_io[ia] = pa;
            p_io[ib] = pb;
            return make_double2(pa, pb);
        } else {
            const int64_t ia = cx.ra + p, ib = ia + nf;
            const double qa = fma(-coef, raw[2], raw[0]), qb = fma(-coef, raw[3], raw[1]);
            q_out[ia] = qa;
            q_out[ib] = qb;
            return make_double2(raw[0] + qa, raw[1] + qb);
        }
    }
    __device__ __forceinline__ double2 spec(const Ctx &, int, double2 V) const { return V; }
    __device__ __forceinline__ void store(const Ctx &, int, double2, double *) const {}
    __device__ __forceinline__ void store_half(const Ctx &cx, int k, double2 A, double2 Bv) const {
        Z[cx.hb + k] = A;
        Z[cx.hb + W + k] = Bv;
    }
    // TR: the tile's B pairs (rows 2 c0 .. 2 c0 + 2B - 1) from their LDS slabs
    // (natural order) to Z[k * nx + row], thread t taking k = idx / 2B, row
    // 2 c0 + idx % 2B, so consecutive threads write consecutive rows
    __device__ __forceinline__ void store_half_t(const double2 *lds, int LS, int B, int64_t c0, int64_t npairs,
                                                 int t, int nt) const {
        const int R = 2 * B;
        const int P = (int)nf;
        for (int idx = t; idx < (int)W * R; idx += nt) {
            const int k = idx / R, r = idx % R, q = r >> 1;
            if (c0 + q >= npairs) continue;
            const double2 *sl = lds + q * LS;
            const double2 Zk = sl[lpad(k)], Zc = sl[lpad((P - k) & (P - 1))];
            Z[(int64_t)k * nx + 2 * c0 + r] = (r & 1) ? make_double2(0.5 * (Zk.y + Zc.y), -0.5 * (Zk.x - Zc.x))
                                                      : make_double2(0.5 * (Zk.x + Zc.x), 0.5 * (Zk.y - Zc.y));
        }
    }
};

template <int PRE> HalfFwdOp<PRE, true> transposed(const HalfFwdOp<PRE, false> &f, int64_t nx) {
    HalfFwdOp<PRE, true> t{};
    t.x = f.x;
    t.q_in = f.q_in;
    t.p_io = f.p_io;
    t.u_out = f.u_out;
    t.q_out = f.q_out;
    t.Z = f.Z;
    t.nf = f.nf;
    t.W = f.W;
    t.nx = nx;
    t.fpart = f.fpart;
    t.fnp = f.fnp;
    t.k = f.k;
    t.fresh = f.fresh;
    t.pred = f.pred;
    return t;
}

// P^{-1}, pass along a middle axis (3D: y) of the half spectra, in place,
// forward (DIR -1) or inverse (DIR +1).  Line l: base (l / W) * n W + l % W,
// stride W.
template <int DIR_> struct CplxOp {
    static constexpr int NFFT = 1, DIR = DIR_, NRAW = 2, FOLD = 0, NACC = 0;
    static constexpr bool HALF = false, HALF_T = false, IN_T = false;
    struct Ctx {
        int64_t base;
    };
    double2 *Z;
    int64_t s, ns;
    double *part;
    int pred;
    __device__ void prep(const Sc *) {}
    __device__ bool fold(Sc *) { return false; }
    __device__ __forceinline__ Ctx ctx(int64_t l) const { return Ctx{line_base(l, s, ns)}; }
    __device__ __forceinline__ void fetch(const Ctx &cx, int p, double *raw) const {
        const double2 z = Z[cx.base + p * s];
        raw[0] = z.x;
        raw[1] = z.y;
    }
    __device__ __forceinline__ double2 finish(const Ctx &, int, const double *raw) const {
        return make_double2(raw[0], raw[1]);
    }
    __device__ __forceinline__ double2 spec(const Ctx &, int, double2 V) const { return V; }
    __device__ __forceinline__ void store(const Ctx &cx, int p, double2 V, double *) const { Z[cx.base + p * s] = V; }
    __device__ void store_half(const Ctx &, int, double2, double2) const {}
};

// P^{-1}, pass along the slow axis x of the half spectra, in place: the DFT,
// the division by eta - sigma (mu_x(k) + mu_other), the inverse DFT.  Line l
// (element p at l + p * nl) carries the frequencies kf = l % W of the fast
// axis and, in 3D, km = l / W of the middle axis; mu_other is their symbols'
// sum (Strang circulants' eigenvalues).
struct DivOp {
    static constexpr int NFFT = 2, DIR = 0, NRAW = 2, FOLD = 0, NACC = 0;
    static constexpr bool HALF = false, HALF_T = false, IN_T = false;
    struct Ctx {
        int64_t l;
        double2 mo;
    };
    double2 *Z;
    int64_t nl, W;  // element p of line l at l * ll + p * nl
    int64_t ll = 1;
    int mid;  // 1 in 3D
    Sym sx, sm, sf;
    double eta, sigma;
    double *part;
    int pred;
    __device__ void prep(const Sc *) {}
    __device__ bool fold(Sc *) { return false; }
    __device__ __forceinline__ Ctx ctx(int64_t l) const {
        double2 mo = sf(l % W);
        if (mid) {
            const double2 m2 = sm(l / W);
            mo.x += m2.x;
            mo.y += m2.y;
        }
        return Ctx{l * ll, mo};
    }
    __device__ __forceinline__ void fetch(const Ctx &cx, int p, double *raw) const {
        const double2 z = Z[cx.l + p * nl];
        raw[0] = z.x;
        raw[1] = z.y;
    }
    __device__ __forceinline__ double2 finish(const Ctx &, int, const double *raw) const {
        return make_double2(raw[0], raw[1]);
    }
    __device__ __forceinline__ double2 spec(const Ctx &cx, int k, double2 V) const {
        const double2 mx = sx(k);
        const double er = eta - sigma * (mx.x + cx.mo.x), ei = -sigma * (mx.y + cx.mo.y);
        const double q = 1.0 / fma(er, er, ei * ei);
        return make_double2(fma(V.x, er, V.y * ei) * q, fma(V.y, er, -V.x * ei) * q);
    }
    __device__ __forceinline__ void store(const Ctx &cx, int p, double2 V, double *) const { Z[cx.l + p * nl] = V; }
    __device__ void store_half(const Ctx &, int, double2, double2) const {}
};

// P^{-1}, fast-axis inverse pass: the half spectra of rows 2c and 2c+1
// extended by conjugate symmetry (X_{nf-k} = conj X_k; the k = 0 and k = nf/2
// values of a real row are real) into Z = X_a + i X_b, the inverse DFT, real
// part -> row 2c, imaginary part -> row 2c+1, scaled by 1/N.
struct HalfInvOp {
    static constexpr int NFFT = 1, DIR = 1, NRAW = 4, FOLD = 0, NACC = 0;
    static constexpr bool HALF = false, HALF_T = false, IN_T = false;
    struct Ctx {
        int64_t ra, hb;
    };
    const double2 *Z;
    double *y;
    double *x;  // non-NULL: also x += alpha y (CGS, the second solve of an iteration)
    int64_t nf, W;
    double scale, alpha;
    double *part;
    int pred;
    __device__ void prep(const Sc *sc) {
        if (x) alpha = sc->alpha;
    }
    __device__ bool fold(Sc *) { return false; }
    __device__ __forceinline__ Ctx ctx(int64_t c) const { return Ctx{2 * c * nf, 2 * c * W}; }
    __device__ __forceinline__ void fetch(const Ctx &cx, int p, double *raw) const {
        const int64_t k = p <= nf / 2 ? p : nf - p;
        const double2 a = Z[cx.hb + k], b = Z[cx.hb + W + k];
        raw[0] = a.x;
        raw[1] = a.y;
        raw[2] = b.x;
        raw[3] = b.y;
    }
    __device__ __forceinline__ double2 finish(const Ctx &, int p, const double *raw) const {
        double ay = raw[1], by = raw[3];
        if (p == 0 || p == nf / 2) {
            ay = 0.0;
            by = 0.0;
        } else if (p > nf / 2) {
            ay = -ay;
            by = -by;
        }
        return make_double2(raw[0] - by, ay + raw[2]);
    }
    __device__ __forceinline__ double2 spec(const Ctx &, int, double2 V) const { return V; }
    __device__ __forceinline__ void store(const Ctx &cx, int p, double2 V, double *) const {
        const int64_t ia = cx.ra + p, ib = ia + nf;
        const double ya = V.x * scale, yb = V.y * scale;
        y[ia] = ya;
        y[ib] = yb;
        if (x) {
            x[ia] = fma(alpha, ya, x[ia]);
            x[ib] = fma(alpha, yb, x[ib]);
        }
    }
    __device__ void store_half(const Ctx &, int, double2, double2) const {}
};

// P^{-1}, fast-axis inverse pass from transposed half spectra (two
// dimensions, Z[k * nx + row]): the workgroup first copies its pairs' half
// spectra into LDS (consecutive threads, consecutive rows of one k; row 2c's
// values at slab[k], row 2c+1's at slab[W + k], 2W <= LS slots), then works
// as HalfInvOp.
struct HalfInvTOp {
    static constexpr int NFFT = 1, DIR = 1, NRAW = 4, FOLD = 0, NACC = 0;
    static constexpr bool HALF = false, HALF_T = false, IN_T = true;
    struct Ctx {
        int64_t ra;
        const double2 *slab;
    };
    const double2 *Z;
    double *y;
    double *x;  // non-NULL: also x += alpha y, as in HalfInvOp
    int64_t nf, W, nx;
    double scale, alpha;
    double *part;
    int pred;
    __device__ void prep(const Sc *sc) {
        if (x) alpha = sc->alpha;
    }
    __device__ bool fold(Sc *) { return false; }
    __device__ __forceinline__ Ctx ctx(int64_t c) const { return Ctx{2 * c * nf, nullptr}; }
    __device__ __forceinline__ void stage_in(double2 *lds, int LS, int B, int64_t c0, int64_t npairs, int t,
                                             int nt) const {
        const int R = 2 * B;
        for (int idx = t; idx < (int)W * R; idx += nt) {
            const int k = idx / R, r = idx % R, q = r >> 1;
            if (c0 + q >= npairs) continue;
            lds[q * LS + (r & 1) * (int)W + k] = Z[(int64_t)k * nx + 2 * c0 + r];
        }
    }
    __device__ __forceinline__ void fetch(const Ctx &cx, int p, double *raw) const {
        const int k = p <= nf / 2 ? p : (int)nf - p;
        const double2 a = cx.slab[k], b = cx.slab[W + k];
        raw[0] = a.x;
        raw[1] = a.y;
        raw[2] = b.x;
        raw[3] = b.y;
    }
    __device__ __forceinline__ double2 finish(const Ctx &, int p, const double *raw) const {
        double ay = raw[1], by = raw[3];
        if (p == 0 || p == nf / 2) {
            ay = 0.0;
            by = 0.0;
        } else if (p > nf / 2) {
            ay = -ay;
            by = -by;
        }
        return make_double2(raw[0] - by, ay + raw[2]);
    }
    __device__ __forceinline__ double2 spec(const Ctx &, int, double2 V) const { return V; }
    __device__ __forceinline__ void store(const Ctx &cx, int p, double2 V, double *) const {
        const int64_t ia = cx.ra + p, ib = ia + nf;
        const double ya = V.x * scale, yb = V.y * scale;
        y[ia] = ya;
        y[ib] = yb;
        if (x) {
            x[ia] = fma(alpha, ya, x[ia]);
            x[ib] = fma(alpha, yb, x[ib]);
        }
    }
    __device__ void store_half(const Ctx &, int, double2, double2) const {}
};

// Forward DFT of one real column of `len` values zero-padded to P (spectra).
struct SpecOp {
    static constexpr int NFFT = 1, DIR = -1, NRAW = 1, FOLD = 0, NACC = 0;
    static constexpr bool HALF = false, HALF_T = false, IN_T = false;
    struct Ctx {
        int dummy;
    };
    const double *col;
    double2 *out;
    int64_t len;
    double *part;
    int pred;
    __device__ void prep(const Sc *) {}
    __device__ bool fold(Sc *) { return false; }
    __device__ __forceinline__ Ctx ctx(int64_t) const { return Ctx{0}; }
    __device__ __forceinline__ void fetch(const Ctx &, int p, double *raw) const {
        raw[0] = p < len ? col[p] : 0.0;
    }
    __device__ __forceinline__ double2 finish(const Ctx &, int, const double *raw) const {
        return make_double2(raw[0], 0.0);
    }
    __device__ __forceinline__ double2 spec(const Ctx &, int, double2 V) const { return V; }
    __device__ __forceinline__ void store(const Ctx &, int p, double2 V, double *) const { out[p] = V; }
    __device__ void store_half(const Ctx &, int, double2, double2) const {}
};

// ---------------------------------------------------------------------------
// Vector kernels (right-hand side, history, acceptance check, finishing
// steps).
// ---------------------------------------------------------------------------
#define TSFND_LOOP(i, N) for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < (N); i += (int64_t)gridDim.x * RB)

__global__ void __launch_bounds__(RB) k_fill(double *x, int64_t N, double val) {
    TSFND_LOOP(i, N) x[i] = val;
}

// History of (3.1): H_L = kappa sum_{s<L} c_{L-s}^(L) (u^{s+1} - u^s), with
// c_L^(L) = clast_L (the s = 0 term) and c_m^(L) = cbase[m] for 1 <= m < L
// (Lemma 1), summed in blocks of HB levels: at a block's first level b the
// sweep forms, in one pass over u^0..u^{b-1}, the part of every level
// L = b..b+HB-1 that uses only those levels (s <= b-2); each level L then
// adds the terms s = b-1..L-1 (the catch-up).  About b + HB vectors per
// block plus L - b + 3 per level, against L + 2 per level for the whole sum.
constexpr int HB = 8;
struct HbLast {
    double c[HB];  // clast of the block's levels
};

__global__ void __launch_bounds__(RB) k_hist_sweep(const double *__restrict__ U, int64_t N, int b, int nl,
                                                   const double *__restrict__ cbase, HbLast cl,
                                                   double *__restrict__ Q) {
    TSFND_LOOP(i, N) {
        double acc[HB];
#pragma unroll
        for (int q = 0; q < HB; ++q) acc[q] = 0.0;
        double prev = U[i];
        for (int s = 0; s <= b - 2; ++s) {
            const double next = U[(int64_t)(s + 1) * N + i];
            const double d = next - prev;
            prev = next;
#pragma unroll
            for (int q = 0; q < HB; ++q) acc[q] = fma(s == 0 ? cl.c[q] : cbase[b + q - s], d, acc[q]);
        }
#pragma unroll
        for (int q = 0; q < HB; ++q)
            if (q < nl) Q[(int64_t)q * N + i] = acc[q];
    }
}

// catch-up of level L in the block starting at b: Q_L (NULL in the first
// block) plus the terms s = max(b-1, 0)..L-1, times kappa
__global__ void __launch_bounds__(RB) k_hist_catch(const double *__restrict__ U, int64_t N, int L, int b,
                                                   const double *__restrict__ cbase, double clast_L, double kappa,
                                                   const double *__restrict__ QL, double *__restrict__ H) {
    const int s0 = b - 1 > 0 ? b - 1 : 0;
    TSFND_LOOP(i, N) {
        double acc = QL ? QL[i] : 0.0;
        for (int s = s0; s < L; ++s)
            acc = fma(s == 0 ? clast_L : cbase[L - s], U[(int64_t)(s + 1) * N + i] - U[(int64_t)s * N + i], acc);
        H[i] = kappa * acc;
    }
}

// initial guess of level j: u^j (mode 1) or 3u^j - 3u^{j-1} + u^{j-2} (mode 2)
__global__ void __launch_bounds__(RB) k_guess(const double *__restrict__ U, int64_t N, int j, int mode,
                                              double *__restrict__ x) {
    const double *uj = U + (int64_t)j * N;
    if (mode == 1) {
        TSFND_LOOP(i, N) x[i] = uj[i];
    } else {
        const double *u1 = uj - N, *u2 = uj - 2 * N;  // mode 2 only at j >= 2
        TSFND_LOOP(i, N) x[i] = fma(3.0, uj[i] - u1[i], u2[i]);
    }
}

// g = B u^j - H + f; r = rt = g (zero initial guess); partial |g|^2
__global__ void __launch_bounds__(RB) k_rhs(const double *__restrict__ Bu, const double *__restrict__ H,
                                            const double *__restrict__ f, double *__restrict__ g,
                                            double *__restrict__ r, double *__restrict__ rt, int64_t N,
                                            double *partials) {
    double acc[1] = {0.0};
    TSFND_LOOP(i, N) {
        double v = Bu[i];
        if (H) v -= H[i];
        if (f) v += f[i];
        g[i] = v;
        r[i] = v;
        rt[i] = v;
        acc[0] = fma(v, v, acc[0]);
    }
    block_partial<1>(acc, partials, blockIdx.x);
}

__global__ void __launch_bounds__(RB) k_fin_rhs(const double *partials, int np, Sc *sc, double rtol) {
    double tot[1];
    reduce_partials<1>(partials, np, tot);
    if (threadIdx.x == 0) {
        Sc s{};
        s.gnorm2 = tot[0];
        s.rnorm2 = tot[0];
        s.rho[0] = tot[0];
        s.tol2 = rtol * rtol * tot[0];
        s.aux0 = tot[0];
        s.status = finite(tot[0]) ? ST_OK : ST_NONFINITE;
        s.done = (tot[0] == 0.0 || !finite(tot[0])) ? 1 : 0;
        *sc = s;
    }
}

// chunk end: the finishing step of iteration k-1's r update (what the next
// iteration's first pass would fold), so a poll sees convergence at once
__global__ void __launch_bounds__(RB) k_fold_rho(const double *partials, int np, Sc *sc, int k) {
    if (sc->done) return;
    double tot[2];
    reduce_partials<2>(partials, np, tot);
    if (threadIdx.x == 0) {
        sc->rho[k & 1] = tot[0];
        sc->rnorm2 = tot[1];
        sc->iter = k;
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
__global__ void __launch_bounds__(RB) k_true(const double *__restrict__ g, const double *__restrict__ Ax,
                                             const double *__restrict__ x, double *__restrict__ r,
                                             double *__restrict__ rt, int64_t N, double *partials) {
    double acc[2] = {0.0, 0.0};
    TSFND_LOOP(i, N) {
        const double ri = g[i] - Ax[i];
        r[i] = ri;
        rt[i] = ri;
        acc[0] = fma(ri, ri, acc[0]);
        acc[1] = fma(x[i], x[i], acc[1]);
    }
    block_partial<2>(acc, partials, blockIdx.x);
}

// accept x at |r| <= rtol |g| or backward error |r| / (anorm |x| + |g|) <=
// bwtol; otherwise restart CGS from x at iteration k (r = rt = g - A x)
__global__ void __launch_bounds__(RB) k_fin_true(const double *partials, int np, Sc *sc, double anorm, double bwtol,
                                                 int k) {
    double tot[2];
    reduce_partials<2>(partials, np, tot);
    if (threadIdx.x == 0) {
        sc->nchecks += 1;
        sc->aux0 = tot[0];
        sc->aux1 = tot[1];
        sc->rnorm2 = tot[0];
        sc->rho[k & 1] = tot[0];
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

// the partials of a large reducing pass summed into NA values (in the
// fixed order of reduce_partials), which the folding pass then reads
template <int NA> __global__ void __launch_bounds__(RB) k_squash(const double *partials, int np, double *out, const Sc *sc) {
    if (sc->done) return;
    double tot[NA];
    reduce_partials<NA>(partials, np, tot);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int a = 0; a < NA; ++a) out[a] = tot[a];
    }
}

#undef TSFND_LOOP

}  // namespace tsfnd

// ===========================================================================
// Host side.
// ===========================================================================
using namespace tsfnd;

namespace {

constexpr double BW_TOL = 1e-13;
constexpr int MAX_RESTARTS = 3;

// One plan of either dimension.  Axis 0 is x (slowest), axis d-1 the fast
// (contiguous) axis.
struct NdPlan {
    int d = 2;
    hipStream_t stream = nullptr;
    int64_t n[3] = {1, 1, 1}, N = 0, M = 0, level = 0, W = 0, Nh = 0;
    double alpha = 0, T = 0, tau = 0, sigma = 0, kappa = 0, rtol = 1e-10;
    double beta[3] = {}, lo[3] = {}, h[3] = {}, hb[3] = {};
    int maxit = 500, last_iters = 8, warm = TSFCDE_WS_ZERO;
    std::vector<double> eta, anorm, cbase, clast, gam[3], dp[3], dm[3];
    tsfcde2d_src_fn f2 = nullptr;
    tsfcde3d_src_fn f3 = nullptr;
    void *fuser = nullptr;
    double *h_f = nullptr;  // pinned staging of callback sources
    Sc *h_sc = nullptr;     // pinned copy of the device scalars
    // device (inside the caller's workspace)
    double *U = nullptr, *g = nullptr, *r = nullptr, *rt = nullptr, *u = nullptr, *p = nullptr, *q = nullptr,
           *phat = nullptr, *uhat = nullptr, *vhat = nullptr, *t = nullptr, *w = nullptr, *H = nullptr,
           *fbuf = nullptr, *part1 = nullptr, *part2 = nullptr, *partv = nullptr, *sq = nullptr,
           *d_cbase = nullptr, *cols = nullptr;
    double2 *Z = nullptr, *lam[3] = {}, *ls[3] = {}, *tw = nullptr;
    Sc *sc = nullptr;
    double2 *symE[3] = {}, *symS[3] = {};  // level sym_level's symbols (embedding, Strang)
    int64_t sym_level = -1;
    double *Q = nullptr;  // the current history block's partial sums (HB vectors)
    int64_t qblock = 0;   // first level of the block Q holds (0: none)
    // what the folding passes read: rt.vhat (fold1) and rt.r, r.r (fold2)
    // partials, nfold1 / nfold2 of them
    const double *fold1 = nullptr, *fold2 = nullptr;
    int nfold1 = 0, nfold2 = 0;
};

}  // namespace

struct tsfcde2d_plan_s : NdPlan {};
struct tsfcde3d_plan_s : NdPlan {};

namespace {

bool pow2_in(int64_t v, int64_t lo, int64_t hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int NVEC = 13;  // g r rt u p q phat uhat vhat t w H fbuf

struct Layout {
    size_t U, vec, Z, lam, sym, tw, part, sc, cb, Q, cols, total;
};

int64_t spec_len(const int64_t *n, int d) {
    int64_t s = 0;
    for (int a = 0; a < d; ++a) s += 3 * n[a];  // embedding (2n) and Strang (n) spectra
    return s;
}

// partials of a reducing pass along x, per accumulator: at most one per
// workgroup of B >= 1 lines of 2 n_x points over 8 values per lane and at
// least 256 lanes, i.e. N / 2048
int64_t part_len(int64_t N) { return N / 1024 + 64; }

Layout layout(const int64_t *n, int d, int64_t M) {
    int64_t N = 1;
    for (int a = 0; a < d; ++a) N *= n[a];
    const int64_t W = n[d - 1] / 2 + 1, Nh = N / n[d - 1] * W;
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = al256(o + bytes);
        return at;
    };
    L.U = take(sizeof(double) * (size_t)(M + 1) * (size_t)N);
    L.vec = take(sizeof(double) * NVEC * (size_t)N);
    L.Z = take(sizeof(double2) * (size_t)Nh);
    L.lam = take(sizeof(double2) * (size_t)spec_len(n, d));
    L.sym = take(sizeof(double2) * (size_t)spec_len(n, d));
    L.tw = take(sizeof(double2) * (size_t)((int64_t(1) << (PMAX_LOG2 + 1)) - 2));
    L.part = take(sizeof(double) * (size_t)(2 * 2 * part_len(N) + 2 * RBLK + 4));
    L.sc = take(sizeof(Sc));
    L.cb = take(sizeof(double) * (size_t)(M + 2 + HB));
    L.Q = take(sizeof(double) * HB * (size_t)N);
    L.cols = take(sizeof(double) * (size_t)spec_len(n, d));
    L.total = o;
    return L;
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

double level_time(const NdPlan *pl, int64_t j) { return ((double)j + pl->sigma) * pl->tau; }

int nblocks(int64_t N) { return (int)std::min<int64_t>(RBLK, (N + RB - 1) / RB); }

#define HIPCHK(x)                                    \
    do {                                             \
        if ((x) != hipSuccess) return TSFCDE_EDEVICE; \
    } while (0)

// Launch of k_line, one tile per workgroup; returns the grid through
// *grid_out.  Row passes take workgroups of 256 threads: half the LDS per
// workgroup, twice the workgroups per CU, whose load, transform and store
// phases overlap better (1.7% less time per CGS iteration at 256^3; at
// 1024 x 1024 the same waves spread over more CUs); rows of 4096 points (512
// lanes each) take 512.  Strided passes keep 512 threads, whose wider tiles
// (more adjacent lines) read longer runs of each row (11% less time per CGS
// iteration at 1024 x 1024; 256 threads in the strided passes of up to 512
// points were 3% slower at 256^3).
// Eight values per lane in every pass: sixteen in the Toeplitz passes of 256
// points and more (half the exchanges at 256, 1024 and 2048 points, twice the
// LDS per workgroup) measured 13% slower per CGS iteration at 1024 x 1024 and
// 22% at 256^3.
template <class Op, int P> constexpr int line_e() { return 8; }

template <int P, bool ROWS, int NTL, class Op>
hipError_t line_g(NdPlan *pl, const Op &op, int64_t nlines, int *grid_out) {
    constexpr int EV = line_e<Op, P>();
    using G = LineGeo<P, NTL, EV>;
    const int64_t grid = (nlines + G::B - 1) / G::B;
    if (grid < 1 || grid > INT32_MAX) return hipErrorInvalidValue;
    if (grid_out) *grid_out = (int)grid;
    hipLaunchKernelGGL((k_line<P, ROWS, NTL, Op, EV>), dim3((unsigned)grid), dim3(NTL), 0, pl->stream, op, nlines,
                       (const double2 *)pl->tw, pl->sc);
    return hipGetLastError();
}

template <class Op, class = void> struct WideTile {
    static constexpr bool value = false;
};
template <class Op> struct WideTile<Op, decltype(void(Op::WIDE))> {
    static constexpr bool value = Op::WIDE;
};

template <int P, bool ROWS, class Op>
hipError_t line_t(NdPlan *pl, const Op &op, int64_t nlines, int *grid_out) {
    if constexpr (ROWS && P / 8 <= 256) {
        return line_g<P, ROWS, 256>(pl, op, nlines, grid_out);
    } else if constexpr (!ROWS && (P == 1024 || P == 4096) && WideTile<Op>::value) {
        // slow-axis products on 1024- and 4096-point embeddings (axes of 512
        // and 2048): 1024 threads hold twice the lines of 512, so each row
        // run is twice as long (at 512^3 whole 128-byte lines: 12% and 8%
        // less time for the two CGS forms; 8% less per CGS iteration at
        // 2048^2).  The middle-axis pass was 14% slower that way, and at 2048
        // points (axes of 1024) the wider form spills: 8% slower per CGS
        // iteration at 1024^2; both keep 512.
        return line_g<P, ROWS, 1024>(pl, op, nlines, grid_out);
    } else {
        return line_g<P, ROWS, NT>(pl, op, nlines, grid_out);
    }
}

template <bool ROWS, class Op>
hipError_t line(NdPlan *pl, int64_t P, const Op &op, int64_t nlines, int *grid_out = nullptr) {
    switch (P) {
        case 16: return line_t<16, ROWS>(pl, op, nlines, grid_out);
        case 32: return line_t<32, ROWS>(pl, op, nlines, grid_out);
        case 64: return line_t<64, ROWS>(pl, op, nlines, grid_out);
        case 128: return line_t<128, ROWS>(pl, op, nlines, grid_out);
        case 256: return line_t<256, ROWS>(pl, op, nlines, grid_out);
        case 512: return line_t<512, ROWS>(pl, op, nlines, grid_out);
        case 1024: return line_t<1024, ROWS>(pl, op, nlines, grid_out);
        case 2048: return line_t<2048, ROWS>(pl, op, nlines, grid_out);
        case 4096: return line_t<4096, ROWS>(pl, op, nlines, grid_out);
        default: return hipErrorInvalidValue;
    }
}

// The partials of a reducing pass as the folding pass reads them: in place
// up to MAXPART, else summed first into NA values at `sq`.
template <int NA>
hipError_t finish_partials(NdPlan *pl, double *part, int np, double *sq, const double **f, int *fn) {
    if (np <= MAXPART) {
        *f = part;
        *fn = np;
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_squash<NA>, dim3(1), dim3(RB), 0, pl->stream, (const double *)part, np, sq,
                       (const Sc *)pl->sc);
    *f = sq;
    *fn = 1;
    return hipGetLastError();
}

// stride of axis a and the symbol of L_axis at level j: on the embedding
// (length 2n, emb) or of the Strang circulant (length n)
int64_t stride_of(const NdPlan *pl, int a) {
    int64_t s = 1;
    for (int b = a + 1; b < pl->d; ++b) s *= pl->n[b];
    return s;
}

// The symbol tables of level j (all axes), computed when the plan's tables
// hold another level.
hipError_t ensure_symbols(NdPlan *pl, int64_t j) {
    if (pl->sym_level == j) return hipSuccess;
    SymTabs t{};
    for (int a = 0; a < pl->d; ++a) {
        for (int emb = 0; emb < 2; ++emb) {
            const int e = t.count++;
            const int64_t P = emb ? 2 * pl->n[a] : pl->n[a];
            t.lam[e] = emb ? pl->lam[a] : pl->ls[a];
            t.tw[e] = pl->tw + tw_offset((int)P);
            t.out[e] = emb ? pl->symE[a] : pl->symS[a];
            t.P[e] = P;
            t.cre[e] = pl->hb[a] * (pl->dp[a][j] + pl->dm[a][j]);
            t.cim[e] = pl->hb[a] * (pl->dp[a][j] - pl->dm[a][j]);
            t.cq[e] = pl->gam[a][j] / pl->h[a];
        }
    }
    hipLaunchKernelGGL(k_symbols, dim3(16, (unsigned)t.count), dim3(256), 0, pl->stream, t);
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) pl->sym_level = j;
    return e;
}

// level j's symbol of axis a (ensure_symbols(pl, j) queued before)
Sym symbol(const NdPlan *pl, int a, int64_t, bool emb) {
    Sym s{};
    s.tab = emb ? pl->symE[a] : pl->symS[a];
    return s;
}

enum class Fin { Y, DOT, XR };

// y = ca v + cb L v at level j, L = sum_axes L_axis: the fast axis first
// (w = L v), a middle axis adds (w += L v), the slow axis finishes (with
// ca/cb folded into its symbol) with the epilogue `fin` (Y: store y; DOT:
// store y = vhat and reduce rt.y into part1; XR: update r from y = A v and
// reduce rt.r, r.r into part2).  cb must not be 0.
hipError_t product(NdPlan *pl, int64_t j, const double *v, double *y, double ca, double cb, int pred, Fin fin) {
    const int d = pl->d;
    hipError_t e;
    for (int a = d - 1; a >= 1; --a) {
        const int64_t n = pl->n[a], s = stride_of(pl, a), nlines = pl->N / n / 2;
        if (a == d - 1) {
            ToepOp<EPI_W> o{};
            o.v = v;
            o.n = n;
            o.s = s;
            o.ns = n * s;
            o.sym = symbol(pl, a, j, true);
            o.invP = 1.0 / (double)(2 * n);
            o.w = pl->w;
            o.pred = pred;
            e = line<true>(pl, 2 * n, o, nlines);
        } else {
            ToepOp<EPI_WADD> o{};
            o.v = v;
            o.n = n;
            o.s = s;
            o.ns = n * s;
            o.sym = symbol(pl, a, j, true);
            o.invP = 1.0 / (double)(2 * n);
            o.w = pl->w;
            o.pred = pred;
            e = line<false>(pl, 2 * n, o, nlines);
        }
        if (e != hipSuccess) return e;
    }
    const int64_t n = pl->n[0], s = stride_of(pl, 0), nlines = pl->N / n / 2;
    auto fill = [&](auto &o) {
        o.v = v;
        o.n = n;
        o.s = s;
        o.ns = n * s;
        o.sym = symbol(pl, 0, j, true);
        o.sym.c0 = ca / cb;
        o.invP = 1.0 / (double)(2 * n);
        o.w = pl->w;
        o.y = y;
        o.cb = cb;
        o.rt = pl->rt;
        o.pred = pred;
    };
    if (fin == Fin::Y) {
        ToepOp<EPI_Y> o{};
        fill(o);
        return line<false>(pl, 2 * n, o, nlines);
    }
    int np = 0;
    if (fin == Fin::DOT) {
        ToepOp<EPI_DOT> o{};
        fill(o);
        o.part = pl->part1;
        if ((e = line<false>(pl, 2 * n, o, nlines, &np)) != hipSuccess) return e;
        return finish_partials<1>(pl, pl->part1, np, pl->sq, &pl->fold1, &pl->nfold1);
    }
    ToepOp<EPI_XR> o{};
    fill(o);
    o.r = pl->r;
    o.part = pl->part2;
    if ((e = line<false>(pl, 2 * n, o, nlines, &np)) != hipSuccess) return e;
    return finish_partials<2>(pl, pl->part2, np, pl->sq + 2, &pl->fold2, &pl->nfold2);
}

// y = P^{-1} (input of the first pass) at level j: the fast-axis forward pass
// `first` (built by the caller), the middle axis (3D), the slow axis with
// the division, the middle axis back, the fast axis back into y.
template <class First>
hipError_t psolve_from(NdPlan *pl, int64_t j, const First &first, double *y, int pred, double *x_upd = nullptr) {
    const int d = pl->d;
    const int64_t nf = pl->n[d - 1], W = pl->W, rows2 = pl->N / nf / 2;
    hipError_t e;
    if (d == 2) {
        // two dimensions: the half spectrum kept transposed (Z[ky * nx + kx]),
        // so the division pass runs along contiguous rows
        const int64_t nx = pl->n[0];
        if ((e = line<true>(pl, nf, transposed(first, nx), rows2)) != hipSuccess) return e;
        DivOp dv{};
        dv.Z = pl->Z;
        dv.nl = 1;
        dv.ll = nx;
        dv.W = W;
        dv.mid = 0;
        dv.sx = symbol(pl, 0, j, false);
        dv.sf = symbol(pl, 1, j, false);
        dv.eta = pl->eta[j];
        dv.sigma = pl->sigma;
        dv.pred = pred;
        if ((e = line<true>(pl, nx, dv, W)) != hipSuccess) return e;
        HalfInvTOp hi{};
        hi.Z = pl->Z;
        hi.y = y;
        hi.x = x_upd;
        hi.nf = nf;
        hi.W = W;
        hi.nx = nx;
        hi.scale = 1.0 / (double)pl->N;
        hi.pred = pred;
        return line<true>(pl, nf, hi, rows2);
    }
    e = line<true>(pl, nf, first, rows2);
    if (e != hipSuccess) return e;
    if (d == 3) {
        CplxOp<-1> o{};
        o.Z = pl->Z;
        o.s = W;
        o.ns = pl->n[1] * W;
        o.pred = pred;
        if ((e = line<false>(pl, pl->n[1], o, pl->Nh / pl->n[1])) != hipSuccess) return e;
    }
    DivOp dv{};
    dv.Z = pl->Z;
    dv.nl = pl->Nh / pl->n[0];
    dv.W = W;
    dv.mid = d == 3;
    dv.sx = symbol(pl, 0, j, false);
    dv.sf = symbol(pl, d - 1, j, false);
    if (d == 3) dv.sm = symbol(pl, 1, j, false);
    dv.eta = pl->eta[j];
    dv.sigma = pl->sigma;
    dv.pred = pred;
    if ((e = line<false>(pl, pl->n[0], dv, dv.nl)) != hipSuccess) return e;
    if (d == 3) {
        CplxOp<1> o{};
        o.Z = pl->Z;
        o.s = W;
        o.ns = pl->n[1] * W;
        o.pred = pred;
        if ((e = line<false>(pl, pl->n[1], o, pl->Nh / pl->n[1])) != hipSuccess) return e;
    }
    HalfInvOp hi{};
    hi.Z = pl->Z;
    hi.y = y;
    hi.x = x_upd;
    hi.nf = nf;
    hi.W = W;
    hi.scale = 1.0 / (double)pl->N;
    hi.pred = pred;
    return line<true>(pl, nf, hi, rows2);
}

hipError_t psolve(NdPlan *pl, int64_t j, const double *v, double *y, int pred) {
    HalfFwdOp<PRE_X> f{};
    f.x = v;
    f.Z = pl->Z;
    f.nf = pl->n[pl->d - 1];
    f.W = pl->W;
    f.pred = pred;
    return psolve_from(pl, j, f, y, pred);
}

// CGS iteration k (Barrett et al., Templates), right preconditioned:
//   u = r + beta q, p = u + beta (q + beta p)  (u = p = r when fresh)
//   phat = P^{-1} p, vhat = A phat, alpha = rho / rt.vhat
//   q = u - alpha vhat, uhat = P^{-1} (u + q)
//   x += alpha uhat, r -= alpha A uhat, rho' = rt.r
hipError_t cgs_iteration(NdPlan *pl, int64_t j, double *x, int k, bool fresh) {
    hipError_t e;
    const double eta = pl->eta[j], sg = pl->sigma;
    HalfFwdOp<PRE_UP> a{};
    a.x = pl->r;
    a.q_in = pl->q;
    a.p_io = pl->p;
    a.u_out = pl->u;
    a.Z = pl->Z;
    a.nf = pl->n[pl->d - 1];
    a.W = pl->W;
    a.fpart = pl->fold2;
    a.fnp = pl->nfold2;
    a.k = k;
    a.fresh = fresh ? 1 : 0;
    a.pred = 1;
    if ((e = psolve_from(pl, j, a, pl->phat, 1)) != hipSuccess) return e;
    if ((e = product(pl, j, pl->phat, pl->vhat, eta, -sg, 1, Fin::DOT)) != hipSuccess) return e;
    HalfFwdOp<PRE_Q> c{};
    c.x = pl->u;
    c.q_in = pl->vhat;
    c.q_out = pl->q;
    c.Z = pl->Z;
    c.nf = pl->n[pl->d - 1];
    c.W = pl->W;
    c.fpart = pl->fold1;
    c.fnp = pl->nfold1;
    c.k = k;
    c.pred = 1;
    if ((e = psolve_from(pl, j, c, pl->uhat, 1, x)) != hipSuccess) return e;  // and x += alpha uhat
    return product(pl, j, pl->uhat, nullptr, eta, -sg, 1, Fin::XR);
}

int poll(NdPlan *pl) {
    HIPCHK(hipMemcpyAsync(pl->h_sc, pl->sc, sizeof(Sc), hipMemcpyDeviceToHost, pl->stream));
    HIPCHK(hipStreamSynchronize(pl->stream));
    return TSFCDE_OK;
}

int status_code(int st) {
    if (st == ST_BREAKDOWN) return TSFCDE_EBREAKDOWN;
    if (st == ST_NONFINITE) return TSFCDE_ENONFINITE;
    return TSFCDE_OK;
}

void node_coords(const NdPlan *pl, int a, int64_t i, double *out) { *out = pl->lo[a] + (double)(i + 1) * pl->h[a]; }

int callback_source(NdPlan *pl, int64_t j, const double **d_f) {
    *d_f = nullptr;
    if (!pl->f2 && !pl->f3) return TSFCDE_OK;
    if (!pl->h_f && hipHostMalloc(reinterpret_cast<void **>(&pl->h_f), sizeof(double) * (size_t)pl->N) != hipSuccess) {
        pl->h_f = nullptr;
        return TSFCDE_EDEVICE;
    }
    HIPCHK(hipStreamSynchronize(pl->stream));  // the last copy out of h_f has finished
    const double t = level_time(pl, j);
    if (pl->d == 2) {
        for (int64_t i = 0; i < pl->n[0]; ++i) {
            double x, y;
            node_coords(pl, 0, i, &x);
            for (int64_t k = 0; k < pl->n[1]; ++k) {
                node_coords(pl, 1, k, &y);
                pl->h_f[i * pl->n[1] + k] = pl->f2(x, y, t, pl->fuser);
            }
        }
    } else {
        for (int64_t i = 0; i < pl->n[0]; ++i) {
            double x, y, z;
            node_coords(pl, 0, i, &x);
            for (int64_t k = 0; k < pl->n[1]; ++k) {
                node_coords(pl, 1, k, &y);
                for (int64_t l = 0; l < pl->n[2]; ++l) {
                    node_coords(pl, 2, l, &z);
                    pl->h_f[(i * pl->n[1] + k) * pl->n[2] + l] = pl->f3(x, y, z, t, pl->fuser);
                }
            }
        }
    }
    HIPCHK(hipMemcpyAsync(pl->fbuf, pl->h_f, sizeof(double) * (size_t)pl->N, hipMemcpyHostToDevice, pl->stream));
    *d_f = pl->fbuf;
    return TSFCDE_OK;
}

int level_step(NdPlan *pl, const double *d_f, double *d_u_out, tsfcde_stats *st) {
    if (pl->level >= pl->M) return TSFCDE_EDONE;
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t j = pl->level, N = pl->N;
    const int nb = nblocks(N);
    if (!d_f) {
        if (int rc = callback_source(pl, j, &d_f)) return rc;
    }
    double *x = pl->U + (size_t)(j + 1) * (size_t)N;
    HIPCHK(ensure_symbols(pl, j));
    // history sum and right-hand side g = B u^j - H + f
    if (j >= 1) {
        const int64_t b = 1 + HB * ((j - 1) / HB);
        if (b > 1 && pl->qblock != b) {
            HbLast cl{};
            const int nl = (int)std::min<int64_t>(HB, pl->M - b);
            for (int q = 0; q < nl; ++q) cl.c[q] = pl->clast[b + q];
            hipLaunchKernelGGL(k_hist_sweep, dim3(nb), dim3(RB), 0, pl->stream, (const double *)pl->U, N, (int)b, nl,
                               (const double *)pl->d_cbase, cl, pl->Q);
            HIPCHK(hipGetLastError());
            pl->qblock = b;
        }
        hipLaunchKernelGGL(k_hist_catch, dim3(nb), dim3(RB), 0, pl->stream, (const double *)pl->U, N, (int)j, (int)b,
                           (const double *)pl->d_cbase, pl->clast[j], pl->kappa,
                           (const double *)(b > 1 ? pl->Q + (size_t)(j - b) * (size_t)N : nullptr), pl->H);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(product(pl, j, pl->U + (size_t)j * (size_t)N, pl->t, pl->eta[j], 1.0 - pl->sigma, 0, Fin::Y));
    hipLaunchKernelGGL(k_rhs, dim3(nb), dim3(RB), 0, pl->stream, (const double *)pl->t,
                       (const double *)(j >= 1 ? pl->H : nullptr), d_f, pl->g, pl->r, pl->rt, N, pl->partv);
    hipLaunchKernelGGL(k_fin_rhs, dim3(1), dim3(RB), 0, pl->stream, (const double *)pl->partv, nb, pl->sc, pl->rtol);
    // initial guess: zero, or u^j / the quadratic extrapolation, which goes
    // through the acceptance check at once (the CGS passes are predicated off
    // when it is accepted; otherwise CGS starts from it with r = g - A x0)
    const int mode = pl->warm == TSFCDE_WS_PREV ? 1 : pl->warm == TSFCDE_WS_EXTRAP ? (j >= 2 ? 2 : (j >= 1 ? 1 : 0)) : 0;
    const int guess = mode == 2 ? TSFCDE_WS_EXTRAP : (mode == 1 ? TSFCDE_WS_PREV : TSFCDE_WS_ZERO);
    if (mode > 0) {
        hipLaunchKernelGGL(k_guess, dim3(nb), dim3(RB), 0, pl->stream, (const double *)pl->U, N, (int)j, mode, x);
        HIPCHK(hipGetLastError());
        HIPCHK(product(pl, j, x, pl->t, pl->eta[j], -pl->sigma, 0, Fin::Y));
        hipLaunchKernelGGL(k_true, dim3(nb), dim3(RB), 0, pl->stream, (const double *)pl->g, (const double *)pl->t,
                           (const double *)x, pl->r, pl->rt, N, pl->partv);
        hipLaunchKernelGGL(k_fin_true, dim3(1), dim3(RB), 0, pl->stream, (const double *)pl->partv, nb, pl->sc,
                           pl->anorm[j], BW_TOL, 0);
    } else {
        hipLaunchKernelGGL(k_fill, dim3(nb), dim3(RB), 0, pl->stream, x, N, 0.0);
    }
    HIPCHK(hipGetLastError());
    // CGS in chunks between polls; a stopped solve is checked on its true
    // residual and backward error and restarted from x when it fails
    int restarts = 0, chunk = std::max(2, pl->last_iters), code = TSFCDE_OK;
    int k = 0, seg = 0;  // iterations issued; the current segment's first
    bool accepted = false, checked = false;
    for (;;) {
        const int todo = std::min(chunk, pl->maxit - k);
        for (int m = 0; m < todo; ++m, ++k) HIPCHK(cgs_iteration(pl, j, x, k, k == seg));
        if (todo > 0) {
            hipLaunchKernelGGL(k_fold_rho, dim3(1), dim3(RB), 0, pl->stream, pl->fold2, pl->nfold2, pl->sc, k);
            HIPCHK(hipGetLastError());
        }
        if (int rc = poll(pl)) return rc;
        const Sc &h = *pl->h_sc;
        if (!h.done) {
            if (k >= pl->maxit || todo <= 0) {
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
        // the check: r = g - A x and the acceptance test; a restart begins
        // at the iteration where CGS stopped
        k = h.iter;
        HIPCHK(product(pl, j, x, pl->t, pl->eta[j], -pl->sigma, 0, Fin::Y));
        hipLaunchKernelGGL(k_true, dim3(nb), dim3(RB), 0, pl->stream, (const double *)pl->g, (const double *)pl->t,
                           (const double *)x, pl->r, pl->rt, N, pl->partv);
        hipLaunchKernelGGL(k_fin_true, dim3(1), dim3(RB), 0, pl->stream, (const double *)pl->partv, nb, pl->sc,
                           pl->anorm[j], BW_TOL, k);
        HIPCHK(hipGetLastError());
        if (int rc = poll(pl)) return rc;
        checked = true;
        if (pl->h_sc->done) {
            code = status_code(pl->h_sc->status);
            accepted = code == TSFCDE_OK;
            break;
        }
        if (restarts >= MAX_RESTARTS || k >= pl->maxit) break;
        ++restarts;
        seg = k;
        chunk = std::max(2, pl->last_iters / 2);
    }
    const Sc &h = *pl->h_sc;
    const int iters = h.done ? h.iter : k;
    if (code == TSFCDE_OK && !accepted) code = checked ? TSFCDE_EACCEPT : TSFCDE_ENOCONV;
    pl->last_iters = std::max(1, iters / (restarts + 1));
    if (d_u_out) HIPCHK(hipMemcpyAsync(d_u_out, x, sizeof(double) * (size_t)N, hipMemcpyDeviceToDevice, pl->stream));
    HIPCHK(hipStreamSynchronize(pl->stream));
    if (st) {
        st->iters = iters;
        st->outer_iters = 1;
        st->restarts = restarts;
        st->status = code;
        st->relres = h.gnorm2 > 0 ? std::sqrt(h.rnorm2 / h.gnorm2) : 0.0;
        st->relres_true = checked ? (h.gnorm2 > 0 ? std::sqrt(h.aux0 / h.gnorm2) : 0.0) : -1.0;
        const double den = pl->anorm[j] * std::sqrt(h.aux1) + std::sqrt(h.gnorm2);
        st->backward_err = checked ? (den > 0 ? std::sqrt(h.aux0) / den : 0.0) : -1.0;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        st->precision_used = TSFCDE_FP64;
        st->guess = guess;
        st->method = 0;
        st->pad = 0;
    }
    pl->level = j + 1;
    return code;
}

// Problem data common to both dimensions, gathered by the entry points.
struct NdProblem {
    int d;
    double alpha, beta[3], lo[3], hi[3], T, rtol;
    int64_t n[3], M;
    tsfcde_coef_fn gam[3], dp[3], dm[3];
    void *coef_user;
    int maxit, warm;
};

int validate(const NdProblem &p) {
    if (!(p.alpha > 0.0 && p.alpha <= 1.0)) return TSFCDE_EINVAL;
    if (!(p.T > 0.0) || !std::isfinite(p.T) || p.M < 1) return TSFCDE_EINVAL;
    if (p.warm != TSFCDE_WS_ZERO && p.warm != TSFCDE_WS_PREV && p.warm != TSFCDE_WS_EXTRAP) return TSFCDE_EINVAL;
    for (int a = 0; a < p.d; ++a) {
        if (!(p.beta[a] > 1.0 && p.beta[a] <= 2.0)) return TSFCDE_EINVAL;
        if (!(p.hi[a] > p.lo[a]) || !std::isfinite(p.lo[a]) || !std::isfinite(p.hi[a])) return TSFCDE_EINVAL;
        if (!p.gam[a] || !p.dp[a] || !p.dm[a]) return TSFCDE_EINVAL;
        if (p.n[a] < 1) return TSFCDE_EINVAL;
    }
    for (int a = 0; a < p.d; ++a)
        if (!pow2_in(p.n[a], 16, 2048)) return TSFCDE_EUNSUPPORTED;
    if (p.M > (int64_t(1) << 20)) return TSFCDE_EUNSUPPORTED;
    int64_t N = 1;
    for (int a = 0; a < p.d; ++a) N *= p.n[a];
    if (N > (int64_t(1) << 30)) return TSFCDE_EUNSUPPORTED;
    return TSFCDE_OK;
}

NdProblem from2(const tsfcde2d_problem *p) {
    NdProblem q{};
    q.d = 2;
    q.alpha = p->alpha;
    q.beta[0] = p->beta_x;
    q.beta[1] = p->beta_y;
    q.lo[0] = p->a;
    q.hi[0] = p->b;
    q.lo[1] = p->c;
    q.hi[1] = p->d;
    q.T = p->T;
    q.n[0] = p->nx;
    q.n[1] = p->ny;
    q.M = p->M;
    q.gam[0] = p->gamma_x;
    q.gam[1] = p->gamma_y;
    q.dp[0] = p->dplus_x;
    q.dp[1] = p->dplus_y;
    q.dm[0] = p->dminus_x;
    q.dm[1] = p->dminus_y;
    q.coef_user = p->coef_user;
    q.rtol = p->rtol;
    q.maxit = p->maxit;
    q.warm = p->warm_start;
    return q;
}

NdProblem from3(const tsfcde3d_problem *p) {
    NdProblem q{};
    q.d = 3;
    q.alpha = p->alpha;
    for (int a = 0; a < 3; ++a) {
        q.beta[a] = p->beta[a];
        q.lo[a] = p->lo[a];
        q.hi[a] = p->hi[a];
        q.n[a] = p->n[a];
        q.gam[a] = p->gamma[a];
        q.dp[a] = p->dplus[a];
        q.dm[a] = p->dminus[a];
    }
    q.T = p->T;
    q.M = p->M;
    q.coef_user = p->coef_user;
    q.rtol = p->rtol;
    q.maxit = p->maxit;
    q.warm = p->warm_start;
    return q;
}

template <class PlanT>
int plan_create(const NdProblem &prob, void *d_workspace, size_t bytes, void *stream, PlanT **out,
                const std::vector<double> *u0) {
    *out = nullptr;
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255)) return TSFCDE_EINVAL;
    const int d = prob.d;
    const Layout L = layout(prob.n, d, prob.M);
    if (bytes < L.total) return TSFCDE_ENOMEM;
    PlanT *pl = new (std::nothrow) PlanT();
    if (!pl) return TSFCDE_ENOMEM;
    auto fail = [&](int code) {
        if (pl->h_sc) (void)hipHostFree(pl->h_sc);
        if (pl->h_f) (void)hipHostFree(pl->h_f);
        delete pl;
        return code;
    };
    pl->d = d;
    pl->stream = reinterpret_cast<hipStream_t>(stream);
    pl->N = 1;
    for (int a = 0; a < d; ++a) {
        pl->n[a] = prob.n[a];
        pl->N *= prob.n[a];
        pl->beta[a] = prob.beta[a];
        pl->lo[a] = prob.lo[a];
        pl->h[a] = (prob.hi[a] - prob.lo[a]) / (double)(prob.n[a] + 1);
        pl->hb[a] = std::pow(pl->h[a], -prob.beta[a]);
    }
    const int64_t M = prob.M, N = pl->N;
    pl->W = pl->n[d - 1] / 2 + 1;
    pl->Nh = N / pl->n[d - 1] * pl->W;
    pl->M = M;
    pl->alpha = prob.alpha;
    pl->T = prob.T;
    pl->tau = prob.T / (double)M;
    pl->sigma = 1.0 - prob.alpha / 2.0;
    pl->kappa = std::pow(pl->tau, -prob.alpha) / std::tgamma(2.0 - prob.alpha);
    pl->rtol = prob.rtol > 0 ? prob.rtol : 1e-10;
    pl->maxit = prob.maxit > 0 ? prob.maxit : 500;
    pl->warm = prob.warm;
    // coefficients at t_{j+sigma}
    for (int a = 0; a < d; ++a) {
        pl->gam[a].resize(M);
        pl->dp[a].resize(M);
        pl->dm[a].resize(M);
    }
    for (int64_t j = 0; j < M; ++j) {
        const double t = level_time(pl, j);
        for (int a = 0; a < d; ++a) {
            const double g = prob.gam[a](t, prob.coef_user), p = prob.dp[a](t, prob.coef_user),
                         m = prob.dm[a](t, prob.coef_user);
            if (!std::isfinite(g) || !std::isfinite(p) || !std::isfinite(m) || p < 0 || m < 0)
                return fail(TSFCDE_EINVAL);
            pl->gam[a][j] = g;
            pl->dp[a][j] = p;
            pl->dm[a][j] = m;
        }
    }
    // L2-1sigma tables (Lemma 1): eta_j = kappa c_0^(j), c_m = a_m + b_{m+1} - b_m
    // (1 <= m < j), c_j = a_j - b_j
    {
        const double al = prob.alpha, sg = pl->sigma;
        std::vector<double> av(M + 2), bv(M + 2, 0.0);
        av[0] = std::pow(sg, 1.0 - al);
        for (int64_t l = 1; l <= M + 1; ++l) {
            av[l] = std::pow(l + sg, 1.0 - al) - std::pow(l - 1 + sg, 1.0 - al);
            bv[l] = (std::pow(l + sg, 2.0 - al) - std::pow(l - 1 + sg, 2.0 - al)) / (2.0 - al) -
                    0.5 * (std::pow(l + sg, 1.0 - al) + std::pow(l - 1 + sg, 1.0 - al));
        }
        pl->eta.resize(M);
        pl->cbase.assign(M + 2 + HB, 0.0);  // zeros past M for the sweep's last block
        pl->clast.assign(M + 1, 0.0);
        for (int64_t j = 0; j < M; ++j) pl->eta[j] = pl->kappa * (j == 0 ? av[0] : av[0] + bv[1]);
        for (int64_t m = 1; m <= M; ++m) pl->cbase[m] = av[m] + bv[m + 1] - bv[m];
        for (int64_t j = 1; j <= M; ++j) pl->clast[j] = av[j] - bv[j];
    }
    // weights, embedding and Strang columns of every axis; |A| bound
    std::vector<double> cols((size_t)spec_len(pl->n, d), 0.0);
    double wsum[3] = {};
    {
        size_t off = 0;
        for (int a = 0; a < d; ++a) {
            const int64_t n = pl->n[a];
            const std::vector<double> w = wsgd(prob.beta[a], n + 1);
            for (double v : w) wsum[a] += std::fabs(v);
            // embedding column of W (length 2n): c_m = omega_{m+1} (m < n), c_{2n-1} = omega_0;
            // Strang column (length n): c_k = omega_{k+1} (k <= n/2), c_{n-1} = omega_0, else 0
            double *e = cols.data() + off, *s = e + 2 * n;
            for (int64_t m = 0; m < n; ++m) e[m] = w[m + 1];
            e[2 * n - 1] = w[0];
            for (int64_t k = 0; k <= n / 2; ++k) s[k] = w[k + 1];
            s[n - 1] = w[0];
            off += 3 * n;
        }
    }
    pl->anorm.resize(M);
    for (int64_t j = 0; j < M; ++j) {
        double tot = 0.0;
        for (int a = 0; a < d; ++a)
            tot += std::fabs(pl->gam[a][j]) / pl->h[a] + (pl->dp[a][j] + pl->dm[a][j]) * pl->hb[a] * wsum[a];
        pl->anorm[j] = pl->eta[j] + pl->sigma * tot;
    }
    // device buffers
    char *ws = reinterpret_cast<char *>(d_workspace);
    pl->U = reinterpret_cast<double *>(ws + L.U);
    double *vec = reinterpret_cast<double *>(ws + L.vec);
    double **bufs[NVEC] = {&pl->g, &pl->r, &pl->rt, &pl->u, &pl->p, &pl->q, &pl->phat,
                           &pl->uhat, &pl->vhat, &pl->t, &pl->w, &pl->H, &pl->fbuf};
    for (int k = 0; k < NVEC; ++k) *bufs[k] = vec + (size_t)k * (size_t)N;
    pl->Z = reinterpret_cast<double2 *>(ws + L.Z);
    {
        double2 *sp = reinterpret_cast<double2 *>(ws + L.lam), *sy = reinterpret_cast<double2 *>(ws + L.sym);
        for (int a = 0; a < d; ++a) {
            pl->lam[a] = sp;
            pl->ls[a] = sp + 2 * pl->n[a];
            pl->symE[a] = sy;
            pl->symS[a] = sy + 2 * pl->n[a];
            sp += 3 * pl->n[a];
            sy += 3 * pl->n[a];
        }
    }
    pl->tw = reinterpret_cast<double2 *>(ws + L.tw);
    pl->part1 = reinterpret_cast<double *>(ws + L.part);
    pl->part2 = pl->part1 + 2 * part_len(N);
    pl->partv = pl->part2 + 2 * part_len(N);
    pl->sq = pl->partv + 2 * RBLK;
    pl->sc = reinterpret_cast<Sc *>(ws + L.sc);
    pl->d_cbase = reinterpret_cast<double *>(ws + L.cb);
    pl->Q = reinterpret_cast<double *>(ws + L.Q);
    pl->cols = reinterpret_cast<double *>(ws + L.cols);
    if (hipHostMalloc(reinterpret_cast<void **>(&pl->h_sc), sizeof(Sc)) != hipSuccess) {
        pl->h_sc = nullptr;
        return fail(TSFCDE_EDEVICE);
    }
    std::memset(pl->h_sc, 0, sizeof(Sc));
    bool ok = hipMemcpyAsync(pl->d_cbase, pl->cbase.data(), sizeof(double) * (size_t)(M + 2 + HB), hipMemcpyHostToDevice,
                             pl->stream) == hipSuccess &&
              hipMemcpyAsync(pl->cols, cols.data(), sizeof(double) * cols.size(), hipMemcpyHostToDevice, pl->stream) ==
                  hipSuccess &&
              hipMemcpyAsync(pl->sc, pl->h_sc, sizeof(Sc), hipMemcpyHostToDevice, pl->stream) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(k_twiddles, dim3(16), dim3(256), 0, pl->stream, pl->tw, PMAX_LOG2);
        ok = hipGetLastError() == hipSuccess;
    }
    // spectra: DFT of the embedding columns (2n points) and Strang columns (n points)
    {
        size_t off = 0;
        for (int a = 0; a < d && ok; ++a) {
            const int64_t n = pl->n[a];
            const double *e = pl->cols + off, *s = e + 2 * n;
            SpecOp o1{e, pl->lam[a], 2 * n, nullptr, 0};
            SpecOp o2{s, pl->ls[a], n, nullptr, 0};
            ok = line<true>(pl, 2 * n, o1, 1) == hipSuccess && line<true>(pl, n, o2, 1) == hipSuccess;
            off += 3 * n;
        }
    }
    // u^0 = phi at the nodes (or 0)
    if (ok) {
        if (u0) {
            ok = hipMemcpyAsync(pl->U, u0->data(), sizeof(double) * (size_t)N, hipMemcpyHostToDevice, pl->stream) ==
                 hipSuccess;
        } else {
            hipLaunchKernelGGL(k_fill, dim3(nblocks(N)), dim3(RB), 0, pl->stream, pl->U, N, 0.0);
            ok = hipGetLastError() == hipSuccess;
        }
    }
    if (ok) ok = hipStreamSynchronize(pl->stream) == hipSuccess;
    if (!ok) return fail(TSFCDE_EDEVICE);
    *out = pl;
    return TSFCDE_OK;
}

int set_state(NdPlan *pl, int64_t level, const double *d_U) {
    if (!pl || !d_U || level < 0 || level >= pl->M) return TSFCDE_EINVAL;
    HIPCHK(hipMemcpyAsync(pl->U, d_U, sizeof(double) * (size_t)((level + 1) * pl->N), hipMemcpyDeviceToDevice,
                          pl->stream));
    HIPCHK(hipStreamSynchronize(pl->stream));
    pl->level = level;
    pl->qblock = 0;  // the history block sums are rebuilt from the new levels
    return TSFCDE_OK;
}

int solve_all(NdPlan *pl, const double *d_F, int64_t ldF, double *d_U_out, tsfcde_stats *stats) {
    if (!pl) return TSFCDE_EINVAL;
    if (d_F && ldF < pl->N) return TSFCDE_EINVAL;
    if (pl->level >= pl->M) return TSFCDE_EDONE;
    int first = TSFCDE_OK;
    const int64_t j0 = pl->level;
    while (pl->level < pl->M) {
        const int64_t j = pl->level;
        const int rc = level_step(pl, d_F ? d_F + (size_t)j * (size_t)ldF : nullptr, nullptr,
                                  stats ? stats + (j - j0) : nullptr);
        if (rc == TSFCDE_EDEVICE) return rc;
        if (rc && !first) first = rc;
    }
    if (d_U_out) {
        HIPCHK(hipMemcpyAsync(d_U_out, pl->U, sizeof(double) * (size_t)((pl->M + 1) * pl->N), hipMemcpyDeviceToDevice,
                              pl->stream));
        HIPCHK(hipStreamSynchronize(pl->stream));
    }
    return first;
}

int apply_op(NdPlan *pl, int32_t op, int64_t j, const double *d_x, double *d_y) {
    if (!pl || !d_x || !d_y || d_x == d_y || j < 0 || j >= pl->M) return TSFCDE_EINVAL;
    if (op != TSFCDE_OP_A && op != TSFCDE_OP_B && op != TSFCDE_OP_PINV) return TSFCDE_EINVAL;
    hipError_t e = ensure_symbols(pl, j);
    if (e != hipSuccess) return TSFCDE_EDEVICE;
    if (op == TSFCDE_OP_A) {
        e = product(pl, j, d_x, d_y, pl->eta[j], -pl->sigma, 0, Fin::Y);
    } else if (op == TSFCDE_OP_B) {
        e = product(pl, j, d_x, d_y, pl->eta[j], 1.0 - pl->sigma, 0, Fin::Y);
    } else if (op == TSFCDE_OP_PINV) {
        e = psolve(pl, j, d_x, d_y, 0);
    } else {
        return TSFCDE_EINVAL;
    }
    return e == hipSuccess ? TSFCDE_OK : TSFCDE_EDEVICE;
}

int destroy(NdPlan *pl) {
    if (!pl) return TSFCDE_EINVAL;
    (void)hipStreamSynchronize(pl->stream);
    if (pl->h_sc) (void)hipHostFree(pl->h_sc);
    if (pl->h_f) (void)hipHostFree(pl->h_f);
    return TSFCDE_OK;
}

}  // namespace

extern "C" {

// ---- two dimensions ---------------------------------------------------------

int tsfcde2d_workspace_bytes(const tsfcde2d_problem *prob, size_t *bytes) {
    if (!bytes || !prob) return TSFCDE_EINVAL;
    const NdProblem p = from2(prob);
    if (int rc = validate(p)) return rc;
    *bytes = layout(p.n, 2, p.M).total;
    return TSFCDE_OK;
}

int tsfcde2d_plan(const tsfcde2d_problem *prob, void *d_workspace, size_t bytes, void *stream, tsfcde2d_plan_t *out) {
    if (!out) return TSFCDE_EINVAL;
    *out = nullptr;
    if (!prob) return TSFCDE_EINVAL;
    const NdProblem p = from2(prob);
    if (int rc = validate(p)) return rc;
    std::vector<double> u0;
    if (prob->phi) {
        u0.resize((size_t)(p.n[0] * p.n[1]));
        const double hx = (p.hi[0] - p.lo[0]) / (double)(p.n[0] + 1), hy = (p.hi[1] - p.lo[1]) / (double)(p.n[1] + 1);
        for (int64_t i = 0; i < p.n[0]; ++i)
            for (int64_t k = 0; k < p.n[1]; ++k)
                u0[(size_t)(i * p.n[1] + k)] =
                    prob->phi(p.lo[0] + (double)(i + 1) * hx, p.lo[1] + (double)(k + 1) * hy, prob->phi_user);
    }
    tsfcde2d_plan_s *pl = nullptr;
    const int rc = plan_create(p, d_workspace, bytes, stream, &pl, prob->phi ? &u0 : nullptr);
    if (rc) return rc;
    pl->f2 = prob->f;
    pl->fuser = prob->f_user;
    *out = pl;
    return TSFCDE_OK;
}

int tsfcde2d_set_state(tsfcde2d_plan_t pl, int64_t level, const double *d_U) { return set_state(pl, level, d_U); }

int tsfcde2d_step(tsfcde2d_plan_t pl, const double *d_f, double *d_u_out, tsfcde_stats *stats) {
    if (!pl) return TSFCDE_EINVAL;
    return level_step(pl, d_f, d_u_out, stats);
}

int tsfcde2d_solve(tsfcde2d_plan_t pl, const double *d_F, int64_t ldF, double *d_U_out, tsfcde_stats *stats) {
    return solve_all(pl, d_F, ldF, d_U_out, stats);
}

int tsfcde2d_apply(tsfcde2d_plan_t pl, int32_t op, int64_t j, const double *d_x, double *d_y) {
    return apply_op(pl, op, j, d_x, d_y);
}

int tsfcde2d_nodes(tsfcde2d_plan_t pl, double *h_x, double *h_y) {
    if (!pl) return TSFCDE_EINVAL;
    double *outs[2] = {h_x, h_y};
    for (int a = 0; a < 2; ++a)
        if (outs[a])
            for (int64_t i = 0; i < pl->n[a]; ++i) node_coords(pl, a, i, outs[a] + i);
    return TSFCDE_OK;
}

double tsfcde2d_level_time(tsfcde2d_plan_t pl, int64_t j) {
    if (!pl || j < 0 || j >= pl->M) return std::nan("");
    return level_time(pl, j);
}

int64_t tsfcde2d_level(tsfcde2d_plan_t pl) { return pl ? pl->level : -1; }

const double *tsfcde2d_history(tsfcde2d_plan_t pl) { return pl ? pl->U : nullptr; }

int tsfcde2d_destroy(tsfcde2d_plan_t pl) {
    const int rc = destroy(pl);
    if (rc == TSFCDE_OK) delete pl;
    return rc;
}

// ---- three dimensions -------------------------------------------------------

int tsfcde3d_workspace_bytes(const tsfcde3d_problem *prob, size_t *bytes) {
    if (!bytes || !prob) return TSFCDE_EINVAL;
    const NdProblem p = from3(prob);
    if (int rc = validate(p)) return rc;
    *bytes = layout(p.n, 3, p.M).total;
    return TSFCDE_OK;
}

int tsfcde3d_plan(const tsfcde3d_problem *prob, void *d_workspace, size_t bytes, void *stream, tsfcde3d_plan_t *out) {
    if (!out) return TSFCDE_EINVAL;
    *out = nullptr;
    if (!prob) return TSFCDE_EINVAL;
    const NdProblem p = from3(prob);
    if (int rc = validate(p)) return rc;
    std::vector<double> u0;
    if (prob->phi) {
        u0.resize((size_t)(p.n[0] * p.n[1] * p.n[2]));
        double h[3];
        for (int a = 0; a < 3; ++a) h[a] = (p.hi[a] - p.lo[a]) / (double)(p.n[a] + 1);
        for (int64_t i = 0; i < p.n[0]; ++i)
            for (int64_t k = 0; k < p.n[1]; ++k)
                for (int64_t l = 0; l < p.n[2]; ++l)
                    u0[(size_t)((i * p.n[1] + k) * p.n[2] + l)] =
                        prob->phi(p.lo[0] + (double)(i + 1) * h[0], p.lo[1] + (double)(k + 1) * h[1],
                                  p.lo[2] + (double)(l + 1) * h[2], prob->phi_user);
    }
    tsfcde3d_plan_s *pl = nullptr;
    const int rc = plan_create(p, d_workspace, bytes, stream, &pl, prob->phi ? &u0 : nullptr);
    if (rc) return rc;
    pl->f3 = prob->f;
    pl->fuser = prob->f_user;
    *out = pl;
    return TSFCDE_OK;
}

int tsfcde3d_set_state(tsfcde3d_plan_t pl, int64_t level, const double *d_U) { return set_state(pl, level, d_U); }

int tsfcde3d_step(tsfcde3d_plan_t pl, const double *d_f, double *d_u_out, tsfcde_stats *stats) {
    if (!pl) return TSFCDE_EINVAL;
    return level_step(pl, d_f, d_u_out, stats);
}

int tsfcde3d_solve(tsfcde3d_plan_t pl, const double *d_F, int64_t ldF, double *d_U_out, tsfcde_stats *stats) {
    return solve_all(pl, d_F, ldF, d_U_out, stats);
}

int tsfcde3d_apply(tsfcde3d_plan_t pl, int32_t op, int64_t j, const double *d_x, double *d_y) {
    return apply_op(pl, op, j, d_x, d_y);
}

int tsfcde3d_nodes(tsfcde3d_plan_t pl, double *h_x, double *h_y, double *h_z) {
    if (!pl) return TSFCDE_EINVAL;
    double *outs[3] = {h_x, h_y, h_z};
    for (int a = 0; a < 3; ++a)
        if (outs[a])
            for (int64_t i = 0; i < pl->n[a]; ++i) node_coords(pl, a, i, outs[a] + i);
    return TSFCDE_OK;
}

double tsfcde3d_level_time(tsfcde3d_plan_t pl, int64_t j) {
    if (!pl || j < 0 || j >= pl->M) return std::nan("");
    return level_time(pl, j);
}

int64_t tsfcde3d_level(tsfcde3d_plan_t pl) { return pl ? pl->level : -1; }

const double *tsfcde3d_history(tsfcde3d_plan_t pl) { return pl ? pl->U : nullptr; }

int tsfcde3d_destroy(tsfcde3d_plan_t pl) {
    const int rc = destroy(pl);
    if (rc == TSFCDE_OK) delete pl;
    return rc;
}

}  // extern "C"
