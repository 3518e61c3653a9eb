// kernels.hpp -- gfx950 kernels of the TSFCDE time-level solver.
//
// Real transforms of length L = 2N run as complex transforms of length
// N = R x C (R rows, C columns, row-major, N complex values) in three passes:
//   pass A (k_col, forward): length-R FFTs down the columns of the packed
//     input z[m] = x[2m] + i x[2m+1], times the four-step twiddle
//     W_N^(col*row); a workgroup owns B adjacent columns so every row
//     segment it reads/writes is B*16 contiguous bytes.
//   middle (k_mid): per pair of rows (k1, R-k1) -- the rows that hold
//     frequencies k and N-k -- forward length-C FFTs, the real-to-complex
//     untangle, the per-level symbol multiply (Toeplitz matvec through the
//     circulant embedding) or divide (Strang preconditioner solve), the
//     complex-to-real retangle, and inverse length-C FFTs.  The spectrum is
//     never written out in natural order: position k1*C + k2 holds frequency
//     k1 + R*k2, and the stored symbol tables use the same layout.
//   pass C (k_col, inverse): conjugate twiddle, inverse length-R FFTs down the
//     columns, unpack to real.
// Vector updates of the Krylov iteration are fused into pass A (prologue) and
// pass C (epilogue); dot products are reduced per workgroup and finished, in
// a fixed order (deterministic results), by a one-workgroup kernel or inside
// the pass that follows (see InCgsUPT::fold).
#pragma once
#include "fft_core.hpp"

namespace tsf {

// ---------------------------------------------------------------------------
// Device scalars of the CGS iteration (one struct per plan).
// ---------------------------------------------------------------------------
struct DevScalars {
    double rho, rho_prev, alpha, beta, rtv, rnorm2, gnorm2, tol2;
    double aux0, aux1, rtol2, r0sq;  // r0sq: |g - A x0|^2 of the right-hand side's initial guess
    int iter, done, status, fresh;  // fresh: next CGS iteration starts from r (u = p = r)
    int better;   // the last restart's |g - A x|^2 was below r0sq
    int netkept;  // the learned guess was kept at this level (set by k_keep_better)
    // rho of the iterations of a chunk whose finishing steps are folded into
    // the next pass (see InCgsUPT::fold): rho_i sits in rho2[i & 1] for i >= 1
    // (rho_0 in rho), so a pass never reads the slot it writes
    double rho2[2];
    // residual checks: `checked` says the current done state was confirmed by
    // a restart pass (cleared by the right-hand side); nchecks counts the
    // acceptance checks of the level, prestat keeps the status CGS stopped with
    int checked, nchecks, prestat;
    double omega;  // BiCGSTAB's omega of the last iteration
};

enum : int { ST_OK = 0, ST_BREAKDOWN = 1, ST_NONFINITE = 2 };

// Predication of a launch on the device scalars: pred 0 always runs, pred 1
// skips once the solve is done, pred 2 skips when the last restart found its
// guess better than the right-hand side's (a second restart is then moot),
// pred 3 runs only when the solve is done and no residual check has
// confirmed that yet (an acceptance check queued behind a chunk of CGS).
// Kernels test it before their first load: a skipped workgroup (a converged
// level, or a converged instance of a batch) then costs almost nothing.
__device__ __forceinline__ bool skip(int pred, const DevScalars *sc) {
    return (pred == 1 && sc->done) || (pred == 2 && sc->better) || (pred == 3 && !(sc->done && !sc->checked));
}

// Loaders that can fold the previous pass's finishing step (see InCgsUPT).
template <class T, class = void> struct HasFold {
    static constexpr bool value = false;
};
template <class T> struct HasFold<T, decltype(void(static_cast<T *>(nullptr)->fold(static_cast<DevScalars *>(nullptr))))> {
    static constexpr bool value = true;
};

// Symbol of one level: S(k) = s0 + cre*Re(L_k) + i*(cim*Im(L_k) + cq*sin(2 pi k / L)),
// where L_k is the stored spectrum of W_beta (embedding or Strang).  For a
// product (MODE 0) y = S * x * scale; for a solve (MODE 1) y = x / (S * scale).
struct SymParams {
    double s0, cre, cim, cq, scale;
};

// ---------------------------------------------------------------------------
// Reductions in two launches: each workgroup of a pass sums its lanes (wave64
// shuffles, then LDS across waves) and stores one partial per accumulator
// (indexed by the tile it covers);
// a one-workgroup finishing kernel then sums the partials in index order.
// The kernel boundary makes the partials visible, so no device-scope fence
// (which on gfx950 writes back and invalidates the XCD's L2) is needed.  The
// summation order is fixed by the pass geometry and a 256-wide layout of the
// final sum, so results are reproducible.
// ---------------------------------------------------------------------------
template <int NACC>
__device__ __forceinline__ void block_partial(double (&acc)[NACC], double *partials, int64_t slot) {
    __shared__ double red[NACC][16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwave = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int a = 0; a < NACC; ++a) {
        double v = acc[a];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[a][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int a = 0; a < NACC; ++a) {
            double s = 0.0;
            for (int w = 0; w < nwave; ++w) s += red[a][w];
            partials[(size_t)slot * NACC + a] = s;
        }
    }
}

// Sum of nparts partials; every thread gets the same totals.  The order is
// fixed by a 256-wide layout whatever the workgroup size (at least 256
// threads): thread t < 256 adds partials t, t + 256, ... in turn, then the
// 64-lane trees of waves 0..3 and their four sums.  A finishing kernel and a
// pass of another thread count that folds the same step therefore agree bit
// for bit.
constexpr int RED_WIDTH = 256;
template <int NACC>
__device__ __forceinline__ void reduce_partials(const double *partials, int nparts, double (&tot)[NACC]) {
    __shared__ double red[NACC][RED_WIDTH / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double loc[NACC];
#pragma unroll
    for (int a = 0; a < NACC; ++a) loc[a] = 0.0;
    if (threadIdx.x < RED_WIDTH) {
        for (int i = threadIdx.x; i < nparts; i += RED_WIDTH) {
#pragma unroll
            for (int a = 0; a < NACC; ++a) loc[a] += partials[(size_t)i * NACC + a];
        }
    }
#pragma unroll
    for (int a = 0; a < NACC; ++a) {
        double v = loc[a];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0 && wave < RED_WIDTH / 64) red[a][wave] = v;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < NACC; ++a) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < RED_WIDTH / 64; ++w) s += red[a][w];
        tot[a] = s;
    }
}

__device__ __forceinline__ bool finite(double x) { return isfinite(x); }

// Workgroups are dispatched to the chip's eight XCDs round-robin by index, and
// each XCD has its own L2.  Column tiles narrower than a 128-byte line share
// lines with their neighbours; this permutation gives each XCD a contiguous
// run of tiles so that neighbours meet in the same L2 (identity when the
// grid is not a multiple of eight).
constexpr int XCDS = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t grid) {
    if (grid % XCDS) return bid;
    return (bid % XCDS) * (grid / XCDS) + bid / XCDS;
}

// Element pair (i, i+1) of a real vector of nr values (i even).  Vectors of odd
// length end with a lone element: the pair loads it with a zero partner, and
// a store writes only the element that exists.
__device__ __forceinline__ double2 ld2(const double *p, int64_t i, int64_t nr) {
    if (i + 1 < nr) return *reinterpret_cast<const double2 *>(p + i);
    return make_double2(i < nr ? p[i] : 0.0, 0.0);
}
__device__ __forceinline__ void st2(double *p, int64_t i, int64_t nr, double2 v) {
    if (i + 1 < nr) *reinterpret_cast<double2 *>(p + i) = v;
    else if (i < nr) p[i] = v.x;
}

// The same for vectors stored in FP32 (values are widened on load and rounded
// to nearest on store; all arithmetic stays in FP64 registers).
__device__ __forceinline__ double2 ld2(const float *p, int64_t i, int64_t nr) {
    if (i + 1 < nr) {
        const float2 v = *reinterpret_cast<const float2 *>(p + i);
        return make_double2(v.x, v.y);
    }
    return make_double2(i < nr ? (double)p[i] : 0.0, 0.0);
}
__device__ __forceinline__ void st2(float *p, int64_t i, int64_t nr, double2 v) {
    if (i + 1 < nr) *reinterpret_cast<float2 *>(p + i) = make_float2((float)v.x, (float)v.y);
    else if (i < nr) p[i] = (float)v.x;
}

// Complex buffer element m stored in FP64 or FP32.
__device__ __forceinline__ double2 ldc(const double2 *p, int64_t m) { return p[m]; }
__device__ __forceinline__ double2 ldc(const float2 *p, int64_t m) {
    const float2 v = p[m];
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void stc(double2 *p, int64_t m, double2 v) { p[m] = v; }
__device__ __forceinline__ void stc(float2 *p, int64_t m, double2 v) { p[m] = make_float2((float)v.x, (float)v.y); }

// ---------------------------------------------------------------------------
// Pass-A loaders (forward column pass).  They return packed element
// m = row*C + col of the real input, z[m] = x[2m] + i x[2m+1], in two phases:
// fetch(row, col, raw) only issues the NL loads of the element, and
// finish(row, col, raw) combines them, makes the loader's own stores and
// returns z[m].  A pass fetches all its elements before finishing any, so no
// load waits behind a store that might alias it.
// ---------------------------------------------------------------------------
template <class S> struct InRealT {  // plain real vector, zero beyond nr values
    const S *x;
    int64_t nr, C;
    static constexpr int NL = 1;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *raw) const {
        raw[0] = ld2(x, 2 * (row * C + col), nr);
    }
    __device__ __forceinline__ double2 finish(int, int64_t, const double2 *raw) const { return raw[0]; }
};
using InReal = InRealT<double>;

// CGS: u = r + beta q ; p = u + beta (q + beta p) (first iteration: u = p = r);
// writes u and p, transforms p.
template <class S> struct InCgsUPT {
    const S *r;
    S *u, *p;
    const S *q;
    int64_t nr, C;
    double beta;
    bool first;
    // Folded finishing step of the previous iteration's last pass (fpart set):
    // its partials (|r|^2, rt.r) summed here, in the order and with the thread
    // count of k_final, so the result is bitwise the same.  ci >= 1 is the
    // iteration's index in its chunk.
    const double *fpart = nullptr;
    int fnparts = 0, ci = 0;
    __device__ void prep(const DevScalars *sc) {
        first = fpart ? false : sc->fresh != 0;
        beta = sc->beta;
    }
    // Every thread calls; returns true (uniformly) when the solve is done.
    // Workgroup 0 stores what OutCgsRT::final stores; rho goes to a parity slot.
    __device__ bool fold(DevScalars *sc) {
        if (!fpart) return false;
        double tot[2];
        reduce_partials<2>(fpart, fnparts, tot);
        const double rho_old = ci == 1 ? sc->rho : sc->rho2[(ci - 1) & 1];
        const double b = tot[1] / rho_old;
        int status = ST_OK, done = 0;
        if (!finite(tot[0]) || !finite(tot[1])) {
            status = ST_NONFINITE;
            done = 1;
        } else if (tot[0] <= sc->tol2) {
            done = 1;
        } else if (tot[1] == 0.0) {
            status = ST_BREAKDOWN;
            done = 1;
        }
        if (threadIdx.x == 0 && blockIdx.x == 0) {
            sc->rnorm2 = tot[0];
            sc->rho_prev = rho_old;
            sc->rho2[ci & 1] = tot[1];
            sc->beta = b;
            sc->iter += 1;
            sc->fresh = 0;
            if (done) {
                sc->rho = tot[1];  // the state a poll and a restart read
                sc->done = 1;
                if (status != ST_OK) sc->status = status;
            }
        }
        beta = b;
        return done != 0;
    }
    static constexpr int NL = 3;
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *raw) const {
        int64_t i = 2 * (row * C + col);
        if (i >= nr) return;
        raw[0] = ld2(r, i, nr);
        if (!first) {
            raw[1] = ld2(q, i, nr);
            raw[2] = ld2(p, i, nr);
        }
    }
    __device__ __forceinline__ double2 finish(int row, int64_t col, const double2 *raw) const {
        int64_t i = 2 * (row * C + col);
        if (i >= nr) return make_double2(0.0, 0.0);
        double2 rv = raw[0];
        double2 uv, pv;
        if (first) {
            uv = rv;
            pv = rv;
        } else {
            double2 qv = raw[1];
            double2 po = raw[2];
            uv = make_double2(fma(beta, qv.x, rv.x), fma(beta, qv.y, rv.y));
            pv = make_double2(fma(beta, fma(beta, po.x, qv.x), uv.x), fma(beta, fma(beta, po.y, qv.y), uv.y));
        }
        st2(u, i, nr, uv);
        st2(p, i, nr, pv);
        return pv;
    }
};
using InCgsUP = InCgsUPT<double>;

// CGS: q = u - alpha vhat (written); transforms u + q.
template <class S> struct InCgsQT {
    const S *u, *vhat;
    S *q;
    int64_t nr, C;
    double alpha;
    // Folded finishing step of the iteration's rt.vhat pass (fpart set; ci is
    // the iteration's index in its chunk), as in InCgsUPT.
    const double *fpart = nullptr;
    int fnparts = 0, ci = 0;
    __device__ void prep(const DevScalars *sc) { alpha = sc->alpha; }
    __device__ bool fold(DevScalars *sc) {
        if (!fpart) return false;
        double tot[1];
        reduce_partials<1>(fpart, fnparts, tot);
        const double rho = ci == 0 ? sc->rho : sc->rho2[ci & 1];
        const double a = rho / tot[0];
        int status = ST_OK;
        if (tot[0] == 0.0) status = ST_BREAKDOWN;
        else if (!finite(a)) status = ST_NONFINITE;
        if (threadIdx.x == 0 && blockIdx.x == 0) {
            sc->rtv = tot[0];
            sc->alpha = a;
            if (status != ST_OK) {
                sc->rho = rho;
                sc->status = status;
                sc->done = 1;
            }
        }
        alpha = a;
        return status != ST_OK;
    }
    static constexpr int NL = 2;
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *raw) const {
        int64_t i = 2 * (row * C + col);
        if (i >= nr) return;
        raw[0] = ld2(u, i, nr);
        raw[1] = ld2(vhat, i, nr);
    }
    __device__ __forceinline__ double2 finish(int row, int64_t col, const double2 *raw) const {
        int64_t i = 2 * (row * C + col);
        if (i >= nr) return make_double2(0.0, 0.0);
        double2 uv = raw[0];
        double2 vv = raw[1];
        double2 qv = make_double2(fma(-alpha, vv.x, uv.x), fma(-alpha, vv.y, uv.y));
        st2(q, i, nr, qv);
        return make_double2(uv.x + qv.x, uv.y + qv.y);
    }
};
using InCgsQ = InCgsQT<double>;

// CGS: x = x + alpha uhat (written); transforms uhat.
template <class S> struct InCgsXT {
    const S *uhat;
    S *x;
    int64_t nr, C;
    double alpha;
    __device__ void prep(const DevScalars *sc) { alpha = sc->alpha; }
    static constexpr int NL = 2;
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *raw) const {
        int64_t i = 2 * (row * C + col);
        if (i >= nr) return;
        raw[0] = ld2(uhat, i, nr);
        raw[1] = ld2(x, i, nr);
    }
    __device__ __forceinline__ double2 finish(int row, int64_t col, const double2 *raw) const {
        int64_t i = 2 * (row * C + col);
        if (i >= nr) return make_double2(0.0, 0.0);
        double2 uh = raw[0];
        double2 xv = raw[1];
        st2(x, i, nr, make_double2(fma(alpha, uh.x, xv.x), fma(alpha, uh.y, xv.y)));
        return uh;
    }
};
using InCgsX = InCgsXT<double>;

// Pass-A store: spectrum buffer y[row*C + col] = val * W_N^(row*col).
template <class CS> struct OutSpecT {
    CS *y;
    Tw2 tw;  // table for exp(-2 pi i m / L), L = 2N
    int64_t C;
    static constexpr int NACC = 0, NPRE = 2;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *pre) const {
        tw.fetch(2 * (int64_t)row * col, pre);
    }
    __device__ __forceinline__ void store(int row, int64_t col, double2 val, double *, const double2 *pre) const {
        stc(y, row * C + col, cmul(val, cmul(pre[0], pre[1])));
    }
    // with the twiddle from a running product (TwRec) instead of prefetched entries
    static constexpr bool REC = true;
    __device__ __forceinline__ void store_tw(int row, int64_t col, double2 val, double2 w) const {
        stc(y, row * C + col, cmul(val, w));
    }
    __device__ void final(const double *, DevScalars *) const {}
    double *partials;
};
using OutSpec = OutSpecT<double2>;

// ---------------------------------------------------------------------------
// Pass-C loader and stores (inverse column pass).
// ---------------------------------------------------------------------------
template <class CS> struct InSpecT {
    const CS *y;
    Tw2 tw;
    int64_t C;
    static constexpr int NL = 3;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *raw) const {
        raw[0] = ldc(y, row * C + col);
        tw.fetch(2 * (int64_t)row * col, raw + 1);
    }
    __device__ __forceinline__ double2 finish(int, int64_t, const double2 *raw) const {
        return cmul(raw[0], cconj(cmul(raw[1], raw[2])));
    }
    // the value alone, its twiddle then from a running product (TwRec)
    static constexpr bool REC = true;
    __device__ __forceinline__ double2 value(int row, int64_t col) const { return ldc(y, row * C + col); }
    __device__ __forceinline__ double2 finish_tw(double2 val, double2 w) const { return cmul(val, cconj(w)); }
};
using InSpec = InSpecT<double2>;

template <class S> struct OutRealT {  // x[2m], x[2m+1] for 2m < nr
    S *x;
    int64_t nr, C;
    static constexpr int NACC = 0, NPRE = 0;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int, int64_t, double2 *) const {}
    __device__ __forceinline__ void store(int row, int64_t col, double2 val, double *, const double2 *) const {
        st2(x, 2 * (row * C + col), nr, val);
    }
    __device__ void final(const double *, DevScalars *) const {}
    double *partials;
};
using OutReal = OutRealT<double>;

// ---------------------------------------------------------------------------
// BiCGSTAB (van der Vorst 1992; the right-preconditioned form of Barrett et
// al., Templates 1994), on the same passes as CGS: per iteration
//   p = r + beta (p - omega v)  (p = r when fresh), beta = (rho/rho_prev)(alpha/omega)
//   phat = P^-1 p ; v = A phat ; alpha = rho / (rt . v)
//   s = r - alpha v ; shat = P^-1 s ; t = A shat ; omega = (t . s) / (t . t)
//   x += alpha phat + omega shat ; r = s - omega t ; rho' = rt . r
// The scalars stay on the device: each reducing pass's finishing step writes
// them, the next pass reads them.
// ---------------------------------------------------------------------------
struct InBiP {  // p (written), transformed for the preconditioner solve
    const double *r, *v;
    double *p;
    int64_t nr, C;
    double beta = 0.0, omega = 0.0;
    bool first = true;
    __device__ void prep(const DevScalars *sc) {
        first = sc->fresh != 0;
        omega = sc->omega;
        beta = first ? 0.0 : (sc->rho / sc->rho_prev) * (sc->alpha / sc->omega);
    }
    static constexpr int NL = 3;
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *raw) const {
        const int64_t i = 2 * (row * C + col);
        if (i >= nr) return;
        raw[0] = ld2(r, i, nr);
        if (!first) {
            raw[1] = ld2(p, i, nr);
            raw[2] = ld2(v, i, nr);
        }
    }
    __device__ __forceinline__ double2 finish(int row, int64_t col, const double2 *raw) const {
        const int64_t i = 2 * (row * C + col);
        if (i >= nr) return make_double2(0.0, 0.0);
        double2 pv = raw[0];
        if (!first) {
            const double2 po = raw[1], vv = raw[2];
            pv.x = fma(beta, fma(-omega, vv.x, po.x), pv.x);
            pv.y = fma(beta, fma(-omega, vv.y, po.y), pv.y);
        }
        st2(p, i, nr, pv);
        return pv;
    }
};

struct OutBiV {  // v = A phat (written); alpha = rho / (rt . v)
    double *v;
    const double *rt;
    int64_t nr, C;
    static constexpr int NACC = 1, NPRE = 1;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *pre) const {
        const int64_t i = 2 * (row * C + col);
        if (i < nr) pre[0] = ld2(rt, i, nr);
    }
    __device__ __forceinline__ void store(int row, int64_t col, double2 val, double *acc, const double2 *pre) const {
        const int64_t i = 2 * (row * C + col);
        if (i < nr) {
            if (i + 1 >= nr) val.y = 0.0;
            st2(v, i, nr, val);
            acc[0] = fma(pre[0].x, val.x, fma(pre[0].y, val.y, acc[0]));
        }
    }
    __device__ void final(const double *tot, DevScalars *sc) const {
        sc->rtv = tot[0];
        sc->alpha = sc->rho / tot[0];
        if (tot[0] == 0.0) {
            sc->status = ST_BREAKDOWN;
            sc->done = 1;
        } else if (!finite(sc->alpha)) {
            sc->status = ST_NONFINITE;
            sc->done = 1;
        }
    }
    double *partials;
};

struct InBiS {  // s = r - alpha v (written), transformed for the preconditioner solve
    const double *r, *v;
    double *s;
    int64_t nr, C;
    double alpha = 0.0;
    __device__ void prep(const DevScalars *sc) { alpha = sc->alpha; }
    static constexpr int NL = 2;
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *raw) const {
        const int64_t i = 2 * (row * C + col);
        if (i >= nr) return;
        raw[0] = ld2(r, i, nr);
        raw[1] = ld2(v, i, nr);
    }
    __device__ __forceinline__ double2 finish(int row, int64_t col, const double2 *raw) const {
        const int64_t i = 2 * (row * C + col);
        if (i >= nr) return make_double2(0.0, 0.0);
        const double2 sv = make_double2(fma(-alpha, raw[1].x, raw[0].x), fma(-alpha, raw[1].y, raw[0].y));
        st2(s, i, nr, sv);
        return sv;
    }
};

struct OutBiT {  // t = A shat (written); omega = (t . s) / (t . t)
    double *t;
    const double *s;
    int64_t nr, C;
    static constexpr int NACC = 2, NPRE = 1;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *pre) const {
        const int64_t i = 2 * (row * C + col);
        if (i < nr) pre[0] = ld2(s, i, nr);
    }
    __device__ __forceinline__ void store(int row, int64_t col, double2 val, double *acc, const double2 *pre) const {
        const int64_t i = 2 * (row * C + col);
        if (i < nr) {
            if (i + 1 >= nr) val.y = 0.0;
            st2(t, i, nr, val);
            acc[0] = fma(val.x, pre[0].x, fma(val.y, pre[0].y, acc[0]));
            acc[1] = fma(val.x, val.x, fma(val.y, val.y, acc[1]));
        }
    }
    __device__ void final(const double *tot, DevScalars *sc) const {
        // t = 0 means s = 0: x + alpha phat is the answer, and omega = 0
        // leaves r = s for the update's convergence test
        sc->omega = tot[1] > 0.0 ? tot[0] / tot[1] : 0.0;
        if (!finite(tot[0]) || !finite(tot[1])) {
            sc->status = ST_NONFINITE;
            sc->done = 1;
        }
    }
    double *partials;
};

// x += alpha phat + omega shat ; r = s - omega t ; partial sums of |r|^2 and
// rt . r per workgroup (256 threads).
__global__ void __launch_bounds__(256) k_bicg_update(double *__restrict__ x, double *__restrict__ r,
                                                     const double *__restrict__ rt, const double *__restrict__ phat,
                                                     const double *__restrict__ shat, const double *__restrict__ s,
                                                     const double *__restrict__ t, int64_t n, const DevScalars *sc,
                                                     double *partials, int pred) {
    if (skip(pred, sc)) return;
    const double alpha = sc->alpha, omega = sc->omega;
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] = fma(omega, shat[i], fma(alpha, phat[i], x[i]));
        const double ri = fma(-omega, t[i], s[i]);
        r[i] = ri;
        acc[0] = fma(ri, ri, acc[0]);
        acc[1] = fma(rt[i], ri, acc[1]);
    }
    block_partial<2>(acc, partials, blockIdx.x);
}

// Finishing step of k_bicg_update: rho_prev = rho, rho = rt . r, |r|^2, the
// iteration count and the stopping, breakdown and non-finite tests.
__global__ void __launch_bounds__(256) k_bicg_final(const double *partials, int nparts, DevScalars *sc, int pred) {
    if (skip(pred, sc)) return;
    double tot[2];
    reduce_partials<2>(partials, nparts, tot);
    if (threadIdx.x == 0) {
        sc->rnorm2 = tot[0];
        sc->rho_prev = sc->rho;
        sc->rho = tot[1];
        sc->iter += 1;
        sc->fresh = 0;
        if (!finite(tot[0]) || !finite(tot[1])) {
            sc->status = ST_NONFINITE;
            sc->done = 1;
        } else if (tot[0] <= sc->tol2) {
            sc->done = 1;
        } else if (tot[1] == 0.0 || sc->omega == 0.0) {
            sc->status = ST_BREAKDOWN;
            sc->done = 1;
        }
    }
}

// Fast history (the L2-1sigma weights c_m, m >= 2, as sum_k w_k rho_k^m +
// sum_p C_p m^p).  At level L >= 2 (write_p):
//   P_L = kappa [sum_k w_k S_k + sum_p C_p T_p + c_L^(L) (u^1 - u^0) - c_1 u^{L-1}]
// with S_k = sum_{m=2}^{L-1} rho_k^m delta_{L-m}, T_p = sum_{m=2}^{L-1} m^p delta_{L-m},
// delta_s = u^{s+1} - u^s; then (advance) the recursions move to level L+1:
//   S_k <- rho_k (S_k + rho_k delta_{L-1}),  T_p <- 2^p delta_{L-1} + sum_{q<=p} C(p,q) T_q.
// S holds K + 4 rows of ld values (the K exponentials, then T_0..T_3).
struct SoePoly {
    double c[4];
};
__global__ void __launch_bounds__(256) k_hist_soe(const double *__restrict__ U, int64_t n, int64_t ld, int L,
                                                  double *__restrict__ S, int K, const double *__restrict__ rho,
                                                  const double *__restrict__ w, SoePoly poly, double kappa, double c1,
                                                  double cL, double *__restrict__ P, int write_p, int advance) {
    const double *uL = U + (size_t)L * ld, *uLm = U + (size_t)(L - 1) * ld;
    double *T = S + (size_t)K * ld;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double um = uLm[i], d = uL[i] - um;
        double t0 = T[i], t1 = T[ld + i], t2 = T[2 * ld + i], t3 = T[3 * ld + i];
        double acc = poly.c[0] * t0 + poly.c[1] * t1 + poly.c[2] * t2 + poly.c[3] * t3;
        for (int k = 0; k < K; ++k) {
            double sk = S[(size_t)k * ld + i];
            acc = fma(w[k], sk, acc);
            if (advance) S[(size_t)k * ld + i] = rho[k] * fma(rho[k], d, sk);
        }
        if (write_p) P[i] = kappa * (acc + cL * (U[ld + i] - U[i]) - c1 * um);
        if (advance) {
            T[3 * ld + i] = 8.0 * d + t0 + 3.0 * t1 + 3.0 * t2 + t3;
            T[2 * ld + i] = 4.0 * d + t0 + 2.0 * t1 + t2;
            T[ld + i] = 2.0 * d + t0 + t1;
            T[i] = d + t0;
        }
    }
}

// Last step of the Gohberg-Semencul product (Algorithm 1): the pass that
// forms z3 = L0_p z1 stores x = (z4 - z3) / xi_0.
struct OutGsfCombine {
    const double *z4;
    double *x;
    int64_t nr, C;
    double inv_xi0;
    static constexpr int NACC = 0, NPRE = 1;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *pre) const {
        const int64_t i = 2 * (row * C + col);
        if (i < nr) pre[0] = ld2(z4, i, nr);
    }
    __device__ __forceinline__ void store(int row, int64_t col, double2 val, double *, const double2 *pre) const {
        const int64_t i = 2 * (row * C + col);
        if (i < nr) st2(x, i, nr, make_double2((pre[0].x - val.x) * inv_xi0, (pre[0].y - val.y) * inv_xi0));
    }
    __device__ void final(const double *, DevScalars *) const {}
    double *partials;
};

// vhat = A phat; accumulates rt . vhat; the last workgroup sets alpha = rho / (rt . vhat).
template <class S> struct OutCgsDotT {
    S *vhat;
    const S *rt;
    int64_t nr, C;
    static constexpr int NACC = 1, NPRE = 1;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *pre) const {
        int64_t i = 2 * (row * C + col);
        if (i < nr) pre[0] = ld2(rt, i, nr);
    }
    __device__ __forceinline__ void store(int row, int64_t col, double2 val, double *acc, const double2 *pre) const {
        int64_t i = 2 * (row * C + col);
        if (i < nr) {
            if (i + 1 >= nr) val.y = 0.0;
            st2(vhat, i, nr, val);
            double2 t = pre[0];
            acc[0] = fma(t.x, val.x, fma(t.y, val.y, acc[0]));
        }
    }
    __device__ void final(const double *tot, DevScalars *sc) const {
        sc->rtv = tot[0];
        double a = sc->rho / tot[0];
        if (tot[0] == 0.0) {
            sc->status = ST_BREAKDOWN;
            sc->done = 1;
        } else if (!finite(a)) {
            sc->status = ST_NONFINITE;
            sc->done = 1;
        }
        sc->alpha = a;
    }
    double *partials;
};
using OutCgsDot = OutCgsDotT<double>;

// r = r - alpha (A uhat); accumulates r.r and rt.r; the last workgroup advances
// the recurrence scalars and tests |r| <= rtol |g|.
template <class S> struct OutCgsRT {
    S *r;
    const S *rt;
    int64_t nr, C;
    double alpha;
    static constexpr int NACC = 2, NPRE = 2;
    __device__ void prep(const DevScalars *sc) { alpha = sc->alpha; }
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *pre) const {
        int64_t i = 2 * (row * C + col);
        if (i < nr) {
            pre[0] = ld2(r, i, nr);
            pre[1] = ld2(rt, i, nr);
        }
    }
    __device__ __forceinline__ void store(int row, int64_t col, double2 val, double *acc, const double2 *pre) const {
        int64_t i = 2 * (row * C + col);
        if (i < nr) {
            if (i + 1 >= nr) val.y = 0.0;
            double2 rv = pre[0];
            rv.x = fma(-alpha, val.x, rv.x);
            rv.y = fma(-alpha, val.y, rv.y);
            st2(r, i, nr, rv);
            double2 t = pre[1];
            acc[0] = fma(rv.x, rv.x, fma(rv.y, rv.y, acc[0]));
            acc[1] = fma(t.x, rv.x, fma(t.y, rv.y, acc[1]));
        }
    }
    __device__ void final(const double *tot, DevScalars *sc) const {
        sc->rnorm2 = tot[0];
        sc->rho_prev = ci == 0 ? sc->rho : sc->rho2[ci & 1];
        sc->rho = tot[1];
        sc->beta = tot[1] / sc->rho_prev;
        sc->iter += 1;
        sc->fresh = 0;
        if (!finite(tot[0]) || !finite(tot[1])) {
            sc->status = ST_NONFINITE;
            sc->done = 1;
        } else if (tot[0] <= sc->tol2) {
            sc->done = 1;
        } else if (tot[1] == 0.0) {
            sc->status = ST_BREAKDOWN;
            sc->done = 1;
        }
    }
    double *partials;
    int ci = 0;  // index in its chunk of the iteration this finishes (0: rho_old is rho)
};
using OutCgsR = OutCgsRT<double>;

// Right-hand side of (3.3) from y = A u^j:
//   g = (eta/sigma) u^j - ((1-sigma)/sigma) y - H + f     (= B u^j - H + f)
// with H = P + kappa c_1 u^j (P the history kernels' partial sum), i.e.
//   g = (eta/sigma - kappa c_1) u^j - ((1-sigma)/sigma) y - P + f,
// c_u holding the first coefficient and H pointing at P;
//   x0 = u^j (warm) or 0;  r = g - A x0 ;  rt = r.
// The finishing kernel initialises the CGS scalars for the level.
// warm: 0 -> x0 = 0; 1 -> x0 = u^j; 2 -> x0 = 3u^j - 3u^{j-1} + u^{j-2}
// (quadratic extrapolation in t; r is then recomputed from x0 by a restart).
struct OutRhs {
    const double *uj, *H, *f;
    double *g, *r, *rt, *x;
    int64_t nr, C;
    double c_u, c_y;  // eta/sigma - kappa c_1 (or eta/sigma at level 0), (1-sigma)/sigma
    int warm, has_hist;
    const double *ujm1, *ujm2;  // u^{j-1}, u^{j-2} for warm == 2
    // u^j, H and f are fetched ahead; the extrapolation's two older levels
    // are read in the store (once per level, and it keeps the pass unspilled)
    static constexpr int NACC = 2, NPRE = 3;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *pre) const {
        int64_t i = 2 * (row * C + col);
        if (i < nr) {
            pre[0] = ld2(uj, i, nr);
            if (has_hist) pre[1] = ld2(H, i, nr);
            if (f) pre[2] = ld2(f, i, nr);
        }
    }
    __device__ __forceinline__ void store(int row, int64_t col, double2 val, double *acc, const double2 *pre) const {
        int64_t i = 2 * (row * C + col);
        if (i < nr) {
            if (i + 1 >= nr) val.y = 0.0;
            double2 u = pre[0];
            double2 gv = make_double2(fma(c_u, u.x, -c_y * val.x), fma(c_u, u.y, -c_y * val.y));
            if (has_hist) {
                double2 hv = pre[1];
                gv.x -= hv.x;
                gv.y -= hv.y;
            }
            if (f) {
                double2 fv = pre[2];
                gv.x += fv.x;
                gv.y += fv.y;
            }
            double2 rv = warm == 1 ? make_double2(gv.x - val.x, gv.y - val.y) : gv;
            double2 xv = make_double2(0.0, 0.0);
            if (warm == 1) {
                xv = u;
            } else if (warm == 2) {
                const double2 a = ld2(ujm1, i, nr);
                const double2 b = ld2(ujm2, i, nr);
                xv = make_double2(fma(3.0, u.x - a.x, b.x), fma(3.0, u.y - a.y, b.y));
            }
            st2(g, i, nr, gv);
            st2(r, i, nr, rv);
            st2(rt, i, nr, rv);
            st2(x, i, nr, xv);
            acc[0] = fma(gv.x, gv.x, fma(gv.y, gv.y, acc[0]));
            acc[1] = fma(rv.x, rv.x, fma(rv.y, rv.y, acc[1]));
        }
    }
    __device__ void final(const double *tot, DevScalars *sc) const {
        sc->gnorm2 = tot[0];
        sc->rnorm2 = tot[1];
        sc->rho = tot[1];
        sc->rho_prev = 1.0;
        sc->beta = 0.0;
        sc->alpha = 0.0;
        sc->tol2 = sc->rtol2 * tot[0];
        sc->iter = 0;
        sc->fresh = 1;
        sc->aux0 = tot[1];
        sc->r0sq = tot[1];
        sc->status = ST_OK;
        sc->checked = 0;
        sc->nchecks = 0;
        sc->done = (tot[1] <= sc->tol2) ? 1 : 0;
        if (!finite(tot[0]) || !finite(tot[1])) {
            sc->status = ST_NONFINITE;
            sc->done = 1;
        }
    }
    double *partials;
};

// |g - A x|^2 into aux0.
struct OutTrueRes {
    const double *g;
    int64_t nr, C;
    static constexpr int NACC = 1, NPRE = 1;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *pre) const {
        int64_t i = 2 * (row * C + col);
        if (i < nr) pre[0] = ld2(g, i, nr);
    }
    __device__ __forceinline__ void store(int row, int64_t col, double2 val, double *acc, const double2 *pre) const {
        int64_t i = 2 * (row * C + col);
        if (i < nr) {
            if (i + 1 >= nr) val.y = 0.0;
            double2 gv = pre[0];
            double dx = gv.x - val.x, dy = gv.y - val.y;
            acc[0] = fma(dx, dx, fma(dy, dy, acc[0]));
        }
    }
    __device__ void final(const double *tot, DevScalars *sc) const { sc->aux0 = tot[0]; }
    double *partials;
};

// Restart of CGS from the current iterate x (true-residual verification and
// breakdown recovery): y = A x, r = g - y, rt = r; the last workgroup resets
// the recurrence and records |r|^2 in aux0.
struct OutRestart {
    const double *g, *x;
    double *r, *rt;
    int64_t nr, C;
    double anorm, bwtol;  // bound on |A|_2; accept x at backward error <= bwtol (0: never)
    static constexpr int NACC = 2, NPRE = 2;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *pre) const {
        int64_t i = 2 * (row * C + col);
        if (i < nr) {
            pre[0] = ld2(g, i, nr);
            pre[1] = ld2(x, i, nr);
        }
    }
    __device__ __forceinline__ void store(int row, int64_t col, double2 val, double *acc, const double2 *pre) const {
        int64_t i = 2 * (row * C + col);
        if (i < nr) {
            if (i + 1 >= nr) val.y = 0.0;
            double2 gv = pre[0];
            double2 rv = make_double2(gv.x - val.x, gv.y - val.y);
            st2(r, i, nr, rv);
            st2(rt, i, nr, rv);
            acc[0] = fma(rv.x, rv.x, fma(rv.y, rv.y, acc[0]));
            acc[1] = fma(pre[1].x, pre[1].x, fma(pre[1].y, pre[1].y, acc[1]));
        }
    }
    // aux0 = |g - A x|^2 (true residual), aux1 = |x|^2.  x is accepted (done)
    // when |g - A x| <= rtol |g|, or when the normwise backward error
    // |g - A x| / (|A| |x| + |g|) is at most bwtol.
    __device__ void final(const double *tot, DevScalars *sc) const {
        if (check) {  // an acceptance check: count it, keep how CGS stopped
            sc->nchecks += 1;
            sc->prestat = sc->status;
        }
        sc->aux0 = tot[0];
        sc->aux1 = tot[1];
        sc->better = (tot[0] < sc->r0sq) ? 1 : 0;  // isfinite by comparison
        sc->rnorm2 = tot[0];
        sc->rho = tot[0];
        sc->rho_prev = 1.0;
        sc->beta = 0.0;
        sc->alpha = 0.0;
        sc->fresh = 1;
        sc->status = ST_OK;
        const double den = anorm * sqrt(tot[1]) + sqrt(sc->gnorm2);
        const bool bw_ok = bwtol > 0.0 && sqrt(tot[0]) <= bwtol * den;
        sc->done = (tot[0] <= sc->tol2 || bw_ok) ? 1 : 0;
        if (!finite(tot[0])) {
            sc->status = ST_NONFINITE;
            sc->done = 1;
        }
        sc->checked = sc->done;
    }
    double *partials;
    int check = 0;  // 1: an acceptance check of a converged solve (counted in nchecks)
};

// Iterative refinement (FP64 outer loop around an FP32-stored inner solve):
// x += d (the inner solve's correction, FP32) in FP64; transforms x.
struct InIR {
    double *x;
    const float *d;
    int64_t nr, C;
    static constexpr int NL = 2;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *raw) const {
        int64_t i = 2 * (row * C + col);
        if (i >= nr) return;
        raw[0] = ld2(x, i, nr);
        raw[1] = ld2(d, i, nr);
    }
    __device__ __forceinline__ double2 finish(int row, int64_t col, const double2 *raw) const {
        int64_t i = 2 * (row * C + col);
        if (i >= nr) return make_double2(0.0, 0.0);
        const double2 xv = make_double2(raw[0].x + raw[1].x, raw[0].y + raw[1].y);
        st2(x, i, nr, xv);
        return xv;
    }
};

// Outer residual r = g - A x in FP64: |r|^2 and |x|^2 accumulate in FP64, r is
// handed to the inner solve rounded to FP32 (r = rt = r, d = 0).  The last
// workgroup's epilogue stops the level when |r| <= rtol |g|, and otherwise
// starts the inner CGS with tolerance irtol |r|.
struct OutIR {
    const double *g, *x;
    float *r, *rt, *d;
    int64_t nr, C;
    double irtol2;
    static constexpr int NACC = 2, NPRE = 2;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *pre) const {
        int64_t i = 2 * (row * C + col);
        if (i < nr) {
            pre[0] = ld2(g, i, nr);
            pre[1] = ld2(x, i, nr);
        }
    }
    __device__ __forceinline__ void store(int row, int64_t col, double2 val, double *acc, const double2 *pre) const {
        int64_t i = 2 * (row * C + col);
        if (i < nr) {
            if (i + 1 >= nr) val.y = 0.0;
            const double2 gv = pre[0];
            const double2 rv = make_double2(gv.x - val.x, gv.y - val.y);
            st2(r, i, nr, rv);
            st2(rt, i, nr, rv);
            st2(d, i, nr, make_double2(0.0, 0.0));
            acc[0] = fma(rv.x, rv.x, fma(rv.y, rv.y, acc[0]));
            acc[1] = fma(pre[1].x, pre[1].x, fma(pre[1].y, pre[1].y, acc[1]));
        }
    }
    // aux1 = |g - A x|^2, aux0 = |x|^2
    __device__ void final(const double *tot, DevScalars *sc) const {
        sc->aux1 = tot[0];
        sc->aux0 = tot[1];
        sc->rnorm2 = tot[0];
        sc->rho = tot[0];
        sc->rho_prev = 1.0;
        sc->beta = 0.0;
        sc->alpha = 0.0;
        sc->tol2 = irtol2 * tot[0];
        sc->iter = 0;
        sc->fresh = 1;
        sc->status = ST_OK;
        sc->done = (tot[0] <= sc->rtol2 * sc->gnorm2) ? 1 : 0;
        if (!finite(tot[0])) {
            sc->status = ST_NONFINITE;
            sc->done = 1;
        }
    }
    double *partials;
};

// ---------------------------------------------------------------------------
// Values per lane of the FFT passes (4, 8 or 16); fewer values per lane give
// more waves per SIMD.  Chosen per kernel family at build time.
// ---------------------------------------------------------------------------
#ifndef TSF_E_COL
#define TSF_E_COL 8
#endif
#ifndef TSF_E_MID
#define TSF_E_MID 8
#endif
#ifndef TSF_E_FUSE
#define TSF_E_FUSE 8
#endif
// Column passes of length 512 (single plans) run four columns of 64 lanes
// at eight values per lane, four waves per CU at n = 2^20; four values per
// lane double the waves and were 4-6% faster (measured).
#ifndef TSF_E_COL_512
#define TSF_E_COL_512 4
#endif
#ifndef TSF_E_COL_1024  // column passes of length 1024 (single plans)
#define TSF_E_COL_1024 TSF_E_COL
#endif
// Columns of 2048 at sixteen values per lane: four columns per workgroup
// (64-byte row segments) instead of two.  With the four-step twiddles from
// running products the passes do not spill, and the march ran 8.5% faster
// at n = 2^22 and 7% at n = 2^24 than at eight (measured).
#ifndef TSF_E_COL_2048  // column passes of length 2048 (single plans)
#define TSF_E_COL_2048 16
#endif
// Columns of 4096 at eight values per lane fit one per workgroup (16-byte
// row segments); at sixteen, two columns of 256 lanes, with the twiddles
// read from the global table (measured 6% faster per iteration at n = 2^24
// even when these passes still spilled registers).
#ifndef TSF_E_COL_4096  // column passes of length 4096 (single plans)
#define TSF_E_COL_4096 16
#endif
// The preconditioner's middle pass has half the rows of the product's (one
// workgroup per CU at n = 2^20); four values per lane give it twice the
// waves, which outweighs its unpaired last stage (5% faster, measured), for
// rows of up to 1024 points.
// Rows of 4096 at eight values per lane need 1024-thread workgroups (128
// VGPRs a lane, spilling); sixteen values per lane give 512 threads with no
// spill, and the pass ran 32% faster (measured at n = 2^24).
#ifndef TSF_E_MID_4096  // middle passes with rows of 4096 (single plans)
#define TSF_E_MID_4096 16
#endif
#ifndef TSF_MID_PAIRS  // row pairs per workgroup of a single plan's middle passes (1 or 2)
#define TSF_MID_PAIRS 2
#endif
#ifndef TSF_E_MID_2048  // middle passes with rows of 2048 (single plans)
#define TSF_E_MID_2048 TSF_E_MID
#endif
#ifndef TSF_E_MID_SOLVE  // middle pass of the preconditioner solve (single plans)
#define TSF_E_MID_SOLVE 4
#endif

// ---------------------------------------------------------------------------
// Column pass: length-R FFTs down B adjacent columns per workgroup, B * R =
// 4096 values (64 KiB), except for columns of 512: four of them, so that the
// 1024 columns of a 2^20-point problem's preconditioner transform give a
// workgroup per CU (eight left half the CUs idle; measured 8% slower).
// Narrower tiles split the 128-byte lines of a row (measured slower).
// ---------------------------------------------------------------------------
constexpr int LDS_VALUES = 163840 / 16;  // complex doubles in a CU's LDS
template <int R, int EMAX> struct ColGeo {
    static constexpr int E = Geo<R, EMAX>::E;
    static constexpr int T = Geo<R, EMAX>::T;
    // at sixteen values per lane, columns of 2048 and 4096 take 8192 values
    // per workgroup (four and two columns at 512 threads)
    static constexpr int B0 = R == 512 ? 4 : (R >= 2048 && E >= 16 ? 8192 / R : 4096 / R);
    static constexpr int B = (B0 * T > 1024) ? 1024 / T : B0;  // columns per workgroup
    static constexpr int NT = B * T;                            // threads per workgroup
    // the twiddle table is staged in LDS when it fits beside the data
    static constexpr bool TWL = R > E && lpad_size(R) * B + R <= LDS_VALUES - 64;
    // the partial sums reduce in a fixed 256-wide order (reduce_partials)
    static_assert(NT >= 256 && NT <= 1024, "column pass workgroup size");
    static_assert(lpad_size(R) * B <= LDS_VALUES - 64, "data slab fits in LDS");
};

// Loaders and stores whose per-value operands are only the four-step
// twiddle can take it from a running product instead (TwRec), in passes of
// at least TSF_REC_MIN_E values per lane: there it removed the register
// spills at sixteen, and at eight it cut the headline march's time by 2.8%
// and the batch's by 3.7% (fewer table loads); at four it gained less
// (measured).
#ifndef TSF_REC_MIN_E
#define TSF_REC_MIN_E 8
#endif
template <class T, class = void> struct HasRec {
    static constexpr bool value = false;
};
template <class T> struct HasRec<T, decltype(void(T::REC))> {
    static constexpr bool value = T::REC;
};

// Last-stage outputs of butterfly group q (slots q + NB r) sit at positions
// pos(j, q) + NS r: one running product per group.
template <class Out, int NB> struct ColRecSink {
    const Out *out;
    int64_t c;
    TwRec *tr;
    __device__ __forceinline__ void operator()(int pos, double2 val, int slot) const {
        out->store_tw(pos, c, val, tr[slot % NB].next());
    }
};

// ColSink whose epilogue operands are fetched late (prefetch(), before the
// exchange that precedes the last stage) rather than before the transform.
template <class Out, int NP, int R, int E> struct ColLateSink {
    Out *out;
    int64_t c;
    double *acc;
    double2 (*pre)[NP];
    int j;
    bool active;
    __device__ __forceinline__ void prefetch() const {
        if (active) {
#pragma unroll
            for (int m = 0; m < E; ++m) out->fetch(LastStage<R, E>::pos(j, m), c, pre[m]);
        }
    }
    __device__ __forceinline__ void operator()(int pos, double2 val, int slot) const {
        out->store(pos, c, val, acc, pre[slot]);
    }
};

template <class Out, int NP> struct ColSink {
    Out *out;
    int64_t c;
    double *acc;
    const double2 (*pre)[NP];
    __device__ __forceinline__ void operator()(int pos, double2 val, int slot) const {
        out->store(pos, c, val, acc, pre[slot]);
    }
};

template <int R, int EMAX, int DIR, class In, class Out>
__device__ __forceinline__ void col_body(int64_t C, In in, Out out, const double2 *__restrict__ tw_all, DevScalars *sc,
                                         int pred) {
    if (skip(pred, sc)) return;
    using G = ColGeo<R, EMAX>;
    constexpr int E = G::E, T = G::T, B = G::B;
    __shared__ double2 lds[lpad_size(R) * B];
    __shared__ double2 twl[G::TWL ? R : 1];
    const int t = threadIdx.x;
    const int b = t % B, j = t / B;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t c = tile * B + b;
    const bool active = c < C;
    in.prep(sc);
    out.prep(sc);
    // The four-step twiddles of the input and of the output come from
    // running products (TwRec) rather than two table entries per value (at
    // sixteen values per lane those entries did not fit beside the values in
    // the register file): the lane's rows form arithmetic progressions
    // j + T m, and in the last stage pos(j, q) + NS r for each of a lane's
    // butterfly groups q.
    constexpr bool REC_IN = E >= TSF_REC_MIN_E && HasRec<In>::value;
    constexpr bool REC_OUT = E >= TSF_REC_MIN_E && HasRec<Out>::value;
    constexpr int NBL = LastStage<R, E>::NB;
    // every load of the pass is issued before the first store: the inputs,
    // then the operands the last stage's stores combine with each output
    double2 raw[E][REC_IN ? 1 : In::NL];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        if (active) {
            if constexpr (REC_IN) {
                raw[m][0] = in.value(j + T * m, c);
            } else {
                in.fetch(j + T * m, c, raw[m]);
            }
        }
    }
    TwRec trin, trout[REC_OUT ? NBL : 1];
    if constexpr (REC_IN) {
        if (active) trin.init(in.tw, j, T, c);
    }
    if constexpr (REC_OUT) {
#pragma unroll
        for (int q = 0; q < NBL; ++q)
            if (active) trout[q].init(out.tw, LastStage<R, E>::pos(j, q), LastStage<R, E>::NS, c);
    }
    // the same width leaves no room for the epilogue's operands across the
    // transform either: they are fetched before its last exchange instead
    constexpr bool LATE = E >= 16 && Out::NPRE > 0 && !REC_OUT;
    constexpr int NP = Out::NPRE > 0 && !REC_OUT ? Out::NPRE : 1;
    double2 pre[REC_OUT ? 1 : E][NP];
    if constexpr (Out::NPRE > 0 && !REC_OUT && !LATE) {
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (active) out.fetch(LastStage<R, E>::pos(j, m), c, pre[m]);
    }
    // a folded finishing step runs while the loads are in flight; the solve
    // may end there (the decision is the same in every workgroup)
    if constexpr (HasFold<In>::value) {
        if (in.fold(sc)) return;
    }
    double2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        if constexpr (REC_IN) {
            v[m] = active ? in.finish_tw(raw[m][0], trin.next()) : make_double2(0.0, 0.0);
        } else {
            v[m] = active ? in.finish(j + T * m, c, raw[m]) : make_double2(0.0, 0.0);
        }
    }
    // the first barrier inside the transform orders these writes before any use
    if constexpr (G::TWL) stage_twiddles<R>(twl, tw_all, t, G::NT);
    double acc[Out::NACC > 0 ? Out::NACC : 1];
#pragma unroll
    for (int a = 0; a < (Out::NACC > 0 ? Out::NACC : 1); ++a) acc[a] = 0.0;
    if constexpr (REC_OUT) {
        static_assert(Out::NACC == 0, "running-product twiddles serve plain spectrum stores");
        ColRecSink<Out, NBL> sink{&out, c, trout};
        if constexpr (G::TWL) {
            fft_t<R, E, DIR, 1>(v, j, active, twl, lds + b, B, sink);
        } else {
            fft<R, E, DIR>(v, j, active, tw_all, lds + b, B, sink);
        }
    } else if constexpr (LATE) {
        ColLateSink<Out, NP, R, E> sink{&out, c, acc, pre, j, active};
        if constexpr (G::TWL) {
            fft_t<R, E, DIR, 1>(v, j, active, twl, lds + b, B, sink);
        } else {
            fft<R, E, DIR>(v, j, active, tw_all, lds + b, B, sink);
        }
    } else {
        ColSink<Out, NP> sink{&out, c, acc, pre};
        if constexpr (G::TWL) {
            fft_t<R, E, DIR, 1>(v, j, active, twl, lds + b, B, sink);
        } else {
            fft<R, E, DIR>(v, j, active, tw_all, lds + b, B, sink);
        }
    }
    if constexpr (Out::NACC > 0) block_partial<Out::NACC>(acc, out.partials, tile);
}

// Finishing kernel of a reducing pass (one workgroup of the pass's size NT).
template <int NT, class Out>
__global__ void __launch_bounds__(NT) k_final(Out out, int nparts, DevScalars *sc, int pred) {
    if (skip(pred, sc)) return;
    double tot[Out::NACC];
    reduce_partials<Out::NACC>(out.partials, nparts, tot);
    if (threadIdx.x == 0) out.final(tot, sc);
}

template <int R, int EMAX, int DIR, class In, class Out>
__global__ void __launch_bounds__((ColGeo<R, EMAX>::NT)) k_col(int64_t C, In in, Out out,
                                                             const double2 *__restrict__ tw_all, DevScalars *sc,
                                                             int pred) {
    col_body<R, EMAX, DIR, In, Out>(C, in, out, tw_all, sc, pred);
}

// Batched form: one launch for a group of instances with the same transform
// geometry; blockIdx.y selects the instance, whose loader, store and scalars
// come from a descriptor in device memory.  With an index list `act` the
// launch covers only the listed instances (descriptor act[blockIdx.y]), so a
// group's converged instances cost no workgroups at all.
__device__ __forceinline__ int batch_member(const int *__restrict__ act) {
    return act ? act[blockIdx.y] : (int)blockIdx.y;
}

template <class In, class Out> struct ColDesc {
    int64_t C;
    In in;
    Out out;
    DevScalars *sc;
};

template <int R, int EMAX, int DIR, class In, class Out>
__global__ void __launch_bounds__((ColGeo<R, EMAX>::NT)) k_col_b(const ColDesc<In, Out> *__restrict__ d,
                                                               const int *__restrict__ act,
                                                               const double2 *__restrict__ tw_all, int pred) {
    const ColDesc<In, Out> D = d[batch_member(act)];
    col_body<R, EMAX, DIR, In, Out>(D.C, D.in, D.out, tw_all, D.sc, pred);
}

template <int NT, class In, class Out>
__global__ void __launch_bounds__(NT) k_final_b(const ColDesc<In, Out> *__restrict__ d,
                                                 const int *__restrict__ act, int nparts, int pred) {
    const ColDesc<In, Out> &D = d[batch_member(act)];
    if (skip(pred, D.sc)) return;
    double tot[Out::NACC];
    reduce_partials<Out::NACC>(D.out.partials, nparts, tot);
    if (threadIdx.x == 0) D.out.final(tot, D.sc);
}

// ---------------------------------------------------------------------------
// Fused column pass: inverse length-RP column FFTs of the preconditioner
// transform (R_P x C) followed, for the same columns, by the forward
// length-2RP column FFTs of the following Toeplitz product (R_A = 2R_P rows,
// same C).  The packed preconditioner output z'[m] = y[2m] + i y[2m+1],
// m = row*C + col, is exactly the nonzero half of the product's packed input,
// so the solve's result never goes through memory.  `op` may apply a vector
// update to it (x += alpha * uhat) and returns the product's input.
// ---------------------------------------------------------------------------
struct OpIdent {
    static constexpr bool FETCH = false;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int, int64_t, double2 &) const {}
    __device__ __forceinline__ double2 operator()(int, int64_t, double2 v, double2) const { return v; }
};

template <class S> struct OpCgsXT {  // x += alpha * uhat at real indices 2m, 2m+1 (x fetched at kernel start)
    static constexpr bool FETCH = true;
    S *x;
    int64_t C;
    double alpha;
    __device__ void prep(const DevScalars *sc) { alpha = sc->alpha; }
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 &xv) const {
        const int64_t i = 2 * (row * C + col);
        xv = ld2(x, i, i + 2);
    }
    __device__ __forceinline__ double2 operator()(int row, int64_t col, double2 uh, double2 xv) const {
        const int64_t i = 2 * (row * C + col);
        st2(x, i, i + 2, make_double2(fma(alpha, uh.x, xv.x), fma(alpha, uh.y, xv.y)));
        return uh;
    }
};
using OpCgsX = OpCgsXT<double>;

template <class CS, int NB> struct BufRecSink {  // y[pos*C + c] = val * tw(2*pos*c), twiddles from running products
    CS *y;
    TwRec *tr;  // one per butterfly group of the last stage
    int64_t C, c;
    __device__ __forceinline__ void operator()(int pos, double2 val, int slot) const {
        stc(y, pos * C + c, cmul(val, tr[slot % NB].next()));
    }
};

template <int NS_, class CS> struct BufSink {  // y[pos*C + c] = val * tw(2*pos*c), table entries fetched per slot
    CS *y;
    const double2 (*tw)[2];
    int64_t C, c;
    __device__ __forceinline__ void operator()(int pos, double2 val, int slot) const {
        stc(y, pos * C + c, cmul(val, cmul(tw[slot][0], tw[slot][1])));
    }
};

// Fused passes whose product columns have 4096 points: sixteen values per
// lane give two columns per workgroup (global twiddles), 1.3% faster per
// iteration at n = 2^24 (measured).
#ifndef TSF_E_FUSE_4096
#define TSF_E_FUSE_4096 16
#endif
// ... and with 2048 points: four columns per workgroup, 1.2% faster per
// iteration at n = 2^22 (measured).
#ifndef TSF_E_FUSE_2048
#define TSF_E_FUSE_2048 16
#endif
#ifndef TSF_E_FUSE_P  // values per lane of the fused pass's preconditioner transform
#define TSF_E_FUSE_P 8
#endif
template <int RP, int EMAX> struct FuseGeo {
    static constexpr int RA = 2 * RP;
    using GA = ColGeo<RA, EMAX>;
    static constexpr int EA = GA::E, TA = GA::T, B = GA::B, NT = GA::NT;
    static constexpr int EPM = TSF_E_FUSE_P < EA ? TSF_E_FUSE_P : EA;
    static constexpr int EP = Geo<RP, EPM>::E, TP = Geo<RP, EPM>::T;
    static_assert(TP <= TA, "the preconditioner transform's lanes fit in the workgroup");
};

template <int RP, int EMAX, class Op, class CS>
__global__ void __launch_bounds__((FuseGeo<RP, EMAX>::NT)) k_fuse(int64_t C, const CS *__restrict__ bufP, Tw2 twP,
                                                                CS *__restrict__ bufA, Tw2 twA, Op op,
                                                                const double2 *__restrict__ tw_all, DevScalars *sc,
                                                                int pred) {
    if (skip(pred, sc)) return;
    using G = FuseGeo<RP, EMAX>;
    constexpr int RA = G::RA, EA = G::EA, TA = G::TA, B = G::B, EP = G::EP, TP = G::TP;
    constexpr bool TWL = G::GA::TWL;
    __shared__ double2 lds[lpad_size(RA) * B];
    __shared__ double2 twl[TWL ? RA : 1];
    const int t = threadIdx.x;
    const int b = t % B, j = t / B;
    const int64_t c = xcd_tile(blockIdx.x, gridDim.x) * B + b;
    const bool colok = c < C;
    const bool activeP = colok && j < TP;
    op.prep(sc);
    // the four-step twiddles come from running products (TwRec), as in the
    // column passes
    constexpr bool RECP = EA >= TSF_REC_MIN_E;
    constexpr bool RECA = EA >= TSF_REC_MIN_E;
    constexpr int NBA = LastStage<RA, EA>::NB;
    // inverse preconditioner column FFT (conjugate four-step twiddle first)
    double2 rp[EP][RECP ? 1 : 3];
#pragma unroll
    for (int m = 0; m < EP; ++m) {
        const int row = j + TP * m;
        if (activeP) {
            rp[m][0] = ldc(bufP, row * C + c);
            if constexpr (!RECP) twP.fetch(2 * (int64_t)row * c, rp[m] + 1);
        }
    }
    TwRec trp, tra[NBA];
    if constexpr (RECP) {
        if (activeP) trp.init(twP, j, TP, c);
    }
    if constexpr (RECA) {
#pragma unroll
        for (int q = 0; q < NBA; ++q)
            if (colok) tra[q].init(twA, LastStage<RA, EA>::pos(j, q), LastStage<RA, EA>::NS, c);
    }
    // operands of the update and of the product's four-step twiddle, fetched now
    double2 xo[EA];
    if constexpr (Op::FETCH) {
#pragma unroll
        for (int m = 0; m < EA; ++m) {
            const int row = j + TA * m;
            if (colok && row < RP) op.fetch(row, c, xo[m]);
        }
    }
    double2 twa[RECA ? 1 : EA][2];
    if constexpr (!RECA) {
#pragma unroll
        for (int m = 0; m < EA; ++m)
            if (colok) twA.fetch(2 * (int64_t)LastStage<RA, EA>::pos(j, m) * c, twa[m]);
    }
    double2 vp[EP];
#pragma unroll
    for (int m = 0; m < EP; ++m) {
        if constexpr (RECP) {
            vp[m] = activeP ? cmul(rp[m][0], cconj(trp.next())) : make_double2(0.0, 0.0);
        } else {
            vp[m] = activeP ? cmul(rp[m][0], cconj(cmul(rp[m][1], rp[m][2]))) : make_double2(0.0, 0.0);
        }
    }
    if constexpr (TWL) stage_twiddles<RA>(twl, tw_all, t, G::NT);
    __syncthreads();
    LdsSink lsink{lds + b, B};
    if constexpr (TWL) {
        fft_t<RP, EP, 1, 2>(vp, j, activeP, twl, lds + b, B, lsink);
    } else {
        fft<RP, EP, 1>(vp, j, activeP, tw_all, lds + b, B, lsink);
    }
    __syncthreads();
    // product input: rows < RP carry the solve's output, rows >= RP are zero
    double2 va[EA];
#pragma unroll
    for (int m = 0; m < EA; ++m) {
        const int row = j + TA * m;
        double2 val = make_double2(0.0, 0.0);
        if (colok && row < RP) val = op(row, c, lds[lpad(row) * B + b], Op::FETCH ? xo[m] : val);
        va[m] = val;
    }
    __syncthreads();
    if constexpr (RECA) {
        BufRecSink<CS, NBA> bsink{bufA, tra, C, c};
        if constexpr (TWL) {
            fft_t<RA, EA, -1, 1>(va, j, colok, twl, lds + b, B, bsink);
        } else {
            fft<RA, EA, -1>(va, j, colok, tw_all, lds + b, B, bsink);
        }
    } else {
        BufSink<EA, CS> bsink{bufA, twa, C, c};
        if constexpr (TWL) {
            fft_t<RA, EA, -1, 1>(va, j, colok, twl, lds + b, B, bsink);
        } else {
            fft<RA, EA, -1>(va, j, colok, tw_all, lds + b, B, bsink);
        }
    }
}

// ---------------------------------------------------------------------------
// Middle pass: row pairs, untangle, symbol, retangle.
// MODE 0: y = S x (product); MODE 1: y = x / S (solve); MODE 2: write the
// forward spectrum X (natural-frequency values at native positions) to `spec`
// (k = 0 and k = N packed as (X_0, X_N) at position 0) and stop.
// ---------------------------------------------------------------------------
template <int MODE>
__device__ __forceinline__ void pair_update(double2 &za, double2 &zb, double2 w, double2 La, double2 Lb,
                                            const SymParams &sp, double2 *xa_out, double2 *xb_out) {
    const double2 A = za, Bc = cconj(zb);
    const double2 E2 = cadd(A, Bc);
    const double2 O2 = mul_i<-1>(csub(A, Bc));  // (A - Bc) / i
    const double2 wO = cmul(w, O2);
    const double2 Xa = cadd(E2, wO);           // 2 X_k
    const double2 Xb = cconj(csub(E2, wO));    // 2 X_{N-k}
    if constexpr (MODE == 2) {
        *xa_out = cscale(Xa, 0.5);
        *xb_out = cscale(Xb, 0.5);
        return;
    } else {
        const double s = -w.y;  // sin(2 pi k / L)
        const double2 Sa = make_double2(fma(sp.cre, La.x, sp.s0), fma(sp.cim, La.y, sp.cq * s));
        const double2 Sb = make_double2(fma(sp.cre, Lb.x, sp.s0), fma(sp.cim, Lb.y, sp.cq * s));
        double2 Ya, Yb;
        if constexpr (MODE == 0) {
            Ya = cscale(cmul(Sa, Xa), sp.scale);
            Yb = cscale(cmul(Sb, Xb), sp.scale);
        } else {
            const double2 Da = cscale(Sa, sp.scale), Db = cscale(Sb, sp.scale);
            const double ia = 1.0 / fma(Da.x, Da.x, Da.y * Da.y);
            const double ib = 1.0 / fma(Db.x, Db.x, Db.y * Db.y);
            Ya = cscale(cmul(Xa, cconj(Da)), ia);
            Yb = cscale(cmul(Xb, cconj(Db)), ib);
        }
        const double2 E2n = cadd(Ya, cconj(Yb));
        const double2 O2n = cmul(csub(Ya, cconj(Yb)), cconj(w));
        za = cadd(E2n, mul_i<1>(O2n));
        zb = cadd(cconj(E2n), mul_i<1>(cconj(O2n)));
    }
}

template <int C_, int EMAX> struct MidGeo {
    // two rows per workgroup, at most 1024 threads
    static constexpr int E0 = Geo<C_, EMAX>::E;
    static constexpr int E = (2 * (C_ / E0) > 1024) ? C_ / 512 : E0;
    static constexpr int T = C_ / E;
    static constexpr int NT = (2 * T + 63) / 64 * 64;  // threads per workgroup
    static constexpr int LS = lpad_size(C_);
};

template <class CS> struct RowSinkT {  // Y[row*C + pos] = val
    CS *Y;
    int64_t base;
    __device__ __forceinline__ void operator()(int pos, double2 val, int) const { stc(Y, base + pos, val); }
};
using RowSink = RowSinkT<double2>;

// One row pair (k1, R - k1) of a middle pass: the thread's row values and
// the pair step's operands, loaded before the pair's transform starts.
template <int C_, int EMAX, int MODE, class CS> struct MidPair {
    using G = MidGeo<C_, EMAX>;
    static constexpr int E = G::E, T = G::T;
    static constexpr int NPT = (C_ + G::NT - 1) / G::NT;
    // rows of 4096 would hold the pair step's operands across the transform
    // in more registers than a 1024-thread workgroup has; they load them in
    // the pair step instead
    static constexpr bool PF = C_ <= 2048;
    // rows of 2 * 8^k run their last (radix-2) stage on registers, with the
    // row's logical lanes placed so that partners share a row of 16 lanes
    static constexpr int PAIR = Paired<C_, E>::OK ? (T >= 16 ? 8 : 1) : 0;
    int64_t wg, ra, rb, row;
    int j, sel;
    bool active;
    double2 v[E];
    double2 pLa[PF ? NPT : 1], pLb[PF ? NPT : 1], pW[PF ? NPT : 1];

    // pair index w: rows (w, R - w), and for w = 0 the self-paired rows 0, R/2
    __device__ __forceinline__ void fetch(int64_t w, int64_t R, const CS *Y, const CS *spec, const Tw2 &twL) {
        constexpr int64_t C = C_;
        wg = w;
        ra = w == 0 ? 0 : w;
        rb = w == 0 ? R / 2 : R - w;
        const int t = threadIdx.x;
        sel = t / T;
        j = PAIR ? paired_lane<T>(t % T) : t % T;
        active = sel < 2;
        row = sel == 0 ? ra : rb;
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = active ? ldc(Y, row * C + j + T * m) : make_double2(0.0, 0.0);
        // Everything the pair step needs is fetched now, so its latency overlaps
        // the row loads and the forward transform: spectrum values and untangle
        // twiddles of this thread's pairs (rows ra, rb with ra != 0).
        if constexpr (PF) {
            if (wg != 0) {
#pragma unroll
                for (int i = 0; i < NPT; ++i) {
                    const int k2 = t + G::NT * i;
                    pLa[i] = pLb[i] = pW[i] = make_double2(0.0, 0.0);
                    if (k2 < C_) {
                        if constexpr (MODE != 2) {
                            pLa[i] = ldc(spec, ra * C + k2);
                            pLb[i] = ldc(spec, rb * C + (C_ - 1 - k2));
                        }
                        pW[i] = twL(ra + R * k2);
                    }
                }
            }
        }
    }
};

// The transform of one fetched row pair: forward row FFTs, untangle, symbol,
// retangle, inverse row FFTs (MODE 2 stops after the untangle).  twl holds
// the stage twiddles when TWL (staged by the caller).
template <int C_, int EMAX, int MODE, class CS, bool TWL>
__device__ __forceinline__ void mid_transform(MidPair<C_, EMAX, MODE, CS> &P, int64_t R, CS *Y, const CS *spec,
                                              double2 *spec_out, const Tw2 &twL, const SymParams &sp,
                                              const double2 *__restrict__ tw_all, double2 *lds, const double2 *twl) {
    using G = MidGeo<C_, EMAX>;
    using MP = MidPair<C_, EMAX, MODE, CS>;
    constexpr int E = G::E, T = G::T, LS = G::LS, NPT = MP::NPT, PAIR = MP::PAIR;
    constexpr bool PF = MP::PF;
    constexpr int64_t C = C_;
    const int64_t wg = P.wg, ra = P.ra, rb = P.rb, row = P.row;
    const int t = threadIdx.x, j = P.j;
    const bool active = P.active;
    double2 *slab = lds + (P.sel < 2 ? P.sel : 0) * LS;
    LdsSink lsink{slab, 1};
    if constexpr (TWL) {
        fft_t<C_, E, -1, 1, LdsSink, PAIR>(P.v, j, active, twl, slab, 1, lsink);
    } else {
        fft<C_, E, -1, LdsSink, PAIR>(P.v, j, active, tw_all, slab, 1, lsink);
    }
    __syncthreads();
    double2 *s0 = lds, *s1 = lds + LS;
    const int nthr = blockDim.x;
    if (wg != 0) {
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int k2 = t + G::NT * i;
            if (k2 >= C_) break;
            const int k2b = C_ - 1 - k2;
            double2 za = s0[lpad(k2)], zb = s1[lpad(k2b)];
            const int64_t pa = ra * C + k2, pb = rb * C + k2b;
            double2 xa, xb;
            if constexpr (PF) {
                pair_update<MODE>(za, zb, P.pW[i], P.pLa[i], P.pLb[i], sp, &xa, &xb);
            } else {
                const double2 La = MODE != 2 ? ldc(spec, pa) : make_double2(0.0, 0.0);
                const double2 Lb = MODE != 2 ? ldc(spec, pb) : make_double2(0.0, 0.0);
                pair_update<MODE>(za, zb, twL(ra + R * k2), La, Lb, sp, &xa, &xb);
            }
            if constexpr (MODE == 2) {
                spec_out[pa] = xa;
                spec_out[pb] = xb;
            } else {
                s0[lpad(k2)] = za;
                s1[lpad(k2b)] = zb;
            }
        }
    } else {
        // rows 0 and R/2 pair with themselves.
        const int ntask = C_ + 1;
        for (int task = t; task < ntask; task += nthr) {
            if (task <= C_ / 2) {
                const int k2 = task;
                const int k2b = (C_ - k2) & (C_ - 1);
                double2 za = s0[lpad(k2)], zb = s0[lpad(k2b)];
                const int64_t k = R * k2;
                double2 La = make_double2(0, 0), Lb = make_double2(0, 0);
                if constexpr (MODE != 2) {
                    if (k2 == 0) {
                        const double2 L0 = ldc(spec, 0);
                        La = make_double2(L0.x, 0.0);  // lambda_0
                        Lb = make_double2(L0.y, 0.0);  // lambda_N
                    } else {
                        La = ldc(spec, k2);
                        Lb = ldc(spec, k2b);
                    }
                }
                const double2 w = k2 == 0 ? make_double2(1.0, 0.0) : twL(k);
                double2 xa, xb;
                pair_update<MODE>(za, zb, w, La, Lb, sp, &xa, &xb);
                if constexpr (MODE == 2) {
                    if (k2 == 0) {
                        spec_out[0] = make_double2(xa.x, xb.x);
                    } else {
                        spec_out[k2] = xa;
                        spec_out[k2b] = xb;
                    }
                } else {
                    s0[lpad(k2)] = za;
                    if (k2 != 0 && k2b != k2) s0[lpad(k2b)] = zb;
                }
            } else {
                const int k2 = task - (C_ / 2 + 1);
                const int k2b = C_ - 1 - k2;
                double2 za = s1[lpad(k2)], zb = s1[lpad(k2b)];
                const int64_t k = R / 2 + R * k2;
                const int64_t pa = (R / 2) * C + k2, pb = (R / 2) * C + k2b;
                double2 La = make_double2(0, 0), Lb = make_double2(0, 0);
                if constexpr (MODE != 2) {
                    La = ldc(spec, pa);
                    Lb = ldc(spec, pb);
                }
                double2 xa, xb;
                pair_update<MODE>(za, zb, twL(k), La, Lb, sp, &xa, &xb);
                if constexpr (MODE == 2) {
                    spec_out[pa] = xa;
                    spec_out[pb] = xb;
                } else {
                    s1[lpad(k2)] = za;
                    s1[lpad(k2b)] = zb;
                }
            }
        }
    }
    if constexpr (MODE == 2) return;
    __syncthreads();
    double2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = active ? slab[lpad(j + T * m)] : make_double2(0.0, 0.0);
    __syncthreads();
    RowSinkT<CS> rsink{Y, row * C};
    if constexpr (TWL) {
        fft_t<C_, E, 1, 1, RowSinkT<CS>, PAIR>(v, j, active, twl, slab, 1, rsink);
    } else {
        fft<C_, E, 1, RowSinkT<CS>, PAIR>(v, j, active, tw_all, slab, 1, rsink);
    }
}

// A middle pass over NPAIR row pairs per workgroup (pairs NPAIR*b ...).  With
// two, the second pair's loads are issued before the first pair's transform,
// so its memory traffic overlaps the first pair's LDS and arithmetic work,
// and the first pair's stores overlap the second's transform.
template <int C_, int EMAX, int MODE, class CS, int NPAIR = 1>
__device__ __forceinline__ void mid_body(int64_t R, CS *Y, const CS *spec, double2 *spec_out, Tw2 twL,
                                         SymParams sp, const double2 *__restrict__ tw_all, DevScalars *sc, int pred) {
    if (skip(pred, sc)) return;
    using G = MidGeo<C_, EMAX>;
    constexpr int LS = G::LS;
    // stage twiddles in LDS when both rows and the table fit in 160 KiB
    constexpr bool TWL = C_ > G::E && (2 * LS + C_) * 16 <= 163840;
    __shared__ double2 lds[2 * LS];
    __shared__ double2 twl[TWL ? C_ : 1];
    using MP = MidPair<C_, EMAX, MODE, CS>;
    MP A;
    A.fetch((int64_t)NPAIR * blockIdx.x, R, Y, spec, twL);
    if constexpr (NPAIR == 2) {
        MP B;
        B.fetch(2 * (int64_t)blockIdx.x + 1, R, Y, spec, twL);
        // the first barrier inside the transform orders these writes before any use
        if constexpr (TWL) stage_twiddles<C_>(twl, tw_all, threadIdx.x, G::NT);
        mid_transform<C_, EMAX, MODE, CS, TWL>(A, R, Y, spec, spec_out, twL, sp, tw_all, lds, twl);
        __syncthreads();  // the slabs are free again
        mid_transform<C_, EMAX, MODE, CS, TWL>(B, R, Y, spec, spec_out, twL, sp, tw_all, lds, twl);
    } else {
        if constexpr (TWL) stage_twiddles<C_>(twl, tw_all, threadIdx.x, G::NT);
        mid_transform<C_, EMAX, MODE, CS, TWL>(A, R, Y, spec, spec_out, twL, sp, tw_all, lds, twl);
    }
}

template <int C_, int EMAX, int MODE, class CS, int NPAIR = 1>
__global__ void __launch_bounds__((MidGeo<C_, EMAX>::NT)) k_mid(int64_t R, CS *Y, const CS *spec,
                                                              double2 *spec_out, Tw2 twL, SymParams sp,
                                                              const double2 *__restrict__ tw_all, DevScalars *sc,
                                                              int pred) {
    mid_body<C_, EMAX, MODE, CS, NPAIR>(R, Y, spec, spec_out, twL, sp, tw_all, sc, pred);
}

struct MidDesc {
    int64_t R;
    double2 *Y;
    const double2 *spec;
    double2 *spec_out;
    Tw2 twL;
    SymParams sp;
    DevScalars *sc;
};

template <int C_, int EMAX, int MODE>
__global__ void __launch_bounds__((MidGeo<C_, EMAX>::NT)) k_mid_b(const MidDesc *__restrict__ d,
                                                                const int *__restrict__ act,
                                                                const double2 *__restrict__ tw_all, int pred) {
    const MidDesc D = d[batch_member(act)];
    mid_body<C_, EMAX, MODE, double2>(D.R, D.Y, D.spec, D.spec_out, D.twL, D.sp, tw_all, D.sc, pred);
}

// ---------------------------------------------------------------------------
// Complex transforms (Bluestein's chirp-z DFT of arbitrary length n, used to
// build the Strang preconditioner when n is not a power of two).
// ---------------------------------------------------------------------------
// Complex loader: v[m] = z[m] (or zr[m] real) for m < nv, else 0, optionally
// times conj(chirp[m]).
struct InCplx {
    const double2 *z;
    const double *zr;
    const double2 *chirp;
    int64_t nv, C;
    static constexpr int NL = 2;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *raw) const {
        const int64_t m = row * C + col;
        if (m >= nv) return;
        raw[0] = z ? z[m] : make_double2(zr[m], 0.0);
        if (chirp) raw[1] = chirp[m];
    }
    __device__ __forceinline__ double2 finish(int row, int64_t col, const double2 *raw) const {
        const int64_t m = row * C + col;
        if (m >= nv) return make_double2(0.0, 0.0);
        return chirp ? cmul(raw[0], cconj(raw[1])) : raw[0];
    }
};

// Complex store: z[m] = val (optionally times conj(chirp[m])) for m < nv.
struct OutCplx {
    double2 *z;
    const double2 *chirp;
    int64_t nv, C;
    static constexpr int NACC = 0, NPRE = 1;
    __device__ void prep(const DevScalars *) {}
    __device__ __forceinline__ void fetch(int row, int64_t col, double2 *pre) const {
        const int64_t m = row * C + col;
        if (m < nv && chirp) pre[0] = chirp[m];
    }
    __device__ __forceinline__ void store(int row, int64_t col, double2 val, double *, const double2 *pre) const {
        const int64_t m = row * C + col;
        if (m < nv) z[m] = chirp ? cmul(val, cconj(pre[0])) : val;
    }
    __device__ void final(const double *, DevScalars *) const {}
    double *partials;
};

template <int C_, int EMAX> struct RowGeo {
    static constexpr int E0 = Geo<C_, EMAX>::E;
    static constexpr int E = (C_ / E0 > 1024) ? C_ / 1024 : E0;
    static constexpr int T = C_ / E;
    static constexpr int NT = (T + 63) / 64 * 64;
    static constexpr int LS = lpad_size(C_);
};

// One row of a complex R x C transform per workgroup.  MODE 3: forward row
// FFT, multiply by the stored spectrum (native order), inverse row FFT (the
// middle of a circular convolution).  MODE 4: forward row FFT, spectrum out.
template <int C_, int EMAX, int MODE>
__device__ __forceinline__ void row_body(double2 *Y, const double2 *spec, double2 *spec_out,
                                         const double2 *__restrict__ tw_all) {
    using G = RowGeo<C_, EMAX>;
    constexpr int E = G::E, T = G::T;
    __shared__ double2 lds[G::LS];
    const int64_t row = blockIdx.x;
    const int j = threadIdx.x;
    const bool active = j < T;
    double2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = active ? Y[row * C_ + j + T * m] : make_double2(0.0, 0.0);
    LdsSink lsink{lds, 1};
    fft<C_, E, -1>(v, j, active, tw_all, lds, 1, lsink);
    __syncthreads();
    if constexpr (MODE == 4) {
        if (active) {
#pragma unroll
            for (int m = 0; m < E; ++m) spec_out[row * C_ + j + T * m] = lds[lpad(j + T * m)];
        }
        return;
    } else {
#pragma unroll
        for (int m = 0; m < E; ++m)
            v[m] = active ? cmul(lds[lpad(j + T * m)], spec[row * C_ + j + T * m]) : make_double2(0.0, 0.0);
        __syncthreads();
        RowSink rsink{Y, row * C_};
        fft<C_, E, 1>(v, j, active, tw_all, lds, 1, rsink);
    }
}

template <int C_, int EMAX, int MODE>
__global__ void __launch_bounds__((RowGeo<C_, EMAX>::NT)) k_row(double2 *Y, const double2 *spec, double2 *spec_out,
                                                                const double2 *__restrict__ tw_all) {
    row_body<C_, EMAX, MODE>(Y, spec, spec_out, tw_all);
}

struct RowDesc {
    double2 *Y;
    const double2 *spec;
    double2 *spec_out;
};

template <int C_, int EMAX, int MODE>
__global__ void __launch_bounds__((RowGeo<C_, EMAX>::NT)) k_row_b(const RowDesc *__restrict__ d,
                                                                  const int *__restrict__ act,
                                                                  const double2 *__restrict__ tw_all) {
    const RowDesc D = d[batch_member(act)];
    row_body<C_, EMAX, MODE>(D.Y, D.spec, D.spec_out, tw_all);
}

// x = fallback where the device scalars say the last restart's x did not
// beat the right-hand side's initial guess (learned warm start).
__global__ void k_keep_better(double *__restrict__ x, const double *__restrict__ fallback, int64_t n,
                              DevScalars *sc) {
    const int keep = sc->better;
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->netkept = keep;  // no block reads netkept
    if (keep) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = fallback[i];
}

// FP32 copy (round to nearest) of a complex FP64 array.
__global__ void k_to_f32(const double2 *src, float2 *dst, int64_t m) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x)
        dst[k] = make_float2((float)src[k].x, (float)src[k].y);
}

// Chirp b_m = exp(i pi m^2 / n), m < n (m^2 reduced modulo 2n exactly).
__global__ void k_chirp(double2 *b, int64_t n) {
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < n; m += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = (m * m) % (2 * n);
        double sn, cs;
        sincospi((double)q / (double)n, &sn, &cs);
        b[m] = make_double2(cs, sn);
    }
}

// Circular arrangement of the chirp for a length-L convolution:
// bb[l] = bb[L-l] = scale * b_l (1 <= l < n), bb[0] = scale * b_0, else 0.
__global__ void k_chirp_embed(const double2 *b, int64_t n, int64_t L, double scale, double2 *bb) {
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < L; m += (int64_t)gridDim.x * blockDim.x) {
        double2 v = make_double2(0.0, 0.0);
        if (m < n) v = cscale(b[m], scale);
        else if (L - m < n) v = cscale(b[L - m], scale);
        bb[m] = v;
    }
}

// Strang preconditioner at one level: w_k = conj(1 / lambda_k) with
// lambda_k = s0 + cre Re(Ls_k) + i (cim Im(Ls_k) + cq sin(2 pi k / n)).
__global__ void k_pc_column(const double2 *Ls, int64_t n, SymParams sp, double2 *w) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        double sn, cs;
        sincospi(2.0 * (double)k / (double)n, &sn, &cs);
        const double2 L = Ls[k];
        const double2 lam = make_double2(fma(sp.cre, L.x, sp.s0), fma(sp.cim, L.y, sp.cq * sn));
        const double d = 1.0 / fma(lam.x, lam.x, lam.y * lam.y);
        w[k] = make_double2(lam.x * d, lam.y * d);  // conj(1/lam) = lam / |lam|^2
    }
}

// First column of the length-L embedding of the circulant with first column
// p_m = Re(Wt_m) / n (the inverse Strang circulant): lag l -> p[l mod n].
__global__ void k_pc_embed(const double2 *Wt, int64_t n, int64_t L, double *e) {
    const double inv = 1.0 / (double)n;
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < L; m += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        if (m < n) v = Wt[m].x * inv;
        else if (L - m < n) v = Wt[n - (L - m)].x * inv;
        e[m] = v;
    }
}

// ---------------------------------------------------------------------------
// History sum of (3.3):  H_L = kappa * sum_{s=0}^{L-1} c_{L-s}^(L) (u^{s+1} - u^s)
// with c_L^(L) = clast[L] (s = 0) and c_m^(L) = cbase[m] (1 <= m <= L-1).
// The kernels form every term but the newest level's,
//   P_L = kappa * [ sum_{s=0}^{L-2} c_{L-s} (u^{s+1} - u^s) - c_1 u^{L-1} ],
// so that H_L = P_L + kappa c_1 u^L and the right-hand side folds
// kappa c_1 u^L into its coefficient of u^L.
//
// Blocked evaluation.  The weights depend on L - s only (and on L through the
// s = 0 weight), so one pass over the stored levels can serve several future
// levels.  Levels are grouped in blocks of HB from level 1; for a block that
// starts at level b and a level L of it,
//   P_L = Q_L + kappa * [ sum_{s=b-1}^{L-2} c_{L-s} (u^{s+1} - u^s) - c_1 u^{L-1} ]   (L > b),
//   Q_L = kappa * sum_{s=0}^{b-2} c_{L-s}^(L) (u^{s+1} - u^s),      P_b = Q_b - kappa c_1^(b) u^{b-1}.
// The sweep (k_hist_sweep) reads u^0..u^{b-1} once and writes Q_L for every
// level of the block (P_b for the first); the catch-up (k_hist_catch) of level
// L > b reads the L - b + 1 newest levels u^{b-1}..u^{L-1} and Q_L and writes
// P_L.  Per level that is about 1/HB of the stored levels instead of all of
// them.  The arithmetic of each element does not depend on the grid, so
// every path (side stream, main stream, batch) gives bitwise the same sums.
// Each lane streams two adjacent unknowns through the stored levels (rows of
// U are ldu >= n doubles apart, ldu even; an odd n reads the zero pad).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double hist_c(int s, int j, const double *cbase, double clast) {
    return s == 0 ? clast : cbase[j - s];
}

constexpr int HB = 8;  // levels per history block

struct HistBlock {
    double clast[HB];  // clast[b + l]: the s = 0 weight of level b + l
    double c1b;        // c_1^(b)
    int b, nl;         // first level of the block, levels in it (<= HB)
};

// The sweep reads every stored level once per block; with TSF_HIST_NT its
// loads carry the non-temporal hint, so that the stream does not displace the
// solve's working set from the caches.
#ifndef TSF_HIST_NT
#define TSF_HIST_NT 0
#endif
__device__ __forceinline__ double2 ld_sweep(const double *p) {
#if TSF_HIST_NT
    typedef double v2d __attribute__((ext_vector_type(2)));
    const v2d v = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(p));
    return make_double2(v.x, v.y);
#else
    return *reinterpret_cast<const double2 *>(p);
#endif
}

__device__ __forceinline__ void hist_sweep_pair(const double *__restrict__ U, int64_t ldu,
                                                const double *__restrict__ cbase, const HistBlock &hb, double kappa,
                                                double *__restrict__ Q, int64_t i) {
    double2 prev = *reinterpret_cast<const double2 *>(U + i);
    double2 acc[HB];
#pragma unroll
    for (int l = 0; l < HB; ++l) acc[l] = make_double2(0.0, 0.0);
    const int b = hb.b, nl = hb.nl;
    auto add = [&](int s, double2 x) {
        const double2 d = make_double2(x.x - prev.x, x.y - prev.y);
#pragma unroll
        for (int l = 0; l < HB; ++l) {
            if (l < nl) {
                const double c = s == 0 ? hb.clast[l] : cbase[b + l - s];
                acc[l].x = fma(c, d.x, acc[l].x);
                acc[l].y = fma(c, d.y, acc[l].y);
            }
        }
        prev = x;
    };
    int s = 0;
    const int full = b - 1;  // differences s = 0..b-2
    constexpr int U8 = 8;    // eight levels in flight per step
    for (; s + U8 <= full; s += U8) {
        double2 x[U8];
#pragma unroll
        for (int q = 0; q < U8; ++q) x[q] = ld_sweep(U + (int64_t)(s + 1 + q) * ldu + i);
#pragma unroll
        for (int q = 0; q < U8; ++q) add(s + q, x[q]);
    }
    for (; s < full; ++s) add(s, ld_sweep(U + (int64_t)(s + 1) * ldu + i));
    acc[0].x = fma(-hb.c1b, prev.x, acc[0].x);  // prev = u^{b-1}
    acc[0].y = fma(-hb.c1b, prev.y, acc[0].y);
#pragma unroll
    for (int l = 0; l < HB; ++l)
        if (l < nl)
            *reinterpret_cast<double2 *>(Q + (int64_t)l * ldu + i) = make_double2(kappa * acc[l].x, kappa * acc[l].y);
}

__device__ __forceinline__ void hist_catch_pair(const double *__restrict__ U, int64_t ldu,
                                                const double *__restrict__ cbase, int b, int L, double clastL,
                                                double c1L, double kappa, const double *__restrict__ QL,
                                                double *__restrict__ P, int64_t i) {
    double2 prev = *reinterpret_cast<const double2 *>(U + (int64_t)(b - 1) * ldu + i);
    const double2 q = *reinterpret_cast<const double2 *>(QL + i);
    double2 acc = make_double2(0.0, 0.0);
    for (int s = b - 1; s <= L - 2; ++s) {
        const double2 x = *reinterpret_cast<const double2 *>(U + (int64_t)(s + 1) * ldu + i);
        const double c = hist_c(s, L, cbase, clastL);
        acc.x = fma(c, x.x - prev.x, acc.x);
        acc.y = fma(c, x.y - prev.y, acc.y);
        prev = x;
    }
    acc.x = fma(-c1L, prev.x, acc.x);  // prev = u^{L-1}
    acc.y = fma(-c1L, prev.y, acc.y);
    *reinterpret_cast<double2 *>(P + i) = make_double2(fma(kappa, acc.x, q.x), fma(kappa, acc.y, q.y));
}

// Grid-stride over pairs: a small grid runs as a background job beside the solve.
__global__ void __launch_bounds__(256) k_hist_sweep(const double *__restrict__ U, int64_t n, int64_t ldu,
                                                    const double *__restrict__ cbase, HistBlock hb, double kappa,
                                                    double *__restrict__ Q) {
    for (int64_t i = 2 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x); i < n;
         i += 2 * (int64_t)gridDim.x * blockDim.x)
        hist_sweep_pair(U, ldu, cbase, hb, kappa, Q, i);
}

__global__ void __launch_bounds__(256) k_hist_catch(const double *__restrict__ U, int64_t n, int64_t ldu,
                                                    const double *__restrict__ cbase, int b, int L, double clastL,
                                                    double c1L, double kappa, const double *__restrict__ QL,
                                                    double *__restrict__ P) {
    for (int64_t i = 2 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x); i < n;
         i += 2 * (int64_t)gridDim.x * blockDim.x)
        hist_catch_pair(U, ldu, cbase, b, L, clastL, c1L, kappa, QL, P, i);
}

// Batched element-wise kernels: descriptor per instance (blockIdx.y), a
// grid-stride loop over that instance's length in blockIdx.x.  An instance
// with nothing to do at this level has n = 0.
struct HistDesc {
    const double *U;
    int64_t n, ldu;
    const double *cbase;
    HistBlock hb;     // sweep
    int L;            // catch-up level
    double clastL, c1L, kappa;
    const double *QL;
    double *out;      // Q (sweep) or P (catch-up)
};

__global__ void __launch_bounds__(256) k_hist_sweep_b(const HistDesc *__restrict__ d) {
    const HistDesc &D = d[blockIdx.y];
    for (int64_t i = 2 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x); i < D.n;
         i += 2 * (int64_t)gridDim.x * blockDim.x)
        hist_sweep_pair(D.U, D.ldu, D.cbase, D.hb, D.kappa, D.out, i);
}

__global__ void __launch_bounds__(256) k_hist_catch_b(const HistDesc *__restrict__ d) {
    const HistDesc &D = d[blockIdx.y];
    for (int64_t i = 2 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x); i < D.n;
         i += 2 * (int64_t)gridDim.x * blockDim.x)
        hist_catch_pair(D.U, D.ldu, D.cbase, D.hb.b, D.L, D.clastL, D.c1L, D.kappa, D.QL, D.out, i);
}

struct PcDesc {
    const double2 *Ls;
    double2 *w;
    const double2 *Wt;
    double *e;
    int64_t n, L;
    SymParams sp;
};

__global__ void k_pc_column_b(const PcDesc *__restrict__ d) {
    const PcDesc D = d[blockIdx.y];
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < D.n; k += (int64_t)gridDim.x * blockDim.x) {
        double sn, cs;
        sincospi(2.0 * (double)k / (double)D.n, &sn, &cs);
        const double2 L = D.Ls[k];
        const double2 lam = make_double2(fma(D.sp.cre, L.x, D.sp.s0), fma(D.sp.cim, L.y, D.sp.cq * sn));
        const double q = 1.0 / fma(lam.x, lam.x, lam.y * lam.y);
        D.w[k] = make_double2(lam.x * q, lam.y * q);
    }
}

__global__ void k_pc_embed_b(const PcDesc *__restrict__ d) {
    const PcDesc D = d[blockIdx.y];
    const double inv = 1.0 / (double)D.n;
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < D.L; m += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        if (m < D.n) v = D.Wt[m].x * inv;
        else if (D.L - m < D.n) v = D.Wt[D.n - (D.L - m)].x * inv;
        D.e[m] = v;
    }
}

// Convergence state of every instance of a batch, gathered for one host read:
// out[i] = (done, status, iter, 0).
__global__ void k_gather_done(DevScalars *const *__restrict__ scs, int count, int4 *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        const DevScalars *s = scs[i];
        out[i] = make_int4(s->done, s->status, s->iter, 0);
    }
}

// ---------------------------------------------------------------------------
// Plan-time kernels.
// ---------------------------------------------------------------------------

// Packed tables tw_P[m] = exp(-2 pi i m / P) for P = 2, 4, ..., PMAX.
__global__ void k_twiddle_packed(double2 *tw, int pmax_log2) {
    const int64_t total = (int64_t(1) << (pmax_log2 + 1)) - 2;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        // idx = (P - 2) + m with P the largest power of two such that P - 2 <= idx
        int lg = 1;
        while (((int64_t(1) << (lg + 1)) - 2) <= idx) ++lg;
        const int64_t P = int64_t(1) << lg;
        const int64_t m = idx - (P - 2);
        double s, c;
        sincospi(2.0 * (double)m / (double)P, &s, &c);
        tw[idx] = make_double2(c, -s);
    }
}

// Two-level table for exp(-2 pi i m / L): lo[e] = w(e), e < 2^shift;
// hi[e] = w(e * 2^shift), e < nhi.
__global__ void k_twiddle_tw2(double2 *lo, double2 *hi, int64_t L, int shift, int64_t nhi) {
    const int64_t nlo = int64_t(1) << shift;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < nlo + nhi;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = idx < nlo ? idx : (idx - nlo) << shift;
        // reduce m/L to [0, 1) exactly (L is a power of two)
        const double frac = (double)(m & (L - 1)) / (double)L;
        double s, c;
        sincospi(2.0 * frac, &s, &c);
        if (idx < nlo) lo[idx] = make_double2(c, -s);
        else hi[idx - nlo] = make_double2(c, -s);
    }
}

// g_k = prod_{i=1..k} (1 - (beta+1)/i), k = 0..K (Lemma 3 recurrence), by a
// single-workgroup chunked product scan.
__global__ void __launch_bounds__(1024) k_grunwald(double beta, int64_t K, double *g) {
    __shared__ double pre[1024];
    const int t = threadIdx.x;
    const int64_t tot = K + 1;
    const int64_t chunk = (tot + 1023) / 1024;
    const int64_t k0 = t * chunk, k1 = min(tot, k0 + chunk);
    double p = 1.0;
    for (int64_t k = k0; k < k1; ++k) p *= (k == 0) ? 1.0 : (1.0 - (beta + 1.0) / (double)k);
    pre[t] = p;
    __syncthreads();
    // inclusive Hillis-Steele product scan over the 1024 chunk products
    for (int d = 1; d < 1024; d <<= 1) {
        double other = t >= d ? pre[t - d] : 1.0;
        __syncthreads();
        pre[t] *= other;
        __syncthreads();
    }
    double run = t == 0 ? 1.0 : pre[t - 1];
    for (int64_t k = k0; k < k1; ++k) {
        run *= (k == 0) ? 1.0 : (1.0 - (beta + 1.0) / (double)k);
        g[k] = run;
    }
}

// omega_k = l1 g_k + l0 g_{k-1} + lm1 g_{k-2}  (Lemma 2), k = 0..K.
__global__ void k_wsgd(const double *g, int64_t K, double l1, double l0, double lm1, double *w) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= K; k += (int64_t)gridDim.x * blockDim.x) {
        double v = l1 * g[k];
        if (k >= 1) v = fma(l0, g[k - 1], v);
        if (k >= 2) v = fma(lm1, g[k - 2], v);
        w[k] = v;
    }
}

// First column of the length-L circulant embedding of W_beta:
// c_m = omega_{m+1} (m < n), c_{L-1} = omega_0, else 0.
__global__ void k_embed_column(const double *w, int64_t n, int64_t L, double *c) {
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < L; m += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        if (m < n) v = w[m + 1];
        if (m == L - 1) v += w[0];
        c[m] = v;
    }
}

// First column of T. Chan's optimal circulant of W_beta (the circulant nearest
// to W_beta in the Frobenius norm): c_k = ((n - k) t_k + k t_{k-n}) / n with
// t_lag = omega_{lag+1} for lag >= -1, else 0; t_{k-n} is nonzero only at
// k = n - 1 (lag -1, omega_0).
__global__ void k_tchan_column(const double *w, int64_t n, double *c) {
    const double inv = 1.0 / (double)n;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        double v = (double)(n - k) * w[k + 1];
        if (k == n - 1) v = fma((double)k, w[0], v);
        c[k] = v * inv;
    }
}

// First column of the Strang circulant s(W_beta): lag k for 0 <= k <= n/2,
// lag k - n otherwise; W has lags -1..n-1 with entry omega_{lag+1}.
__global__ void k_strang_column(const double *w, int64_t n, double *c) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t lag = k <= n / 2 ? k : k - n;
        c[k] = lag >= -1 ? w[lag + 1] : 0.0;
    }
}

// Columns of the length-L circulant embeddings of the four triangular
// Toeplitz factors of the Gohberg-Semencul formula (Sec. 3.1), from
// x = A^-1 e_1 and y = A^-1 e_n; lag m = i - k >= 0 sits at index m, lag
// m < 0 at L + m (L >= 2n keeps the two ranges apart):
//   which 0: L_p,  lags 0..n-1,      entry x_m;
//   which 1: R_p,  lags -(n-1)..0,   entry y_{n-1+m};
//   which 2: L0_p, lags 1..n-1,      entry y_{m-1};
//   which 3: R0_p, lags -(n-1)..-1,  entry x_{n+m}.
__global__ void k_gsf_column(const double *x, const double *y, int64_t n, int64_t L, int which, double *c) {
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < L; m += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        if (m < n) {
            if (which == 0) v = x[m];
            else if (which == 1 && m == 0) v = y[n - 1];
            else if (which == 2 && m >= 1) v = y[m - 1];
        } else if (L - m < n) {
            const int64_t lag = m - L;  // -(n-1) .. -1
            if (which == 1) v = y[n - 1 + lag];
            else if (which == 3) v = x[n + lag];
        }
        c[m] = v;
    }
}

// g = e_pos, x = 0, r = rt = e_pos (rows of ld values, pads zero), and the
// device scalars of a fresh CGS solve of A x = g to |r| <= tol |g| (|g| = 1),
// as the right-hand side pass leaves them.
__global__ void k_unit_rhs(double *g, double *x, double *r, double *rt, int64_t ld, int64_t pos, double tol,
                           DevScalars *sc) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ld; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = i == pos ? 1.0 : 0.0;
        g[i] = v;
        x[i] = 0.0;
        r[i] = v;
        rt[i] = v;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->gnorm2 = 1.0;
        sc->rnorm2 = 1.0;
        sc->rho = 1.0;
        sc->rho_prev = 1.0;
        sc->beta = 0.0;
        sc->alpha = 0.0;
        sc->tol2 = tol * tol;
        sc->iter = 0;
        sc->fresh = 1;
        sc->aux0 = 1.0;
        sc->r0sq = 1.0;
        sc->status = ST_OK;
        sc->checked = 0;
        sc->nchecks = 0;
        sc->done = 0;
    }
}

// Native-order spectrum (position k1*C + k2 <-> frequency k1 + R*k2, X_0/X_N
// packed at position 0) to natural order k = 0..N.
__global__ void k_spec_export(const double2 *spec, int64_t R, int64_t C, double2 *out) {
    const int64_t N = R * C;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= N; k += (int64_t)gridDim.x * blockDim.x) {
        double2 v;
        if (k == 0) v = make_double2(spec[0].x, 0.0);
        else if (k == N) v = make_double2(spec[0].y, 0.0);
        else v = spec[(k % R) * C + k / R];
        out[k] = v;
    }
}

__global__ void k_copy(const double *__restrict__ src, double *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

template <class S>
__global__ void k_fill(S *__restrict__ dst, S v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = v;
}

}  // namespace tsf
