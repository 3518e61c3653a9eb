// fft_core.hpp -- register/LDS Stockham FFT building blocks for gfx950.
//
// A transform of length P (power of two, 2..4096) is held by T = P/E lanes,
// each lane owning E complex values (E is a tuning parameter: 4, 8 or 16;
// fewer values per lane means more waves per SIMD to hide memory latency).
// Lane j holds the elements at positions j + T*m, m = 0..E-1 ("canonical
// layout").  One Stockham stage of radix RAD combines, for butterfly index
// bf, the inputs bf + (P/RAD)*r; with bf = j + T*q these are exactly the
// lane's own values v[q + (E/RAD)*r], so every stage starts from registers.
// The outputs of a stage go to the self-sorting position
// (bf/NS)*NS*RAD + bf%NS + r*NS: to LDS for all but the last stage, and to a
// caller-supplied sink for the last one (global memory, or LDS in natural
// frequency order).
//
// Twiddles come from a table tw_P[m] = exp(-2 pi i m / P) (FP64, built on the
// device at plan time) for the power-of-two multiples of a butterfly's base
// angle, and as products of two of those for the rest; the inverse transform
// uses conjugates.  Butterfly
// constants are exact algebraic values of cos/sin(2 pi k/16).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsf {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// multiply by -i (DIR < 0) or +i (DIR > 0)
template <int DIR> __device__ __forceinline__ double2 mul_i(double2 a) {
    return DIR < 0 ? make_double2(a.y, -a.x) : make_double2(-a.y, a.x);
}

// exp(DIR * 2 pi i * K / 16) applied to a, K compile-time in [0, 16).
template <int K, int DIR> __device__ __forceinline__ double2 rot16(double2 a) {
    constexpr double C1 = 0.92387953251128675613;  // cos(pi/8)
    constexpr double S1 = 0.38268343236508977173;  // sin(pi/8)
    constexpr double H = 0.70710678118654752440;   // sqrt(1/2)
    constexpr int k = K & 15;
    if constexpr (k == 0) return a;
    else if constexpr (k == 4) return mul_i<DIR>(a);
    else if constexpr (k == 8) return make_double2(-a.x, -a.y);
    else if constexpr (k == 12) return mul_i<-DIR>(a);
    else {
        constexpr double cs[16] = {1, C1, H, S1, 0, -S1, -H, -C1, -1, -C1, -H, -S1, 0, S1, H, C1};
        constexpr double sn[16] = {0, S1, H, C1, 1, C1, H, S1, 0, -S1, -H, -C1, -1, -C1, -H, -S1};
        const double c = cs[k];
        const double s = DIR > 0 ? sn[k] : -sn[k];
        return make_double2(fma(a.x, c, -a.y * s), fma(a.x, s, a.y * c));
    }
}

// In-place DFT of length R (1, 2, 4, 8, 16) on a[0..R), natural order in and
// out, kernel exp(DIR * 2 pi i jk / R).  Radix-2 decimation in time, unrolled.
template <int R, int DIR> struct Dft {
    static __device__ __forceinline__ void run(double2 *a) {
        if constexpr (R == 1) {
            return;
        } else if constexpr (R == 2) {
            double2 t = a[1];
            a[1] = csub(a[0], t);
            a[0] = cadd(a[0], t);
        } else {
            constexpr int H = R / 2;
            double2 e[H], o[H];
#pragma unroll
            for (int i = 0; i < H; ++i) { e[i] = a[2 * i]; o[i] = a[2 * i + 1]; }
            Dft<H, DIR>::run(e);
            Dft<H, DIR>::run(o);
            apply<0>(a, e, o);
        }
    }
    template <int K> static __device__ __forceinline__ void apply(double2 *a, const double2 *e, const double2 *o) {
        if constexpr (K < R / 2) {
            double2 t = rot16<K * (16 / R), DIR>(o[K]);
            a[K] = cadd(e[K], t);
            a[K + R / 2] = csub(e[K], t);
            apply<K + 1>(a, e, o);
        }
    }
};

// Geometry of a length-P transform at (at most) EMAX values per lane.
template <int P, int EMAX> struct Geo {
    static constexpr int E = P < EMAX ? P : EMAX;  // values per lane
    static constexpr int T = P / E;               // lanes per transform
};

// LDS index padding: one spare slot every 16 elements breaks the bank
// pattern of the power-of-two strides in the stage write-back.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lpad_size(int P) { return P + (P >> 4) + 1; }

// Offset of the length-P sub-table inside the packed twiddle array
// (tables for P = 2, 4, 8, ... are stored back to back).
__host__ __device__ constexpr int tw_offset(int P) { return P - 2; }

// twP[m * TS] = exp(-2 pi i m / P): the twiddle table of a length-P transform
// (TS > 1 when a longer table, e.g. one staged in LDS, is shared).
template <int P, int E, int RAD, int NS, int DIR, int TS>
__device__ __forceinline__ void stage_bfly(double2 (&v)[E], int j, const double2 *twP) {
    constexpr int NB = E / RAD;
    constexpr int T = P / E;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        double2 a[RAD];
#pragma unroll
        for (int r = 0; r < RAD; ++r) a[r] = v[q + NB * r];
        if constexpr (NS > 1) {
            const int bf = j + T * q;
            const int k = bf & (NS - 1);
            constexpr int STRIDE = P / (NS * RAD);
            // w^r for the power-of-two r from the table, the others as
            // products of two of those (w^3 = w^2 w, w^5 = w^4 w, ...): fewer
            // table reads for about one more rounding per derived twiddle
            double2 w[RAD];
#pragma unroll
            for (int r = 1; r < RAD; r *= 2) w[r] = twP[r * k * (STRIDE * TS)];
#pragma unroll
            for (int r = 3; r < RAD; ++r) {
                const int hb = 1 << (31 - __builtin_clz(r));
                if (hb != r) w[r] = cmul(w[hb], w[r - hb]);
            }
#pragma unroll
            for (int r = 1; r < RAD; ++r) {
                double2 wr = w[r];
                if (DIR > 0) wr.y = -wr.y;
                a[r] = cmul(a[r], wr);
            }
        }
        Dft<RAD, DIR>::run(a);
#pragma unroll
        for (int r = 0; r < RAD; ++r) v[q + NB * r] = a[r];
    }
}

// Runs the stages of a length-P transform from sub-length NS upwards on the
// canonical register layout.  Intermediate results are exchanged through the
// LDS slab `lds` (element p at lds[lpad(p) * LS]; several transforms may
// share a slab, interleaved with stride LS).  The outputs of the last stage
// are handed to sink(pos, value, slot) (natural frequency order pos; slot is
// the register index m of the value, see LastStage).  Every lane
// of the workgroup must call this (it contains barriers); lanes with
// active == false only take part in the barriers.
// Exchange of one value between partner lanes of a wave, register to register
// (DPP, no LDS): lanes l and l ^ 8 for SD = 8 (row rotation by 8 within each
// row of 16 lanes), lanes l and l ^ 1 for SD = 1 (quad permutation [1,0,3,2]).
// Every lane of the wave must execute it.
template <int SD> __device__ __forceinline__ double swap_lane_pair(double x) {
    static_assert(SD == 1 || SD == 8, "partner lanes 1 or 8 apart");
    constexpr int CTRL = SD == 8 ? 0x128 : 0xB1;
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int SD> __device__ __forceinline__ double2 swap_lane_pair(double2 v) {
    return make_double2(swap_lane_pair<SD>(v.x), swap_lane_pair<SD>(v.y));
}

// Paired layout of a length-P transform at E = 8 values per lane whose last
// Stockham stage is radix 2 (P = 2 * 8^k, so T = P/8 is 2, 16 or 128): that
// stage combines the outputs of logical lanes j and j + T/2.  When those two
// logical lanes sit in partner hardware lanes (paired_lane), the stage runs on
// registers with a lane swap instead of a round trip through LDS between two
// barriers.  In a row transform (one transform per T lanes) with T >= 16 the
// hardware lanes of each row of 16 hold 8 consecutive logical lanes and their
// 8 partners, so every group of 8 lanes still reads or writes one whole
// 128-byte line of a row; for T = 2 the mapping is the identity and the
// partners are adjacent (swap distance 1).
template <int P, int E> struct Paired {
    static constexpr bool pow8(int q) {
        while (q > 1 && q % 8 == 0) q /= 8;
        return q == 1;
    }
    static constexpr bool OK = E == 8 && P >= 16 && pow8(P / 2) && (P / E == 2 || (P / E) % 16 == 0);
};
template <int T> __device__ __forceinline__ int paired_lane(int u) {
    if constexpr (T >= 16) return ((u >> 4) << 3) + (u & 7) + ((u & 8) ? T / 2 : 0);
    else return u;
}

// The last, radix-2 stage in the paired layout.  After the preceding radix-8
// stage (sub-length T/2), slot r of logical lane j < T/2 holds position
// p = j + (T/2) r and slot r of lane j + T/2 holds p + P/2; the butterfly is
// y_p = x_p + w^p x_{p+P/2}, y_{p+P/2} = x_p - w^p x_{p+P/2}, w = exp(DIR 2 pi i / P).
template <int P, int E, int DIR, int TS, int SD, class Sink>
__device__ __forceinline__ void pair_stage(double2 (&v)[E], int j, bool active, const double2 *twP, Sink &sink) {
    constexpr int T = P / E, H = T / 2;
    const bool hi = j >= H;
    const int jl = hi ? j - H : j;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int p = jl + H * r;
        double2 w = twP[p * TS];
        if (DIR > 0) w.y = -w.y;
        const double2 sv = hi ? cmul(v[r], w) : v[r];  // what this lane contributes
        const double2 o = swap_lane_pair<SD>(sv);     // the partner's contribution
        const double2 y = hi ? csub(o, sv) : cadd(v[r], o);
        if (active) sink(hi ? p + P / 2 : p, y, r);
    }
}

// PAIR != 0: the transform runs in the paired layout (see Paired), with
// partner lanes PAIR (1 or 8) hardware lanes apart; every lane of each wave
// must call.
// Sinks with a prefetch() hook get it called before the exchange that
// precedes the last stage, so that the operands their stores combine with
// are in flight during that exchange but do not occupy registers across the
// whole transform.
template <class T, class = void> struct HasPrefetch {
    static constexpr bool value = false;
};
template <class T> struct HasPrefetch<T, decltype(void(static_cast<T *>(nullptr)->prefetch()))> {
    static constexpr bool value = true;
};

template <int P, int E, int NS, int DIR, int TS, class Sink, int PAIR = 0>
__device__ __forceinline__ void fft_stages(double2 (&v)[E], int j, bool active, const double2 *twP, double2 *lds,
                                           int LS, Sink &sink) {
    constexpr int T = P / E;
    constexpr int REM = P / NS;
    constexpr int RAD = REM >= E ? E : REM;
    constexpr int NB = E / RAD;
    stage_bfly<P, E, RAD, NS, DIR, TS>(v, j, twP);
    if constexpr (PAIR && NS * RAD * 2 == P) {
        static_assert(RAD == E && NB == 1 && NS == T / 2, "paired layout: radix-8 stage before the radix-2 one");
        pair_stage<P, E, DIR, TS, PAIR>(v, j, active, twP, sink);
    } else if constexpr (NS * RAD == P) {
        if (active) {
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int bf = j + T * q;
                const int base = (bf & ~(NS - 1)) * RAD + (bf & (NS - 1));
#pragma unroll
                for (int r = 0; r < RAD; ++r) sink(base + r * NS, v[q + NB * r], q + NB * r);
            }
        }
    } else {
        constexpr int NS2 = NS * RAD;
        constexpr int RAD2 = P / NS2 >= E ? E : P / NS2;
        if constexpr (HasPrefetch<Sink>::value && NS2 * RAD2 == P) sink.prefetch();
        if (active) {
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int bf = j + T * q;
                const int base = (bf & ~(NS - 1)) * RAD + (bf & (NS - 1));
#pragma unroll
                for (int r = 0; r < RAD; ++r) lds[lpad(base + r * NS) * LS] = v[q + NB * r];
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = lds[lpad(j + T * m) * LS];
        }
        __syncthreads();
        fft_stages<P, E, NS * RAD, DIR, TS, Sink, PAIR>(v, j, active, twP, lds, LS, sink);
    }
}

// Where the last stage of a length-P transform at E values per lane puts its
// outputs: value slot m of lane j goes to natural-order position pos(j, m).
// Callers use it to fetch, before the transform starts, the operands that the
// sink will combine with each output (so no load waits behind the stores).
template <int P, int E> struct LastStage {
    static constexpr int rad_at(int ns) { return (P / ns >= E) ? E : P / ns; }
    static constexpr int ns_last() {
        int ns = 1;
        while (ns * rad_at(ns) < P) ns *= rad_at(ns);
        return ns;
    }
    static constexpr int NS = ns_last(), RAD = rad_at(NS), NB = E / RAD, T = P / E;
    static __device__ __forceinline__ int pos(int j, int m) {
        const int q = m % NB, r = m / NB;
        const int bf = j + T * q;
        return (bf & ~(NS - 1)) * RAD + (bf & (NS - 1)) + r * NS;
    }
};

// Transform with twiddles from the packed global table.
template <int P, int E, int DIR, class Sink, int PAIR = 0>
__device__ __forceinline__ void fft(double2 (&v)[E], int j, bool active, const double2 *__restrict__ tw_all,
                                    double2 *lds, int LS, Sink &sink) {
    fft_stages<P, E, 1, DIR, 1, Sink, PAIR>(v, j, active, tw_all + tw_offset(P), lds, LS, sink);
}

// Transform with twiddles from a table of length P * TS (typically staged in
// LDS at kernel start, so no stage waits on a global load).
template <int P, int E, int DIR, int TS, class Sink, int PAIR = 0>
__device__ __forceinline__ void fft_t(double2 (&v)[E], int j, bool active, const double2 *tw, double2 *lds, int LS,
                                      Sink &sink) {
    fft_stages<P, E, 1, DIR, TS, Sink, PAIR>(v, j, active, tw, lds, LS, sink);
}

// Cooperative copy of the length-P twiddle table into LDS (P entries).
template <int P>
__device__ __forceinline__ void stage_twiddles(double2 *dst, const double2 *__restrict__ tw_all, int t, int nt) {
    const double2 *src = tw_all + tw_offset(P);
    for (int i = t; i < P; i += nt) dst[i] = src[i];
}

// Sink writing the transform in natural order into an LDS slab.
struct LdsSink {
    double2 *lds;
    int LS;
    __device__ __forceinline__ void operator()(int pos, double2 val, int) const { lds[lpad(pos) * LS] = val; }
};

// Two-level twiddle table for exp(-2 pi i m / L), m < L:
// w(m) = hi[m >> shift] * lo[m & ((1 << shift) - 1)].
struct Tw2 {
    const double2 *lo;
    const double2 *hi;
    int shift;
    __device__ __forceinline__ double2 operator()(int64_t m) const {
        return cmul(hi[m >> shift], lo[m & ((int64_t(1) << shift) - 1)]);
    }
    // the two table entries of w(m), loaded without combining them
    __device__ __forceinline__ void fetch(int64_t m, double2 *hl) const {
        hl[0] = hi[m >> shift];
        hl[1] = lo[m & ((int64_t(1) << shift) - 1)];
    }
};

// Four-step twiddles w(2 (r0 + S m) c), m = 0, 1, 2, ..., of one lane's
// values (their rows form an arithmetic progression) as a running product
// w(2 r0 c) * w(2 S c)^m: two table lookups per lane instead of two per
// value.  Each step adds about one rounding unit, so after the at most 15
// steps of a lane the twiddle errs by a few units, the size of the FFT's own
// rounding.  next() returns the current twiddle and advances.
struct TwRec {
    double2 w, step;
    __device__ __forceinline__ void init(const Tw2 &tw, int64_t r0, int64_t S, int64_t c) {
        w = tw(2 * r0 * c);
        step = tw(2 * S * c);
    }
    __device__ __forceinline__ double2 next() {
        const double2 cur = w;
        w = cmul(w, step);
        return cur;
    }
};

}  // namespace tsf
