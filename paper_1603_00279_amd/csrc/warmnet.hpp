// warmnet.hpp -- kernels of the learned Krylov warm start.
//
// A four-layer 1-D convolutional network (7 -> 32 -> 32 -> 32 -> 1 channels,
// width 5, zero padding, tanh after the first three layers) predicts the next
// time level as a correction to quadratic extrapolation in t:
//   x0 = 3 (u^j - u^{j-1}) + u^{j-2} + y * e2,
// (a correction that is smooth and vanishes where u is fixed in time, as at
// the Dirichlet boundary), where y is the network output for the inputs
//   e1 / s, e2 / s  (e1 = u^j - u^{j-1}, e2 = u^j - 2u^{j-1} + u^{j-2},
//                    s = RMS of e2 over the grid, 1 if e2 vanishes),
// and five channels constant in x that describe the level (alpha, beta and
// the sizes of the convection and two diffusion terms of sigma L_j relative
// to eta_j, see (3.3)).
//
// Precision: bfloat16 weights (rounded to nearest even from FP32 master
// weights kept for the optimiser) and FP32 accumulation everywhere.  The two
// hidden 32 -> 32 layers run on the matrix cores (v_mfma_f32_32x32x8_bf16),
// so their inputs (tanh outputs in [-1, 1]) are rounded to bfloat16 too; the
// input layer (whose first channel grows like the level index, which bfloat16
// would quantise in steps of up to 1/2) and the output layer take FP32 inputs
// on FP32 vector FMAs, as do the backward passes.  Biases, activations and
// gradients are FP32; the extrapolation and the scale s FP64.
//
// Layout: activations of a batch of B samples as [B][channels][n] (FP32);
// parameters as one flat vector, layer by layer W[c_out][c_in][5] then
// b[c_out] (the same order as the CPU reference of the network).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsf {
namespace net {

constexpr int CIN = 7, WIDTH = 32, KS = 5, HALF = 2, NLAYER = 4;

struct Sample {              // one training or inference sample
    const double *un;        // u^{j+1} (target), may be null
    const double *u0, *u1, *u2;  // u^j, u^{j-1}, u^{j-2}
    float feat[5];           // channels 2..6
    float pad;
};

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {  // round to nearest, ties to even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float round_bf16(float f) { return bf16_to_f32(f32_to_bf16(f)); }

// Block sum of a double (every thread passes its part; result valid in thread 0).
template <int NT>
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[NT / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) s += red[w];
    return s;
}

// s_b = RMS of e2 over the grid (1 when it vanishes), one workgroup per sample.
// The samples come from a device array `smp`, or, when it is null, from the
// single sample `one` passed by value (inference needs no upload).
// s_b = RMS of e2 over the grid (1 when it vanishes): workgroup (x, b) sums
// a slice of sample b into part[b][x]; k_net_inputs adds the slices up.
template <int NT>
__global__ void __launch_bounds__(NT) k_net_scale(const Sample *__restrict__ smp, Sample one, int64_t n,
                                                  double *part) {
    const int b = blockIdx.y;
    const Sample S = smp ? smp[b] : one;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const double e2 = S.u0[i] - 2.0 * S.u1[i] + S.u2[i];
        acc = fma(e2, e2, acc);
    }
    const double tot = block_sum<NT>(acc);
    if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = tot;
}

// s of sample b from its slices, formed once per workgroup (the first wave
// reads the slices, thread 0 adds them in slice order and shares the result).
__device__ __forceinline__ double net_scale(const double *part, int nparts, int b, int64_t n) {
    __shared__ double sl[64];
    __shared__ double sv;
    if (threadIdx.x < 64) sl[threadIdx.x] = (int)threadIdx.x < nparts ? part[(size_t)b * nparts + threadIdx.x] : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < nparts; ++k) t += sl[k];
        const double s = sqrt(t / (double)n);
        sv = s > 0.0 ? s : 1.0;
    }
    __syncthreads();
    return sv;
}

// Network inputs X[b][c][i] and, when the sample has u^{j+1}, the target
// Y*[b][i] = (u^{j+1} - base) / s (every thread forms s from the slices).
__global__ void k_net_inputs(const Sample *__restrict__ smp, Sample one, int64_t n, const double *__restrict__ part,
                             int nparts, float *__restrict__ X, float *__restrict__ Ystar) {
    const int b = blockIdx.y;
    const Sample S = smp ? smp[b] : one;
    const double inv = 1.0 / net_scale(part, nparts, b, n);
    float *Xb = X + (size_t)b * CIN * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double a0 = S.u0[i], a1 = S.u1[i], a2 = S.u2[i];
        const double e1 = a0 - a1, e2 = a0 - 2.0 * a1 + a2;
        Xb[i] = (float)(e1 * inv);
        Xb[n + i] = (float)(e2 * inv);
#pragma unroll
        for (int c = 0; c < 5; ++c) Xb[(2 + c) * n + i] = S.feat[c];
        if (Ystar && S.un) {
            const double base = fma(3.0, a0 - a1, a2);
            Ystar[(size_t)b * n + i] = (float)((S.un[i] - base) * inv);
        }
    }
}

// x0 = base + y e2 for one sample (FP64 out).
__global__ void k_net_output(Sample S, int64_t n, const float *__restrict__ y, double *__restrict__ x0) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double a0 = S.u0[i], a1 = S.u1[i], a2 = S.u2[i];
        const double base = fma(3.0, a0 - a1, a2);
        x0[i] = fma((double)y[i], a0 - 2.0 * a1 + a2, base);
    }
}

// Cooperative load of TOT tile elements by NT threads: element e = it*NT + t
// is src(e) (a global load, or 0), stored by put(e, value).  The pass count
// is a compile-time constant, so every load of the tile is in flight before
// the first LDS store.
template <int TOT, int NT, class Src, class Put>
__device__ __forceinline__ void tile_load(Src src, Put put) {
    constexpr int IT = (TOT + NT - 1) / NT;
    float v[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int e = it * NT + (int)threadIdx.x;
        v[it] = e < TOT ? src(e) : 0.0f;
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int e = it * NT + (int)threadIdx.x;
        if (e < TOT) put(e, v[it]);
    }
}

// ---------------------------------------------------------------------------
// Convolution out[b][co][p] = sum_ci sum_k W[co][ci][k] in[b][ci][p + k - 2]
// (zero outside 0 <= p + k - 2 < n), then an epilogue:
//   EPI 0: + bias, tanh;  EPI 1: + bias;  EPI 2: times (1 - act^2) (the
//   backward pass through tanh, act = the layer's stored activation).
// A workgroup covers TX positions of one sample; thread t takes position
// t % TX and output channels [OPT * (t / TX), +OPT).  Lanes of a wave share
// the channel group, so weight reads from LDS are broadcasts.
// The weights come in as `Wt[ci][k][co]` (FP32, already widened from
// bfloat16, see k_net_widen) so each thread reads its OPT channels together.
// ---------------------------------------------------------------------------
template <int CI, int CO> struct ConvGeo {
    static constexpr int OPT = CO < 8 ? CO : 8;
    static constexpr int G = CO / OPT;
    static constexpr int TX = G >= 4 ? 64 : (G == 2 ? 128 : 64);
    static constexpr int NT = TX * G;
};

template <int CI, int CO, int EPI, bool ROUND = false>
__global__ void __launch_bounds__((ConvGeo<CI, CO>::NT)) k_conv(const float *__restrict__ in,
                                                               const float *__restrict__ Wt,
                                                               const float *__restrict__ bias,
                                                               const float *__restrict__ act, float *__restrict__ out,
                                                               int64_t n) {
    using G = ConvGeo<CI, CO>;
    constexpr int TX = G::TX, OPT = G::OPT, NT = G::NT;
    __shared__ float tile[CI][TX + 2 * HALF];
    __shared__ float wl[CI * KS * CO];
    const int b = blockIdx.y;
    const int64_t p0 = (int64_t)blockIdx.x * TX;
    const float *inb = in + (size_t)b * CI * n;
    constexpr int TW = TX + 2 * HALF;
    tile_load<CI * TW, NT>(
        [&](int e) {
            const int64_t p = p0 + e % TW - HALF;
            return (p >= 0 && p < n) ? inb[(size_t)(e / TW) * n + p] : 0.0f;
        },
        [&](int e, float v) { tile[e / TW][e % TW] = ROUND ? round_bf16(v) : v; });
    tile_load<CI * KS * CO, NT>([&](int e) { return Wt[e]; }, [&](int e, float v) { wl[e] = v; });
    __syncthreads();
    const int tp = threadIdx.x % TX, cg = threadIdx.x / TX;
    const int64_t p = p0 + tp;
    float acc[OPT];
#pragma unroll
    for (int o = 0; o < OPT; ++o) acc[o] = 0.0f;
    // one input channel per iteration: the loop kept rolled holds one
    // channel's KS * OPT weights at a time
#pragma unroll 1
    for (int ci = 0; ci < CI; ++ci) {
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const float x = tile[ci][tp + k];
            const float *w = wl + (ci * KS + k) * CO + cg * OPT;
#pragma unroll
            for (int o = 0; o < OPT; ++o) acc[o] = fmaf(w[o], x, acc[o]);
        }
    }
    if (p < n) {
        float *ob = out + (size_t)b * CO * n;
#pragma unroll
        for (int o = 0; o < OPT; ++o) {
            const int co = cg * OPT + o;
            float v = acc[o];
            if constexpr (EPI == 0) v = tanhf(v + bias[co]);
            else if constexpr (EPI == 1) v = v + bias[co];
            else {
                const float a = act[(size_t)b * CO * n + (size_t)co * n + p];
                v = v * (1.0f - a * a);
            }
            ob[(size_t)co * n + p] = v;
        }
    }
}

// Widen a layer's bfloat16 weights W[co][ci][k] to FP32 in the order the
// convolution reads: forward Wt[ci][k][co]; for the backward pass through the
// data (a convolution from co channels to ci channels with the taps reversed)
// Wb[co][k][ci] = W[co][ci][KS-1-k].
__global__ void k_net_widen(const uint16_t *__restrict__ W, int ci_n, int co_n, float *__restrict__ Wt,
                            float *__restrict__ Wb) {
    const int tot = ci_n * co_n * KS;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < tot; idx += gridDim.x * blockDim.x) {
        const int co = idx / (ci_n * KS), ci = (idx / KS) % ci_n, k = idx % KS;
        const float w = bf16_to_f32(W[idx]);
        Wt[(ci * KS + k) * co_n + co] = w;
        if (Wb) Wb[(co * KS + (KS - 1 - k)) * ci_n + ci] = w;
    }
}

// Loss of a sample: the relative error of its correction,
//   sum_p (y_p X1_p - T_p)^2 / D,  D = sum_p T_p^2 + n EPS_D,
// with X1 = e2 / s (input channel 1) and T = Y* (the scaled extrapolation
// error); the batch loss is the mean over samples.  k_net_den forms D per
// sample (one workgroup each), k_net_loss dL/dy and per-workgroup partial
// sums of the loss.
constexpr double EPS_D = 1e-12;  // X1 has unit RMS: errors below 1e-6 RMS(e2) count as none

template <int NT>
__global__ void __launch_bounds__(NT) k_net_den(const float *__restrict__ ystar, int64_t n, double *__restrict__ den) {
    const float *t = ystar + (size_t)blockIdx.x * n;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += NT) acc = fma((double)t[i], (double)t[i], acc);
    const double s = block_sum<NT>(acc);
    if (threadIdx.x == 0) den[blockIdx.x] = s + (double)n * EPS_D;
}

template <int NT>
__global__ void __launch_bounds__(NT) k_net_loss(const float *__restrict__ y, const float *__restrict__ ystar,
                                                 const float *__restrict__ X, const double *__restrict__ den,
                                                 int count, int64_t n, float *__restrict__ dy,
                                                 double *__restrict__ part) {
    double acc = 0.0;
    const int64_t total = (int64_t)count * n;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < total; i += (int64_t)gridDim.x * NT) {
        const int64_t b = i / n, p = i - b * n;
        const float x1 = X[(size_t)b * CIN * n + n + p];
        const double d = den[b];
        const float r = y[i] * x1 - ystar[i];
        dy[i] = (float)(2.0 * (double)r * (double)x1 / (d * (double)count));
        acc += (double)r * (double)r / d;
    }
    const double s = block_sum<NT>(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// Weight and bias gradients of one layer:
//   dW[co][ci][k] = sum_b sum_p dZ[b][co][p] a[b][ci][p + k - 2],
//   db[co]        = sum_b sum_p dZ[b][co][p].
// Thread (ci, cb) accumulates a block of COB output channels x KS taps for
// input channel ci (and, for ci = 0, the biases of its channels) over the
// positions of its workgroup; the partial sums of every workgroup are summed
// in a fixed order by k_net_wgrad_reduce.
// ---------------------------------------------------------------------------
template <int CI, int CO> struct WgradGeo {
    static constexpr int COB = CO < 4 ? CO : 4;
    static constexpr int NTH = CI * (CO / COB);
    static constexpr int NT = NTH <= 64 ? 64 : (NTH <= 128 ? 128 : 256);
    static constexpr int TX = 128;
    static constexpr int NE = CO * CI * KS + CO;  // entries per layer
};

template <int CI, int CO, bool ROUND>
__global__ void __launch_bounds__((WgradGeo<CI, CO>::NT)) k_net_wgrad(const float *__restrict__ dz,
                                                                     const float *__restrict__ a, int64_t n,
                                                                     float *__restrict__ part) {
    using G = WgradGeo<CI, CO>;
    constexpr int TX = G::TX, COB = G::COB, NT = G::NT;
    __shared__ float ta[CI][TX + 2 * HALF];
    __shared__ float tz[CO][TX];
    const int b = blockIdx.y;
    const float *ab = a + (size_t)b * CI * n;
    const float *zb = dz + (size_t)b * CO * n;
    const int t = threadIdx.x;
    const bool own = t < G::NTH;
    const int ci = own ? t % CI : 0, cb = own ? t / CI : 0;
    float acc[COB][KS];
    float accb[COB];
#pragma unroll
    for (int o = 0; o < COB; ++o) {
        accb[o] = 0.0f;
#pragma unroll
        for (int k = 0; k < KS; ++k) acc[o][k] = 0.0f;
    }
    for (int64_t p0 = (int64_t)blockIdx.x * TX; p0 < n; p0 += (int64_t)gridDim.x * TX) {
        __syncthreads();
        constexpr int TW = TX + 2 * HALF;
        tile_load<CI * TW, NT>(
            [&](int e) {
                const int64_t p = p0 + e % TW - HALF;
                return (p >= 0 && p < n) ? ab[(size_t)(e / TW) * n + p] : 0.0f;
            },
            [&](int e, float v) { ta[e / TW][e % TW] = ROUND ? round_bf16(v) : v; });  // as the forward pass saw it
        tile_load<CO * TX, NT>(
            [&](int e) {
                const int64_t p = p0 + e % TX;
                return p < n ? zb[(size_t)(e / TX) * n + p] : 0.0f;
            },
            [&](int e, float v) { tz[e / TX][e % TX] = v; });
        __syncthreads();
        if (own) {
            for (int q = 0; q < TX; ++q) {
                float av[KS];
#pragma unroll
                for (int k = 0; k < KS; ++k) av[k] = ta[ci][q + k];
#pragma unroll
                for (int o = 0; o < COB; ++o) {
                    const float z = tz[cb * COB + o][q];
                    accb[o] += z;
#pragma unroll
                    for (int k = 0; k < KS; ++k) acc[o][k] = fmaf(z, av[k], acc[o][k]);
                }
            }
        }
    }
    if (own) {
        float *pw = part + (size_t)(blockIdx.y * gridDim.x + blockIdx.x) * G::NE;
#pragma unroll
        for (int o = 0; o < COB; ++o) {
            const int co = cb * COB + o;
#pragma unroll
            for (int k = 0; k < KS; ++k) pw[(co * CI + ci) * KS + k] = acc[o][k];
            if (ci == 0) pw[CO * CI * KS + co] = accb[o];
        }
    }
}

// grad[e] = sum over workgroups w (in index order) of part[w][e].
__global__ void k_net_wgrad_reduce(const float *__restrict__ part, int nwg, int ne, float *__restrict__ grad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    float s = 0.0f;
    for (int w = 0; w < nwg; ++w) s += part[(size_t)w * ne + e];
    grad[e] = s;
}

// ---------------------------------------------------------------------------
// Forward convolution to 32 channels on the matrix cores.  As a product,
//   out[co][p] = sum_k Wm[co][k] * T[k][p],  k = tap * CIP + ci (tap-major),
// with T[k][p] = bf16(in[ci][p + tap - 2]) (zero outside the grid and for the
// padding channels ci >= CI) and Wm the bfloat16 weights in that k order.
// A wave computes 32 channels x 32 positions with v_mfma_f32_32x32x8_bf16:
//   A (32 x 8): lane l holds Wm[l % 32][kb*8 + 4(l/32) + t], t = 0..3,
//   B (8 x 32): lane l holds T[kb*8 + 4(l/32) + t][l % 32],
//   D (32 x 32): lane l, register r holds out[8(r/4) + 4(l/32) + r%4][l % 32],
// (layout checked on the device against a CPU product).  Four consecutive k
// share a tap and are four adjacent channels, so the input tile is kept in
// LDS channel-last and every B operand is one 8-byte read.  Epilogue: bias,
// tanh, FP32 store (coalesced along positions).
// ---------------------------------------------------------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int MFMA_WAVES = 2;  // waves (of 32 positions each) per workgroup

template <int CI, int CIP>
__global__ void __launch_bounds__(64 * MFMA_WAVES) k_conv_mfma(const float *__restrict__ in,
                                                               const uint16_t *__restrict__ Wm,
                                                               const float *__restrict__ bias, float *__restrict__ out,
                                                               int64_t n) {
    constexpr int NT = 64 * MFMA_WAVES, TX = 32 * MFMA_WAVES, K = KS * CIP, KB = K / 8;
    constexpr int RS = CIP + 4;  // padded LDS row (bf16 units)
    static_assert(CIP % 8 == 0 || CIP == 8, "channel padding");
    __shared__ __align__(16) uint16_t tin[(TX + 2 * HALF) * RS];
    const int b = blockIdx.y;
    const int64_t p0 = (int64_t)blockIdx.x * TX;
    const float *inb = in + (size_t)b * CI * n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, c32 = lane & 31;
    // the wave's weights (A operands) straight from global memory
    bf16x4 aw[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) aw[kb] = *reinterpret_cast<const bf16x4 *>(Wm + c32 * K + kb * 8 + 4 * h);
    constexpr int TW = TX + 2 * HALF;
    tile_load<CIP * TW, NT>(
        [&](int e) {
            const int ci = e / TW;
            const int64_t p = p0 + e % TW - HALF;
            return (ci < CI && p >= 0 && p < n) ? inb[(size_t)ci * n + p] : 0.0f;
        },
        [&](int e, float v) { tin[(e % TW) * RS + e / TW] = f32_to_bf16(v); });
    __syncthreads();
    const int pw = wave * 32 + c32;  // this lane's position column within the tile
    f32x16 acc = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const int k0 = kb * 8 + 4 * h, tap = k0 / CIP, ci0 = k0 % CIP;
        const bf16x4 bv = *reinterpret_cast<const bf16x4 *>(tin + (pw + tap) * RS + ci0);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(aw[kb], bv, acc, 0, 0, 0);
    }
    const int64_t p = p0 + pw;
    if (p < n) {
        float *ob = out + (size_t)b * 32 * n;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int co = 8 * (r / 4) + 4 * h + (r % 4);
            ob[(size_t)co * n + p] = tanhf(acc[r] + bias[co]);
        }
    }
}

// bfloat16 weights W[co][ci][k] (32 outputs) -> Wm[co][k * CIP + ci], zero for
// the padding channels.
__global__ void k_net_widen_mfma(const uint16_t *__restrict__ W, int ci_n, int cip, uint16_t *__restrict__ Wm) {
    const int tot = 32 * KS * cip;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < tot; idx += gridDim.x * blockDim.x) {
        const int co = idx / (KS * cip), rem = idx % (KS * cip), k = rem / cip, ci = rem % cip;
        Wm[idx] = ci < ci_n ? W[(co * ci_n + ci) * KS + k] : (uint16_t)0;
    }
}

// Adam (Kingma and Ba 2015, Algorithm 1) on the FP32 master parameters, then
// the bfloat16 copy the convolutions read.
__global__ void k_net_adam(float *__restrict__ theta, float *__restrict__ m, float *__restrict__ v,
                           const float *__restrict__ g, uint16_t *__restrict__ wbf, int count, float lr, float b1,
                           float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float th = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    theta[i] = th;
    wbf[i] = f32_to_bf16(th);
}

__global__ void k_net_round(const float *__restrict__ theta, uint16_t *__restrict__ wbf, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) wbf[i] = f32_to_bf16(theta[i]);
}

}  // namespace net
}  // namespace tsf
