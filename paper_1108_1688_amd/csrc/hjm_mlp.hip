// Learned surrogate of the caplet price: an MLP 8 -> 256 -> 256 -> 256 -> 256 -> 1
// with GELU activations, trained on prices of the Douglas-ADI solver and used
// inside its training box (the ADI solver is the fallback outside it).
//
// Arithmetic: matrix products take BF16 operands (activations, weights and
// back-propagated gradients rounded to BF16 at fixed points) and accumulate
// in FP32 on the matrix cores (v_mfma_f32_16x16x32_bf16); biases, the output
// layer's dot product, the loss, the weight gradients and the Adam state are
// FP32, with FP32 master weights.
//
// MFMA fragment layout (16 x 16 x 32): lane l holds row l % 16 of A and column
// l % 16 of B, each at k = 8 (l / 16) .. 8 (l / 16) + 7, and rows
// 4 (l / 16) .. 4 (l / 16) + 3 of column l % 16 of the product.
#include "hjm.h"
#include "hjm_mlp.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace hjm_nn {
namespace {

typedef __attribute__((ext_vector_type(4))) float f4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf8;
typedef unsigned short bf16_t;  // BF16 bit pattern in memory

constexpr int H = kHidden;   // 256
constexpr int KIN = kInPad;  // 32: the 8 inputs padded with zeros

__device__ __forceinline__ bf16_t f2bf(float f)
{
    // round to nearest even (finite inputs)
    unsigned int u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t b) { return __uint_as_float((unsigned int)b << 16); }

// GELU(z) = z Phi(z), Phi the standard normal CDF; derivative Phi(z) + z phi(z)
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z)
{
    const float Phi = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
    const float phi = 0.39894228040143268f * expf(-0.5f * z * z);
    return Phi + z * phi;
}

// Gaussian caplet baseline (optional control variate of the output): with it
// the network learns ln(price / B(x)) and reports B(x) exp(y scale + shift).
// B is the textbook Gaussian (Hull-White) caplet, the zero-coupon bond put,
// with the rate volatility frozen at lambda f(0,T)^gamma on the mean path
// 1 + (v0 - 1) e^{-theta_v t} of the variance factor; the row's curve is
// f(0,t) = level + slope (1 - e^{-decay t}), payment one tenor after expiry,
// strike = at-the-money (simple compounding) + offset.  FP64 throughout.
struct BaseK {
    double lam, two_gam, theta_v, decay, tenor;
    int on;
};

__device__ __forceinline__ double ncdf(double z) { return 0.5 * erfc(-z * 0.70710678118654752440); }

__device__ double caplet_baseline(const float* __restrict__ xr, const BaseK& b)
{
    const double kap = xr[0], v0 = xr[3], a = xr[4], sl = xr[5], dk = xr[6], T = xr[7];
    const double c = b.decay, tau = b.tenor;
    // integral of f(0, .) over [0, t]
    const double iT = a * T + sl * (T + expm1(-c * T) / c);
    const double iM = a * (T + tau) + sl * ((T + tau) + expm1(-c * (T + tau)) / c);
    const double PT = exp(-iT), PM = exp(-iM);
    const double D = 1.0 + tau * ((PT / PM - 1.0) / tau + dk);  // 1 + tau K
    const double G = kap > 0.0 ? -expm1(-kap * tau) / kap : tau;
    const double fT = a - sl * expm1(-c * T);
    // integral over [0, T] of the mean variance path against e^{-2 kappa (T - t)}
    const double I1 = kap > 0.0 ? -expm1(-2.0 * kap * T) / (2.0 * kap) : T;
    const double d = 2.0 * kap - b.theta_v;
    const double I2 = exp(-2.0 * kap * T) * (d != 0.0 ? expm1(d * T) / d : T);
    const double var = b.lam * b.lam * pow(fT, b.two_gam) * G * G * (I1 + (v0 - 1.0) * I2);
    const double sd = sqrt(var);
    const double h = log(D * PM / PT) / sd + 0.5 * sd;
    return PT * ncdf(sd - h) - D * PM * ncdf(-h);
}

__device__ __forceinline__ bf8 load8(const bf16_t* p)
{
    // 16-byte aligned load of 8 BF16 values
    return *reinterpret_cast<const bf8*>(p);
}

// one input mapped to [-1, 1] over its box side, rounded to BF16
__device__ __forceinline__ bf16_t norm_in(float v, float lo, float hi)
{
    return f2bf(2.0f * (v - lo) / (hi - lo) - 1.0f);
}

// ---------------------------------------------------------------------------
// Input: normalise to [-1, 1] over the box, flag rows outside it, pad to 32.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_input(const float* __restrict__ x, int64_t n, const float* __restrict__ lo,
                                               const float* __restrict__ hi, bf16_t* __restrict__ xp,
                                               uint8_t* __restrict__ in_box)
{
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    bool inside = true;
    bf16_t row[KIN];
    for (int c = 0; c < KIN; ++c) row[c] = 0;
    for (int c = 0; c < kIn; ++c) {
        const float v = x[s * kIn + c];
        inside = inside && v >= lo[c] && v <= hi[c];
        row[c] = norm_in(v, lo[c], hi[c]);
    }
    for (int c = 0; c < KIN; ++c) xp[s * KIN + c] = row[c];
    if (in_box) in_box[s] = inside ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Forward layer: Z = Hin W^T + b (FP32), Hout = BF16(GELU(Z)).
// Hin is n x K (BF16, row-major), W is 256 x K (BF16, row-major).  A
// workgroup is one wave: 64 samples (blockIdx.x) and features
// [64 w, 64 w + 64), w = blockIdx.y: 4 x 4 MFMA tiles of 16 x 16.  One wave
// per workgroup keeps four times as many compute units busy on the small
// training batches as a workgroup holding all four feature blocks would.
// ---------------------------------------------------------------------------
template <int K>
__global__ __launch_bounds__(64) void k_fwd(const bf16_t* __restrict__ hin, const bf16_t* __restrict__ w,
                                            const float* __restrict__ b, int64_t n, float* __restrict__ z,
                                            bf16_t* __restrict__ hout)
{
    const int lane = threadIdx.x;
    const int wave = blockIdx.y;
    const int64_t s0 = (int64_t)blockIdx.x * 64;
    const int f0 = wave * 64;
    const int r = lane & 15;
    const int kq = (lane >> 4) * 8;
    f4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf8 av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            int64_t srow = s0 + a * 16 + r;
            srow = srow < n ? srow : n - 1;  // tail rows repeat the last sample, not stored
            av[a] = load8(hin + srow * K + k0 + kq);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) bv[c] = load8(w + (int64_t)(f0 + c * 16 + r) * K + k0 + kq);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[c], acc[a][c], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int f = f0 + c * 16 + r;
        const float bias = b[f];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t s = s0 + a * 16 + (lane >> 4) * 4 + v;
                if (s < n) {
                    const float zz = acc[a][c][v] + bias;
                    if (z) z[s * H + f] = zz;
                    hout[s * H + f] = f2bf(gelu(zz));
                }
            }
    }
}

// Output layer of the training pass: y = H4 . w5 + b5 (BF16 operands, FP32
// sum) in network units.  One thread per sample.
__global__ __launch_bounds__(256) void k_out(const bf16_t* __restrict__ h4, const bf16_t* __restrict__ w5,
                                             const float* __restrict__ b5, int64_t n, float* __restrict__ y)
{
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    float acc = 0.0f;
    for (int f = 0; f < H; f += 8) {
        const bf8 hv = load8(h4 + s * H + f);
        const bf8 wv = load8(w5 + f);
#pragma unroll
        for (int e = 0; e < 8; ++e) acc += (float)hv[e] * (float)wv[e];
    }
    y[s] = acc + b5[0];
}

// Training targets in network units: (ln(price / B(x)) - shift) / scale with
// the baseline, (price - shift) / scale without.  One thread per row.
__global__ __launch_bounds__(256) void k_targets(const float* __restrict__ x, const double* __restrict__ price,
                                                 int64_t n, float scale, float shift, BaseK base,
                                                 float* __restrict__ t)
{
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const double p = price[s];
    if (base.on && !(p > 0.0)) {
        t[s] = __builtin_nanf("");  // no logarithm: the row must be dropped
        return;
    }
    const double y = base.on ? log(p / caplet_baseline(x + s * kIn, base)) : p;
    t[s] = (float)((y - (double)shift) / (double)scale);
}

// ---------------------------------------------------------------------------
// Inference in one kernel.  A workgroup takes 64 rows through the input map,
// the four hidden layers and the output layer; the rows' activations stay in
// LDS (BF16, 64 x 256, rows padded by 16 bytes so that the fragment reads of
// a wave spread over the banks), so HBM sees only the inputs, the weights
// (from L2 after the first workgroups) and the prices.  Each layer is the
// k_fwd tiling (wave w: features [64 w, 64 w + 64) of all 64 rows, 4 x 4 MFMA
// tiles, k in steps of 32) with its A operand read from LDS, then bias, GELU
// and BF16 rounding as k_fwd; the output is k_out's sum.  Same operations in
// the same order as k_input, k_fwd and k_out: the same results.
// ---------------------------------------------------------------------------
constexpr int kXP = KIN + 8;  // LDS row pitch of the input tile (BF16 values)
constexpr int kHP = H + 8;    // LDS row pitch of the activation tile

// acc = A W^T over K for the wave's 64 features; A is the LDS tile (pitch ap)
template <int K>
__device__ __forceinline__ void tile_layer(const bf16_t* __restrict__ a_lds, int ap, const bf16_t* __restrict__ w,
                                           int f0, int r, int kq, f4 (&acc)[4][4])
{
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf8 av[4], bv[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) bv[c] = load8(w + (int64_t)(f0 + c * 16 + r) * K + k0 + kq);
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = *reinterpret_cast<const bf8*>(a_lds + (a * 16 + r) * ap + k0 + kq);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[c], acc[a][c], 0, 0, 0);
    }
}

// H tile = BF16(GELU(acc + b)) for the wave's features
__device__ __forceinline__ void tile_gelu(bf16_t* __restrict__ h_lds, const float* __restrict__ b, int f0, int r,
                                          int lane, const f4 (&acc)[4][4])
{
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int f = f0 + c * 16 + r;
        const float bias = b[f];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = a * 16 + (lane >> 4) * 4 + v;
                h_lds[row * kHP + f] = f2bf(gelu(acc[a][c][v] + bias));
            }
    }
}

__global__ __launch_bounds__(256, 4) void k_infer(const float* __restrict__ x, int64_t n, const float* __restrict__ box,
                                               const bf16_t* __restrict__ w1, const bf16_t* __restrict__ w2,
                                               const bf16_t* __restrict__ w3, const bf16_t* __restrict__ w4,
                                               const bf16_t* __restrict__ w5, const float* __restrict__ p,
                                               float scale, float shift, BaseK base, float* __restrict__ y,
                                               uint8_t* __restrict__ in_box)
{
    __shared__ __attribute__((aligned(16))) bf16_t xs[64 * kXP];
    __shared__ __attribute__((aligned(16))) bf16_t hs[64 * kHP];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int64_t s0 = (int64_t)blockIdx.x * 64;
    if (t < 64) {
        // row s0 + t; tail rows repeat the last sample (never stored)
        const bool live = s0 + t < n;
        const int64_t s = live ? s0 + t : n - 1;
        bool inside = true;
#pragma unroll
        for (int c = 0; c < KIN; ++c) {
            bf16_t q = 0;
            if (c < kIn) {
                const float v = x[s * kIn + c];
                inside = inside && v >= box[c] && v <= box[kIn + c];
                q = norm_in(v, box[c], box[kIn + c]);
            }
            xs[t * kXP + c] = q;
        }
        if (in_box && live) in_box[s] = inside ? 1 : 0;
    }
    __syncthreads();
    const int r = lane & 15;
    const int kq = (lane >> 4) * 8;
    const int f0 = wave * 64;
    f4 acc[4][4];
    tile_layer<KIN>(xs, kXP, w1, f0, r, kq, acc);
    tile_gelu(hs, p + kOffB1, f0, r, lane, acc);
    __syncthreads();
    const bf16_t* ws[3] = {w2, w3, w4};
    const int64_t bo[3] = {kOffB2, kOffB3, kOffB4};
#pragma unroll 1
    for (int l = 0; l < 3; ++l) {
        tile_layer<H>(hs, kHP, ws[l], f0, r, kq, acc);
        __syncthreads();  // every wave has read the layer's inputs
        tile_gelu(hs, p + bo[l], f0, r, lane, acc);
        __syncthreads();
    }
    if (t < 64 && s0 + t < n) {
        const int64_t s = s0 + t;
        float a = 0.0f;
        for (int f = 0; f < H; f += 8) {
            const bf8 hv = *reinterpret_cast<const bf8*>(hs + t * kHP + f);
            const bf8 wv = load8(w5 + f);
#pragma unroll
            for (int e = 0; e < 8; ++e) a += (float)hv[e] * (float)wv[e];
        }
        if (base.on)
            y[s] = (float)(caplet_baseline(x + s * kIn, base) * exp((double)(a + p[kOffB5]) * scale + shift));
        else
            y[s] = (a + p[kOffB5]) * scale + shift;
    }
}

// ---------------------------------------------------------------------------
// Backward.
// ---------------------------------------------------------------------------
// Loss (mean squared error in network units, y already in network units) and
// its gradient dy = 2 (y - t) / n; per-block partial sums of the squared error.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, const float* __restrict__ t, int64_t n,
                                              float* __restrict__ dy, float* __restrict__ part)
{
    __shared__ float red[256];
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float e2 = 0.0f;
    if (s < n) {
        const float e = y[s] - t[s];
        dy[s] = 2.0f * e / (float)n;
        e2 = e * e;
    }
    red[threadIdx.x] = e2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Output layer backward: dZ4 = BF16(dy w5 GELU'(Z4)), and per-block partials
// of dw5 = sum_s dy H4 and db5 = sum_s dy (block = kOutSub samples: many
// blocks, short serial loops).
constexpr int kOutSub = 16;
__global__ __launch_bounds__(256) void k_out_bwd(const float* __restrict__ dy, const bf16_t* __restrict__ h4,
                                                 const float* __restrict__ z4, const bf16_t* __restrict__ w5,
                                                 int64_t n, bf16_t* __restrict__ dz4, float* __restrict__ part)
{
    // thread = feature f; loop over the block's samples
    const int f = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * kOutSub;
    const float wf = bf2f(w5[f]);
    float gw = 0.0f, gb = 0.0f;
    for (int q = 0; q < kOutSub; ++q) {
        const int64_t s = s0 + q;
        if (s >= n) break;
        const float d = dy[s];
        gw += d * bf2f(h4[s * H + f]);
        gb += d;
        dz4[s * H + f] = f2bf(d * wf * gelu_d(z4[s * H + f]));
    }
    part[(int64_t)blockIdx.x * (H + 1) + f] = gw;
    if (f == 0) part[(int64_t)blockIdx.x * (H + 1) + H] = gb;
}

// dH = dZ W (n x 256 times 256 x K) with dZ_prev = BF16(dH GELU'(Z_prev)).
// wt is W^T (K x 256, BF16 row-major), so B = W^T^T reads rows of wt.
// Same tiling as k_fwd (one wave per workgroup, blockIdx.y the column
// block) with K = 256 features of the output side.
__global__ __launch_bounds__(64) void k_bwd_dh(const bf16_t* __restrict__ dz, const bf16_t* __restrict__ wt,
                                               const float* __restrict__ zprev, int64_t n,
                                               bf16_t* __restrict__ dzprev)
{
    const int lane = threadIdx.x;
    const int wave = blockIdx.y;
    const int64_t s0 = (int64_t)blockIdx.x * 64;
    const int f0 = wave * 64;  // output column block (input features of the layer)
    const int r = lane & 15;
    const int kq = (lane >> 4) * 8;
    f4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < H; k0 += 32) {
        bf8 av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            int64_t srow = s0 + a * 16 + r;
            srow = srow < n ? srow : n - 1;
            av[a] = load8(dz + srow * H + k0 + kq);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) bv[c] = load8(wt + (int64_t)(f0 + c * 16 + r) * H + k0 + kq);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[c], acc[a][c], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int k = f0 + c * 16 + r;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t s = s0 + a * 16 + (lane >> 4) * 4 + v;
                if (s < n) dzprev[s * H + k] = f2bf(acc[a][c][v] * gelu_d(zprev[s * H + k]));
            }
    }
}

// Weight gradient partials: P[chunk] = dZ^T Hprev over the chunk's samples
// (256 x K, FP32), and the bias partials sum_s dZ.  Workgroup = one chunk of
// kChunk samples and a 64 x 64 tile of (feature f, input k); the chunk's rows
// are staged through LDS and read back transposed for the MFMA operands.
template <int K>
__global__ __launch_bounds__(256) void k_bwd_dw(const bf16_t* __restrict__ dz, const bf16_t* __restrict__ hprev,
                                                int64_t n, float* __restrict__ part, float* __restrict__ bpart)
{
    constexpr int TK = K < 64 ? K : 64;  // tile width along k
    __shared__ bf16_t sdz[32][64 + 8];
    __shared__ bf16_t sh[32][64 + 8];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tiles_k = K / TK;
    const int tf = blockIdx.y / tiles_k;  // feature tile
    const int tk = blockIdx.y % tiles_k;  // input tile
    const int f0 = tf * 64, k0 = tk * TK;
    const int64_t c0 = (int64_t)blockIdx.x * kChunk;
    const int r = lane & 15;
    const int kq = (lane >> 4) * 8;
    // wave w: features f0 + 16 w .. +16, all TK inputs (TK / 16 tiles)
    f4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.0f;
    for (int q0 = 0; q0 < kChunk; q0 += 32) {
        // stage 32 samples x 64 features of dZ and 32 x TK of Hprev
        for (int e = threadIdx.x; e < 32 * 64; e += 256) {
            const int q = e / 64, c = e % 64;
            const int64_t s = c0 + q0 + q;
            sdz[q][c] = s < n ? dz[s * H + f0 + c] : (bf16_t)0;
        }
        for (int e = threadIdx.x; e < 32 * TK; e += 256) {
            const int q = e / TK, c = e % TK;
            const int64_t s = c0 + q0 + q;
            sh[q][c] = s < n ? hprev[s * K + k0 + c] : (bf16_t)0;
        }
        __syncthreads();
        // A = dZ^T tile: row f = 16 w + r, k (sample) = kq .. kq + 7
        bf8 av;
#pragma unroll
        for (int e = 0; e < 8; ++e) av[e] = __builtin_bit_cast(__bf16, sdz[kq + e][16 * wave + r]);
        if (lane < 16) {
            // bias partial of feature f0 + 16 w + lane over these 32 samples
            float t = 0.0f;
            for (int q = 0; q < 32; ++q) t += bf2f(sdz[q][16 * wave + lane]);
            bsum += t;
        }
#pragma unroll
        for (int c = 0; c < TK / 16; ++c) {
            bf8 bv;
#pragma unroll
            for (int e = 0; e < 8; ++e) bv[e] = __builtin_bit_cast(__bf16, sh[kq + e][16 * c + r]);
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[c], 0, 0, 0);
        }
        __syncthreads();
    }
    float* P = part + (int64_t)blockIdx.x * H * K;
#pragma unroll
    for (int c = 0; c < TK / 16; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int f = f0 + 16 * wave + (lane >> 4) * 4 + v;
            const int k = k0 + 16 * c + r;
            P[f * K + k] = acc[c][v];
        }
    if (tk == 0 && lane < 16) bpart[(int64_t)blockIdx.x * H + f0 + 16 * wave + lane] = bsum;
}

// Sum partials over chunks: out[i] = sum_c part[c * len + i] (fixed order).
__global__ __launch_bounds__(256) void k_sum(const float* __restrict__ part, int chunks, int64_t len,
                                             float* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    float a = 0.0f;
    for (int c = 0; c < chunks; ++c) a += part[(int64_t)c * len + i];
    out[i] = a;
}

// Layer-1 weight gradient: the partials cover the 32 padded inputs; only the
// first kIn are parameters.  out[f kIn + k] = sum_c part[c][f][k].
__global__ __launch_bounds__(256) void k_sum_w1(const float* __restrict__ part, int chunks, float* __restrict__ out)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kHidden * kIn) return;
    const int f = i / kIn, k = i % kIn;
    float a = 0.0f;
    for (int c = 0; c < chunks; ++c) a += part[(int64_t)c * kHidden * KIN + f * KIN + k];
    out[i] = a;
}

// Adam on the flat FP32 parameters, then refresh the BF16 operand copies.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, int64_t len, float lr, float b1,
                                              float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 copies of the weights: W (256 x K, K = 32 for layer 1 with zero
// padding) and W^T (K x 256) for the backward products, and w5.
__global__ __launch_bounds__(256) void k_cast(const float* __restrict__ p, bf16_t* __restrict__ w1,
                                              bf16_t* __restrict__ w2, bf16_t* __restrict__ w3,
                                              bf16_t* __restrict__ w4, bf16_t* __restrict__ w2t,
                                              bf16_t* __restrict__ w3t, bf16_t* __restrict__ w4t,
                                              bf16_t* __restrict__ w5)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < (int64_t)H * KIN) {
        const int f = (int)(i / KIN), k = (int)(i % KIN);
        w1[i] = k < kIn ? f2bf(p[kOffW1 + f * kIn + k]) : (bf16_t)0;
    }
    if (i < (int64_t)H * H) {
        const int f = (int)(i / H), k = (int)(i % H);
        const bf16_t a = f2bf(p[kOffW2 + i]), b = f2bf(p[kOffW3 + i]), c = f2bf(p[kOffW4 + i]);
        w2[i] = a; w3[i] = b; w4[i] = c;
        w2t[(int64_t)k * H + f] = a; w3t[(int64_t)k * H + f] = b; w4t[(int64_t)k * H + f] = c;
    }
    if (i < H) w5[i] = f2bf(p[kOffW5 + i]);
}

}  // namespace
}  // namespace hjm_nn

using namespace hjm_nn;

// ---------------------------------------------------------------------------
// Host side and C ABI.
// ---------------------------------------------------------------------------
struct hjm_mlp {
    hipStream_t stream = nullptr;
    int64_t max_batch = 0;
    float lo[kIn], hi[kIn];
    float scale = 1.0f, shift = 0.0f;
    BaseK base{};  // off until hjm_mlp_set_baseline
    int64_t adam_t = 0;
    // device pointers (all inside the caller's workspace)
    float *p, *m, *v, *g, *box;
    bf16_t *w1, *w2, *w3, *w4, *w2t, *w3t, *w4t, *w5;
    bf16_t *xp, *h1, *h2, *h3, *h4, *dz4, *dz3, *dz2, *dz1;
    float *z1, *z2, *z3, *z4, *y, *dy, *part, *bpart, *lpart;
    std::vector<float> lpart_host;
};

namespace {

hjm_status mfail(hjm_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return hjm::report_error(code, buf);
}

hjm_status mhip(hipError_t e, const char* where) { return mfail(HJM_EDEVICE, "%s: %s", where, hipGetErrorString(e)); }

struct MlpLayout {
    size_t total = 0;
    size_t take(size_t bytes)
    {
        const size_t at = total;
        total = (total + bytes + 255) & ~(size_t)255;
        return at;
    }
};

int64_t chunks_of(int64_t n) { return (n + kChunk - 1) / kChunk; }

// Lay out (or only size, base == nullptr) the workspace.
size_t mlp_layout(hjm_mlp* h, char* base, int64_t nb)
{
    MlpLayout L;
    // addresses from integers: sizing (base null) forms no pointer from a null one
    const uintptr_t b0 = reinterpret_cast<uintptr_t>(base);
    auto F = [&](size_t count) { return reinterpret_cast<float*>(b0 + L.take(count * 4)); };
    auto B = [&](size_t count) { return reinterpret_cast<bf16_t*>(b0 + L.take(count * 2)); };
    const int64_t ch = chunks_of(nb);
    const size_t rows = (size_t)((nb + 63) / 64 * 64);
    float* p = F(kParams);
    float* m = F(kParams);
    float* v = F(kParams);
    float* g = F(kParams);
    float* box = F(2 * kIn);
    bf16_t* w1 = B((size_t)H * KIN);
    bf16_t* w2 = B((size_t)H * H);
    bf16_t* w3 = B((size_t)H * H);
    bf16_t* w4 = B((size_t)H * H);
    bf16_t* w2t = B((size_t)H * H);
    bf16_t* w3t = B((size_t)H * H);
    bf16_t* w4t = B((size_t)H * H);
    bf16_t* w5 = B(H);
    bf16_t* xp = B(rows * KIN);
    bf16_t* hs[4];
    float* zs[4];
    bf16_t* dzs[4];
    for (int l = 0; l < 4; ++l) { hs[l] = B(rows * H); zs[l] = F(rows * H); dzs[l] = B(rows * H); }
    float* y = F(rows);
    float* dy = F(rows);
    float* part = F((size_t)ch * H * H + (size_t)ch * (H + 1));
    float* bpart = F((size_t)ch * H);
    float* lpart = F((size_t)(nb + 255) / 256);
    if (h) {
        h->p = p; h->m = m; h->v = v; h->g = g; h->box = box;
        h->w1 = w1; h->w2 = w2; h->w3 = w3; h->w4 = w4; h->w2t = w2t; h->w3t = w3t; h->w4t = w4t; h->w5 = w5;
        h->xp = xp;
        h->h1 = hs[0]; h->h2 = hs[1]; h->h3 = hs[2]; h->h4 = hs[3];
        h->z1 = zs[0]; h->z2 = zs[1]; h->z3 = zs[2]; h->z4 = zs[3];
        h->dz1 = dzs[0]; h->dz2 = dzs[1]; h->dz3 = dzs[2]; h->dz4 = dzs[3];
        h->y = y; h->dy = dy; h->part = part; h->bpart = bpart; h->lpart = lpart;
    }
    return L.total;
}

unsigned blocks256(int64_t n) { return (unsigned)((n + 255) / 256); }

// training forward pass from raw inputs (inference runs k_infer instead);
// z arrays kept for the backward pass when keep_z
hipError_t forward(hjm_mlp* h, const float* x, int64_t n, uint8_t* in_box, bool keep_z)
{
    hipStream_t st = h->stream;
    const unsigned gb = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL(k_input, dim3(blocks256(n)), dim3(256), 0, st, x, n, h->box, h->box + kIn, h->xp, in_box);
    const dim3 grid(gb, H / 64);  // (64-sample tile, feature block)
    hipLaunchKernelGGL(k_fwd<KIN>, grid, dim3(64), 0, st, h->xp, h->w1, h->p + kOffB1, n,
                       keep_z ? h->z1 : nullptr, h->h1);
    hipLaunchKernelGGL(k_fwd<H>, grid, dim3(64), 0, st, h->h1, h->w2, h->p + kOffB2, n,
                       keep_z ? h->z2 : nullptr, h->h2);
    hipLaunchKernelGGL(k_fwd<H>, grid, dim3(64), 0, st, h->h2, h->w3, h->p + kOffB3, n,
                       keep_z ? h->z3 : nullptr, h->h3);
    hipLaunchKernelGGL(k_fwd<H>, grid, dim3(64), 0, st, h->h3, h->w4, h->p + kOffB4, n,
                       keep_z ? h->z4 : nullptr, h->h4);
    return hipGetLastError();
}

hipError_t cast_weights(hjm_mlp* h)
{
    hipLaunchKernelGGL(k_cast, dim3(blocks256((int64_t)H * H)), dim3(256), 0, h->stream, h->p, h->w1, h->w2, h->w3,
                       h->w4, h->w2t, h->w3t, h->w4t, h->w5);
    return hipGetLastError();
}

// loss and gradients of a minibatch (t in network units); returns the summed
// squared error in *sse (after a stream synchronisation) when sse != nullptr
hjm_status gradients(hjm_mlp* h, const float* x, const float* t, int64_t n, double* sse)
{
    hipStream_t st = h->stream;
    hipError_t e = forward(h, x, n, nullptr, true);
    if (e) return mhip(e, "mlp forward");
    // network units (the loss compares them with targets in the same units)
    hipLaunchKernelGGL(k_out, dim3(blocks256(n)), dim3(256), 0, st, h->h4, h->w5, h->p + kOffB5, n, h->y);
    hipLaunchKernelGGL(k_loss, dim3(blocks256(n)), dim3(256), 0, st, h->y, t, n, h->dy, h->lpart);
    // (n / 16) (H + 1) partials fit the ceil(n / 256) (H H + H + 1) floats of part
    const int64_t nsub = (n + kOutSub - 1) / kOutSub;
    hipLaunchKernelGGL(k_out_bwd, dim3((unsigned)nsub), dim3(256), 0, st, h->dy, h->h4, h->z4, h->w5, n, h->dz4,
                       h->part);
    // dw5, db5
    hipLaunchKernelGGL(k_sum, dim3(blocks256(H + 1)), dim3(256), 0, st, h->part, (int)nsub, (int64_t)(H + 1),
                       h->g + kOffW5);
    const unsigned gb = (unsigned)((n + 63) / 64);
    const int64_t ch = chunks_of(n);
    struct L { const bf16_t* dz; const bf16_t* hprev; int K; int64_t offW, offB; const bf16_t* wt; const float* zprev;
               bf16_t* dzprev; };
    const L layers[4] = {{h->dz4, h->h3, H, kOffW4, kOffB4, h->w4t, h->z3, h->dz3},
                         {h->dz3, h->h2, H, kOffW3, kOffB3, h->w3t, h->z2, h->dz2},
                         {h->dz2, h->h1, H, kOffW2, kOffB2, h->w2t, h->z1, h->dz1},
                         {h->dz1, h->xp, KIN, kOffW1, kOffB1, nullptr, nullptr, nullptr}};
    for (const L& ly : layers) {
        if (ly.K == H) {
            hipLaunchKernelGGL(k_bwd_dw<H>, dim3((unsigned)ch, (H / 64) * (H / 64)), dim3(256), 0, st, ly.dz, ly.hprev,
                               n, h->part, h->bpart);
            hipLaunchKernelGGL(k_sum, dim3(blocks256((int64_t)H * H)), dim3(256), 0, st, h->part, (int)ch,
                               (int64_t)H * H, h->g + ly.offW);
        } else {
            hipLaunchKernelGGL(k_bwd_dw<KIN>, dim3((unsigned)ch, (H / 64)), dim3(256), 0, st, ly.dz, ly.hprev, n,
                               h->part, h->bpart);
            hipLaunchKernelGGL(k_sum_w1, dim3(blocks256((int64_t)H * kIn)), dim3(256), 0, st, h->part, (int)ch,
                               h->g + ly.offW);
        }
        hipLaunchKernelGGL(k_sum, dim3(blocks256(H)), dim3(256), 0, st, h->bpart, (int)ch, (int64_t)H, h->g + ly.offB);
        if (ly.wt)
            hipLaunchKernelGGL(k_bwd_dh, dim3(gb, H / 64), dim3(64), 0, st, ly.dz, ly.wt, ly.zprev, n, ly.dzprev);
    }
    if ((e = hipGetLastError())) return mhip(e, "mlp backward");
    if (sse) {
        const int64_t nl = (n + 255) / 256;
        h->lpart_host.resize(nl);
        if ((e = hipMemcpyAsync(h->lpart_host.data(), h->lpart, nl * 4, hipMemcpyDeviceToHost, st)) ||
            (e = hipStreamSynchronize(st)))
            return mhip(e, "mlp loss");
        double a = 0.0;
        for (float q : h->lpart_host) a += q;
        *sse = a;
    }
    return HJM_OK;
}

}  // namespace

extern "C" {

hjm_status hjm_mlp_workspace_bytes(int64_t max_batch, size_t* bytes)
{
    if (!bytes) return mfail(HJM_EINVAL, "null argument");
    if (max_batch < 1 || max_batch > ((int64_t)1 << 26)) return mfail(HJM_EINVAL, "max_batch outside [1, 2^26]");
    *bytes = mlp_layout(nullptr, nullptr, max_batch);
    return HJM_OK;
}

hjm_status hjm_mlp_create(const float box_lo[8], const float box_hi[8], float out_scale, float out_shift,
                          int64_t max_batch, void* d_workspace, size_t ws_bytes, void* hip_stream, hjm_mlp** out)
{
    if (!out) return mfail(HJM_EINVAL, "null output handle");
    *out = nullptr;
    if (!box_lo || !box_hi || !d_workspace) return mfail(HJM_EINVAL, "null argument");
    if (max_batch < 1 || max_batch > ((int64_t)1 << 26)) return mfail(HJM_EINVAL, "max_batch outside [1, 2^26]");
    for (int c = 0; c < kIn; ++c)
        if (!(std::isfinite(box_lo[c]) && std::isfinite(box_hi[c]) && box_lo[c] < box_hi[c]))
            return mfail(HJM_EINVAL, "box coordinate %d: need finite lo < hi", c);
    if (!(std::isfinite(out_scale) && std::isfinite(out_shift) && out_scale != 0.0f))
        return mfail(HJM_EINVAL, "output scale must be finite and nonzero");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256) return mfail(HJM_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = mlp_layout(nullptr, nullptr, max_batch);
    if (ws_bytes < need) return mfail(HJM_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    hjm_mlp* h = new (std::nothrow) hjm_mlp;
    if (!h) return mfail(HJM_EINVAL, "host allocation failed");
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    h->max_batch = max_batch;
    std::memcpy(h->lo, box_lo, sizeof h->lo);
    std::memcpy(h->hi, box_hi, sizeof h->hi);
    h->scale = out_scale;
    h->shift = out_shift;
    mlp_layout(h, reinterpret_cast<char*>(d_workspace), max_batch);
    float box[2 * kIn];
    std::memcpy(box, box_lo, kIn * 4);
    std::memcpy(box + kIn, box_hi, kIn * 4);
    hipError_t e;
    if ((e = hipMemcpyAsync(h->box, box, sizeof box, hipMemcpyHostToDevice, h->stream)) ||
        (e = hipMemsetAsync(h->p, 0, kParams * 4, h->stream)) || (e = hipMemsetAsync(h->m, 0, kParams * 4, h->stream)) ||
        (e = hipMemsetAsync(h->v, 0, kParams * 4, h->stream)) || (e = hipMemsetAsync(h->g, 0, kParams * 4, h->stream)) ||
        (e = cast_weights(h)) ||
        (e = hipStreamSynchronize(h->stream))) {
        delete h;
        return mhip(e, "hjm_mlp_create");
    }
    *out = h;
    return HJM_OK;
}

hjm_status hjm_mlp_set_params(hjm_mlp* h, const float* params, int64_t n)
{
    if (!h || !params) return mfail(HJM_EINVAL, "null argument");
    if (n != kParams) return mfail(HJM_EINVAL, "expected %lld parameters, got %lld", (long long)kParams, (long long)n);
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(params[i])) return mfail(HJM_EINVAL, "non-finite parameter %lld", (long long)i);
    hipError_t e;
    h->adam_t = 0;
    if ((e = hipMemcpyAsync(h->p, params, kParams * 4, hipMemcpyHostToDevice, h->stream)) ||
        (e = hipMemsetAsync(h->m, 0, kParams * 4, h->stream)) || (e = hipMemsetAsync(h->v, 0, kParams * 4, h->stream)) ||
        (e = cast_weights(h)) ||
        (e = hipStreamSynchronize(h->stream)))
        return mhip(e, "hjm_mlp_set_params");
    return HJM_OK;
}

hjm_status hjm_mlp_get_params(hjm_mlp* h, float* params, int64_t n)
{
    if (!h || !params) return mfail(HJM_EINVAL, "null argument");
    if (n != kParams) return mfail(HJM_EINVAL, "expected %lld parameters, got %lld", (long long)kParams, (long long)n);
    hipError_t e;
    if ((e = hipMemcpyAsync(params, h->p, kParams * 4, hipMemcpyDeviceToHost, h->stream)) ||
        (e = hipStreamSynchronize(h->stream)))
        return mhip(e, "hjm_mlp_get_params");
    return HJM_OK;
}

hjm_status hjm_mlp_gradients(hjm_mlp* h, const float* d_x, const float* d_t, int64_t n, double* sse)
{
    if (!h || !d_x || !d_t) return mfail(HJM_EINVAL, "null argument");
    if (n < 1 || n > h->max_batch) return mfail(HJM_EINVAL, "n=%lld outside [1, max_batch]", (long long)n);
    return gradients(h, d_x, d_t, n, sse);
}

hjm_status hjm_mlp_get_grads(hjm_mlp* h, float* grads, int64_t n)
{
    if (!h || !grads) return mfail(HJM_EINVAL, "null argument");
    if (n != kParams) return mfail(HJM_EINVAL, "expected %lld gradients, got %lld", (long long)kParams, (long long)n);
    hipError_t e;
    if ((e = hipMemcpyAsync(grads, h->g, kParams * 4, hipMemcpyDeviceToHost, h->stream)) ||
        (e = hipStreamSynchronize(h->stream)))
        return mhip(e, "hjm_mlp_get_grads");
    return HJM_OK;
}

hjm_status hjm_mlp_adam(hjm_mlp* h, float lr, float beta1, float beta2, float eps)
{
    if (!h) return mfail(HJM_EINVAL, "null handle");
    if (!(lr > 0.0f && beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f))
        return mfail(HJM_EINVAL, "invalid Adam hyper-parameters");
    h->adam_t += 1;
    const float c1 = 1.0f - std::pow(beta1, (float)h->adam_t);
    const float c2 = 1.0f - std::pow(beta2, (float)h->adam_t);
    hipLaunchKernelGGL(k_adam, dim3(blocks256(kParams)), dim3(256), 0, h->stream, h->p, h->m, h->v, h->g,
                       (int64_t)kParams, lr, beta1, beta2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    if (!e) e = cast_weights(h);
    if (e) return mhip(e, "hjm_mlp_adam");
    return HJM_OK;
}

hjm_status hjm_mlp_train_epoch(hjm_mlp* h, const float* d_x, const float* d_t, int64_t n, int64_t batch, float lr,
                               double* mean_loss)
{
    if (!h || !d_x || !d_t) return mfail(HJM_EINVAL, "null argument");
    if (n < 1 || batch < 1 || batch > h->max_batch) return mfail(HJM_EINVAL, "need n >= 1 and 1 <= batch <= max_batch");
    double sse = 0.0;
    for (int64_t s0 = 0; s0 < n; s0 += batch) {
        const int64_t nb = std::min(batch, n - s0);
        double part = 0.0;
        hjm_status st = gradients(h, d_x + s0 * kIn, d_t + s0, nb, mean_loss ? &part : nullptr);
        if (st) return st;
        sse += part;
        if ((st = hjm_mlp_adam(h, lr, 0.9f, 0.999f, 1e-8f))) return st;
    }
    if (mean_loss) *mean_loss = sse / (double)n;
    return HJM_OK;
}

hjm_status hjm_mlp_infer(hjm_mlp* h, const float* d_x, int64_t n, float* d_y, uint8_t* d_in_box)
{
    if (!h || !d_x || !d_y) return mfail(HJM_EINVAL, "null argument");
    if (n < 0) return mfail(HJM_EINVAL, "negative n");
    for (int64_t s0 = 0; s0 < n; s0 += h->max_batch) {
        const int64_t nb = std::min(h->max_batch, n - s0);
        hipLaunchKernelGGL(k_infer, dim3((unsigned)((nb + 63) / 64)), dim3(256), 0, h->stream, d_x + s0 * kIn, nb,
                           h->box, h->w1, h->w2, h->w3, h->w4, h->w5, h->p, h->scale, h->shift, h->base, d_y + s0,
                           d_in_box ? d_in_box + s0 : nullptr);
        hipError_t e = hipGetLastError();
        if (e) return mhip(e, "hjm_mlp_infer");
    }
    return HJM_OK;
}

hjm_status hjm_mlp_set_baseline(hjm_mlp* h, const hjm_mlp_baseline* b)
{
    if (!h) return mfail(HJM_EINVAL, "null handle");
    if (!b) {
        h->base = BaseK{};
        return HJM_OK;
    }
    if (!(std::isfinite(b->lambda) && std::isfinite(b->gamma) && std::isfinite(b->theta_v) &&
          std::isfinite(b->f_decay) && std::isfinite(b->tenor)))
        return mfail(HJM_EINVAL, "baseline constants must be finite");
    if (!(b->lambda > 0.0 && b->gamma >= 0.0 && b->gamma <= 1.0 && b->theta_v >= 0.0 && b->f_decay > 0.0 &&
          b->tenor > 0.0))
        return mfail(HJM_EINVAL, "baseline: need lambda > 0, gamma in [0, 1], theta_v >= 0, f_decay > 0, tenor > 0");
    h->base = BaseK{b->lambda, 2.0 * b->gamma, b->theta_v, b->f_decay, b->tenor, 1};
    return HJM_OK;
}

hjm_status hjm_mlp_targets(hjm_mlp* h, const float* d_x, const double* d_price, int64_t n, float* d_t)
{
    if (!h || !d_x || !d_price || !d_t) return mfail(HJM_EINVAL, "null argument");
    if (n < 0 || n > ((int64_t)1 << 31)) return mfail(HJM_EINVAL, "n outside [0, 2^31]");
    if (n == 0) return HJM_OK;
    hipLaunchKernelGGL(k_targets, dim3(blocks256(n)), dim3(256), 0, h->stream, d_x, d_price, n, h->scale, h->shift,
                       h->base, d_t);
    hipError_t e = hipGetLastError();
    if (e) return mhip(e, "hjm_mlp_targets");
    return HJM_OK;
}

hjm_status hjm_mlp_destroy(hjm_mlp* h)
{
    delete h;
    return HJM_OK;
}

}  // extern "C"
