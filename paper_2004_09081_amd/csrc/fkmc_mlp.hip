// Learned surrogate of the kMC diffusion coefficients: an ensemble of MLPs
// 4 -> 128 -> 128 -> 2 (SiLU), inputs (1000/T, x_H, log10 x_V, E_z/1e7 V/m),
// outputs (log10 D_O, log10 D_H), trained with Adam on a masked mean-square
// error of standardised targets.  Weights are used in BF16 with FP32
// accumulation; the 128x128 layer's forward product, its input gradient and
// its weight gradient run on MFMA (v_mfma_f32_16x16x32_bf16), the two thin
// layers (K = 4 and N = 2) on FP32 FMA.  One workgroup per ensemble member
// keeps the whole network and a 32-sample tile in LDS and runs every training
// step of a call in one launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fkmc.h"

namespace surrogate {

constexpr int kIn = 4, kH = 128, kOut = 2;
constexpr int kTile = 32;  // samples per tile
constexpr int kMaxBatch = 1024;
constexpr int kThreads = 256;
// parameter vector: W1[4][128], b1[128], W2[128][128] (in, out), b2[128], W3[128][2], b3[2]
constexpr int oW1 = 0, ob1 = oW1 + kIn * kH, oW2 = ob1 + kH, ob2 = oW2 + kH * kH,
              oW3 = ob2 + kH, ob3 = oW3 + kH * kOut, kParams = ob3 + kOut;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// fp32 -> bf16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float bf16_round(float f) { return from_bf16(to_bf16(f)); }

__device__ __forceinline__ float sigmoidf(float z) { return 1.0f / (1.0f + __expf(-z)); }

struct Norm {
    float xm[kIn], xs[kIn], ym[kOut], ys[kOut];
};

struct MlpDev {
    float* params;   // [members][kParams] fp32 masters
    float* adam_m;
    float* adam_v;
    float* grads;    // [members][kParams] (gradient mode)
    float* loss;     // [members]
    Norm* norm;
    const float* X;  // [n][4]
    const float* Y;  // [n][2]
    const float* M;  // [n][2] mask (1 valid, 0 ignored)
    int n;
    int members;
    uint32_t seed;
};

// LDS layout (bytes)
constexpr int L_W2 = 0;                                  // bf16 [in][out]
constexpr int L_W2T = L_W2 + kH * kH * 2;                // bf16 [out][in]
constexpr int L_Z1 = L_W2T + kH * kH * 2;                // f32 [32][128]
constexpr int L_Z2 = L_Z1 + kTile * kH * 4;              // f32 [32][128] (z2, later dh1)
constexpr int L_H1 = L_Z2 + kTile * kH * 4;              // bf16 [32][128]
constexpr int L_H1T = L_H1 + kTile * kH * 2;             // bf16 [128][32]
constexpr int L_DZ = L_H1T + kTile * kH * 2;             // bf16 dz2 [32][128] + dz2T [128][32]
                                                         // (holds h2 f32 [32][128] before)
constexpr int L_W1 = L_DZ + kTile * kH * 4;              // f32 (bf16-rounded) [4][128]
constexpr int L_B1 = L_W1 + kIn * kH * 4;
constexpr int L_B2 = L_B1 + kH * 4;
constexpr int L_W3 = L_B2 + kH * 4;                      // f32 (bf16-rounded) [128][2]
constexpr int L_B3 = L_W3 + kH * kOut * 4;               // 4 floats
constexpr int L_X = L_B3 + 16;                           // f32 [32][4]
constexpr int L_T = L_X + kTile * kIn * 4;               // f32 [32][2]
constexpr int L_MK = L_T + kTile * kOut * 4;
constexpr int L_DY = L_MK + kTile * kOut * 4;
constexpr int L_GW1 = L_DY + kTile * kOut * 4;           // grads of the thin layers
constexpr int L_GB1 = L_GW1 + kIn * kH * 4;
constexpr int L_GB2 = L_GB1 + kH * 4;
constexpr int L_GW3 = L_GB2 + kH * 4;
constexpr int L_GB3 = L_GW3 + kH * kOut * 4;             // 4 floats
constexpr int L_IDX = L_GB3 + 16;                        // int [kMaxBatch]
constexpr int L_RED = L_IDX + kMaxBatch * 4;             // 16 floats
constexpr int kLdsBytes = L_RED + 64;

struct Lds {
    unsigned char* base;
    __device__ uint16_t* W2() const { return (uint16_t*)(base + L_W2); }
    __device__ uint16_t* W2T() const { return (uint16_t*)(base + L_W2T); }
    __device__ float* Z1() const { return (float*)(base + L_Z1); }
    __device__ float* Z2() const { return (float*)(base + L_Z2); }
    __device__ uint16_t* H1() const { return (uint16_t*)(base + L_H1); }
    __device__ uint16_t* H1T() const { return (uint16_t*)(base + L_H1T); }
    __device__ float* H2() const { return (float*)(base + L_DZ); }
    __device__ uint16_t* DZ() const { return (uint16_t*)(base + L_DZ); }
    __device__ uint16_t* DZT() const { return (uint16_t*)(base + L_DZ + kTile * kH * 2); }
    __device__ float* W1() const { return (float*)(base + L_W1); }
    __device__ float* B1() const { return (float*)(base + L_B1); }
    __device__ float* B2() const { return (float*)(base + L_B2); }
    __device__ float* W3() const { return (float*)(base + L_W3); }
    __device__ float* B3() const { return (float*)(base + L_B3); }
    __device__ float* X() const { return (float*)(base + L_X); }
    __device__ float* T() const { return (float*)(base + L_T); }
    __device__ float* MK() const { return (float*)(base + L_MK); }
    __device__ float* DY() const { return (float*)(base + L_DY); }
    __device__ float* GW1() const { return (float*)(base + L_GW1); }
    __device__ float* GB1() const { return (float*)(base + L_GB1); }
    __device__ float* GB2() const { return (float*)(base + L_GB2); }
    __device__ float* GW3() const { return (float*)(base + L_GW3); }
    __device__ float* GB3() const { return (float*)(base + L_GB3); }
    __device__ int* IDX() const { return (int*)(base + L_IDX); }
    __device__ float* RED() const { return (float*)(base + L_RED); }
};

__device__ __forceinline__ bf16x8 load8(const uint16_t* p)
{
    return *(const bf16x8*)p;
}

// Philox4x32-10 (Salmon et al., SC'11) for minibatch sampling and init.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; r++) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Copy member's weights (bf16-rounded) into LDS.
__device__ void load_weights(const Lds& S, const float* p, int tid)
{
    for (int e = tid; e < kH * kH; e += kThreads) {
        const int i = e / kH, j = e % kH;
        const uint16_t h = to_bf16(p[oW2 + e]);
        S.W2()[i * kH + j] = h;
        S.W2T()[j * kH + i] = h;
    }
    for (int e = tid; e < kIn * kH; e += kThreads) S.W1()[e] = bf16_round(p[oW1 + e]);
    for (int e = tid; e < kH * kOut; e += kThreads) S.W3()[e] = bf16_round(p[oW3 + e]);
    if (tid < kH) {
        S.B1()[tid] = p[ob1 + tid];
        S.B2()[tid] = p[ob2 + tid];
    }
    if (tid < kOut) S.B3()[tid] = p[ob3 + tid];
}

__device__ void zero_small_grads(const Lds& S, int tid)
{
    for (int e = tid; e < kIn * kH; e += kThreads) S.GW1()[e] = 0.f;
    for (int e = tid; e < kH * kOut; e += kThreads) S.GW3()[e] = 0.f;
    if (tid < kH) {
        S.GB1()[tid] = 0.f;
        S.GB2()[tid] = 0.f;
    }
    if (tid < 4) S.GB3()[tid] = 0.f;
}

// Forward through layers 1-2 for the 32 samples in S.X: z1, h1 (bf16,
// both layouts), z2 (MFMA).  Ends with a barrier.
__device__ void forward12(const Lds& S, int tid, int wave, int lane)
{
    for (int e = tid; e < kTile * kH; e += kThreads) {
        const int r = e / kH, i = e % kH;
        float z = S.B1()[i];
#pragma unroll
        for (int a = 0; a < kIn; a++) z = __fmaf_rn(S.X()[r * kIn + a], S.W1()[a * kH + i], z);
        S.Z1()[e] = z;
        const uint16_t h = to_bf16(z * sigmoidf(z));
        S.H1()[r * kH + i] = h;
        S.H1T()[i * kTile + r] = h;
    }
    __syncthreads();
    // z2 = h1 . W2 + b2: 2 x 8 output tiles of 16x16, 4 per wave, K = 128
    const int q = lane >> 4, c = lane & 15;
    for (int t = wave; t < 16; t += 4) {
        const int rm = t >> 3, cn = t & 7;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < kH / 32; kk++) {
            const bf16x8 a = load8(S.H1() + (rm * 16 + c) * kH + kk * 32 + 8 * q);
            const bf16x8 b = load8(S.W2T() + (cn * 16 + c) * kH + kk * 32 + 8 * q);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
        }
        const int col = cn * 16 + c;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int row = rm * 16 + 4 * q + e;
            S.Z2()[row * kH + col] = acc[e] + S.B2()[col];
        }
    }
    __syncthreads();
}

// y = h2 . W3 + b3 for the tile (h2 = silu(z2) stored in S.H2()).
__device__ void forward3(const Lds& S, int tid, float* y_out /* [32][2] or null */)
{
    for (int e = tid; e < kTile * kH; e += kThreads) {
        const float z = S.Z2()[e];
        S.H2()[e] = z * sigmoidf(z);
    }
    __syncthreads();
    if (tid < kTile * kOut) {
        const int r = tid >> 1, o = tid & 1;
        float y = S.B3()[o];
        for (int j = 0; j < kH; j++) y = __fmaf_rn(S.H2()[r * kH + j], S.W3()[j * kOut + o], y);
        if (y_out) y_out[tid] = y;
        S.DY()[tid] = y;  // raw output, turned into dL/dy by the caller
    }
    __syncthreads();
}

// Backward of one tile given dL/dy in S.DY(); accumulates the thin-layer
// gradients in LDS and the 128x128 weight gradient in gw2 (registers).
__device__ void backward_tile(const Lds& S, int tid, int wave, int lane, f32x4 (&gw2)[16])
{
    // thin layer 3
    if (tid < kH * kOut) {
        const int j = tid >> 1, o = tid & 1;
        float g = 0.f;
        for (int r = 0; r < kTile; r++) g = __fmaf_rn(S.H2()[r * kH + j], S.DY()[r * kOut + o], g);
        S.GW3()[j * kOut + o] += g;
    }
    if (tid < kOut) {
        float g = 0.f;
        for (int r = 0; r < kTile; r++) g += S.DY()[r * kOut + tid];
        S.GB3()[tid] += g;
    }
    __syncthreads();
    // dz2 = (dy . W3^T) * silu'(z2); gb2; bf16 copies in both layouts
    if (tid < kH) {
        const int j = tid;
        float gb = 0.f;
        for (int r = 0; r < kTile; r++) {
            const float dh = S.DY()[r * kOut] * S.W3()[j * kOut] + S.DY()[r * kOut + 1] * S.W3()[j * kOut + 1];
            const float z = S.Z2()[r * kH + j];
            const float s = sigmoidf(z);
            const float d = dh * (s * (1.f + z * (1.f - s)));
            gb += d;
            const uint16_t h = to_bf16(d);
            S.DZ()[r * kH + j] = h;
            S.DZT()[j * kTile + r] = h;
        }
        S.GB2()[j] += gb;
    }
    __syncthreads();
    const int q = lane >> 4, c = lane & 15;
    // gW2 += h1^T . dz2 (8 x 8 tiles of 16x16, 16 per wave, K = 32)
#pragma unroll
    for (int u = 0; u < 16; u++) {
        const int t = wave + 4 * u;
        const int rm = t >> 3, cn = t & 7;
        const bf16x8 a = load8(S.H1T() + (rm * 16 + c) * kTile + 8 * q);
        const bf16x8 b = load8(S.DZT() + (cn * 16 + c) * kTile + 8 * q);
        gw2[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, gw2[u], 0, 0, 0);
    }
    // dh1 = dz2 . W2^T into the z2 buffer (2 x 8 tiles, K = 128)
    for (int t = wave; t < 16; t += 4) {
        const int rm = t >> 3, cn = t & 7;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < kH / 32; kk++) {
            const bf16x8 a = load8(S.DZ() + (rm * 16 + c) * kH + kk * 32 + 8 * q);
            const bf16x8 b = load8(S.W2() + (cn * 16 + c) * kH + kk * 32 + 8 * q);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
        }
        // z2 was last read in the dz2 pass, which ended with a barrier
        const int col = cn * 16 + c;
#pragma unroll
        for (int e = 0; e < 4; e++) S.Z2()[(rm * 16 + 4 * q + e) * kH + col] = acc[e];
    }
    __syncthreads();
    // dz1 = dh1 * silu'(z1); gb1, gW1
    if (tid < kH) {
        const int i = tid;
        float gb = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f;
        for (int r = 0; r < kTile; r++) {
            const float z = S.Z1()[r * kH + i];
            const float s = sigmoidf(z);
            const float d = S.Z2()[r * kH + i] * (s * (1.f + z * (1.f - s)));
            gb += d;
            g0 = __fmaf_rn(S.X()[r * kIn + 0], d, g0);
            g1 = __fmaf_rn(S.X()[r * kIn + 1], d, g1);
            g2 = __fmaf_rn(S.X()[r * kIn + 2], d, g2);
            g3 = __fmaf_rn(S.X()[r * kIn + 3], d, g3);
        }
        S.GB1()[i] += gb;
        S.GW1()[0 * kH + i] += g0;
        S.GW1()[1 * kH + i] += g1;
        S.GW1()[2 * kH + i] += g2;
        S.GW1()[3 * kH + i] += g3;
    }
    __syncthreads();
}

// Load tile rows idx[0..cnt) (standardised inputs/targets, masks).
__device__ void load_tile(const Lds& S, const MlpDev& P, const int* idx, int cnt, int tid)
{
    const Norm& N = *P.norm;
    if (tid < kTile * kIn) {
        const int r = tid / kIn, a = tid % kIn;
        S.X()[tid] = r < cnt ? (P.X[(size_t)idx[r] * kIn + a] - N.xm[a]) / N.xs[a] : 0.f;
    }
    if (tid < kTile * kOut) {
        const int r = tid / kOut, o = tid % kOut;
        const bool ok = r < cnt;
        const size_t g = ok ? (size_t)idx[r] * kOut + o : 0;
        const float mk = ok ? P.M[g] : 0.f;
        S.MK()[tid] = mk;
        S.T()[tid] = (ok && mk != 0.f) ? (P.Y[g] - N.ym[o]) / N.ys[o] : 0.f;
    }
    __syncthreads();
}

// mode 0: `steps` Adam steps on minibatches of `batch` samples drawn with
// replacement (batch 0: the whole data set in order).  mode 1: gradient of
// the loss over the whole data set, written to P.grads, no update.
__global__ __launch_bounds__(kThreads) void k_train(MlpDev P, int mode, int steps, int batch,
                                                    float lr, int step0)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Lds S{smem};
    const int member = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    float* p = P.params + (size_t)member * kParams;
    float* am = P.adam_m + (size_t)member * kParams;
    float* av = P.adam_v + (size_t)member * kParams;
    const bool full = batch <= 0 || mode == 1;
    const int B = full ? P.n : batch;
    float loss_last = 0.f;
    for (int st = 0; st < steps; st++) {
        load_weights(S, p, tid);
        zero_small_grads(S, tid);
        if (tid < 8) S.RED()[tid] = 0.f;
        __syncthreads();
        // minibatch indices and per-output valid counts
        if (!full) {
            for (int r = tid; r < B; r += kThreads) {
                const uint4 x = philox((uint32_t)r, (uint32_t)(step0 + st), (uint32_t)member, 0x5A11u,
                                       P.seed, 0xB10Cu);
                S.IDX()[r] = (int)__umulhi(x.x, (uint32_t)P.n);
            }
            __syncthreads();
        }
        {
            float c0 = 0.f, c1 = 0.f;
            for (int r = tid; r < B; r += kThreads) {
                const int i = full ? r : S.IDX()[r];
                c0 += P.M[(size_t)i * kOut];
                c1 += P.M[(size_t)i * kOut + 1];
            }
            atomicAdd(&S.RED()[0], c0);
            atomicAdd(&S.RED()[1], c1);
        }
        __syncthreads();
        const float cnt0 = fmaxf(S.RED()[0], 1.f), cnt1 = fmaxf(S.RED()[1], 1.f);
        f32x4 gw2[16];
#pragma unroll
        for (int u = 0; u < 16; u++) gw2[u] = f32x4{0.f, 0.f, 0.f, 0.f};
        float loss = 0.f;
        for (int t0 = 0; t0 < B; t0 += kTile) {
            const int cnt = B - t0 < kTile ? B - t0 : kTile;
            // indices of this tile
            __shared__ int tidx[kTile];
            if (tid < kTile) tidx[tid] = tid < cnt ? (full ? t0 + tid : S.IDX()[t0 + tid]) : 0;
            __syncthreads();
            load_tile(S, P, tidx, cnt, tid);
            forward12(S, tid, wave, lane);
            forward3(S, tid, nullptr);
            if (tid < kTile * kOut) {
                const int o = tid & 1;
                const float y = S.DY()[tid];
                const float e = (y - S.T()[tid]) * S.MK()[tid];
                loss += e * e / (o ? cnt1 : cnt0);
                S.DY()[tid] = 2.f * e / (o ? cnt1 : cnt0);
            }
            __syncthreads();
            backward_tile(S, tid, wave, lane, gw2);
        }
        atomicAdd(&S.RED()[2], loss);
        __syncthreads();
        loss_last = S.RED()[2];
        if (mode == 1) {
            float* g = P.grads + (size_t)member * kParams;
            const int q = lane >> 4, c = lane & 15;
#pragma unroll
            for (int u = 0; u < 16; u++) {
                const int t = wave + 4 * u, rm = t >> 3, cn = t & 7;
#pragma unroll
                for (int e = 0; e < 4; e++)
                    g[oW2 + (rm * 16 + 4 * q + e) * kH + cn * 16 + c] = gw2[u][e];
            }
            for (int e = tid; e < kIn * kH; e += kThreads) g[oW1 + e] = S.GW1()[e];
            for (int e = tid; e < kH * kOut; e += kThreads) g[oW3 + e] = S.GW3()[e];
            if (tid < kH) {
                g[ob1 + tid] = S.GB1()[tid];
                g[ob2 + tid] = S.GB2()[tid];
            }
            if (tid < kOut) g[ob3 + tid] = S.GB3()[tid];
            break;
        }
        // Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the fp32 masters
        const int tstep = step0 + st + 1;
        const float c1 = 1.f - powf(0.9f, (float)tstep), c2 = 1.f - powf(0.999f, (float)tstep);
        auto adam = [&](int k, float g) {
            const float m = 0.9f * am[k] + 0.1f * g;
            const float v = 0.999f * av[k] + 0.001f * g * g;
            am[k] = m;
            av[k] = v;
            p[k] -= lr * (m / c1) / (sqrtf(v / c2) + 1e-8f);
        };
        {
            const int q = lane >> 4, c = lane & 15;
#pragma unroll
            for (int u = 0; u < 16; u++) {
                const int t = wave + 4 * u, rm = t >> 3, cn = t & 7;
#pragma unroll
                for (int e = 0; e < 4; e++) adam(oW2 + (rm * 16 + 4 * q + e) * kH + cn * 16 + c, gw2[u][e]);
            }
        }
        for (int e = tid; e < kIn * kH; e += kThreads) adam(oW1 + e, S.GW1()[e]);
        for (int e = tid; e < kH * kOut; e += kThreads) adam(oW3 + e, S.GW3()[e]);
        if (tid < kH) {
            adam(ob1 + tid, S.GB1()[tid]);
            adam(ob2 + tid, S.GB2()[tid]);
        }
        if (tid < kOut) adam(ob3 + tid, S.GB3()[tid]);
        __threadfence_block();
        __syncthreads();
    }
    if (tid == 0) P.loss[member] = loss_last;
}

// Ensemble prediction for samples [blockIdx.x*32, +32): per-member outputs
// de-standardised, then mean and population std across members.
__global__ __launch_bounds__(kThreads) void k_predict(MlpDev P, const float* X, int n, float* mean,
                                                      float* stdev, float* each)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Lds S{smem};
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int t0 = blockIdx.x * kTile;
    const int cnt = n - t0 < kTile ? n - t0 : kTile;
    const Norm& N = *P.norm;
    float s1 = 0.f, s2 = 0.f;
    for (int m = 0; m < P.members; m++) {
        load_weights(S, P.params + (size_t)m * kParams, tid);
        if (tid < kTile * kIn) {
            const int r = tid / kIn, a = tid % kIn;
            S.X()[tid] = r < cnt ? (X[(size_t)(t0 + r) * kIn + a] - N.xm[a]) / N.xs[a] : 0.f;
        }
        __syncthreads();
        forward12(S, tid, wave, lane);
        forward3(S, tid, nullptr);
        if (tid < kTile * kOut) {
            const int o = tid & 1;
            const float y = S.DY()[tid] * N.ys[o] + N.ym[o];
            s1 += y;
            s2 += y * y;
            const int r = tid >> 1;
            if (each && r < cnt) each[((size_t)m * n + t0 + r) * kOut + o] = y;
        }
        __syncthreads();
    }
    if (tid < kTile * kOut) {
        const int r = tid >> 1, o = tid & 1;
        if (r < cnt) {
            const float mu = s1 / (float)P.members;
            const float var = fmaxf(s2 / (float)P.members - mu * mu, 0.f);
            mean[(size_t)(t0 + r) * kOut + o] = mu;
            stdev[(size_t)(t0 + r) * kOut + o] = sqrtf(var);
        }
    }
}

// Mean and population std of the inputs and of the valid targets.
__global__ __launch_bounds__(kThreads) void k_norm(MlpDev P)
{
    __shared__ double acc[16][kThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double s[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    double c0 = 0, c1 = 0;
    for (int i = tid; i < P.n; i += kThreads) {
        for (int a = 0; a < kIn; a++) {
            const double x = P.X[(size_t)i * kIn + a];
            s[a] += x;
            s[4 + a] += x * x;
        }
        for (int o = 0; o < kOut; o++) {
            const double mk = P.M[(size_t)i * kOut + o];
            const double y = mk != 0.0 ? P.Y[(size_t)i * kOut + o] : 0.0;
            s[8 + o] += y;
            s[10 + o] += y * y;
        }
        c0 += P.M[(size_t)i * kOut];
        c1 += P.M[(size_t)i * kOut + 1];
    }
    double v[14];
    for (int k = 0; k < 12; k++) v[k] = s[k];
    v[12] = c0;
    v[13] = c1;
    for (int k = 0; k < 14; k++) {
        double x = v[k];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) acc[k][wave] = x;
    }
    __syncthreads();
    if (tid == 0) {
        double t[14];
        for (int k = 0; k < 14; k++) {
            t[k] = 0;
            for (int w = 0; w < kThreads / 64; w++) t[k] += acc[k][w];
        }
        Norm N;
        for (int a = 0; a < kIn; a++) {
            const double m = t[a] / P.n;
            const double var = t[4 + a] / P.n - m * m;
            N.xm[a] = (float)m;
            N.xs[a] = (float)(var > 1e-24 ? sqrt(var) : 1.0);
        }
        for (int o = 0; o < kOut; o++) {
            const double c = t[12 + o] > 0 ? t[12 + o] : 1.0;
            const double m = t[8 + o] / c;
            const double var = t[10 + o] / c - m * m;
            N.ym[o] = (float)m;
            N.ys[o] = (float)(var > 1e-24 ? sqrt(var) : 1.0);
        }
        *P.norm = N;
    }
}

// He-normal initialisation (Box-Muller on Philox draws), zero biases and
// Adam moments.
__global__ void k_init_params(MlpDev P)
{
    const int member = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kParams) return;
    float* p = P.params + (size_t)member * kParams;
    int fan_in = 0;
    if (k < ob1) fan_in = kIn;
    else if (k >= oW2 && k < ob2) fan_in = kH;
    else if (k >= oW3 && k < ob3) fan_in = kH;
    float w = 0.f;
    if (fan_in) {
        const uint4 x = philox((uint32_t)k, (uint32_t)member, 0u, 0x1E17u, P.seed, 0xB10Cu);
        const float u1 = ((x.x >> 8) + 1) * (1.0f / 16777216.0f);
        const float u2 = (x.y >> 8) * (1.0f / 16777216.0f);
        const float g = sqrtf(-2.f * logf(u1)) * cosf(6.283185307179586f * u2);
        w = g * sqrtf(2.f / (float)fan_in);
    }
    p[k] = w;
    P.adam_m[(size_t)member * kParams + k] = 0.f;
    P.adam_v[(size_t)member * kParams + k] = 0.f;
}

}  // namespace surrogate

// ----------------------------------------------------------------------------
// C ABI (include/fkmc.h)
using namespace surrogate;

struct fkmc_mlp {
    MlpDev P;
    hipStream_t stream;
    uint32_t max_samples;
    int step;
};

namespace {
size_t mlp_align(size_t x) { return (x + 255) & ~(size_t)255; }
}

extern "C" {

uint32_t fkmc_mlp_param_count(void) { return (uint32_t)kParams; }

fkmc_status fkmc_mlp_query_sizes(uint32_t members, uint32_t max_samples, size_t* bytes)
{
    if (!bytes || members == 0 || members > 64 || max_samples == 0) return FKMC_E_INVALID;
    const size_t pb = mlp_align((size_t)members * kParams * 4);
    *bytes = 4 * pb + mlp_align(members * 4) + mlp_align(sizeof(Norm)) +
             mlp_align((size_t)max_samples * 4 * 4);
    return FKMC_OK;
}

fkmc_status fkmc_mlp_create(uint32_t members, uint32_t seed, uint32_t max_samples, void* work,
                            size_t bytes, void* stream, fkmc_mlp** out)
{
    size_t need = 0;
    if (!out || !work) return FKMC_E_INVALID;
    if (fkmc_mlp_query_sizes(members, max_samples, &need) != FKMC_OK) return FKMC_E_INVALID;
    if (bytes < need || ((uintptr_t)work & 255)) return FKMC_E_NOMEM;
    fkmc_mlp* h = new fkmc_mlp();
    char* w = (char*)work;
    const size_t pb = mlp_align((size_t)members * kParams * 4);
    h->P.params = (float*)w;
    h->P.adam_m = (float*)(w + pb);
    h->P.adam_v = (float*)(w + 2 * pb);
    h->P.grads = (float*)(w + 3 * pb);
    h->P.loss = (float*)(w + 4 * pb);
    h->P.norm = (Norm*)(w + 4 * pb + mlp_align(members * 4));
    h->P.members = (int)members;
    h->P.seed = seed;
    h->P.n = 0;
    h->stream = (hipStream_t)stream;
    h->max_samples = max_samples;
    h->step = 0;
    hipLaunchKernelGGL(k_init_params, dim3((kParams + 255) / 256, members), dim3(256), 0, h->stream, h->P);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess) {
        delete h;
        return FKMC_E_DEVICE;
    }
    if (hipFuncSetAttribute((const void*)k_train, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_predict, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes) != hipSuccess) {
        delete h;
        return FKMC_E_DEVICE;
    }
    *out = h;
    return FKMC_OK;
}

fkmc_status fkmc_mlp_destroy(fkmc_mlp* h)
{
    if (h) {
        (void)hipStreamSynchronize(h->stream);
        delete h;
    }
    return FKMC_OK;
}

fkmc_status fkmc_mlp_set_data(fkmc_mlp* h, const float* X, const float* Y, const float* mask, uint32_t n)
{
    if (!h || !X || !Y || !mask || n == 0) return FKMC_E_INVALID;
    h->P.X = X;
    h->P.Y = Y;
    h->P.M = mask;
    h->P.n = (int)n;
    hipLaunchKernelGGL(k_norm, dim3(1), dim3(kThreads), 0, h->stream, h->P);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess) return FKMC_E_DEVICE;
    return FKMC_OK;
}

fkmc_status fkmc_mlp_train(fkmc_mlp* h, uint32_t steps, uint32_t batch, float lr, float* loss_out)
{
    if (!h || h->P.n == 0 || batch > (uint32_t)kMaxBatch) return FKMC_E_INVALID;
    if (steps == 0) return FKMC_OK;
    hipLaunchKernelGGL(k_train, dim3(h->P.members), dim3(kThreads), kLdsBytes, h->stream, h->P, 0,
                       (int)steps, (int)batch, lr, h->step);
    if (hipGetLastError() != hipSuccess) return FKMC_E_DEVICE;
    h->step += (int)steps;
    if (loss_out) {
        if (hipMemcpyAsync(loss_out, h->P.loss, h->P.members * 4, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess)
            return FKMC_E_DEVICE;
    }
    return FKMC_OK;
}

fkmc_status fkmc_mlp_grad(fkmc_mlp* h, float* grads_out, float* loss_out)
{
    if (!h || h->P.n == 0 || !grads_out) return FKMC_E_INVALID;
    hipLaunchKernelGGL(k_train, dim3(h->P.members), dim3(kThreads), kLdsBytes, h->stream, h->P, 1, 1, 0,
                       0.f, h->step);
    if (hipGetLastError() != hipSuccess) return FKMC_E_DEVICE;
    if (hipMemcpyAsync(grads_out, h->P.grads, (size_t)h->P.members * kParams * 4, hipMemcpyDeviceToHost, h->stream) != hipSuccess)
        return FKMC_E_DEVICE;
    if (loss_out && hipMemcpyAsync(loss_out, h->P.loss, h->P.members * 4, hipMemcpyDeviceToHost, h->stream) != hipSuccess)
        return FKMC_E_DEVICE;
    return hipStreamSynchronize(h->stream) == hipSuccess ? FKMC_OK : FKMC_E_DEVICE;
}

fkmc_status fkmc_mlp_predict(fkmc_mlp* h, const float* X, uint32_t n, float* mean, float* stdev, float* each)
{
    if (!h || !X || !mean || !stdev || n == 0) return FKMC_E_INVALID;
    hipLaunchKernelGGL(k_predict, dim3((n + kTile - 1) / kTile), dim3(kThreads), kLdsBytes, h->stream,
                       h->P, X, (int)n, mean, stdev, each);
    return hipGetLastError() == hipSuccess ? FKMC_OK : FKMC_E_DEVICE;
}

fkmc_status fkmc_mlp_get_params(fkmc_mlp* h, float* host, size_t n)
{
    if (!h || !host || n != (size_t)h->P.members * kParams) return FKMC_E_INVALID;
    if (hipMemcpyAsync(host, h->P.params, n * 4, hipMemcpyDeviceToHost, h->stream) != hipSuccess) return FKMC_E_DEVICE;
    return hipStreamSynchronize(h->stream) == hipSuccess ? FKMC_OK : FKMC_E_DEVICE;
}

fkmc_status fkmc_mlp_set_params(fkmc_mlp* h, const float* host, size_t n)
{
    if (!h || !host || n != (size_t)h->P.members * kParams) return FKMC_E_INVALID;
    if (hipMemcpyAsync(h->P.params, host, n * 4, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemsetAsync(h->P.adam_m, 0, n * 4, h->stream) != hipSuccess ||
        hipMemsetAsync(h->P.adam_v, 0, n * 4, h->stream) != hipSuccess)
        return FKMC_E_DEVICE;
    h->step = 0;
    return hipStreamSynchronize(h->stream) == hipSuccess ? FKMC_OK : FKMC_E_DEVICE;
}

fkmc_status fkmc_mlp_get_norm(fkmc_mlp* h, float* host12)
{
    if (!h || !host12) return FKMC_E_INVALID;
    if (hipMemcpyAsync(host12, h->P.norm, sizeof(Norm), hipMemcpyDeviceToHost, h->stream) != hipSuccess) return FKMC_E_DEVICE;
    return hipStreamSynchronize(h->stream) == hipSuccess ? FKMC_OK : FKMC_E_DEVICE;
}

}  // extern "C"
