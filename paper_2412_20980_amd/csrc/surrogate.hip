// Learned screening surrogate (an extension; the paper evaluates every
// offspring exactly).  A generation makes lambda children with the usual
// operators; a small network predicts their fitness from summed node
// embeddings and only the `screen` children with the lowest predictions are
// evaluated exactly and enter elitism.  The network trains online on the
// exactly evaluated children.
//
//   x(S) = sum_{v in S} E[v]                          E [n][64]
//   yhat = w3 . relu(W2 relu(W1 x + b1) + b2) + b3    64 -> 256 -> 256 -> 1
//
// FP32 master weights and Adam moments; bfloat16 copies feed the matrix-core
// products (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  The embedding
// gather is the memory-bound part (k rows of 128 bytes per prediction); the
// MLP is a few hundred MFMAs per 16 samples.  Everything is deterministic:
// fixed summation orders, no floating-point atomics; the embedding gradient
// is a per-node sum over the batch samples that contain the node, in sample
// order, read from node-major membership bit rows.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device_common.h"
#include "internal.h"

namespace gapa {
namespace {

constexpr int kD = 64;
constexpr int kH = 256;
constexpr int kMlpRows = 64;  // samples per MLP block, 16 per wave
constexpr uint32_t kStreamSurrInit = 5, kStreamSurrSample = 6, kStreamSurrRandom = 7;
constexpr int kJudgeMax = 1024;
constexpr int kJudgeExtra = 32;  // unscreened children evaluated for the judge in a screened generation
constexpr int kMaxLambda = 8192;

// flat layout of the MLP parameters after E (weights, gradients, partials)
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH * kD;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kH;
constexpr int kMlpParams = kOffB3 + 1;

// LDS of the MLP kernel (bf16 elements): X [64][72], H1, DZ2, DZ1 [64][264]
constexpr int kSX = 72, kSH = 264;
constexpr size_t kMlpLds = 2 * ((size_t)kMlpRows * kSX + 3 * (size_t)kMlpRows * kSH) + 4 * (4 * kH + 4);

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest, ties to even
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h)
{
    return __uint_as_float((uint32_t)h << 16);
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t *p)  // 16-byte aligned
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p));
}

__device__ __forceinline__ bf16x8 gather8(const uint16_t *p, int stride)
{
    uint16_t t[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) t[e] = p[e * stride];
    uint4 q;
    q.x = t[0] | ((uint32_t)t[1] << 16);
    q.y = t[2] | ((uint32_t)t[3] << 16);
    q.z = t[4] | ((uint32_t)t[5] << 16);
    q.w = t[6] | ((uint32_t)t[7] << 16);
    return __builtin_bit_cast(bf16x8, q);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------ parameters ----

// Initial weights: element (r, c) of tensor t (E 0, W1 1, W2 2, w3 3) is
// bound_t * (2u - 1), u = (w + 1/2) / 2^32 from draw(seed, c, r, t, stream 5),
// in double, rounded to float; biases 0.
__global__ void k_surr_init(float *__restrict__ theta, int64_t n, uint64_t seed, double bE, double bW1, double bW2,
                            double bw3)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nE = n * kD;
    if (i >= nE + kMlpParams) return;
    uint32_t t = 0, r = 0, c = 0;
    double bound = 0.0;
    if (i < nE) {
        t = 0, r = (uint32_t)(i / kD), c = (uint32_t)(i % kD), bound = bE;
    } else {
        const int32_t j = (int32_t)(i - nE);
        if (j < kOffB1) t = 1, r = j / kD, c = j % kD, bound = bW1;
        else if (j >= kOffW2 && j < kOffB2) t = 2, r = (j - kOffW2) / kH, c = (j - kOffW2) % kH, bound = bW2;
        else if (j >= kOffW3 && j < kOffB3) t = 3, r = 0, c = j - kOffW3, bound = bw3;
    }
    float val = 0.f;
    if (bound > 0.0) {
        const Words4 w = draw(seed, c, r, t, kStreamSurrInit, 0);
        const double u = ((double)w.w0 + 0.5) * (1.0 / 4294967296.0);
        val = (float)(bound * (2.0 * u - 1.0));
    }
    theta[i] = val;
}

struct Bf16Copies {
    uint16_t *Eb, *W1b, *W1bT, *W2b, *W2bT, *w3b;
};

// bfloat16 copy of MLP parameter j (and its transposed position).
__device__ __forceinline__ void mlp_copy(const Bf16Copies &o, int32_t j, float x)
{
    const uint16_t h = f2bf(x);
    if (j < kOffB1) {
        const int32_t r = j / kD, c = j % kD;
        o.W1b[j] = h;
        o.W1bT[c * kH + r] = h;
    } else if (j >= kOffW2 && j < kOffB2) {
        const int32_t q = j - kOffW2, r = q / kH, c = q % kH;
        o.W2b[q] = h;
        o.W2bT[c * kH + r] = h;
    } else if (j >= kOffW3 && j < kOffB3) {
        o.w3b[j - kOffW3] = h;
    }
}

__global__ void k_bf16_copies(const float *__restrict__ theta, int64_t n, Bf16Copies o)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nE = n * kD;
    if (i >= nE + kMlpParams) return;
    if (i < nE) o.Eb[i] = f2bf(theta[i]);
    else mlp_copy(o, (int32_t)(i - nE), theta[i]);
}

// ------------------------------------------------------------- embedding ----

// x(S) of each row, rounded to bf16: one 256-thread block per row.  Lane
// (wave w, group g = lane / 16, q = lane % 16) adds dims 4q..4q+3 of genes
// j = 16 i + 4 w + g; the four groups and the four waves are then added in a
// fixed order.
__global__ __launch_bounds__(256) void k_embed(const int32_t *__restrict__ genes, const int32_t *__restrict__ rows,
                                               int32_t k, const uint16_t *__restrict__ Eb, uint16_t *__restrict__ xb)
{
    __shared__ float s_part[4][kD];
    const int32_t row = rows ? rows[blockIdx.x] : (int32_t)blockIdx.x;
    const int32_t *g = genes + (int64_t)row * k;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int grp = lane >> 4, q = lane & 15;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    int32_t j = 4 * wv + grp;
    for (; j + 48 < k; j += 64) {
        uint2 e[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) e[u] = *reinterpret_cast<const uint2 *>(Eb + (int64_t)g[j + 16 * u] * kD + 4 * q);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a0 += bf2f((uint16_t)e[u].x);
            a1 += bf2f((uint16_t)(e[u].x >> 16));
            a2 += bf2f((uint16_t)e[u].y);
            a3 += bf2f((uint16_t)(e[u].y >> 16));
        }
    }
    for (; j < k; j += 16) {
        const uint2 e = *reinterpret_cast<const uint2 *>(Eb + (int64_t)g[j] * kD + 4 * q);
        a0 += bf2f((uint16_t)e.x);
        a1 += bf2f((uint16_t)(e.x >> 16));
        a2 += bf2f((uint16_t)e.y);
        a3 += bf2f((uint16_t)(e.y >> 16));
    }
#pragma unroll
    for (int off = 16; off <= 32; off <<= 1) {
        a0 += __shfl_xor(a0, off, 64);
        a1 += __shfl_xor(a1, off, 64);
        a2 += __shfl_xor(a2, off, 64);
        a3 += __shfl_xor(a3, off, 64);
    }
    if (grp == 0) {
        s_part[wv][4 * q] = a0;
        s_part[wv][4 * q + 1] = a1;
        s_part[wv][4 * q + 2] = a2;
        s_part[wv][4 * q + 3] = a3;
    }
    __syncthreads();
    if (threadIdx.x < kD) {
        const int d = threadIdx.x;
        const float x = ((s_part[0][d] + s_part[1][d]) + s_part[2][d]) + s_part[3][d];
        xb[(int64_t)blockIdx.x * kD + d] = f2bf(x);
    }
}

// ------------------------------------------------------------------- MLP ----

struct MlpArgs {
    const uint16_t *xb;  // [N][64]
    const uint16_t *W1b, *W2b, *W1bT, *W2bT, *w3b;
    const float *b1, *b2, *b3;
    float *yhat;         // [N]
    int32_t N;
    // training
    const float *target; // [N] standardised labels
    float dscale;        // 2 / B
    float *lossv;        // [N] squared errors
    uint16_t *dxT;       // [64][N] gradient of x(S), bf16, dimension-major
    float *partial;      // [blocks][kMlpParams] per-block parameter gradients
};

// Forward for 64 samples per block, 16 per wave (rows r0 + i).  MFMA tiles
// are 16 x 16 with K = 32: lane l holds A[l % 16][8 (l / 16) .. + 7],
// B[8 (l / 16) .. + 7][l % 16] and C[4 (l / 16) + r][l % 16], r = 0..3.
// With kTrain the block also runs the backward pass of its samples:
// dyhat = 2 (yhat - t) / B; dz2 = dyhat w3 [z2 > 0]; dh1 = dz2 W2;
// dz1 = dh1 [z1 > 0]; dx = dz1 W1; and its share of every parameter
// gradient (dW2 = dz2^T h1, dW1 = dz1^T x, biases, w3), written as one
// partial row per block and summed in block order later.
template <bool kTrain>
__global__ __launch_bounds__(256) void k_mlp(MlpArgs a)
{
    extern __shared__ __align__(16) uint16_t lds[];
    uint16_t *sX = lds;
    uint16_t *sH1 = sX + kMlpRows * kSX;
    uint16_t *sDZ2 = sH1 + kMlpRows * kSH;
    uint16_t *sDZ1 = sDZ2 + kMlpRows * kSH;
    float *sW3 = reinterpret_cast<float *>(sDZ1 + kMlpRows * kSH);  // [4][256] wave shares of dw3
    float *sB3 = sW3 + 4 * kH;                                      // [4]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int32_t row0 = blockIdx.x * kMlpRows;
    const int wr0 = wv * 16;

    for (int t = threadIdx.x; t < kMlpRows * 8; t += blockDim.x) {
        const int r = t >> 3, c8 = (t & 7) * 8;
        uint4 v = {0u, 0u, 0u, 0u};
        if (row0 + r < a.N) v = *reinterpret_cast<const uint4 *>(a.xb + (int64_t)(row0 + r) * kD + c8);
        *reinterpret_cast<uint4 *>(sX + r * kSX + c8) = v;
    }
    __syncthreads();

    f32x4 acc[16];
    // layer 1: z1 = x W1^T + b1
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kD / 32; ++ks) {
        const bf16x8 A = ld8(sX + (wr0 + lr) * kSX + ks * 32 + lg * 8);
#pragma unroll
        for (int t = 0; t < 16; ++t) acc[t] = mfma(A, ld8(a.W1b + (t * 16 + lr) * kD + ks * 32 + lg * 8), acc[t]);
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const float b = a.b1[t * 16 + lr];
#pragma unroll
        for (int r = 0; r < 4; ++r) sH1[(wr0 + 4 * lg + r) * kSH + t * 16 + lr] = f2bf(fmaxf(acc[t][r] + b, 0.f));
    }
    __syncthreads();
    // layer 2: z2 = h1 W2^T + b2
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < kH / 32; ++ks) {
        const bf16x8 A = ld8(sH1 + (wr0 + lr) * kSH + ks * 32 + lg * 8);
#pragma unroll
        for (int t = 0; t < 16; ++t) acc[t] = mfma(A, ld8(a.W2b + (t * 16 + lr) * kH + ks * 32 + lg * 8), acc[t]);
    }
    // h2 (as its bf16 value) and yhat = w3 . h2 + b3
    float p[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const float b = a.b2[t * 16 + lr];
        const float w = bf2f(a.w3b[t * 16 + lr]);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float h = bf2f(f2bf(fmaxf(acc[t][r] + b, 0.f)));
            acc[t][r] = h;
            p[r] += h * w;
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) p[r] += __shfl_xor(p[r], off, 64);
    const float b3 = a.b3[0];
    float dy[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int32_t row = row0 + wr0 + 4 * lg + r;
        const float y = p[r] + b3;
        dy[r] = 0.f;
        if (row < a.N) {
            if (lr == 0) a.yhat[row] = y;
            if (kTrain) {
                const float e = y - a.target[row];
                dy[r] = e * a.dscale;
                if (lr == 0) a.lossv[row] = e * e;
            }
        }
    }
    if (!kTrain) return;

    // dz2, and this wave's share of dw3 (cols t*16 + lr) and db3
    float q3[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const float w = bf2f(a.w3b[t * 16 + lr]);
        q3[t] = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float h = acc[t][r];
            q3[t] += dy[r] * h;
            sDZ2[(wr0 + 4 * lg + r) * kSH + t * 16 + lr] = f2bf(h > 0.f ? dy[r] * w : 0.f);
        }
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        q3[t] += __shfl_xor(q3[t], 16, 64);
        q3[t] += __shfl_xor(q3[t], 32, 64);
    }
    if (lg == 0)
#pragma unroll
        for (int t = 0; t < 16; ++t) sW3[wv * kH + t * 16 + lr] = q3[t];
    float sd = ((dy[0] + dy[1]) + dy[2]) + dy[3];
    sd += __shfl_xor(sd, 16, 64);
    sd += __shfl_xor(sd, 32, 64);
    if (lane == 0) sB3[wv] = sd;
    __syncthreads();

    // dh1 = dz2 W2, dz1 = dh1 [h1 > 0]
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < kH / 32; ++ks) {
        const bf16x8 A = ld8(sDZ2 + (wr0 + lr) * kSH + ks * 32 + lg * 8);
#pragma unroll
        for (int t = 0; t < 16; ++t) acc[t] = mfma(A, ld8(a.W2bT + (t * 16 + lr) * kH + ks * 32 + lg * 8), acc[t]);
    }
#pragma unroll
    for (int t = 0; t < 16; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int idx = (wr0 + 4 * lg + r) * kSH + t * 16 + lr;
            sDZ1[idx] = f2bf(bf2f(sH1[idx]) > 0.f ? acc[t][r] : 0.f);
        }
    __syncthreads();

    // dx = dz1 W1
    f32x4 ax[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) ax[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < kH / 32; ++ks) {
        const bf16x8 A = ld8(sDZ1 + (wr0 + lr) * kSH + ks * 32 + lg * 8);
#pragma unroll
        for (int t = 0; t < 4; ++t) ax[t] = mfma(A, ld8(a.W1bT + (t * 16 + lr) * kH + ks * 32 + lg * 8), ax[t]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int32_t row = row0 + wr0 + 4 * lg + r;
        if (row < a.N)
#pragma unroll
            for (int t = 0; t < 4; ++t) a.dxT[(int64_t)(t * 16 + lr) * a.N + row] = f2bf(ax[t][r]);
    }

    // parameter gradients of the block's 64 samples
    float *P = a.partial + (int64_t)blockIdx.x * kMlpParams;
    // dW2[j][i] = sum_s dz2[s][j] h1[s][i]: wave wv takes j tiles 4wv..4wv+3
    {
        bf16x8 A[4][2];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) A[u][ks] = gather8(sDZ2 + (ks * 32 + lg * 8) * kSH + (4 * wv + u) * 16 + lr, kSH);
        for (int it = 0; it < 16; ++it) {
            const bf16x8 B0 = gather8(sH1 + (lg * 8) * kSH + it * 16 + lr, kSH);
            const bf16x8 B1 = gather8(sH1 + (32 + lg * 8) * kSH + it * 16 + lr, kSH);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                f32x4 c = mfma(A[u][0], B0, f32x4{0.f, 0.f, 0.f, 0.f});
                c = mfma(A[u][1], B1, c);
#pragma unroll
                for (int r = 0; r < 4; ++r) P[kOffW2 + ((4 * wv + u) * 16 + 4 * lg + r) * kH + it * 16 + lr] = c[r];
            }
        }
    }
    // dW1[j][d] = sum_s dz1[s][j] x[s][d]
    {
        bf16x8 A[4][2];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) A[u][ks] = gather8(sDZ1 + (ks * 32 + lg * 8) * kSH + (4 * wv + u) * 16 + lr, kSH);
#pragma unroll
        for (int dt = 0; dt < 4; ++dt) {
            const bf16x8 B0 = gather8(sX + (lg * 8) * kSX + dt * 16 + lr, kSX);
            const bf16x8 B1 = gather8(sX + (32 + lg * 8) * kSX + dt * 16 + lr, kSX);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                f32x4 c = mfma(A[u][0], B0, f32x4{0.f, 0.f, 0.f, 0.f});
                c = mfma(A[u][1], B1, c);
#pragma unroll
                for (int r = 0; r < 4; ++r) P[kOffW1 + ((4 * wv + u) * 16 + 4 * lg + r) * kD + dt * 16 + lr] = c[r];
            }
        }
    }
    // biases and w3, one thread per hidden unit, samples in order
    {
        const int j = threadIdx.x;
        float s1 = 0.f, s2 = 0.f;
        for (int s = 0; s < kMlpRows; ++s) {
            s1 += bf2f(sDZ1[s * kSH + j]);
            s2 += bf2f(sDZ2[s * kSH + j]);
        }
        P[kOffB1 + j] = s1;
        P[kOffB2 + j] = s2;
        P[kOffW3 + j] = ((sW3[j] + sW3[kH + j]) + sW3[2 * kH + j]) + sW3[3 * kH + j];
        if (j == 0) P[kOffB3] = ((sB3[0] + sB3[1]) + sB3[2]) + sB3[3];
    }
}

// --------------------------------------------------------------------- Adam --

struct AdamArgs {
    float lr, b1, b2, eps, c1, c2;  // c1 = 1 - b1^t, c2 = 1 - b2^t
};

__device__ __forceinline__ float adam(float &theta, float &m, float &v, float g, const AdamArgs &o)
{
    m = o.b1 * m + (1.f - o.b1) * g;
    v = o.b2 * v + (1.f - o.b2) * g * g;
    theta -= o.lr * (m / o.c1) / (sqrtf(v / o.c2) + o.eps);
    return theta;
}

// MLP parameters: gradient = partial rows summed in block order; Adam; the
// bfloat16 copies.  Block 0 also averages the per-sample squared errors.
__global__ void k_adam_mlp(float *__restrict__ theta, float *__restrict__ m, float *__restrict__ v,
                           const float *__restrict__ partial, int32_t nblk, float *__restrict__ keep, AdamArgs o,
                           Bf16Copies cp, const float *__restrict__ lossv, int32_t B, double *__restrict__ loss_out)
{
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0) {
        __shared__ double s_l[256];
        double acc = 0.0;
        for (int32_t s = threadIdx.x; s < B; s += blockDim.x) acc += (double)lossv[s];
        s_l[threadIdx.x] = acc;
        __syncthreads();
        for (int off = blockDim.x / 2; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) s_l[threadIdx.x] += s_l[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) *loss_out = s_l[0] / B;
    }
    if (j >= kMlpParams) return;
    float g = 0.f;
    for (int32_t b = 0; b < nblk; ++b) g += partial[(int64_t)b * kMlpParams + j];
    if (keep) keep[j] = g;
    float th = theta[j], mm = m[j], vv = v[j];
    adam(th, mm, vv, g, o);
    theta[j] = th;
    m[j] = mm;
    v[j] = vv;
    mlp_copy(cp, j, th);
}

// Embeddings.  dE = M^T dx, M the batch's sample x node membership matrix:
// for the hub nodes that sit in most sets of a converged population this is
// a dense contraction over the batch, so it runs on the matrix cores.  The B
// operand (dx of the whole batch, bf16, dimension-major) is staged once per
// block in LDS, rows padded by 8 elements so that the 16 rows a k-step reads
// fall in different banks; each wave then walks tiles of 16 nodes: the A
// operand is the tile's membership bits (node-major rows, one 32-bit word
// per 32 samples) expanded to bf16 0/1, K = the batch; k-steps whose word is
// zero for the whole tile are skipped.  Rows of nodes in some sample get
// their gradient and touched[v] = 1; the others touched[v] = 0 (Adam is lazy
// on E: those rows keep weights and moments).
__global__ __launch_bounds__(1024) void k_grad_E(const uint32_t *__restrict__ bits, int32_t Wb,
                                                const uint16_t *__restrict__ dxT, int32_t B, float *__restrict__ gE,
                                                uint8_t *__restrict__ touched, int64_t n)
{
    extern __shared__ __align__(16) uint16_t sB[];
    const int32_t SB = B + 8;
    for (int32_t c = threadIdx.x; c < kD * (B / 8); c += blockDim.x) {
        const int32_t d = c / (B / 8), e = (c % (B / 8)) * 8;
        *reinterpret_cast<uint4 *>(sB + d * SB + e) = *reinterpret_cast<const uint4 *>(dxT + (int64_t)d * B + e);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int64_t tiles = (n + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * nw + wv; tile < tiles; tile += (int64_t)gridDim.x * nw) {
        const int64_t v0 = tile * 16;
        const int64_t row = v0 + lr;
        // lane (lr, lg) holds words 8 lg .. 8 lg + 7 of node v0 + lr
        uint32_t w8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int ks = 8 * lg + u;
            w8[u] = (row < n && ks < Wb) ? bits[row * Wb + ks] : 0u;
        }
        uint32_t rowany = 0u;
#pragma unroll
        for (int u = 0; u < 8; ++u) rowany |= w8[u];
        rowany |= (uint32_t)__shfl_xor((int)rowany, 16, 64);
        rowany |= (uint32_t)__shfl_xor((int)rowany, 32, 64);
        if (lg == 0 && row < n) touched[row] = rowany != 0u;
        if (__ballot(rowany != 0u) == 0) continue;
        f32x4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 32; ++ks) {
            // word ks of this lane's row sits in lane lr + 16 (ks / 8), slot ks % 8
            const uint32_t word = ks < Wb ? (uint32_t)__shfl((int)w8[ks & 7], lr + 16 * (ks >> 3), 64) : 0u;
            if (__ballot(word != 0u) == 0) continue;
            const uint32_t byte = (word >> (8 * lg)) & 0xFFu;
            uint4 q;
            q.x = ((byte & 1u) ? 0x3F80u : 0u) | ((byte & 2u) ? 0x3F800000u : 0u);
            q.y = ((byte & 4u) ? 0x3F80u : 0u) | ((byte & 8u) ? 0x3F800000u : 0u);
            q.z = ((byte & 16u) ? 0x3F80u : 0u) | ((byte & 32u) ? 0x3F800000u : 0u);
            q.w = ((byte & 64u) ? 0x3F80u : 0u) | ((byte & 128u) ? 0x3F800000u : 0u);
            const bf16x8 A = __builtin_bit_cast(bf16x8, q);
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = mfma(A, ld8(sB + (t * 16 + lr) * SB + ks * 32 + lg * 8), acc[t]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t node = v0 + 4 * lg + r;
            if (node < n)
#pragma unroll
                for (int t = 0; t < 4; ++t) gE[node * kD + t * 16 + lr] = acc[t][r];
        }
    }
}

size_t grad_E_lds(int32_t B)
{
    return (size_t)kD * (B + 8) * 2;
}

// Lazy Adam on E, four weights per thread: rows with touched[v] = 0 are
// left alone; the others step with the global step count.
__global__ void k_adam_E(const float *__restrict__ gE, const uint8_t *__restrict__ touched, float *__restrict__ E,
                         float *__restrict__ m, float *__restrict__ v, uint16_t *__restrict__ Eb,
                         float *__restrict__ keep, int64_t n, AdamArgs o)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // float4 index
    if (q >= n * (kD / 4)) return;
    const int64_t node = q / (kD / 4);
    if (!touched[node]) {
        if (keep) reinterpret_cast<float4 *>(keep)[q] = float4{0.f, 0.f, 0.f, 0.f};
        return;
    }
    const float4 g = reinterpret_cast<const float4 *>(gE)[q];
    float4 th = reinterpret_cast<float4 *>(E)[q];
    float4 mm = reinterpret_cast<float4 *>(m)[q];
    float4 vv = reinterpret_cast<float4 *>(v)[q];
    adam(th.x, mm.x, vv.x, g.x, o);
    adam(th.y, mm.y, vv.y, g.y, o);
    adam(th.z, mm.z, vv.z, g.z, o);
    adam(th.w, mm.w, vv.w, g.w, o);
    reinterpret_cast<float4 *>(E)[q] = th;
    reinterpret_cast<float4 *>(m)[q] = mm;
    reinterpret_cast<float4 *>(v)[q] = vv;
    uint2 h;
    h.x = f2bf(th.x) | ((uint32_t)f2bf(th.y) << 16);
    h.y = f2bf(th.z) | ((uint32_t)f2bf(th.w) << 16);
    reinterpret_cast<uint2 *>(Eb)[q] = h;
    if (keep) reinterpret_cast<float4 *>(keep)[q] = g;
}

// --------------------------------------------------------- GA-side steps ----

// Orderable key of a prediction (NaN last); ties broken by index.
__device__ __forceinline__ uint64_t pred_key(float y, uint32_t idx)
{
    uint32_t u = __float_as_uint(y);
    if (y != y) u = 0x7FFFFFFFu;
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((uint64_t)u << 32) | idx;
}

__device__ __forceinline__ uint64_t random_key(uint64_t seed, uint32_t gen, uint32_t ind, uint32_t i)
{
    return ((uint64_t)draw(seed, i, ind, gen, kStreamSurrRandom, 0).w0 << 32) | i;
}

// Bitonic sort of key[0, L) ascending (L a power of two); whole block.
__device__ void block_sort(uint64_t *key, int32_t L)
{
    for (int32_t size = 2; size <= L; size <<= 1)
        for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int32_t i = threadIdx.x; i < L; i += blockDim.x) {
                const int32_t p = i ^ stride;
                if (p > i) {
                    const bool up = (i & size) == 0;
                    const uint64_t x = key[i], y = key[p];
                    if ((x > y) == up) {
                        key[i] = y;
                        key[p] = x;
                    }
                }
            }
            __syncthreads();
        }
}

// Indices whose bit is set in bits[0, ceil(lambda / 32)), ascending, to
// out[]; whole block (blockDim.x <= 1024).
__device__ void block_compact(const uint32_t *bits, int32_t lambda, int32_t *out)
{
    __shared__ int32_t s_wave[16];
    const int32_t words = (lambda + 31) / 32;
    const int32_t per = (words + blockDim.x - 1) / blockDim.x;
    const int32_t w0 = min(words, (int32_t)threadIdx.x * per), w1 = min(words, w0 + per);
    int32_t cnt = 0;
    for (int32_t w = w0; w < w1; ++w) cnt += __popc(bits[w]);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t incl = cnt;
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) s_wave[wv] = incl;
    __syncthreads();
    int32_t off = incl - cnt;
    for (int q = 0; q < wv; ++q) off += s_wave[q];
    for (int32_t w = w0; w < w1; ++w)
        for (uint32_t x = bits[w]; x; x &= x - 1) out[off++] = w * 32 + __ffs(x) - 1;
    __syncthreads();
}

// Screening.  pool[0, m): the m children with the smallest (prediction,
// index) or, when yhat is NULL, the smallest (first word of
// draw(seed, o, 0, gen, stream 7), o); ascending.  pool[m, m + extra): the
// judge's unbiased sample, the `extra` other children with the smallest
// (first word of draw(seed, o, 1, gen, stream 7), o); ascending.  One block
// of 1024 threads, keys in LDS, lambda <= 8192.
size_t screen_lds(int32_t lambda)
{
    size_t L = 1;
    while ((int32_t)L < lambda) L <<= 1;
    return L * 8 + (size_t)kMaxLambda / 32 * 4 * 2;
}

__global__ __launch_bounds__(1024) void k_screen(const float *__restrict__ yhat, int32_t lambda, int32_t m,
                                                 int32_t extra, uint64_t seed, uint32_t gen,
                                                 int32_t *__restrict__ pool)
{
    extern __shared__ __align__(16) uint64_t key[];  // [L], then two bit sets
    int32_t L = 1;
    while (L < lambda) L <<= 1;
    uint32_t *chosen = reinterpret_cast<uint32_t *>(key + L);
    uint32_t *judged = chosen + kMaxLambda / 32;
    for (int32_t i = threadIdx.x; i < L; i += blockDim.x)
        key[i] = i < lambda ? (yhat ? pred_key(yhat[i], i) : random_key(seed, gen, 0, i)) : ~0ull;
    for (int32_t i = threadIdx.x; i < kMaxLambda / 32; i += blockDim.x) chosen[i] = judged[i] = 0u;
    __syncthreads();
    block_sort(key, L);
    for (int32_t i = threadIdx.x; i < m; i += blockDim.x) {
        const uint32_t idx = (uint32_t)key[i];
        atomicOr(&chosen[idx >> 5], 1u << (idx & 31));
    }
    __syncthreads();
    block_compact(chosen, lambda, pool);
    if (extra <= 0) return;
    for (int32_t i = threadIdx.x; i < L; i += blockDim.x)
        key[i] = (i < lambda && !((chosen[i >> 5] >> (i & 31)) & 1u)) ? random_key(seed, gen, 1, i) : ~0ull;
    __syncthreads();
    block_sort(key, L);
    for (int32_t i = threadIdx.x; i < extra; i += blockDim.x) {
        const uint32_t idx = (uint32_t)key[i];
        atomicOr(&judged[idx >> 5], 1u << (idx & 31));
    }
    __syncthreads();
    block_compact(judged, lambda, pool + m);
}

__global__ void k_iota(int32_t *__restrict__ out, int32_t count)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = i;
}

// Copies the rows of the selected children (pool entries q) to crows[q].
__global__ void k_gather_pool_rows(const int32_t *__restrict__ pool, const int32_t *__restrict__ children, int32_t k,
                                   int32_t *__restrict__ crows)
{
    const int32_t q = blockIdx.x;
    const int32_t o = pool[q];
    for (int32_t j = threadIdx.x; j < k; j += blockDim.x) crows[(int64_t)q * k + j] = children[(int64_t)o * k + j];
}

// Ring buffer: entry (base + q) mod cap takes child pool[q] (q when pool is
// NULL) and the label ln(1 + F[q]).
__global__ void k_append(const int32_t *__restrict__ children, int32_t k, const int32_t *__restrict__ pool,
                         const int64_t *__restrict__ F, int64_t base, int32_t cap, int32_t *__restrict__ buf_genes,
                         double *__restrict__ buf_y)
{
    const int32_t q = blockIdx.x;
    const int32_t o = pool ? pool[q] : q;
    const int64_t slot = (base + q) % cap;
    for (int32_t j = threadIdx.x; j < k; j += blockDim.x) buf_genes[slot * k + j] = children[(int64_t)o * k + j];
    if (threadIdx.x == 0) buf_y[slot] = log1p((double)F[q]);
}

// Mean and spread of the buffered labels (one block, fixed order): the
// spread is sqrt(variance + floor^2), so that a buffer of (nearly) equal
// labels gives targets near zero rather than amplified rounding noise.
constexpr double kSpreadFloor = 1e-6;
__global__ __launch_bounds__(1024) void k_label_stats(const double *__restrict__ y, int32_t count,
                                                      double *__restrict__ out)
{
    __shared__ double s[1024];
    double a = 0.0;
    for (int32_t i = threadIdx.x; i < count; i += blockDim.x) a += y[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    const double mu = s[0] / count;
    __syncthreads();
    a = 0.0;
    for (int32_t i = threadIdx.x; i < count; i += blockDim.x) a += (y[i] - mu) * (y[i] - mu);
    s[threadIdx.x] = a;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = mu;
        out[1] = sqrt(s[0] / count + kSpreadFloor * kSpreadFloor);
    }
}

// Training batch of step `step` in generation `gen`: entry j is buffer row
// bounded(w, count), w the first word of draw(seed, j, step, gen, stream 6);
// its genes are copied and its label standardised.
__global__ void k_sample(uint64_t seed, uint32_t gen, uint32_t step, int32_t count, const int32_t *__restrict__ buf_genes,
                         const double *__restrict__ buf_y, const double *__restrict__ mu_sd, int32_t k,
                         int32_t *__restrict__ genes, float *__restrict__ target)
{
    __shared__ int32_t s_idx;
    const int32_t j = blockIdx.x;
    if (threadIdx.x == 0) {
        const uint32_t w = draw(seed, (uint32_t)j, step, gen, kStreamSurrSample, 0).w0;
        s_idx = (int32_t)bounded(w, (uint32_t)count);
        target[j] = (float)((buf_y[s_idx] - mu_sd[0]) / mu_sd[1]);
    }
    __syncthreads();
    const int32_t r = s_idx;
    for (int32_t t = threadIdx.x; t < k; t += blockDim.x) genes[(int64_t)j * k + t] = buf_genes[(int64_t)r * k + t];
}

// Judge: over J = min(m, 1024) evaluated children (entry i is pool entry
// floor(i m / J)), Spearman's correlation between predictions and exact PC
// (average ranks), and the mean relative error of expm1(yhat sd + mu).
__global__ __launch_bounds__(1024) void k_judge(const float *__restrict__ yhat, const int32_t *__restrict__ pool,
                                                const int64_t *__restrict__ F, int32_t m,
                                                const double *__restrict__ mu_sd, double *__restrict__ out)
{
    __shared__ float s_y[kJudgeMax];
    __shared__ int64_t s_f[kJudgeMax];
    __shared__ double s_a[1024], s_b[1024], s_c[1024], s_e[1024];
    const int32_t J = min(m, kJudgeMax);
    const int32_t i = threadIdx.x;
    if (i < J) {
        const int32_t q = (int32_t)(((int64_t)i * m) / J);
        s_y[i] = yhat[pool ? pool[q] : q];
        s_f[i] = F[q];
    }
    __syncthreads();
    double ra = 0.0, rb = 0.0, rel = 0.0;
    if (i < J) {
        int32_t la = 0, ea = 0, lb = 0, eb = 0;
        for (int32_t j = 0; j < J; ++j) {
            la += s_y[j] < s_y[i];
            ea += s_y[j] == s_y[i];
            lb += s_f[j] < s_f[i];
            eb += s_f[j] == s_f[i];
        }
        const double mid = (J + 1) / 2.0;
        ra = la + (ea + 1) / 2.0 - mid;
        rb = lb + (eb + 1) / 2.0 - mid;
        const double f = (double)s_f[i];
        const double pred = expm1((double)s_y[i] * mu_sd[1] + mu_sd[0]);
        rel = fabs(pred - f) / fmax(f, 1.0);
    }
    s_a[i] = ra * rb;
    s_b[i] = ra * ra;
    s_c[i] = rb * rb;
    s_e[i] = rel;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if (i < off) {
            s_a[i] += s_a[i + off];
            s_b[i] += s_b[i + off];
            s_c[i] += s_c[i + off];
            s_e[i] += s_e[i + off];
        }
        __syncthreads();
    }
    if (i == 0) {
        const double den = sqrt(s_b[0] * s_c[0]);
        out[0] = den > 0.0 ? s_a[0] / den : 0.0;
        out[1] = s_e[0] / J;
    }
}

}  // namespace

// -------------------------------------------------------------- host side ----

struct SurrogateState {
    gapa_surrogate_params sp{};
    int32_t n = 0, k = 0, lambda = 0, W = 0;
    uint64_t seed = 0;
    int64_t steps = 0;        // Adam steps taken
    int64_t appended = 0;     // pairs appended to the ring buffer
    int32_t low_run = 0;      // consecutive screened generations below min_rho
    int32_t fallbacks = 0;
    bool force_full = false;
    bool stats_pending = false;
    int64_t last_gen = 0;
    int32_t last_evaluated = 0, last_pooled = 0;
    bool last_screened = false, last_predicted = false;
    DevBuf theta, m, v, partial, keep_mlp, keep_E;      // float
    DevBuf Eb, W1b, W2b, w3b, W1bT, W2bT;               // bf16
    DevBuf xb, yhat, ytrain, dxT, target, lossv;        // per sample (yhat: the generation's predictions)
    DevBuf bgenes, bmasks, balive, bflag, brows;        // training batch
    DevBuf gE, touched;                                 // embedding gradient, rows present in the batch
    DevBuf buf_genes, buf_y;                            // ring buffer
    DevBuf pool, crows, cmasks, calive;                 // screened children
    DevBuf dstats;                                      // double [8]: mu, sd, rho, rel_err, loss
    double *hstats = nullptr;                           // pinned copy of dstats
    hipEvent_t ready = nullptr;
    bool have_keep = false;
};

namespace {

bool is_batch_size(int32_t B)
{
    return B >= 32 && B <= 1024 && (B & (B - 1)) == 0;
}

Bf16Copies copies(SurrogateState &st)
{
    return Bf16Copies{st.Eb.as<uint16_t>(), st.W1b.as<uint16_t>(), st.W1bT.as<uint16_t>(), st.W2b.as<uint16_t>(),
                      st.W2bT.as<uint16_t>(), st.w3b.as<uint16_t>()};
}

float *mlp_theta(SurrogateState &st)
{
    return st.theta.as<float>() + (int64_t)st.n * kD;
}

MlpArgs mlp_args(SurrogateState &st, const uint16_t *xb, float *yhat, int32_t N)
{
    MlpArgs a{};
    const float *th = mlp_theta(st);
    a.xb = xb;
    a.W1b = st.W1b.as<uint16_t>();
    a.W2b = st.W2b.as<uint16_t>();
    a.W1bT = st.W1bT.as<uint16_t>();
    a.W2bT = st.W2bT.as<uint16_t>();
    a.w3b = st.w3b.as<uint16_t>();
    a.b1 = th + kOffB1;
    a.b2 = th + kOffB2;
    a.b3 = th + kOffB3;
    a.yhat = yhat;
    a.N = N;
    return a;
}

int predict_rows(SurrogateState &st, const int32_t *genes, const int32_t *rows, int32_t N, float *yhat, hipStream_t s)
{
    if (N <= 0) return GAPA_OK;
    hipLaunchKernelGGL(k_embed, dim3(N), dim3(256), 0, s, genes, rows, st.k, st.Eb.as<uint16_t>(),
                       st.xb.as<uint16_t>());
    MlpArgs a = mlp_args(st, st.xb.as<uint16_t>(), yhat, N);
    hipLaunchKernelGGL(k_mlp<false>, dim3((N + kMlpRows - 1) / kMlpRows), dim3(256), kMlpLds, s, a);
    GAPA_HIP(hipGetLastError());
    return GAPA_OK;
}

AdamArgs adam_args(SurrogateState &st)
{
    const double t = (double)st.steps;
    AdamArgs o;
    o.lr = st.sp.lr;
    o.b1 = 0.9f;
    o.b2 = 0.999f;
    o.eps = 1e-8f;
    o.c1 = (float)(1.0 - std::pow(0.9, t));
    o.c2 = (float)(1.0 - std::pow(0.999, t));
    return o;
}

// One Adam step on B rows of genes (device, [B][k]) with standardised
// targets (device): embeddings, MLP forward and backward, gradients, Adam.
int train_step(gapa_ga *ga, const int32_t *genes, const float *target, int32_t B, bool keep, hipStream_t s)
{
    SurrogateState &st = *ga->surr;
    gapa_graph *g = ga->graph;
    st.steps += 1;
    const AdamArgs o = adam_args(st);
    hipLaunchKernelGGL(k_embed, dim3(B), dim3(256), 0, s, genes, nullptr, st.k, st.Eb.as<uint16_t>(),
                       st.xb.as<uint16_t>());
    MlpArgs a = mlp_args(st, st.xb.as<uint16_t>(), st.ytrain.as<float>(), B);
    a.target = target;
    a.dscale = 2.0f / B;
    a.lossv = st.lossv.as<float>();
    a.dxT = st.dxT.as<uint16_t>();
    a.partial = st.partial.as<float>();
    const int32_t nblk = (B + kMlpRows - 1) / kMlpRows;
    hipLaunchKernelGGL(k_mlp<true>, dim3(nblk), dim3(256), kMlpLds, s, a);
    float *th = mlp_theta(st);
    const int64_t nE = (int64_t)st.n * kD;
    hipLaunchKernelGGL(k_adam_mlp, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, th, st.m.as<float>() + nE,
                       st.v.as<float>() + nE, st.partial.as<float>(), nblk, keep ? st.keep_mlp.as<float>() : nullptr,
                       o, copies(st), st.lossv.as<float>(), B, st.dstats.as<double>() + 4);
    // membership bits of the batch, node-major: removed-node bit sets of the
    // rows, transposed
    int rc = launch_mask_build(genes, B, st.k, g->n, g->words, g->d_noniso, g->n_noniso, st.bmasks.as<uint32_t>(),
                               st.balive.as<int32_t>(), st.bflag.as<int32_t>(), s);
    if (rc != GAPA_OK) return rc;
    const int32_t Wb = B / 32;
    if ((rc = launch_bits_transpose(st.bmasks.as<uint32_t>(), B, g->words, g->n, st.brows.as<uint32_t>(), s)) !=
        GAPA_OK)
        return rc;
    const int64_t tiles = ((int64_t)st.n + 15) / 16;
    // one 16-wave block per compute unit shares one staged copy of dx
    const unsigned eblocks = (unsigned)std::min<int64_t>((tiles + 15) / 16, 256);
    hipLaunchKernelGGL(k_grad_E, dim3(eblocks), dim3(1024), grad_E_lds(B), s, st.brows.as<uint32_t>(), Wb,
                       st.dxT.as<uint16_t>(), B, st.gE.as<float>(), st.touched.as<uint8_t>(), (int64_t)st.n);
    const int64_t quads = (int64_t)st.n * (kD / 4);
    hipLaunchKernelGGL(k_adam_E, dim3((unsigned)((quads + 255) / 256)), dim3(256), 0, s, st.gE.as<float>(),
                       st.touched.as<uint8_t>(), st.theta.as<float>(), st.m.as<float>(), st.v.as<float>(),
                       st.Eb.as<uint16_t>(), keep ? st.keep_E.as<float>() : nullptr, (int64_t)st.n, o);
    GAPA_HIP(hipGetLastError());
    st.have_keep = keep;
    return GAPA_OK;
}

int read_stats(gapa_ga *ga)
{
    SurrogateState &st = *ga->surr;
    if (!st.stats_pending) return GAPA_OK;
    GAPA_HIP(hipEventSynchronize(st.ready));
    st.stats_pending = false;
    if (st.last_predicted && st.last_screened) {  // full generations do not count
        const double rho = st.hstats[2];
        st.low_run = rho < st.sp.min_rho ? st.low_run + 1 : 0;
        if (st.sp.fallback_gens > 0 && st.low_run >= st.sp.fallback_gens) {
            st.force_full = true;
            st.low_run = 0;
        }
    }
    return GAPA_OK;
}

}  // namespace

int surrogate_attach(gapa_ga *ga, const gapa_surrogate_params *sp, hipStream_t s)
{
    if (ga->count != 1 || ga->surr || ga->generation != 0) {
        set_error("a surrogate attaches to a single-instance GA at generation 0, once");
        return GAPA_E_INVALID_ARG;
    }
    const int32_t L = ga->lambda;
    if (sp->emb_dim != kD || sp->hidden != kH || sp->screen < 1 || sp->screen > L || L > kMaxLambda ||
        !is_batch_size(sp->batch) || sp->train_steps < 0 || sp->warmup_gens < 0 || sp->buffer < sp->batch ||
        sp->fallback_gens < 0 || !(sp->lr > 0.f) || (sp->flags & ~(uint32_t)GAPA_SCREEN_RANDOM) != 0 ||
        sp->reserved != 0) {
        set_error("invalid surrogate parameters (emb_dim 64, hidden 256, 1 <= screen <= offspring <= 8192, "
                  "batch a power of two in [32, 1024], buffer >= batch, lr > 0)");
        return GAPA_E_INVALID_ARG;
    }
    if ((int64_t)sp->buffer * ga->params.k >= (1ll << 40)) {
        set_error("replay buffer too large");
        return GAPA_E_INVALID_ARG;
    }
    SurrogateState *st = new (std::nothrow) SurrogateState();
    if (!st) {
        set_error("host allocation failed");
        return GAPA_E_OOM;
    }
    ga->surr = st;
    st->sp = *sp;
    st->n = ga->graph->n;
    st->k = ga->params.k;
    st->lambda = L;
    st->W = ga->graph->words;
    st->seed = ga->params.seed;
    const int64_t nE = (int64_t)st->n * kD;
    const int64_t P = nE + kMlpParams;
    const int32_t B = sp->batch;
    const int32_t rows = std::max(L, B);
    const int32_t nblk = (B + kMlpRows - 1) / kMlpRows;
    int rc = GAPA_OK;
    auto res = [&](DevBuf &b, size_t bytes) {
        if (rc == GAPA_OK) rc = b.reserve(bytes);
    };
    res(st->theta, P * 4);
    res(st->m, P * 4);
    res(st->v, P * 4);
    res(st->partial, (size_t)nblk * kMlpParams * 4);
    res(st->keep_mlp, (size_t)kMlpParams * 4);
    res(st->keep_E, (size_t)nE * 4);
    res(st->Eb, (size_t)nE * 2);
    res(st->W1b, kH * kD * 2);
    res(st->W1bT, kH * kD * 2);
    res(st->W2b, kH * kH * 2);
    res(st->W2bT, kH * kH * 2);
    res(st->w3b, kH * 2);
    res(st->xb, (size_t)rows * kD * 2);
    res(st->yhat, (size_t)rows * 4);
    res(st->ytrain, (size_t)B * 4);
    res(st->dxT, (size_t)B * kD * 2);
    res(st->target, (size_t)B * 4);
    res(st->lossv, (size_t)B * 4);
    res(st->bgenes, (size_t)B * st->k * 4);
    res(st->bmasks, (size_t)B * st->W * 4);
    res(st->balive, (size_t)B * 4);
    res(st->bflag, 16);
    res(st->brows, (size_t)st->n * (B / 32) * 4);
    res(st->gE, (size_t)nE * 4);
    res(st->touched, (size_t)st->n);
    res(st->buf_genes, (size_t)sp->buffer * st->k * 4);
    res(st->buf_y, (size_t)sp->buffer * 8);
    res(st->pool, (size_t)L * 4);
    res(st->crows, (size_t)(sp->screen + kJudgeExtra) * st->k * 4);
    res(st->cmasks, (size_t)(sp->screen + kJudgeExtra) * st->W * 4);
    res(st->calive, (size_t)(sp->screen + kJudgeExtra) * 4);
    res(st->dstats, 64);
    if (rc != GAPA_OK) return rc;
    GAPA_HIP(hipHostMalloc(reinterpret_cast<void **>(&st->hstats), 64, hipHostMallocDefault));
    std::memset(st->hstats, 0, 64);
    GAPA_HIP(hipEventCreateWithFlags(&st->ready, hipEventDisableTiming));
    GAPA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_mlp<false>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMlpLds));
    GAPA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_mlp<true>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMlpLds));
    GAPA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_screen), hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)screen_lds(kMaxLambda)));
    GAPA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_grad_E), hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)grad_E_lds(1024)));
    const unsigned blocks = (unsigned)((P + 255) / 256);
    hipLaunchKernelGGL(k_surr_init, dim3(blocks), dim3(256), 0, s, st->theta.as<float>(), (int64_t)st->n, st->seed,
                       0.05, std::sqrt(6.0 / kD), std::sqrt(6.0 / kH), std::sqrt(3.0 / kH));
    hipLaunchKernelGGL(k_bf16_copies, dim3(blocks), dim3(256), 0, s, st->theta.as<float>(), (int64_t)st->n,
                       copies(*st));
    GAPA_HIP(hipGetLastError());
    if ((rc = launch_fill_u32(st->m.ptr, 0u, P, s)) != GAPA_OK) return rc;
    if ((rc = launch_fill_u32(st->v.ptr, 0u, P, s)) != GAPA_OK) return rc;
    if ((rc = launch_fill_u32(st->dstats.ptr, 0u, 16, s)) != GAPA_OK) return rc;
    if ((rc = launch_fill_u32(st->bflag.ptr, 0u, 4, s)) != GAPA_OK) return rc;
    return GAPA_OK;
}

void surrogate_release(SurrogateState *st)
{
    if (!st) return;
    for (DevBuf *b : {&st->theta, &st->m, &st->v, &st->partial, &st->keep_mlp, &st->keep_E, &st->Eb, &st->W1b,
                      &st->W2b, &st->w3b, &st->W1bT, &st->W2bT, &st->xb, &st->yhat, &st->ytrain, &st->dxT, &st->target,
                      &st->lossv, &st->bgenes, &st->bmasks, &st->balive, &st->bflag, &st->brows, &st->gE, &st->touched,
                      &st->buf_genes,
                      &st->buf_y, &st->pool, &st->crows, &st->cmasks, &st->calive, &st->dstats})
        b->release();
    if (st->hstats) (void)hipHostFree(st->hstats);
    if (st->ready) (void)hipEventDestroy(st->ready);
    delete st;
}

int surrogate_generation(gapa_ga *ga, hipStream_t s)
{
    SurrogateState &st = *ga->surr;
    int rc = read_stats(ga);
    if (rc != GAPA_OK) return rc;
    const uint32_t gen = (uint32_t)(ga->generation + 1);
    const bool random = st.sp.flags & GAPA_SCREEN_RANDOM;
    bool full = (int64_t)gen <= st.sp.warmup_gens || st.force_full;
    if (st.force_full) {
        st.fallbacks += 1;
        st.force_full = false;
    }
    const int32_t L = st.lambda;
    // a screened generation builds bit sets only for the children it evaluates
    if ((rc = ga_launch_offspring(ga, s, !full)) != GAPA_OK) return rc;
    const bool predict = !random && (int64_t)gen > st.sp.warmup_gens;
    float *yhat = st.yhat.as<float>();
    if (predict && (rc = predict_rows(st, ga->children.as<int32_t>(), nullptr, L, yhat, s)) != GAPA_OK) return rc;
    int64_t *F = ga->child_fit.as<int64_t>();
    int32_t npool = L;     // children that enter elitism
    int32_t neval = L;     // children evaluated exactly (the pool, then the judge's extra sample)
    const int32_t *pool = nullptr;
    if (full) {
        if ((rc = eval_masks(ga->graph, ga->masks.as<uint32_t>(), ga->alive.as<int32_t>(), L, F, nullptr, ga->ws,
                             &ga->timer, s)) != GAPA_OK)
            return rc;
        if ((rc = ga_rank_and_gather(ga, false, F, nullptr, 0, s)) != GAPA_OK) return rc;
    } else {
        npool = st.sp.screen;
        const int32_t extra = predict ? std::min(kJudgeExtra, L - npool) : 0;
        neval = npool + extra;
        pool = st.pool.as<int32_t>();
        hipLaunchKernelGGL(k_screen, dim3(1), dim3(1024), screen_lds(L), s, random ? nullptr : yhat, L, npool, extra,
                           st.seed, gen, st.pool.as<int32_t>());
        hipLaunchKernelGGL(k_gather_pool_rows, dim3(neval), dim3(256), 0, s, pool, ga->children.as<int32_t>(), st.k,
                           st.crows.as<int32_t>());
        GAPA_HIP(hipGetLastError());
        gapa_graph *g = ga->graph;
        if ((rc = launch_mask_build(st.crows.as<int32_t>(), neval, st.k, g->n, g->words, g->d_noniso, g->n_noniso,
                                    st.cmasks.as<uint32_t>(), st.calive.as<int32_t>(), st.bflag.as<int32_t>(), s)) !=
            GAPA_OK)
            return rc;
        if ((rc = eval_masks(ga->graph, st.cmasks.as<uint32_t>(), st.calive.as<int32_t>(), neval, F, nullptr, ga->ws,
                             &ga->timer, s)) != GAPA_OK)
            return rc;
        if ((rc = ga_rank_and_gather(ga, false, F, pool, npool, s)) != GAPA_OK) return rc;
    }
    double *ds = st.dstats.as<double>();
    if (predict) hipLaunchKernelGGL(k_judge, dim3(1), dim3(1024), 0, s, yhat, pool, F, neval, ds, ds + 2);
    if (!random) {
        hipLaunchKernelGGL(k_append, dim3(neval), dim3(256), 0, s, ga->children.as<int32_t>(), st.k, pool, F,
                           st.appended, st.sp.buffer, st.buf_genes.as<int32_t>(), st.buf_y.as<double>());
        st.appended += neval;
        const int32_t count = (int32_t)std::min<int64_t>(st.appended, st.sp.buffer);
        hipLaunchKernelGGL(k_label_stats, dim3(1), dim3(1024), 0, s, st.buf_y.as<double>(), count, ds);
        for (int32_t t = 0; t < st.sp.train_steps; ++t) {
            hipLaunchKernelGGL(k_sample, dim3(st.sp.batch), dim3(256), 0, s, st.seed, gen, (uint32_t)t, count,
                               st.buf_genes.as<int32_t>(), st.buf_y.as<double>(), ds, st.k,
                               st.bgenes.as<int32_t>(), st.target.as<float>());
            if ((rc = train_step(ga, st.bgenes.as<int32_t>(), st.target.as<float>(), st.sp.batch, false, s)) !=
                GAPA_OK)
                return rc;
        }
    }
    GAPA_HIP(hipGetLastError());
    GAPA_HIP(hipMemcpyAsync(st.hstats, ds, 64, hipMemcpyDeviceToHost, s));
    GAPA_HIP(hipEventRecord(st.ready, s));
    st.stats_pending = true;
    st.last_gen = gen;
    st.last_evaluated = neval;
    st.last_pooled = npool;
    st.last_screened = !full;
    st.last_predicted = predict;
    if (full) {
        // the pool of a full generation is every child
        hipLaunchKernelGGL(k_iota, dim3((L + 255) / 256), dim3(256), 0, s, st.pool.as<int32_t>(), L);
        GAPA_HIP(hipGetLastError());
    }
    ga->generation += 1;
    return GAPA_OK;
}

int surrogate_predict(gapa_ga *ga, const int32_t *genes, int32_t P, float *yhat, hipStream_t s)
{
    SurrogateState &st = *ga->surr;
    const int32_t chunk = std::max(st.lambda, st.sp.batch);  // rows of the x buffer
    for (int32_t c0 = 0; c0 < P; c0 += chunk) {
        const int32_t cnt = std::min(P - c0, chunk);
        int rc = predict_rows(st, genes + (int64_t)c0 * st.k, nullptr, cnt, yhat + c0, s);
        if (rc != GAPA_OK) return rc;
    }
    return GAPA_OK;
}

int surrogate_train_batch(gapa_ga *ga, const int32_t *genes, const float *target, int32_t B, bool keep_grads,
                          hipStream_t s)
{
    SurrogateState &st = *ga->surr;
    if (B != st.sp.batch) {
        set_error("batch size %d differs from the surrogate's (%d)", B, st.sp.batch);
        return GAPA_E_INVALID_ARG;
    }
    return train_step(ga, genes, target, B, keep_grads, s);
}

int surrogate_tensor(gapa_ga *ga, int32_t which, int32_t kind, float *host, int64_t count, bool set)
{
    SurrogateState &st = *ga->surr;
    const int64_t nE = (int64_t)st.n * kD;
    const int64_t off[7] = {0, nE + kOffW1, nE + kOffB1, nE + kOffW2, nE + kOffB2, nE + kOffW3, nE + kOffB3};
    const int64_t size[7] = {nE, kH * kD, kH, kH * kH, kH, kH, 1};
    if (which < 0 || which > 6 || kind < 0 || kind > 1 || count != size[which] || (set && kind != 0) || !host) {
        set_error("invalid tensor request");
        return GAPA_E_INVALID_ARG;
    }
    if (kind == 1 && !st.have_keep) {
        set_error("no gradients kept (train a batch with keep_grads)");
        return GAPA_E_STATE;
    }
    GAPA_HIP(hipDeviceSynchronize());
    float *dev = kind == 0 ? st.theta.as<float>() + off[which]
                           : (which == 0 ? st.keep_E.as<float>() : st.keep_mlp.as<float>() + (off[which] - nE));
    if (!set) {
        GAPA_HIP(hipMemcpy(host, dev, (size_t)count * 4, hipMemcpyDeviceToHost));
        return GAPA_OK;
    }
    GAPA_HIP(hipMemcpy(dev, host, (size_t)count * 4, hipMemcpyHostToDevice));
    const int64_t P = nE + kMlpParams;
    hipLaunchKernelGGL(k_bf16_copies, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, nullptr, st.theta.as<float>(),
                       (int64_t)st.n, copies(st));
    GAPA_HIP(hipGetLastError());
    GAPA_HIP(hipDeviceSynchronize());
    return GAPA_OK;
}

int surrogate_stats(gapa_ga *ga, gapa_surrogate_report *out)
{
    SurrogateState &st = *ga->surr;
    if (st.stats_pending) GAPA_HIP(hipEventSynchronize(st.ready));
    out->generation = st.last_gen;
    out->evaluated = st.last_evaluated;
    out->pooled = st.last_pooled;
    out->screened = st.last_screened ? 1 : 0;
    out->spearman = st.last_predicted ? st.hstats[2] : 0.0;
    out->rel_err = st.last_predicted ? st.hstats[3] : 0.0;
    out->loss = st.hstats[4];
    out->fallbacks = st.fallbacks;
    out->train_steps = (int32_t)st.steps;
    return GAPA_OK;
}

int surrogate_last_predictions(gapa_ga *ga, float *yhat, int32_t cap, int32_t *count)
{
    SurrogateState &st = *ga->surr;
    const int32_t c = st.last_gen > 0 && st.last_predicted ? st.lambda : 0;
    if (count) *count = c;
    if (yhat && c > 0) {
        GAPA_HIP(hipStreamSynchronize(ga->last_stream));
        GAPA_HIP(hipMemcpy(yhat, st.yhat.ptr, (size_t)std::min(c, cap) * 4, hipMemcpyDeviceToHost));
    }
    return GAPA_OK;
}

int surrogate_last_pool(gapa_ga *ga, int32_t *pool, int32_t cap, int32_t *count)
{
    SurrogateState &st = *ga->surr;
    const int32_t c = st.last_gen > 0 ? st.last_evaluated : 0;
    if (count) *count = c;
    if (pool && c > 0) {
        GAPA_HIP(hipStreamSynchronize(ga->last_stream));
        GAPA_HIP(hipMemcpy(pool, st.pool.ptr, (size_t)std::min(c, cap) * 4, hipMemcpyDeviceToHost));
    }
    return GAPA_OK;
}

}  // namespace gapa
