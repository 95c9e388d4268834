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
constexpr int kMlpRows = 16;  // samples per MLP block (one matrix-core row tile)
constexpr int kMlpWaves = 8;  // waves per MLP block, each with 32 hidden units (two column tiles)
constexpr uint32_t kStreamSurrInit = 5, kStreamSurrSample = 6, kStreamSurrRandom = 7;
constexpr int kJudgeMax = 1024;
constexpr int kJudgeExtra = 32;  // unscreened children evaluated for the judge in a screened generation
constexpr int kMaxLambda = 8192;

// flat layout of the MLP parameters after E (weights, gradients)
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH * kD;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kH;
constexpr int kMlpParams = kOffB3 + 1;

// LDS row strides of the MLP kernel (bf16 elements): X [16][72], H1, DZ2 [16][264]
constexpr int kSX = 72, kSH = 264;

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

// Copies the weights the forward pass reads (bf16 E, W1, W2, w3 and the FP32
// biases) into the prediction snapshot, 16 bytes a thread.
constexpr int kSnapParts = 8;
struct SnapArgs {
    const uint32_t *src[kSnapParts];
    uint32_t *dst[kSnapParts];
    int64_t len[kSnapParts];  // in 4-byte words; parts of a multiple of 4 words are 16-byte aligned
};

__global__ void k_snapshot(SnapArgs a)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int t = 0; t < kSnapParts; ++t) {
        if (a.len[t] % 4 == 0) {
            const uint4 *src = reinterpret_cast<const uint4 *>(a.src[t]);
            uint4 *dst = reinterpret_cast<uint4 *>(a.dst[t]);
            for (int64_t i = t0; i < a.len[t] / 4; i += stride) dst[i] = src[i];
        } else {
            for (int64_t i = t0; i < a.len[t]; i += stride) a.dst[t][i] = a.src[t][i];
        }
    }
}

// ------------------------------------------------------------- embedding ----

// x(S) of each row, rounded to bf16: one 256-thread block per row.  Lane
// (wave w, group g = lane / 16, q = lane % 16) adds dims 4q..4q+3 of genes
// j = 16 i + 4 w + g in ascending i; the four groups and the four waves are
// then added in a fixed order.  The row's gene ids are staged in LDS
// (kEmbedIds at a time, coalesced), so each lane keeps kEmbedUnroll
// embedding rows in flight without waiting on their ids.
constexpr int kEmbedIds = 2048;  // a multiple of 16: a chunk keeps each lane's residue j mod 16
constexpr int kEmbedUnroll = 8;

__global__ __launch_bounds__(256) void k_embed(const int32_t *__restrict__ genes, const int32_t *__restrict__ rows,
                                               int32_t k, const uint16_t *__restrict__ Eb, uint16_t *__restrict__ xb)
{
    __shared__ float s_part[4][kD];
    __shared__ int32_t s_ids[kEmbedIds];
    const int32_t row = rows ? rows[blockIdx.x] : (int32_t)blockIdx.x;
    const int32_t *g = genes + (int64_t)row * k;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int grp = lane >> 4, q = lane & 15;
    const int32_t r = 4 * wv + grp;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    for (int32_t c0 = 0; c0 < k; c0 += kEmbedIds) {
        const int32_t cn = min(kEmbedIds, k - c0);
        __syncthreads();  // the previous chunk's ids are no longer read
        for (int32_t t = threadIdx.x; t < cn; t += blockDim.x) s_ids[t] = g[c0 + t];
        __syncthreads();
        int32_t j = r;
        for (; j + 16 * (kEmbedUnroll - 1) < cn; j += 16 * kEmbedUnroll) {
            uint2 e[kEmbedUnroll];
#pragma unroll
            for (int u = 0; u < kEmbedUnroll; ++u)
                e[u] = *reinterpret_cast<const uint2 *>(Eb + (int64_t)s_ids[j + 16 * u] * kD + 4 * q);
#pragma unroll
            for (int u = 0; u < kEmbedUnroll; ++u) {
                a0 += bf2f((uint16_t)e[u].x);
                a1 += bf2f((uint16_t)(e[u].x >> 16));
                a2 += bf2f((uint16_t)e[u].y);
                a3 += bf2f((uint16_t)(e[u].y >> 16));
            }
        }
        for (; j < cn; j += 16) {
            const uint2 e = *reinterpret_cast<const uint2 *>(Eb + (int64_t)s_ids[j] * kD + 4 * q);
            a0 += bf2f((uint16_t)e.x);
            a1 += bf2f((uint16_t)(e.x >> 16));
            a2 += bf2f((uint16_t)e.y);
            a3 += bf2f((uint16_t)(e.y >> 16));
        }
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
    // training (N = B, a multiple of 16)
    const float *target; // [B] standardised labels
    float dscale;        // 2 / B
    float *lossv;        // [B] squared errors
    float *dy;           // [B] d loss / d yhat
    // feature-major bf16 activations and gradients for the weight gradients:
    // xT [64][B], h1T, h2T, dz1T, dz2T [256][B]; dxT [64][B] for dE
    uint16_t *xT, *h1T, *h2T, *dz1T, *dz2T, *dxT;
    // prediction: the label mean and spread of the weights used, copied for the judge
    const double *musd_src;
    double *musd_dst;
};

// Stores the four rows 4 lg .. 4 lg + 3 of one C-tile column as one 8-byte
// write into a feature-major [features][N] array.
__device__ __forceinline__ void store_col4(uint16_t *T, int32_t N, int32_t feat, int32_t row, uint16_t h0, uint16_t h1,
                                           uint16_t h2, uint16_t h3)
{
    uint2 q;
    q.x = h0 | ((uint32_t)h1 << 16);
    q.y = h2 | ((uint32_t)h3 << 16);
    *reinterpret_cast<uint2 *>(T + (int64_t)feat * N + row) = q;
}

// Forward for 16 samples per block (rows row0 .. row0 + 15); wave wv owns
// hidden units 32 wv .. 32 wv + 31 (two 16-wide column tiles) of each layer.
// MFMA tiles are 16 x 16 with K = 32: lane l holds A[l % 16][8 (l / 16) .. + 7],
// B[8 (l / 16) .. + 7][l % 16] and C[4 (l / 16) + r][l % 16], r = 0..3.
// With kTrain the block also runs the backward pass of its samples:
// dyhat = 2 (yhat - t) / B; dz2 = dyhat w3 [h2 > 0]; dh1 = dz2 W2;
// dz1 = dh1 [h1 > 0]; dx = dz1 W1, and writes the bf16 activations and
// gradients the weight-gradient kernel contracts over the batch.
template <bool kTrain>
__global__ __launch_bounds__(64 * kMlpWaves) void k_mlp(MlpArgs a)
{
    __shared__ __align__(16) uint16_t sX[kMlpRows * kSX];
    __shared__ __align__(16) uint16_t sH1[kMlpRows * kSH];   // h1, then dz1 in place
    __shared__ __align__(16) uint16_t sDZ2[kMlpRows * kSH];
    __shared__ float sY[kMlpWaves][kMlpRows];
    __shared__ float sDy[kMlpRows];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int32_t row0 = blockIdx.x * kMlpRows;
    const int c0 = wv * 32;
    // The wave's weight operands of both forward layers are loaded first:
    // they do not depend on the block's data, and loads after a barrier
    // could not be moved above it.
    bf16x8 w1o[kD / 32][2], w2o[kH / 32][2];
#pragma unroll
    for (int ks = 0; ks < kD / 32; ++ks)
#pragma unroll
        for (int t = 0; t < 2; ++t) w1o[ks][t] = ld8(a.W1b + (c0 + t * 16 + lr) * kD + ks * 32 + lg * 8);
#pragma unroll
    for (int ks = 0; ks < kH / 32; ++ks)
#pragma unroll
        for (int t = 0; t < 2; ++t) w2o[ks][t] = ld8(a.W2b + (c0 + t * 16 + lr) * kH + ks * 32 + lg * 8);

    if (!kTrain && a.musd_dst && blockIdx.x == 0 && threadIdx.x < 2) a.musd_dst[threadIdx.x] = a.musd_src[threadIdx.x];
    if (threadIdx.x < kMlpRows * 8) {
        const int r = threadIdx.x >> 3, c8 = (threadIdx.x & 7) * 8;
        uint4 v = {0u, 0u, 0u, 0u};
        if (row0 + r < a.N) v = *reinterpret_cast<const uint4 *>(a.xb + (int64_t)(row0 + r) * kD + c8);
        *reinterpret_cast<uint4 *>(sX + r * kSX + c8) = v;
    }
    __syncthreads();
    if (kTrain)
        for (int q = threadIdx.x; q < kD * (kMlpRows / 4); q += blockDim.x) {
            const int d = q >> 2, r = (q & 3) * 4;
            store_col4(a.xT, a.N, d, row0 + r, sX[r * kSX + d], sX[(r + 1) * kSX + d], sX[(r + 2) * kSX + d],
                       sX[(r + 3) * kSX + d]);
        }

    // layer 1: z1 = x W1^T + b1, h1 = relu(z1) in bf16
    f32x4 acc[2];
    float h1v[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kD / 32; ++ks) {
        const bf16x8 A = ld8(sX + lr * kSX + ks * 32 + lg * 8);
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[t] = mfma(A, w1o[ks][t], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int c = c0 + t * 16 + lr;
        const float b = a.b1[c];
        uint16_t h[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            h[r] = f2bf(fmaxf(acc[t][r] + b, 0.f));
            h1v[t][r] = bf2f(h[r]);
            sH1[(4 * lg + r) * kSH + c] = h[r];
        }
        if (kTrain) store_col4(a.h1T, a.N, c, row0 + 4 * lg, h[0], h[1], h[2], h[3]);
    }
    __syncthreads();

    // layer 2: z2 = h1 W2^T + b2, h2 = relu(z2) in bf16; yhat = w3 . h2 + b3
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kH / 32; ++ks) {
        const bf16x8 A = ld8(sH1 + lr * kSH + ks * 32 + lg * 8);
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[t] = mfma(A, w2o[ks][t], acc[t]);
    }
    float p[4] = {0.f, 0.f, 0.f, 0.f};
    float w3v[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int c = c0 + t * 16 + lr;
        const float b = a.b2[c];
        w3v[t] = bf2f(a.w3b[c]);
        uint16_t h[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            h[r] = f2bf(fmaxf(acc[t][r] + b, 0.f));
            acc[t][r] = bf2f(h[r]);
            p[r] += acc[t][r] * w3v[t];
        }
        if (kTrain) store_col4(a.h2T, a.N, c, row0 + 4 * lg, h[0], h[1], h[2], h[3]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) p[r] += __shfl_xor(p[r], off, 64);
    if (lr == 0)
#pragma unroll
        for (int r = 0; r < 4; ++r) sY[wv][4 * lg + r] = p[r];
    __syncthreads();
    if (threadIdx.x < kMlpRows) {
        const int r = threadIdx.x;
        const int32_t row = row0 + r;
        float y = 0.f;
#pragma unroll
        for (int w = 0; w < kMlpWaves; ++w) y += sY[w][r];
        y += a.b3[0];
        float d = 0.f;
        if (row < a.N) {
            a.yhat[row] = y;
            if (kTrain) {
                const float e = y - a.target[row];
                d = e * a.dscale;
                a.lossv[row] = e * e;
                a.dy[row] = d;
            }
        }
        sDy[r] = d;
    }
    if (!kTrain) return;
    // the backward pass's W2^T operands (the forward ones are no longer needed)
#pragma unroll
    for (int ks = 0; ks < kH / 32; ++ks)
#pragma unroll
        for (int t = 0; t < 2; ++t) w2o[ks][t] = ld8(a.W2bT + (c0 + t * 16 + lr) * kH + ks * 32 + lg * 8);
    __syncthreads();

    // dz2 = dyhat w3 [h2 > 0]
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int c = c0 + t * 16 + lr;
        uint16_t h[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            h[r] = f2bf(acc[t][r] > 0.f ? sDy[4 * lg + r] * w3v[t] : 0.f);
            sDZ2[(4 * lg + r) * kSH + c] = h[r];
        }
        store_col4(a.dz2T, a.N, c, row0 + 4 * lg, h[0], h[1], h[2], h[3]);
    }
    __syncthreads();

    // dh1 = dz2 W2, dz1 = dh1 [h1 > 0] (into sH1: each element by its owner)
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kH / 32; ++ks) {
        const bf16x8 A = ld8(sDZ2 + lr * kSH + ks * 32 + lg * 8);
#pragma unroll
        for (int t = 0; t < 2; ++t) acc[t] = mfma(A, w2o[ks][t], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int c = c0 + t * 16 + lr;
        uint16_t h[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            h[r] = f2bf(h1v[t][r] > 0.f ? acc[t][r] : 0.f);
            sH1[(4 * lg + r) * kSH + c] = h[r];
        }
        store_col4(a.dz1T, a.N, c, row0 + 4 * lg, h[0], h[1], h[2], h[3]);
    }
    __syncthreads();

    // dx = dz1 W1: waves 0..3, one 16-wide tile of the 64 dimensions each
    if (wv < kD / 16) {
        f32x4 ax = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < kH / 32; ++ks)
            ax = mfma(ld8(sH1 + lr * kSH + ks * 32 + lg * 8), ld8(a.W1bT + (wv * 16 + lr) * kH + ks * 32 + lg * 8), ax);
        store_col4(a.dxT, a.N, wv * 16 + lr, row0 + 4 * lg, f2bf(ax[0]), f2bf(ax[1]), f2bf(ax[2]), f2bf(ax[3]));
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

struct WgradArgs {
    const uint16_t *xT, *h1T, *h2T, *dz1T, *dz2T;  // feature-major [features][B] bf16
    const float *dy, *lossv;                       // [B]
    int32_t B;
    float *theta, *m, *v;                          // MLP parameters (flat layout), moments
    float *keep;                                   // NULL, or the gradient of every parameter
    Bf16Copies cp;
    AdamArgs o;
    double *loss_out;                              // mean squared error of the batch
};

__device__ __forceinline__ void adam_param(const WgradArgs &a, int32_t j, float g)
{
    if (a.keep) a.keep[j] = g;
    float th = a.theta[j], mm = a.m[j], vv = a.v[j];
    adam(th, mm, vv, g, a.o);
    a.theta[j] = th;
    a.m[j] = mm;
    a.v[j] = vv;
    mlp_copy(a.cp, j, th);
}

// MLP parameter gradients over the batch, then Adam and the bfloat16 copies;
// one wave per task.  Tasks 0..255: 16 x 16 tiles of dW2 = dz2^T h1;
// 256..319: tiles of dW1 = dz1^T x (K = the batch, on the matrix cores, eight
// k-steps loaded at a time); then db1 = sum dz1,
// db2 = sum dz2 and dw3 = sum dyhat h2, one entry per task (each lane adds a
// run of samples in order, lanes combined in a fixed tree); the last task:
// db3 = sum dyhat and the loss.
constexpr int kWgradTasks = 320 + 3 * kH + 1;
__global__ __launch_bounds__(64) void k_mlp_wgrad(WgradArgs a)
{
    const int32_t task = blockIdx.x;
    const int lane = threadIdx.x, lr = lane & 15, lg = lane >> 4;
    const int32_t B = a.B;
    if (task < 320) {
        const bool w2 = task < 256;
        const int32_t J = w2 ? task >> 4 : (task - 256) >> 2;  // output rows (hidden unit j)
        const int32_t I = w2 ? task & 15 : (task - 256) & 3;    // output columns
        const uint16_t *At = (w2 ? a.dz2T : a.dz1T) + (int64_t)(J * 16 + lr) * B + lg * 8;
        const uint16_t *Bt = (w2 ? a.h1T : a.xT) + (int64_t)(I * 16 + lr) * B + lg * 8;
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
        constexpr int U = 8;
        for (int32_t ks0 = 0; ks0 < B; ks0 += 32 * U) {
            bf16x8 av[U], bv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t ks = ks0 + 32 * u;
                av[u] = ks < B ? ld8(At + ks) : bf16x8{};
                bv[u] = ks < B ? ld8(Bt + ks) : bf16x8{};
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc = mfma(av[u], bv[u], acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int32_t j = J * 16 + 4 * lg + r, i = I * 16 + lr;
            adam_param(a, w2 ? kOffW2 + j * kH + i : kOffW1 + j * kD + i, acc[r]);
        }
        return;
    }
    if (task < 320 + 3 * kH) {
        const int32_t kind = (task - 320) / kH;  // 0 b1, 1 b2, 2 w3
        const int32_t j = (task - 320) % kH;
        const uint16_t *row = (kind == 0 ? a.dz1T : kind == 1 ? a.dz2T : a.h2T) + (int64_t)j * B;
        // lane l adds samples [l per, (l + 1) per) in order, per = B / 64 (B >= 64)
        // or one sample (B = 32)
        const int32_t per = B >= 64 ? B >> 6 : 1;
        const int32_t s0 = lane * per;
        float g = 0.f;
        if (s0 < B) {
            if ((per & 7) == 0) {
                for (int32_t e0 = 0; e0 < per; e0 += 8) {
                    const uint4 q = *reinterpret_cast<const uint4 *>(row + s0 + e0);
                    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const float x = bf2f((uint16_t)(w[e >> 1] >> (16 * (e & 1))));
                        g += kind == 2 ? a.dy[s0 + e0 + e] * x : x;
                    }
                }
            } else {
                for (int32_t e = 0; e < per; ++e) {
                    const float x = bf2f(row[s0 + e]);
                    g += kind == 2 ? a.dy[s0 + e] * x : x;
                }
            }
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) g += __shfl_xor(g, off, 64);
        if (lane == 0) adam_param(a, kind == 0 ? kOffB1 + j : kind == 1 ? kOffB2 + j : kOffW3 + j, g);
        return;
    }
    // db3 and the loss: lane l takes samples l, l + 64, ...; lanes combined in a fixed tree
    float g = 0.f;
    double l2 = 0.0;
    for (int32_t s0 = lane; s0 < B; s0 += 64) {
        g += a.dy[s0];
        l2 += (double)a.lossv[s0];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        g += __shfl_xor(g, off, 64);
        l2 += __shfl_xor(l2, off, 64);
    }
    if (lane == 0) {
        adam_param(a, kOffB3, g);
        *a.loss_out = l2 / B;
    }
}

// Embeddings.  dE = M^T dx, M the batch's sample x node membership matrix:
// for the hub nodes that sit in most sets of a converged population this is
// a dense contraction over the batch, so it runs on the matrix cores.  The B
// operand (dx of the whole batch, bf16, dimension-major) is staged once per
// block in LDS, rows padded by 8 elements so that the 16 rows a k-step reads
// fall in different banks; each wave then walks tiles of 16 nodes: the A
// operand is the tile's membership bits (node-major rows, one 32-bit word
// per 32 samples) expanded to bf16 0/1, K = the batch; k-steps whose word is
// zero for the whole tile are skipped.  Adam is lazy on E: a node in some
// sample steps with the global step count, straight from the accumulators;
// the others keep weights and moments.
__global__ __launch_bounds__(1024) void k_grad_adam_E(const uint32_t *__restrict__ bits, int32_t Wb,
                                                     const uint16_t *__restrict__ dxT, int32_t B,
                                                     float *__restrict__ E, float *__restrict__ m,
                                                     float *__restrict__ v, uint16_t *__restrict__ Eb,
                                                     float *__restrict__ keep, int64_t n, AdamArgs o)
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
        // every lane (lr, lg) holds all Wb <= 32 words of node v0 + lr's row
        // (the four lanes of a node read the same 128 bytes), so a k-step
        // needs no exchange between lanes
        uint32_t w32[32];
#pragma unroll
        for (int ks = 0; ks < 32; ++ks) w32[ks] = (row < n && ks < Wb) ? bits[row * Wb + ks] : 0u;
        uint32_t rowany = 0u;
#pragma unroll
        for (int ks = 0; ks < 32; ++ks) rowany |= w32[ks];
        if (__ballot(rowany != 0u) == 0) {
            if (keep)
                for (int q = lane; q < 16 * kD; q += 64)
                    if (v0 + q / kD < n) keep[v0 * kD + q] = 0.f;
            continue;
        }
        f32x4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 32; ++ks) {
            const uint32_t word = w32[ks];
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
        // lane (lr, lg) holds dE[v0 + 4 lg + r][16 t + lr]; node v0 + i's
        // membership flag sits in lane i.  The weights and moments of all
        // sixteen entries are loaded before any is updated, so the loads are
        // in flight together.
        bool tch[4];
        float th[4][4], mm[4][4], vv[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t node = v0 + 4 * lg + r;
            const bool touched = __shfl((int)rowany, 4 * lg + r, 64) != 0;
            tch[r] = touched && node < n;
            if (keep && node < n)
#pragma unroll
                for (int t = 0; t < 4; ++t) keep[node * kD + t * 16 + lr] = touched ? acc[t][r] : 0.f;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t base = (v0 + 4 * lg + r) * kD + lr;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                th[r][t] = tch[r] ? E[base + t * 16] : 0.f;
                mm[r][t] = tch[r] ? m[base + t * 16] : 0.f;
                vv[r][t] = tch[r] ? v[base + t * 16] : 0.f;
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (!tch[r]) continue;
            const int64_t base = (v0 + 4 * lg + r) * kD + lr;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                adam(th[r][t], mm[r][t], vv[r][t], acc[t][r], o);
                E[base + t * 16] = th[r][t];
                m[base + t * 16] = mm[r][t];
                v[base + t * 16] = vv[r][t];
                Eb[base + t * 16] = f2bf(th[r][t]);
            }
        }
    }
}

size_t grad_E_lds(int32_t B)
{
    return (size_t)kD * (B + 8) * 2;
}

// --------------------------------------------------------- GA-side steps ----

// Orderable 32-bit key of a prediction (NaN last); ties are broken by index.
__device__ __forceinline__ uint32_t pred_key(float y)
{
    uint32_t u = __float_as_uint(y);
    if (y != y) u = 0x7FFFFFFFu;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ uint32_t random_key(uint64_t seed, uint32_t gen, uint32_t ind, uint32_t i)
{
    return draw(seed, i, ind, gen, kStreamSurrRandom, 0).w0;
}

__device__ __forceinline__ bool bit_of(const uint32_t *bits, int32_t i)
{
    return (bits[i >> 5] >> (i & 31)) & 1u;
}

// Exclusive prefix sum over the block (blockDim.x a multiple of 64, <= 1024);
// also returns the block total.  Every thread must call it.
__device__ int32_t block_scan(int32_t x, int32_t *total)
{
    __shared__ int32_t s_wave[16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) s_wave[wv] = incl;
    __syncthreads();
    int32_t before = 0, sum = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
        if (q < wv) before += s_wave[q];
        sum += s_wave[q];
    }
    __syncthreads();
    *total = sum;
    return before + incl - x;
}

// Sets in sel (a bit set over [0, L), cleared by the caller) the `want`
// entries with the smallest (key[i], i) among those not in excl (NULL: none
// excluded); want must not exceed the entries left.  Radix selection on the
// key, eight bits a pass: each pass counts the candidates' next digit and
// keeps the digit that holds the want-th smallest; the keys equal to the
// final value are then taken in index order.  Whole block.
__device__ void block_select(const uint32_t *key, const uint32_t *excl, int32_t L, int32_t want, uint32_t *sel)
{
    __shared__ int32_t hist[256];
    __shared__ uint32_t s_val;
    __shared__ int32_t s_need;
    if (want <= 0) return;
    uint32_t val = 0;  // digits fixed so far
    int32_t need = want;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int32_t i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
        __syncthreads();
        const uint32_t hi_mask = shift == 24 ? 0u : ~0u << (shift + 8);
        for (int32_t i = threadIdx.x; i < L; i += blockDim.x)
            if (!(excl && bit_of(excl, i)) && (key[i] & hi_mask) == (val & hi_mask))
                atomicAdd(&hist[(key[i] >> shift) & 255u], 1);
        __syncthreads();
        if (threadIdx.x < 64) {
            // lane l holds digits 4l .. 4l + 3
            const int l = threadIdx.x;
            const int32_t c0 = hist[4 * l], c1 = hist[4 * l + 1], c2 = hist[4 * l + 2], c3 = hist[4 * l + 3];
            int32_t incl = c0 + c1 + c2 + c3;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int32_t y = __shfl_up(incl, off, 64);
                if (l >= off) incl += y;
            }
            int32_t before = incl - (c0 + c1 + c2 + c3);
            // the digit whose cumulative count first reaches need
            const int32_t cs[4] = {c0, c1, c2, c3};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (before < need && before + cs[e] >= need) {
                    s_val = val | ((uint32_t)(4 * l + e) << shift);
                    s_need = need - before;
                }
                before += cs[e];
            }
        }
        __syncthreads();
        val = s_val;
        need = s_need;
        __syncthreads();
    }
    // keys below val are taken; of the keys equal to val, the first `need`
    // in index order.  Thread t owns the index range [t per, (t + 1) per).
    const int32_t per = (L + blockDim.x - 1) / blockDim.x;
    const int32_t i0 = min(L, (int32_t)threadIdx.x * per), i1 = min(L, i0 + per);
    int32_t eq = 0;
    for (int32_t i = i0; i < i1; ++i) eq += !(excl && bit_of(excl, i)) && key[i] == val;
    int32_t total = 0;
    int32_t rank = block_scan(eq, &total);
    for (int32_t i = i0; i < i1; ++i) {
        if (excl && bit_of(excl, i)) continue;
        bool take = key[i] < val;
        if (key[i] == val) take = rank++ < need;
        if (take) atomicOr(&sel[i >> 5], 1u << (i & 31));
    }
    __syncthreads();
}

// Indices whose bit is set in bits[0, ceil(lambda / 32)), ascending, to
// out[]; whole block (blockDim.x <= 1024).
__device__ void block_compact(const uint32_t *bits, int32_t lambda, int32_t *out)
{
    const int32_t words = (lambda + 31) / 32;
    const int32_t per = (words + blockDim.x - 1) / blockDim.x;
    const int32_t w0 = min(words, (int32_t)threadIdx.x * per), w1 = min(words, w0 + per);
    int32_t cnt = 0;
    for (int32_t w = w0; w < w1; ++w) cnt += __popc(bits[w]);
    int32_t total = 0;
    int32_t off = block_scan(cnt, &total);
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
__global__ __launch_bounds__(1024) void k_screen(const float *__restrict__ yhat, int32_t lambda, int32_t m,
                                                 int32_t extra, uint64_t seed, uint32_t gen,
                                                 int32_t *__restrict__ pool)
{
    __shared__ uint32_t key[kMaxLambda];
    __shared__ uint32_t chosen[kMaxLambda / 32], judged[kMaxLambda / 32];
    for (int32_t i = threadIdx.x; i < lambda; i += blockDim.x)
        key[i] = yhat ? pred_key(yhat[i]) : random_key(seed, gen, 0, i);
    for (int32_t i = threadIdx.x; i < kMaxLambda / 32; i += blockDim.x) chosen[i] = judged[i] = 0u;
    __syncthreads();
    block_select(key, nullptr, lambda, m, chosen);
    block_compact(chosen, lambda, pool);
    if (extra <= 0) return;
    for (int32_t i = threadIdx.x; i < lambda; i += blockDim.x) key[i] = random_key(seed, gen, 1, i);
    __syncthreads();
    block_select(key, chosen, lambda, extra, judged);
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
// Block 0 also copies the loss of the last finished training step.
__global__ void k_append(const int32_t *__restrict__ children, int32_t k, const int32_t *__restrict__ pool,
                         const int64_t *__restrict__ F, int64_t base, int32_t cap, int32_t *__restrict__ buf_genes,
                         double *__restrict__ buf_y, const double *__restrict__ loss, double *__restrict__ loss_out)
{
    const int32_t q = blockIdx.x;
    const int32_t o = pool ? pool[q] : q;
    const int64_t slot = (base + q) % cap;
    for (int32_t j = threadIdx.x; j < k; j += blockDim.x) buf_genes[slot * k + j] = children[(int64_t)o * k + j];
    if (threadIdx.x == 0) buf_y[slot] = log1p((double)F[q]);
    if (q == 0 && threadIdx.x == 0) *loss_out = *loss;
}

// Mean and spread of the buffered labels (one block, fixed order): the
// spread is sqrt(variance + floor^2), so that a buffer of (nearly) equal
// labels gives targets near zero rather than amplified rounding noise.
constexpr double kSpreadFloor = 1e-6;
__device__ double block_sum_d(double a, double *s_w)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = a;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += s_w[w];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(1024) void k_label_stats(const double *__restrict__ y, int32_t count,
                                                      double *__restrict__ out)
{
    __shared__ double s_w[16];
    // four partial sums per thread, so that four loads are in flight at once
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    const int32_t step = 4 * blockDim.x;
    int32_t i = threadIdx.x;
    for (; i + 3 * (int32_t)blockDim.x < count; i += step)
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] += y[i + u * blockDim.x];
    for (; i < count; i += blockDim.x) a[0] += y[i];
    const double mu = block_sum_d((a[0] + a[1]) + (a[2] + a[3]), s_w) / count;
    double b[4] = {0.0, 0.0, 0.0, 0.0};
    i = threadIdx.x;
    for (; i + 3 * (int32_t)blockDim.x < count; i += step)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double d = y[i + u * blockDim.x] - mu;
            b[u] += d * d;
        }
    for (; i < count; i += blockDim.x) b[0] += (y[i] - mu) * (y[i] - mu);
    const double var = block_sum_d((b[0] + b[1]) + (b[2] + b[3]), s_w) / count;
    if (threadIdx.x == 0) {
        out[0] = mu;
        out[1] = sqrt(var + kSpreadFloor * kSpreadFloor);
    }
}

// Training batch of step `step` in generation `gen`: entry j is buffer row
// bounded(w, count), w the first word of draw(seed, j, step, gen, stream 6);
// its genes are copied and its label standardised.
// Membership bits of a sampled training batch are built per chunk of
// kBitChunk nodes.  k_sample records, for each sample j and each chunk
// boundary c (node c kBitChunk, c = 0 .. nchunks), the position in the
// sample's ascending gene row of the first gene at or above it:
// pos[j][c] (binary searches over the row staged in LDS).
constexpr int kBitChunk = 256;  // 32 KB of LDS per block at a batch of 1024: blocks of other kernels fit beside it
constexpr int kSampleRowLds = 4096;      // longest row staged in LDS for the searches

__global__ void k_sample(uint64_t seed, uint32_t gen, uint32_t step, int32_t count, const int32_t *__restrict__ buf_genes,
                         const double *__restrict__ buf_y, const double *__restrict__ mu_sd, int32_t k,
                         int32_t *__restrict__ genes, float *__restrict__ target, int32_t nchunks,
                         int32_t *__restrict__ pos)
{
    __shared__ int32_t s_idx;
    __shared__ int32_t s_row[kSampleRowLds];
    const int32_t j = blockIdx.x;
    if (threadIdx.x == 0) {
        const uint32_t w = draw(seed, (uint32_t)j, step, gen, kStreamSurrSample, 0).w0;
        s_idx = (int32_t)bounded(w, (uint32_t)count);
        target[j] = (float)((buf_y[s_idx] - mu_sd[0]) / mu_sd[1]);
    }
    __syncthreads();
    const int32_t r = s_idx;
    const int32_t *src = buf_genes + (int64_t)r * k;
    const bool lds = k <= kSampleRowLds;
    for (int32_t t = threadIdx.x; t < k; t += blockDim.x) {
        const int32_t gt = src[t];
        genes[(int64_t)j * k + t] = gt;
        if (lds) s_row[t] = gt;
    }
    __syncthreads();
    const int32_t *row = lds ? s_row : src;
    for (int32_t c = threadIdx.x; c <= nchunks; c += blockDim.x) {
        const int32_t v = c * kBitChunk;
        int32_t lo = 0, hi = k;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (row[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        pos[(int64_t)j * (nchunks + 1) + c] = lo;
    }
}

// Node-major membership bits of a sampled batch: bit (j mod 32) of word
// j / 32 of node v's row is set when v is in sample j.  One block per chunk
// of kBitChunk nodes: each thread loads the genes of its samples that lie in
// the chunk (their span is known from the start positions, so the loads are
// issued together), sets their bits in an LDS tile of the chunk's rows, and
// the tile is written out.
__global__ __launch_bounds__(256) void k_batch_bits(const int32_t *__restrict__ genes, int32_t k, int32_t B,
                                                    const int32_t *__restrict__ pos, int32_t nchunks, int32_t n,
                                                    uint32_t *__restrict__ rows)
{
    extern __shared__ uint32_t tile[];  // [kBitChunk][B / 32]
    const int32_t Wb = B / 32;
    const int32_t c = blockIdx.x;
    const int32_t v0 = c * kBitChunk;
    for (int32_t t = threadIdx.x; t < kBitChunk * Wb; t += blockDim.x) tile[t] = 0u;
    __syncthreads();
    for (int32_t j = threadIdx.x; j < B; j += blockDim.x) {
        const int32_t p0 = pos[(int64_t)j * (nchunks + 1) + c], p1 = pos[(int64_t)j * (nchunks + 1) + c + 1];
        const uint32_t bit = 1u << (j & 31);
        const int32_t *row = genes + (int64_t)j * k;
#pragma unroll 4
        for (int32_t p = p0; p < p1; ++p) atomicOr(&tile[(row[p] - v0) * Wb + (j >> 5)], bit);
    }
    __syncthreads();
    const int32_t words = min(kBitChunk, n - v0) * Wb;
    for (int32_t t = threadIdx.x; t < words; t += blockDim.x) rows[(int64_t)v0 * Wb + t] = tile[t];
}

// Judge: over J = min(m, 1024) evaluated children (entry i is pool entry
// floor(i m / J)), Spearman's correlation between predictions and exact PC
// (average ranks), and the mean relative error of expm1(yhat sd + mu).
// out[0] the correlation, out[1] the error; out_musd (optional) receives the
// label mean and spread the predictions were made in.
constexpr int kJudgeKeys = 64;  // keys per k_judge_part block, 16 threads a key

// Partial sums of the judge's statistics: block b ranks keys [64 b, 64 b + 64)
// of the J evenly spaced evaluated children, each key by 16 threads that
// split the others between them (their counts combined by shuffles), and
// writes its keys' sums of ra rb, ra^2, rb^2 and the relative error to
// part[4 b ..] in a fixed order.  (One block ranking every key by one
// thread took 33 us per screened generation.)
__global__ __launch_bounds__(1024) void k_judge_part(const float *__restrict__ yhat, const int32_t *__restrict__ pool,
                                                     const int64_t *__restrict__ F, int32_t m,
                                                     const double *__restrict__ mu_sd, double *__restrict__ part)
{
    __shared__ float s_y[kJudgeMax];
    __shared__ int64_t s_f[kJudgeMax];
    __shared__ double s_w[4][16];
    const int32_t J = min(m, kJudgeMax);
    for (int32_t i = threadIdx.x; i < J; i += blockDim.x) {
        const int32_t q = (int32_t)(((int64_t)i * m) / J);
        s_y[i] = yhat[pool ? pool[q] : q];
        s_f[i] = F[q];
    }
    __syncthreads();
    const int32_t i = blockIdx.x * kJudgeKeys + (int32_t)(threadIdx.x >> 4), p = threadIdx.x & 15;
    int32_t la = 0, ea = 0, lb = 0, eb = 0;
    if (i < J) {
        const float yi = s_y[i];
        const int64_t fi = s_f[i];
        for (int32_t j = p; j < J; j += 16) {
            la += s_y[j] < yi;
            ea += s_y[j] == yi;
            lb += s_f[j] < fi;
            eb += s_f[j] == fi;
        }
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) {
        la += __shfl_xor(la, off, 64);
        ea += __shfl_xor(ea, off, 64);
        lb += __shfl_xor(lb, off, 64);
        eb += __shfl_xor(eb, off, 64);
    }
    double ra = 0.0, rb = 0.0, rel = 0.0;
    if (i < J && p == 0) {
        const double mid = (J + 1) / 2.0;
        ra = la + (ea + 1) / 2.0 - mid;
        rb = lb + (eb + 1) / 2.0 - mid;
        const double f = (double)s_f[i];
        const double pred = expm1((double)s_y[i] * mu_sd[1] + mu_sd[0]);
        rel = fabs(pred - f) / fmax(f, 1.0);
    }
    // sums: a fixed tree inside each wave, then the waves in order
    double q[4] = {ra * rb, ra * ra, rb * rb, rel};
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) q[t] += __shfl_xor(q[t], off, 64);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int t = 0; t < 4; ++t) s_w[t][threadIdx.x >> 6] = q[t];
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum[4] = {0.0, 0.0, 0.0, 0.0};
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
#pragma unroll
            for (int t = 0; t < 4; ++t) sum[t] += s_w[t][w];
#pragma unroll
        for (int t = 0; t < 4; ++t) part[4 * blockIdx.x + t] = sum[t];
    }
}

// The judge's statistics from the nb blocks' partial sums, added in block
// order: Spearman's rho (Pearson's over the average ranks) and the mean
// relative error; with out_musd, the label mean and spread used.
__global__ void k_judge_final(const double *__restrict__ part, int32_t nb, int32_t m, const double *__restrict__ mu_sd,
                              double *__restrict__ out, double *__restrict__ out_musd)
{
    if (threadIdx.x != 0) return;
    const int32_t J = min(m, kJudgeMax);
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    for (int32_t b = 0; b < nb; ++b)
#pragma unroll
        for (int t = 0; t < 4; ++t) sum[t] += part[4 * b + t];
    const double den = sqrt(sum[1] * sum[2]);
    out[0] = den > 0.0 ? sum[0] / den : 0.0;
    out[1] = sum[3] / J;
    if (out_musd) {
        out_musd[0] = mu_sd[0];
        out_musd[1] = mu_sd[1];
    }
}

int launch_judge(const float *yhat, const int32_t *pool, const int64_t *F, int32_t m, const double *mu_sd,
                 double *part, double *out, double *out_musd, hipStream_t s)
{
    const int32_t J = std::min(m, kJudgeMax);
    const int32_t nb = std::max(1, (J + kJudgeKeys - 1) / kJudgeKeys);
    hipLaunchKernelGGL(k_judge_part, dim3(nb), dim3(1024), 0, s, yhat, pool, F, m, mu_sd, part);
    hipLaunchKernelGGL(k_judge_final, dim3(1), dim3(64), 0, s, part, nb, m, mu_sd, out, out_musd);
    GAPA_HIP(hipGetLastError());
    return GAPA_OK;
}

}  // namespace

// -------------------------------------------------------------- host side ----

struct SurrogateState {
    gapa_surrogate_params sp{};
    int32_t n = 0, k = 0, lambda = 0, W = 0;
    uint64_t seed = 0;
    int64_t steps = 0;        // Adam steps taken
    int64_t appended = 0;     // pairs appended to the ring buffer
    int32_t low_run = 0;      // consecutive judged screened generations below min_rho
    int32_t fallbacks = 0;
    int64_t skip_before = 0;  // judged generations launched before the last forced full one do not count
    int64_t last_gen = 0;
    // Figures of generation g live in slot g & 1 (host metadata, the mapped
    // statistics and the event that marks them final): the host decides the
    // fallback for generation g from the judge of generation g - 2, so it
    // never waits for the generation just launched.
    struct Slot {
        int64_t gen = -1;
        int32_t evaluated = 0, pooled = 0;
        bool screened = false, predicted = false, judged = true;
    } slot[2];
    DevBuf theta, m, v, keep_mlp, keep_E;               // float
    DevBuf Eb, W1b, W2b, w3b, W1bT, W2bT;               // bf16
    DevBuf xb, yhat;                                    // predictions: x(S) and yhat of the generation
    DevBuf snap;                                        // prediction snapshot: Eb, W1b, W2b, w3b, biases
    DevBuf xtrain, ytrain, target, lossv, dy;           // training batch, per sample
    DevBuf xT, h1T, h2T, dz1T, dz2T, dxT;               // feature-major training activations, bf16
    DevBuf bgenes, bmasks, balive, bflag, tflag, brows; // training batch
    DevBuf bpos;                                        // int32 [steps][B][chunks + 1]: chunk starts in the batch rows
    DevBuf buf_genes, buf_y;                            // ring buffer
    DevBuf pool, crows, cmasks, calive;                 // screened children
    DevBuf dstats;                                      // double [2]: label mean and spread of the predictions
    DevBuf jpart;                                       // double [16][4]: the judge's partial sums
    DevBuf dloss;                                       // double [5]: [0] the loss of the last explicit
                                                        // batch; [1 + (g & 3)] the loss of the last step of
                                                        // generation g's training
    DevBuf tstats;                                      // double [2]: label mean and spread the training uses
    double *hstats = nullptr;                           // pinned, mapped, per slot (8 doubles): [2] rho,
                                                        // [3] rel_err, [4] loss,
                                                        // [5, 6] the predictions' label mean and spread
    double *hstats_dev = nullptr;                       // its device address (the judge and k_append write it)
    hipEvent_t ready[2] = {nullptr, nullptr};
    // Generation g's training runs on its own stream beside generation g + 1;
    // the predictions of generation g read a snapshot of the weights trained
    // through generation g - 2.
    hipStream_t ts = nullptr;
    hipEvent_t ev_pred = nullptr;   // main stream: the generation's predictions are made
    hipEvent_t ev_snap = nullptr;   // training stream: training done and snapshot taken
    hipEvent_t ev_data = nullptr;   // main stream: the generation's labels are in the buffer
    hipEvent_t ev_sampled = nullptr;  // training stream: the generation's batches are copied out of the buffer
    bool have_keep = false;
    bool explicit_loss = false;  // the last training step was an explicit batch: its loss is in dloss
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

// The prediction snapshot: bf16 E [n][64], W1 [256][64], W2 [256][256],
// w3 [256] and the FP32 biases b1, b2 (b3 after them), each part 256-byte
// aligned.
struct SnapLayout {
    size_t eb, w1, w2, w3, bias, musd, bytes;
};

SnapLayout snap_layout(int64_t n)
{
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    SnapLayout l{};
    l.eb = 0;
    l.w1 = up((size_t)n * kD * 2);
    l.w2 = l.w1 + up((size_t)kH * kD * 2);
    l.w3 = l.w2 + up((size_t)kH * kH * 2);
    l.bias = l.w3 + up((size_t)kH * 2);
    l.musd = l.bias + up((size_t)(2 * kH + 4) * 4);
    l.bytes = l.musd + 256;
    return l;
}

MlpArgs mlp_args(SurrogateState &st, const uint16_t *xb, float *yhat, int32_t N, bool snapshot = false)
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
    if (snapshot) {
        const SnapLayout l = snap_layout(st.n);
        char *b = static_cast<char *>(st.snap.ptr);
        a.W1b = reinterpret_cast<const uint16_t *>(b + l.w1);
        a.W2b = reinterpret_cast<const uint16_t *>(b + l.w2);
        a.w3b = reinterpret_cast<const uint16_t *>(b + l.w3);
        a.b1 = reinterpret_cast<const float *>(b + l.bias);
        a.b2 = a.b1 + kH;
        a.b3 = a.b1 + 2 * kH;
        a.W1bT = a.W2bT = nullptr;  // forward only
    }
    a.yhat = yhat;
    a.N = N;
    return a;
}

// Copies the live weights into the prediction snapshot (stream s).
int take_snapshot(SurrogateState &st, hipStream_t s)
{
    const SnapLayout l = snap_layout(st.n);
    char *b = static_cast<char *>(st.snap.ptr);
    const float *th = mlp_theta(st);
    SnapArgs a{};
    // bf16 E, W1, W2, w3; the FP32 biases b1, b2, b3 (b2 and b3 are not next
    // to b1 in the parameter layout); the label standardisation the
    // snapshot's predictions are in
    const void *src[kSnapParts] = {st.Eb.ptr, st.W1b.ptr, st.W2b.ptr, st.w3b.ptr, th + kOffB1, th + kOffB2,
                                   th + kOffB3, st.tstats.ptr};
    const size_t off[kSnapParts] = {l.eb, l.w1, l.w2, l.w3, l.bias, l.bias + kH * 4, l.bias + 2 * kH * 4, l.musd};
    const size_t bytes[kSnapParts] = {(size_t)st.n * kD * 2, (size_t)kH * kD * 2, (size_t)kH * kH * 2,
                                      (size_t)kH * 2, (size_t)kH * 4, (size_t)kH * 4, 4, 16};
    for (int t = 0; t < kSnapParts; ++t) {
        a.src[t] = static_cast<const uint32_t *>(src[t]);
        a.dst[t] = reinterpret_cast<uint32_t *>(b + off[t]);
        a.len[t] = (int64_t)(bytes[t] / 4);
    }
    hipLaunchKernelGGL(k_snapshot, dim3(1024), dim3(256), 0, s, a);
    GAPA_HIP(hipGetLastError());
    return GAPA_OK;
}

// Predictions for N rows of genes (rows[] selects rows when not NULL), from
// the live weights or from the snapshot.
int predict_rows(SurrogateState &st, const int32_t *genes, const int32_t *rows, int32_t N, float *yhat, hipStream_t s,
                 bool snapshot = false)
{
    if (N <= 0) return GAPA_OK;
    const uint16_t *Eb = snapshot ? reinterpret_cast<const uint16_t *>(static_cast<char *>(st.snap.ptr) +
                                                                       snap_layout(st.n).eb)
                                  : st.Eb.as<uint16_t>();
    hipLaunchKernelGGL(k_embed, dim3(N), dim3(256), 0, s, genes, rows, st.k, Eb, st.xb.as<uint16_t>());
    MlpArgs a = mlp_args(st, st.xb.as<uint16_t>(), yhat, N, snapshot);
    if (snapshot) {
        a.musd_src = reinterpret_cast<const double *>(static_cast<char *>(st.snap.ptr) + snap_layout(st.n).musd);
        a.musd_dst = st.dstats.as<double>();
    }
    hipLaunchKernelGGL(k_mlp<false>, dim3((N + kMlpRows - 1) / kMlpRows), dim3(64 * kMlpWaves), 0, s, a);
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
int train_step(gapa_ga *ga, const int32_t *genes, const float *target, int32_t B, bool keep, double *loss_out,
               const int32_t *pos, hipStream_t s)
{
    SurrogateState &st = *ga->surr;
    gapa_graph *g = ga->graph;
    st.steps += 1;
    const AdamArgs o = adam_args(st);
    hipLaunchKernelGGL(k_embed, dim3(B), dim3(256), 0, s, genes, nullptr, st.k, st.Eb.as<uint16_t>(),
                       st.xtrain.as<uint16_t>());
    MlpArgs a = mlp_args(st, st.xtrain.as<uint16_t>(), st.ytrain.as<float>(), B);
    a.target = target;
    a.dscale = 2.0f / B;
    a.lossv = st.lossv.as<float>();
    a.dy = st.dy.as<float>();
    a.xT = st.xT.as<uint16_t>();
    a.h1T = st.h1T.as<uint16_t>();
    a.h2T = st.h2T.as<uint16_t>();
    a.dz1T = st.dz1T.as<uint16_t>();
    a.dz2T = st.dz2T.as<uint16_t>();
    a.dxT = st.dxT.as<uint16_t>();
    hipLaunchKernelGGL(k_mlp<true>, dim3(B / kMlpRows), dim3(64 * kMlpWaves), 0, s, a);
    const int64_t nE = (int64_t)st.n * kD;
    WgradArgs w{};
    w.xT = a.xT;
    w.h1T = a.h1T;
    w.h2T = a.h2T;
    w.dz1T = a.dz1T;
    w.dz2T = a.dz2T;
    w.dy = a.dy;
    w.lossv = a.lossv;
    w.B = B;
    w.theta = mlp_theta(st);
    w.m = st.m.as<float>() + nE;
    w.v = st.v.as<float>() + nE;
    w.keep = keep ? st.keep_mlp.as<float>() : nullptr;
    w.cp = copies(st);
    w.o = o;
    w.loss_out = loss_out;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(kWgradTasks), dim3(64), 0, s, w);
    // membership bits of the batch, node-major: straight from the rows and
    // their chunk start positions (batches sampled from the buffer), or else
    // the removed-node bit sets of the rows, transposed
    const int32_t Wb = B / 32;
    int rc = GAPA_OK;
    if (pos) {
        const int32_t nchunks = (st.n + kBitChunk - 1) / kBitChunk;
        hipLaunchKernelGGL(k_batch_bits, dim3(nchunks), dim3(256), (size_t)kBitChunk * Wb * 4, s, genes, st.k, B, pos,
                           nchunks, st.n, st.brows.as<uint32_t>());
    } else {
        rc = launch_mask_build(genes, B, st.k, g->n, g->words, g->d_noniso, g->n_noniso, st.bmasks.as<uint32_t>(),
                               st.balive.as<int32_t>(), st.tflag.as<int32_t>(), s);
        if (rc != GAPA_OK) return rc;
        if ((rc = launch_bits_transpose(st.bmasks.as<uint32_t>(), B, g->words, g->n, st.brows.as<uint32_t>(), s)) !=
            GAPA_OK)
            return rc;
    }
    const int64_t tiles = ((int64_t)st.n + 15) / 16;
    // one 16-wave block per compute unit shares one staged copy of dx
    const unsigned eblocks = (unsigned)std::min<int64_t>((tiles + 15) / 16, 256);
    hipLaunchKernelGGL(k_grad_adam_E, dim3(eblocks), dim3(1024), grad_E_lds(B), s, st.brows.as<uint32_t>(), Wb,
                       st.dxT.as<uint16_t>(), B, st.theta.as<float>(), st.m.as<float>(), st.v.as<float>(),
                       st.Eb.as<uint16_t>(), keep ? st.keep_E.as<float>() : nullptr, (int64_t)st.n, o);
    GAPA_HIP(hipGetLastError());
    st.have_keep = keep;
    return GAPA_OK;
}

// The fallback decision for generation gen, from the judge of generation
// gen - 2 (final by now in all but the first generations, as gen - 1 is
// queued behind it): after fallback_gens consecutive judged screened
// generations with a correlation below min_rho, generation gen evaluates
// every child.  Generation gen - 1 was launched before that decision and is
// not counted when its figures arrive.
int decide_fallback(gapa_ga *ga, int64_t gen, bool *force)
{
    SurrogateState &st = *ga->surr;
    *force = false;
    SurrogateState::Slot &sl = st.slot[gen & 1];
    if (sl.gen != gen - 2 || sl.judged) return GAPA_OK;
    GAPA_HIP(hipEventSynchronize(st.ready[gen & 1]));
    sl.judged = true;
    if (!sl.predicted || !sl.screened || sl.gen < st.skip_before) return GAPA_OK;  // full generations do not count
    const double rho = st.hstats[8 * (gen & 1) + 2];
    st.low_run = rho < st.sp.min_rho ? st.low_run + 1 : 0;
    if (st.sp.fallback_gens > 0 && st.low_run >= st.sp.fallback_gens) {
        *force = true;
        st.low_run = 0;
        st.skip_before = gen;
    }
    return GAPA_OK;
}

}  // namespace

int surrogate_attach(gapa_ga *ga, const gapa_surrogate_params *sp, hipStream_t s)
{
    if (ga->count != 1 || ga->surr || ga->generation != 0 || ga->objective_mcn || ga->objective_forest) {
        set_error("a surrogate attaches to a single-instance GA minimising PC at generation 0, once");
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
    int rc = GAPA_OK;
    auto res = [&](DevBuf &b, size_t bytes) {
        if (rc == GAPA_OK) rc = b.reserve(bytes);
    };
    res(st->theta, P * 4);
    res(st->m, P * 4);
    res(st->v, P * 4);
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
    res(st->snap, snap_layout(st->n).bytes);
    res(st->xtrain, (size_t)B * kD * 2);
    res(st->ytrain, (size_t)B * 4);
    res(st->dy, (size_t)B * 4);
    res(st->xT, (size_t)B * kD * 2);
    res(st->h1T, (size_t)B * kH * 2);
    res(st->h2T, (size_t)B * kH * 2);
    res(st->dz1T, (size_t)B * kH * 2);
    res(st->dz2T, (size_t)B * kH * 2);
    res(st->dxT, (size_t)B * kD * 2);
    // one batch per training step of a generation: all are sampled before
    // the first step runs
    const size_t nbatch = (size_t)std::max(sp->train_steps, 1);
    res(st->target, nbatch * B * 4);
    res(st->lossv, (size_t)B * 4);
    res(st->bgenes, nbatch * B * st->k * 4);
    res(st->bpos, nbatch * B * ((size_t)(st->n + kBitChunk - 1) / kBitChunk + 1) * 4);

    res(st->bmasks, (size_t)B * st->W * 4);
    res(st->balive, (size_t)B * 4);
    res(st->bflag, 16);
    res(st->tflag, 16);
    res(st->brows, (size_t)st->n * (B / 32) * 4);
    res(st->buf_genes, (size_t)sp->buffer * st->k * 4);
    res(st->buf_y, (size_t)sp->buffer * 8);
    res(st->pool, (size_t)L * 4);
    res(st->crows, (size_t)(sp->screen + kJudgeExtra) * st->k * 4);
    res(st->cmasks, (size_t)(sp->screen + kJudgeExtra) * st->W * 4);
    res(st->calive, (size_t)(sp->screen + kJudgeExtra) * 4);
    res(st->dstats, 64);
    res(st->jpart, (size_t)8 * 4 * (kJudgeMax / kJudgeKeys));
    res(st->dloss, 5 * 8);
    res(st->tstats, 16);
    if (rc != GAPA_OK) return rc;
    GAPA_HIP(hipHostMalloc(reinterpret_cast<void **>(&st->hstats), 128, hipHostMallocMapped | hipHostMallocCoherent));
    std::memset(st->hstats, 0, 128);
    GAPA_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&st->hstats_dev), st->hstats, 0));
    GAPA_HIP(hipEventCreateWithFlags(&st->ready[0], hipEventDisableTiming));
    GAPA_HIP(hipEventCreateWithFlags(&st->ready[1], hipEventDisableTiming));
    GAPA_HIP(hipEventCreateWithFlags(&st->ev_pred, hipEventDisableTiming));

    GAPA_HIP(hipEventCreateWithFlags(&st->ev_snap, hipEventDisableTiming));
    GAPA_HIP(hipEventCreateWithFlags(&st->ev_data, hipEventDisableTiming));
    GAPA_HIP(hipEventCreateWithFlags(&st->ev_sampled, hipEventDisableTiming));
    GAPA_HIP(hipStreamCreateWithFlags(&st->ts, hipStreamNonBlocking));
    GAPA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_grad_adam_E), hipFuncAttributeMaxDynamicSharedMemorySize,
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
    if ((rc = launch_fill_u32(st->tflag.ptr, 0u, 4, s)) != GAPA_OK) return rc;
    if ((rc = launch_fill_u32(st->dloss.ptr, 0u, 10, s)) != GAPA_OK) return rc;
    {
        static const double musd0[2] = {0.0, 1.0};  // before any training: unstandardised
        GAPA_HIP(hipMemcpyAsync(st->tstats.ptr, musd0, 16, hipMemcpyHostToDevice, s));
        GAPA_HIP(hipStreamSynchronize(s));
    }
    // the snapshot starts as the initial weights; training waits for set-up
    if ((rc = take_snapshot(*st, s)) != GAPA_OK) return rc;
    GAPA_HIP(hipEventRecord(st->ev_data, s));
    GAPA_HIP(hipStreamWaitEvent(st->ts, st->ev_data, 0));
    GAPA_HIP(hipEventRecord(st->ev_sampled, st->ts));
    return GAPA_OK;
}

void surrogate_release(SurrogateState *st)
{
    if (!st) return;
    if (st->ts) (void)hipStreamSynchronize(st->ts);  // training still queued reads the buffers below
    for (DevBuf *b : {&st->theta, &st->m, &st->v, &st->keep_mlp, &st->keep_E, &st->Eb, &st->W1b, &st->W2b, &st->w3b,
                      &st->W1bT, &st->W2bT, &st->xb, &st->yhat, &st->snap, &st->xtrain, &st->ytrain,
                      &st->target, &st->lossv, &st->dy, &st->tflag, &st->dloss, &st->tstats,
                      &st->xT, &st->h1T, &st->h2T, &st->dz1T, &st->dz2T, &st->dxT, &st->bgenes, &st->bmasks,
                      &st->balive, &st->bflag, &st->brows, &st->buf_genes, &st->buf_y, &st->pool, &st->crows,
                      &st->cmasks, &st->calive, &st->dstats, &st->jpart, &st->bpos})
        b->release();
    if (st->hstats) (void)hipHostFree(st->hstats);
    for (hipEvent_t e : {st->ready[0], st->ready[1], st->ev_pred, st->ev_snap, st->ev_data, st->ev_sampled})
        if (e) (void)hipEventDestroy(e);
    if (st->ts) (void)hipStreamDestroy(st->ts);
    delete st;
}

int surrogate_generation(gapa_ga *ga, hipStream_t s)
{
    SurrogateState &st = *ga->surr;
    st.explicit_loss = false;
    const uint32_t gen = (uint32_t)(ga->generation + 1);
    bool force = false;
    int rc = decide_fallback(ga, gen, &force);
    if (rc != GAPA_OK) return rc;
    const bool random = st.sp.flags & GAPA_SCREEN_RANDOM;
    const bool full = (int64_t)gen <= st.sp.warmup_gens || force;
    if (force && (int64_t)gen > st.sp.warmup_gens) st.fallbacks += 1;
    const int32_t si = (int32_t)(gen & 1u);
    double *hs = st.hstats_dev + 8 * si;
    const int32_t L = st.lambda;
    // a screened generation builds bit sets only for the children it evaluates
    if ((rc = ga_launch_offspring(ga, s, !full)) != GAPA_OK) return rc;
    const bool predict = !random && (int64_t)gen > st.sp.warmup_gens;
    float *yhat = st.yhat.as<float>();
    if (!random) {
        // the snapshot holds the weights trained through generation gen - 2
        GAPA_HIP(hipStreamWaitEvent(s, st.ev_snap, 0));
        if (predict) {
            // (the prediction kernel also copies their label standardisation for the judge)
            if ((rc = predict_rows(st, ga->children.as<int32_t>(), nullptr, L, yhat, s, true)) != GAPA_OK) return rc;
        }
        // once they are made, it takes the weights trained through gen - 1
        GAPA_HIP(hipEventRecord(st.ev_pred, s));
        GAPA_HIP(hipStreamWaitEvent(st.ts, st.ev_pred, 0));
        if ((rc = take_snapshot(st, st.ts)) != GAPA_OK) return rc;
        GAPA_HIP(hipEventRecord(st.ev_snap, st.ts));
    }
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
        hipLaunchKernelGGL(k_screen, dim3(1), dim3(1024), 0, s, random ? nullptr : yhat, L, npool, extra,
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
    if (predict && (rc = launch_judge(yhat, pool, F, neval, ds, st.jpart.as<double>(), hs + 2, hs + 5, s)) != GAPA_OK)
        return rc;
    if (!random) {
        // generation gen - 1's training has copied its batches out of the
        // buffer (it goes on beside this generation); the loss reported is
        // that of generation gen - 2's training, finished before this
        // generation's predictions (the wait on the snapshot above)
        GAPA_HIP(hipStreamWaitEvent(s, st.ev_sampled, 0));
        double *dloss = st.dloss.as<double>();
        hipLaunchKernelGGL(k_append, dim3(neval), dim3(256), 0, s, ga->children.as<int32_t>(), st.k, pool, F,
                           st.appended, st.sp.buffer, st.buf_genes.as<int32_t>(), st.buf_y.as<double>(),
                           dloss + 1 + ((gen + 2u) & 3u), hs + 4);
        st.appended += neval;
        const int32_t count = (int32_t)std::min<int64_t>(st.appended, st.sp.buffer);
        GAPA_HIP(hipGetLastError());
        // this generation's training, on the training stream: label statistics,
        // every step's batch, then the steps
        GAPA_HIP(hipEventRecord(st.ev_data, s));
        GAPA_HIP(hipStreamWaitEvent(st.ts, st.ev_data, 0));
        hipLaunchKernelGGL(k_label_stats, dim3(1), dim3(1024), 0, st.ts, st.buf_y.as<double>(), count,
                           st.tstats.as<double>());
        const int32_t B = st.sp.batch;
        const int32_t nchunks = (st.n + kBitChunk - 1) / kBitChunk;
        const int64_t pstride = (int64_t)B * (nchunks + 1);
        for (int32_t t = 0; t < st.sp.train_steps; ++t)
            hipLaunchKernelGGL(k_sample, dim3(B), dim3(256), 0, st.ts, st.seed, gen, (uint32_t)t, count,
                               st.buf_genes.as<int32_t>(), st.buf_y.as<double>(), st.tstats.as<double>(), st.k,
                               st.bgenes.as<int32_t>() + (int64_t)t * B * st.k, st.target.as<float>() + (int64_t)t * B,
                               nchunks, st.bpos.as<int32_t>() + t * pstride);
        GAPA_HIP(hipEventRecord(st.ev_sampled, st.ts));
        for (int32_t t = 0; t < st.sp.train_steps; ++t)
            if ((rc = train_step(ga, st.bgenes.as<int32_t>() + (int64_t)t * B * st.k,
                                 st.target.as<float>() + (int64_t)t * B, B, false, dloss + 1 + (gen & 3u),
                                 st.bpos.as<int32_t>() + t * pstride, st.ts)) != GAPA_OK)
                return rc;
    }
    if (full) {
        // the pool of a full generation is every child
        hipLaunchKernelGGL(k_iota, dim3((L + 255) / 256), dim3(256), 0, s, st.pool.as<int32_t>(), L);
    }
    GAPA_HIP(hipGetLastError());
    GAPA_HIP(hipEventRecord(st.ready[si], s));
    st.last_gen = gen;
    SurrogateState::Slot &sl = st.slot[si];
    sl.gen = gen;
    sl.evaluated = neval;
    sl.pooled = npool;
    sl.screened = !full;
    sl.predicted = predict;
    sl.judged = false;
    ga->generation += 1;
    return GAPA_OK;
}

int surrogate_predict(gapa_ga *ga, const int32_t *genes, int32_t P, float *yhat, hipStream_t s)
{
    SurrogateState &st = *ga->surr;
    GAPA_HIP(hipStreamSynchronize(st.ts));  // the live weights, after all enqueued training
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
    GAPA_HIP(hipStreamSynchronize(st.ts));
    const int rc = train_step(ga, genes, target, B, keep_grads, st.dloss.as<double>(), nullptr, s);
    if (rc == GAPA_OK) st.explicit_loss = true;
    return rc;
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
    const int32_t si = (int32_t)(st.last_gen & 1);
    const SurrogateState::Slot &sl = st.slot[si];
    const double *hs = st.hstats + 8 * si;
    if (st.last_gen > 0) GAPA_HIP(hipEventSynchronize(st.ready[si]));
    const bool predicted = st.last_gen > 0 && sl.predicted;
    out->generation = st.last_gen;
    out->evaluated = st.last_gen > 0 ? sl.evaluated : 0;
    out->pooled = st.last_gen > 0 ? sl.pooled : 0;
    out->screened = st.last_gen > 0 && sl.screened ? 1 : 0;
    out->spearman = predicted ? hs[2] : 0.0;
    out->rel_err = predicted ? hs[3] : 0.0;
    out->loss = hs[4];
    if (st.explicit_loss) {
        GAPA_HIP(hipDeviceSynchronize());
        GAPA_HIP(hipMemcpy(&out->loss, st.dloss.ptr, 8, hipMemcpyDeviceToHost));
    }
    out->fallbacks = st.fallbacks;
    out->train_steps = (int32_t)st.steps;
    out->label_mean = predicted ? hs[5] : 0.0;
    out->label_spread = predicted ? hs[6] : 0.0;
    return GAPA_OK;
}

int surrogate_judge(const float *yhat, const int32_t *pool, const int64_t *F, int32_t m, double mu, double sd,
                    double *out, hipStream_t s)
{
    DevBuf buf;  // [0, 2) mean and spread in, [2, 4) the statistics out, [4, 4 + 4 * 16) partial sums
    int rc = buf.reserve(8 * (4 + 4 * (kJudgeMax / kJudgeKeys)));
    if (rc != GAPA_OK) return rc;
    const double musd[2] = {mu, sd};
    double res[2] = {0.0, 0.0};
    hipError_t e = hipMemcpyAsync(buf.ptr, musd, 16, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        rc = launch_judge(yhat, pool, F, m, buf.as<double>(), buf.as<double>() + 4, buf.as<double>() + 2, nullptr, s);
        if (rc != GAPA_OK) {
            (void)hipStreamSynchronize(s);
            buf.release();
            return rc;
        }
    }
    if (e == hipSuccess) e = hipMemcpyAsync(res, buf.as<double>() + 2, 16, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    buf.release();
    if (e != hipSuccess) return hip_fail(e, "surrogate judge");
    out[0] = res[0];
    out[1] = res[1];
    return GAPA_OK;
}

int surrogate_last_predictions(gapa_ga *ga, float *yhat, int32_t cap, int32_t *count)
{
    SurrogateState &st = *ga->surr;
    const int32_t c = st.last_gen > 0 && st.slot[st.last_gen & 1].predicted ? st.lambda : 0;
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
    const int32_t c = st.last_gen > 0 ? st.slot[st.last_gen & 1].evaluated : 0;
    if (count) *count = c;
    if (pool && c > 0) {
        GAPA_HIP(hipStreamSynchronize(ga->last_stream));
        GAPA_HIP(hipMemcpy(pool, st.pool.ptr, (size_t)std::min(c, cap) * 4, hipMemcpyDeviceToHost));
    }
    return GAPA_OK;
}

}  // namespace gapa
