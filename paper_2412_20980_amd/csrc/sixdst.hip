// The paper's dense reachability fitness (Sec. III-D, eq. 13-17) on the
// matrix cores.  For each removal set S:
//
//   M1 = A_S + I     A_S: the adjacency with every edge of a removed node
//                    deleted (eq. 13), an n_pad x n_pad 0/1 int8 matrix
//                    (n_pad = n rounded up to 128; padding rows and columns
//                    are zero)
//   M  = Normalizer(M1^hops)   by binary exponentiation, the products
//                    (A+I)(A+I)^2(A+I)^4... of the paper, each normalised
//                    (entries > 0 become 1)
//   pc = (sum M - n) / 2,  mcn = the largest row sum over surviving nodes
//
// With hops at least the diameter of every component this is (PC, MCN)
// exactly; the paper's hops = 6 (eq. 15) truncates.  Every matrix is a
// power of one symmetric matrix, so every product is symmetric and column j
// of the right operand is its row j: both operands of the int8 products
// (v_mfma_i32_16x16x64_i8) are read as rows.  Integer arithmetic throughout:
// the result is exact.
#include <algorithm>

#include "device_common.h"
#include "internal.h"

namespace gapa {
namespace {

constexpr int kTile = 128;   // output tile of a block; matrices are padded to a multiple of it
constexpr int kLd = 80;      // LDS row stride of a 64-byte k-step (16 rows of one read fall in distinct banks)
typedef int i32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bool removed(const uint32_t *mask, int32_t v)
{
    return (mask[v >> 5] >> (v & 31)) & 1u;
}

// Row i of M1 for individual z (block (i, z)).
__global__ __launch_bounds__(256) void k_six_build(const uint32_t *__restrict__ masks, int32_t W,
                                                   const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col, int32_t n, int32_t np,
                                                   uint8_t *__restrict__ M)
{
    const int32_t i = blockIdx.x, z = blockIdx.y;
    uint8_t *row = M + ((int64_t)z * np + i) * np;
    const uint32_t *mask = masks + (int64_t)z * W;
    for (int32_t c = threadIdx.x; c < np / 16; c += blockDim.x) reinterpret_cast<uint4 *>(row)[c] = uint4{0, 0, 0, 0};
    __syncthreads();
    if (i >= n) return;
    if (threadIdx.x == 0) row[i] = 1;
    if (removed(mask, i)) return;
    for (int32_t e = row_ptr[i] + threadIdx.x; e < row_ptr[i + 1]; e += blockDim.x) {
        const int32_t j = col[e];
        if (!removed(mask, j)) row[j] = 1;
    }
}

// C = Normalizer(A B) for individual blockIdx.y, A and B symmetric powers of
// one matrix, so C is symmetric: block t computes the 128 x 128 tile
// (bi, bj), bi <= bj, the t-th of the upper triangle, and writes it and its
// mirror image.  The four waves take 64 x 64 quadrants (4 x 4 MFMA tiles
// each).  Per k-step of 64 bytes the 128 A rows and the 128 B rows (B
// columns) of the step are staged in LDS (80-byte pitch: the 16 rows one
// operand read touches fall in distinct banks), double-buffered: the next
// step's global loads are in flight during the products.  MFMA operands:
// lane l holds bytes 16 (l / 16) .. + 15 of the step for row / column
// l % 16 (the same byte order on both sides); C[4 (l / 16) + r][l % 16].
constexpr int kStage = kTile * kLd;    // one operand tile of one k-step
constexpr int kOutPitch = kTile + 16;  // output tile pitch in LDS
__global__ __launch_bounds__(256) void k_six_gemm(const uint8_t *__restrict__ A, const uint8_t *__restrict__ B,
                                                  uint8_t *__restrict__ C, int32_t np)
{
    __shared__ __align__(16) uint8_t smem[4 * kStage];  // [buffer][A, B][128][kLd]
    const int64_t base = (int64_t)blockIdx.y * np * np;
    // t = bj (bj + 1) / 2 + bi
    const int32_t t_lin = blockIdx.x;
    int32_t bj = (int32_t)((sqrtf(8.f * (float)t_lin + 1.f) - 1.f) * 0.5f);
    while ((bj + 1) * (bj + 2) / 2 <= t_lin) ++bj;
    while (bj * (bj + 1) / 2 > t_lin) --bj;
    const int32_t bi = t_lin - bj * (bj + 1) / 2;
    const int32_t i0 = bi * kTile, j0 = bj * kTile;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, lr = lane & 15, lg = lane >> 4;
    const int wr = wv >> 1, wc = wv & 1;
    // loader: thread t moves bytes 16 (t % 4) .. + 15 of rows t / 4 and 64 + t / 4 of both tiles
    const int lrow = t >> 2, lcol = (t & 3) * 16;
    const uint8_t *ga = A + base + (int64_t)(i0 + lrow) * np + lcol;
    const uint8_t *gb = B + base + (int64_t)(j0 + lrow) * np + lcol;
    const int64_t half = (int64_t)64 * np;
    uint4 ra0 = *reinterpret_cast<const uint4 *>(ga), ra1 = *reinterpret_cast<const uint4 *>(ga + half);
    uint4 rb0 = *reinterpret_cast<const uint4 *>(gb), rb1 = *reinterpret_cast<const uint4 *>(gb + half);
    i32x4 acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = i32x4{0, 0, 0, 0};
    const int32_t steps = np / 64;
    for (int32_t s = 0; s < steps; ++s) {
        uint8_t *sA = smem + (s & 1) * 2 * kStage, *sB = sA + kStage;
        *reinterpret_cast<uint4 *>(&sA[lrow * kLd + lcol]) = ra0;
        *reinterpret_cast<uint4 *>(&sA[(64 + lrow) * kLd + lcol]) = ra1;
        *reinterpret_cast<uint4 *>(&sB[lrow * kLd + lcol]) = rb0;
        *reinterpret_cast<uint4 *>(&sB[(64 + lrow) * kLd + lcol]) = rb1;
        __syncthreads();
        if (s + 1 < steps) {
            const int64_t o = (int64_t)(s + 1) * 64;
            ra0 = *reinterpret_cast<const uint4 *>(ga + o);
            ra1 = *reinterpret_cast<const uint4 *>(ga + half + o);
            rb0 = *reinterpret_cast<const uint4 *>(gb + o);
            rb1 = *reinterpret_cast<const uint4 *>(gb + half + o);
        }
        i32x4 a[4], b[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) a[x] = *reinterpret_cast<const i32x4 *>(&sA[(wr * 64 + 16 * x + lr) * kLd + lg * 16]);
#pragma unroll
        for (int y = 0; y < 4; ++y) b[y] = *reinterpret_cast<const i32x4 *>(&sB[(wc * 64 + 16 * y + lr) * kLd + lg * 16]);
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    // normalised tile through LDS, then written as 16-byte row pieces
    __syncthreads();
    uint8_t *out = smem;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(wr * 64 + 16 * x + 4 * lg + r) * kOutPitch + wc * 64 + 16 * y + lr] = acc[x][y][r] > 0 ? 1 : 0;
    __syncthreads();
    const int orow = t >> 1, ocol = (t & 1) * 64;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        *reinterpret_cast<uint4 *>(C + base + (int64_t)(i0 + orow) * np + j0 + ocol + 16 * q) =
            *reinterpret_cast<const uint4 *>(&out[orow * kOutPitch + ocol + 16 * q]);
    if (bi != bj) {
        // the mirror tile: row orow of it is column orow of this one
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t w[4];
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                w[d] = 0;
#pragma unroll
                for (int e = 0; e < 4; ++e) w[d] |= (uint32_t)out[(ocol + 16 * q + 4 * d + e) * kOutPitch + orow] << (8 * e);
            }
            *reinterpret_cast<uint4 *>(C + base + (int64_t)(j0 + orow) * np + i0 + ocol + 16 * q) =
                uint4{w[0], w[1], w[2], w[3]};
        }
    }
}

// Row sums of M: block (g, z) takes rows 32 g .. 32 g + 31 of individual z,
// one wave per row at a time; the block adds its rows' total and largest
// surviving row into the individual's counters (integer atomics, order-free).
constexpr int kRowsPerBlock = 32;
__global__ __launch_bounds__(256) void k_six_rows(const uint8_t *__restrict__ M, const uint32_t *__restrict__ masks,
                                                  int32_t W, int32_t n, int32_t np,
                                                  unsigned long long *__restrict__ total, int32_t *__restrict__ mcn)
{
    __shared__ uint32_t s_sum[4], s_max[4];
    const int32_t z = blockIdx.y;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t *mask = masks + (int64_t)z * W;
    uint32_t bsum = 0, bmax = 0;
    for (int32_t r = wv; r < kRowsPerBlock; r += 4) {
        const int32_t i = blockIdx.x * kRowsPerBlock + r;
        if (i >= n) break;
        const uint4 *row = reinterpret_cast<const uint4 *>(M + ((int64_t)z * np + i) * np);
        uint32_t sum = 0;
        for (int32_t c = lane; c < np / 16; c += 64) {
            const uint4 q = row[c];
            // entries are 0 or 1: the byte sum of a word is its popcount
            sum += __popc(q.x) + __popc(q.y) + __popc(q.z) + __popc(q.w);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
        bsum += sum;
        if (!removed(mask, i)) bmax = max(bmax, sum);
    }
    if (lane == 0) {
        s_sum[wv] = bsum;
        s_max[wv] = bmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
        const uint32_t m = max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3]));
        if (t) atomicAdd(total + z, (unsigned long long)t);
        if (m) atomicMax(mcn + z, (int32_t)m);
    }
}

__global__ void k_six_final(const unsigned long long *__restrict__ total, int32_t count, int32_t n,
                            int64_t *__restrict__ pc)
{
    const int32_t z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z < count) pc[z] = ((int64_t)total[z] - n) / 2;
}

}  // namespace

size_t sixdst_bytes_per_individual(int32_t n)
{
    const size_t np = ((size_t)n + kTile - 1) / kTile * kTile;
    return 3 * np * np;
}

// pc[P], mcn[P] (device) of the P removal sets given as bit sets masks[P][W]
// (device); mats holds three np x np matrices for each of `chunk`
// individuals, tot `chunk` counters.
int sixdst_eval_masks(gapa_graph *g, const uint32_t *masks, int32_t P, int32_t hops, int32_t chunk, uint8_t *mats,
                      unsigned long long *tot, int64_t *pc, int32_t *mcn, hipStream_t s)
{
    const int32_t n = g->n, W = g->words;
    const int32_t np = (n + kTile - 1) / kTile * kTile;
    const int64_t mat = (int64_t)np * np;
    for (int32_t z0 = 0; z0 < P; z0 += chunk) {
        const int32_t cnt = std::min(chunk, P - z0);
        const uint32_t *mk = masks + (int64_t)z0 * W;
        uint8_t *buf[3] = {mats, mats + (int64_t)cnt * mat, mats + 2 * (int64_t)cnt * mat};
        hipLaunchKernelGGL(k_six_build, dim3(np, cnt), dim3(256), 0, s, mk, W, g->d_row_ptr, g->d_col, n, np, buf[0]);
        // binary exponentiation: b holds M1^(2^j), r the product of the powers taken so far
        int b = 0, r = -1;
        const int32_t nt = np / kTile;
        const dim3 grid(nt * (nt + 1) / 2, cnt);
        for (int32_t h = hops;;) {
            if (h & 1) {
                if (r < 0) {
                    r = b;
                } else {
                    const int f = 3 - r - b;  // the free buffer
                    hipLaunchKernelGGL(k_six_gemm, grid, dim3(256), 0, s, buf[r], buf[b], buf[f], np);
                    r = f;
                }
            }
            h >>= 1;
            if (h == 0) break;
            int f = 0;
            while (f == r || f == b) ++f;
            hipLaunchKernelGGL(k_six_gemm, grid, dim3(256), 0, s, buf[b], buf[b], buf[f], np);
            b = f;
        }
        GAPA_HIP(hipGetLastError());
        int rc = launch_fill_u32(tot, 0u, 2 * (int64_t)cnt, s);
        if (rc == GAPA_OK) rc = launch_fill_u32(reinterpret_cast<uint32_t *>(mcn + z0), 0u, cnt, s);
        if (rc != GAPA_OK) return rc;
        hipLaunchKernelGGL(k_six_rows, dim3((n + kRowsPerBlock - 1) / kRowsPerBlock, cnt), dim3(256), 0, s, buf[r],
                           mk, W, n, np, tot, mcn + z0);
        hipLaunchKernelGGL(k_six_final, dim3((cnt + 255) / 256), dim3(256), 0, s, tot, cnt, n, pc + z0);
        GAPA_HIP(hipGetLastError());
    }
    return GAPA_OK;
}

}  // namespace gapa
