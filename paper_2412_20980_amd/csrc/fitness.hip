// Batched fitness of a population of node-removal sets (Section III-C, eq. 13:
// the perturbations of all individuals applied to one shared graph at once).
//
// Every individual is a bit set over the nodes (bit v set: v removed).  The
// components of G - S are found by lock-free union-find over the surviving
// edges (each undirected edge once, edge-parallel over the COO rows of the
// CSR so that hub rows do not serialise one thread), then compressed; the
// component sizes are counted at their roots and reduced to
// PC = sum |C| (|C| - 1) / 2 (int64) and the largest size MCN.
#include <algorithm>

#include "device_common.h"
#include "internal.h"

namespace gapa {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int32_t load_relaxed(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x.  Parents only ever point to smaller ids, so the walk ends; each
// visited node is re-pointed at its grandparent (path halving).  Concurrent
// hooks can make a re-pointing stale but never wrong: it still names an
// ancestor in the same set.
__device__ __forceinline__ int32_t find_root(int32_t *parent, int32_t x)
{
    int32_t p = load_relaxed(parent + x);
    while (p != x) {
        const int32_t gp = load_relaxed(parent + p);
        if (gp != p) __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = p;
        p = gp;
    }
    return x;
}

// Merge the sets of a and b: the larger root is hooked under the smaller one
// with a compare-and-swap; a failed swap means that root was hooked
// meanwhile, so the walk resumes from its new root.
__device__ __forceinline__ void unite(int32_t *parent, int32_t a, int32_t b)
{
    a = find_root(parent, a);
    b = find_root(parent, b);
    while (a != b) {
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        const int32_t old = atomicCAS(parent + a, a, b);
        if (old == a) return;
        a = find_root(parent, old);
        b = find_root(parent, b);
    }
}

// Removed-node bit set of each row of genes, built in LDS and written out,
// plus the row's count of surviving non-isolated nodes.  One block per row.
__global__ void k_mask_build_lds(const int32_t *__restrict__ genes, int32_t k, int32_t n, int32_t W,
                                 const uint32_t *__restrict__ noniso, int32_t n_noniso, uint32_t *__restrict__ masks,
                                 int32_t *__restrict__ alive, int32_t *__restrict__ flag)
{
    extern __shared__ uint32_t U[];
    __shared__ int32_t part[kBlock / 64];
    const int32_t i = blockIdx.x;
    for (int32_t w = threadIdx.x; w < W; w += blockDim.x) U[w] = 0u;
    __syncthreads();
    // eight genes a thread at a time, their loads in flight together
    const int32_t *row = genes + (int64_t)i * k;
    for (int32_t j0 = threadIdx.x; j0 < k; j0 += 8 * blockDim.x) {
        int32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int32_t j = j0 + u * (int32_t)blockDim.x;
            v[u] = j < k ? row[j] : 0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (j0 + u * (int32_t)blockDim.x >= k) break;
            if (v[u] < 0 || v[u] >= n) atomicOr(flag, 1);
            else atomicOr(U + (v[u] >> 5), 1u << (v[u] & 31));
        }
    }
    __syncthreads();
    // the bit set out and the removed non-isolated nodes counted, eight words
    // a thread at a time
    uint32_t *m = masks + (int64_t)i * W;
    int32_t gone = 0;
    int32_t w = threadIdx.x;
    for (; w + 7 * (int32_t)blockDim.x < W; w += 8 * blockDim.x) {
        uint32_t x[8], y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            x[u] = U[w + u * blockDim.x];
            y[u] = noniso[w + u * blockDim.x];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            m[w + u * blockDim.x] = x[u];
            gone += __popc(x[u] & y[u]);
        }
    }
    for (; w < W; w += blockDim.x) {
        m[w] = U[w];
        gone += __popc(U[w] & noniso[w]);
    }
    for (int off = 32; off > 0; off >>= 1) gone += __shfl_down(gone, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = gone;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += part[q];
        alive[i] = n_noniso - t;
    }
}

// Same with the bit set built in global memory (bit sets too large for LDS).
__global__ void k_mask_build(const int32_t *__restrict__ genes, int32_t k, int32_t n, int32_t W,
                             uint32_t *__restrict__ masks, int32_t *__restrict__ flag)
{
    const int32_t i = blockIdx.x;
    uint32_t *m = masks + (int64_t)i * W;
    for (int32_t w = threadIdx.x; w < W; w += blockDim.x) m[w] = 0u;
    __syncthreads();
    const int32_t *row = genes + (int64_t)i * k;
    for (int32_t j = threadIdx.x; j < k; j += blockDim.x) {
        const int32_t v = row[j];
        if (v < 0 || v >= n) {
            atomicOr(flag, 1);
            continue;
        }
        atomicOr(m + (v >> 5), 1u << (v & 31));
    }
}

__global__ void k_mask_alive(const uint32_t *__restrict__ masks, int32_t W, const uint32_t *__restrict__ noniso,
                             int32_t n_noniso, int32_t *__restrict__ alive)
{
    __shared__ int32_t part[kBlock / 64];
    const int32_t i = blockIdx.x;
    const uint32_t *m = masks + (int64_t)i * W;
    int32_t gone = 0;
    for (int32_t w = threadIdx.x; w < W; w += blockDim.x) gone += __popc(m[w] & noniso[w]);
    for (int off = 32; off > 0; off >>= 1) gone += __shfl_down(gone, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = gone;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += part[q];
        alive[i] = n_noniso - t;
    }
}

// parent[b][v] = v for the B individuals of a chunk.
__global__ void k_cc_init(int32_t *__restrict__ parent, int32_t n)
{
    const int32_t b = blockIdx.y;
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) parent[(int64_t)b * n + v] = v;
}

// One thread per CSR entry (v, u) with v < u, both endpoints surviving.
__global__ void k_cc_hook(const int32_t *__restrict__ src, const int32_t *__restrict__ col, int64_t nnz,
                          const uint32_t *__restrict__ masks, int32_t W, int32_t *__restrict__ parent, int32_t n)
{
    const int32_t b = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int32_t v = src[e];
    const int32_t u = col[e];
    if (u <= v) return;
    const uint32_t *m = masks + (int64_t)b * W;
    if (test_bit(m, v) || test_bit(m, u)) return;
    unite(parent + (int64_t)b * n, v, u);
}

// Counts each surviving node at its root.
__global__ void k_cc_count(int32_t *__restrict__ parent, const uint32_t *__restrict__ masks, int32_t W,
                           int32_t *__restrict__ count, int32_t n)
{
    const int32_t b = blockIdx.y;
    const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    if (test_bit(masks + (int64_t)b * W, v)) return;
    int32_t *pb = parent + (int64_t)b * n;
    const int32_t r = find_root(pb, v);
    atomicAdd(count + (int64_t)b * n + r, 1);
}

// PC (or with `forest` the sum of |C| - 1) and MCN of each individual from its
// root counts; clears the counts for the next chunk.  Grid: (slices, B);
// fitness/mcn zeroed beforehand.
__global__ void k_cc_reduce(int32_t *__restrict__ count, int32_t n, unsigned long long *__restrict__ fitness,
                            int32_t *__restrict__ mcn, int32_t forest)
{
    const int32_t b = blockIdx.y;
    int32_t *cb = count + (int64_t)b * n;
    unsigned long long acc = 0;
    int32_t big = 0;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const int32_t s = cb[v];
        if (s) {
            acc += forest ? (unsigned long long)(s - 1) : (unsigned long long)s * (unsigned long long)(s - 1) / 2ull;
            big = s > big ? s : big;
            cb[v] = 0;
        }
    }
    __shared__ unsigned long long sacc[kBlock / 64];
    __shared__ int32_t sbig[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_down(acc, off, 64);
        const int32_t o = __shfl_down(big, off, 64);
        big = o > big ? o : big;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        sacc[wv] = acc;
        sbig[wv] = big;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x / 64); ++i) {
            acc += sacc[i];
            big = sbig[i] > big ? sbig[i] : big;
        }
        if (acc) atomicAdd(fitness + b, acc);
        if (mcn && big) atomicMax(mcn + b, big);
    }
}

}  // namespace

// Plain fill kernels stand in for hipMemsetAsync so that enqueued sequences
// stay safe to capture into HIP graphs.
__global__ void k_fill_u32(uint32_t *__restrict__ p, uint32_t value, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

int launch_fill_u32(void *p, uint32_t value, int64_t count, hipStream_t s)
{
    if (count <= 0) return GAPA_OK;
    const int64_t blocks = std::min<int64_t>((count + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(kBlock), 0, s, static_cast<uint32_t *>(p), value,
                       count);
    GAPA_HIP(hipGetLastError());
    return GAPA_OK;
}

int launch_mask_build(const int32_t *genes, int32_t P, int32_t k, int32_t n, int32_t W, const uint32_t *noniso,
                      int32_t n_noniso, uint32_t *masks, int32_t *alive, int32_t *flag, hipStream_t s)
{
    if (P <= 0) return GAPA_OK;
    const size_t lds = (size_t)W * 4;
    if (lds <= 64 * 1024) {
        hipLaunchKernelGGL(k_mask_build_lds, dim3(P), dim3(kBlock), lds, s, genes, k, n, W, noniso, n_noniso, masks,
                           alive, flag);
    } else {
        hipLaunchKernelGGL(k_mask_build, dim3(P), dim3(kBlock), 0, s, genes, k, n, W, masks, flag);
        hipLaunchKernelGGL(k_mask_alive, dim3(P), dim3(kBlock), 0, s, masks, W, noniso, n_noniso, alive);
    }
    GAPA_HIP(hipGetLastError());
    return GAPA_OK;
}

int eval_masks(gapa_graph *g, const uint32_t *masks, const int32_t *alive, int32_t P, int64_t *fitness, int32_t *mcn,
               FitnessWorkspace &ws, KernelTimer *timer, hipStream_t s, const InstTable *it, Measure measure)
{
    if (it && it->count > 1) {
        if (g->algorithm != 0) return GAPA_E_INVALID_ARG;
        return eval_masks_bits(g, masks, alive, P, fitness, mcn, ws, timer, s, it, measure);
    }
    if (P <= 0) return GAPA_OK;
    if (g->algorithm == 1) return eval_masks_unionfind(g, masks, P, fitness, mcn, ws, timer, s, measure);
    return eval_masks_bits(g, masks, alive, P, fitness, mcn, ws, timer, s, nullptr, measure);
}

int eval_genes(gapa_graph *g, const int32_t *genes, int32_t P, int32_t k, int64_t *fitness, int32_t *mcn,
               int32_t *flag, FitnessWorkspace &ws, KernelTimer *timer, hipStream_t s, Measure measure)
{
    if (P <= 0) return GAPA_OK;
    int rc;
    if ((rc = ws.masks.reserve((size_t)P * g->words * 4)) != GAPA_OK) return rc;
    if ((rc = ws.alive.reserve((size_t)P * 4)) != GAPA_OK) return rc;
    {
        TimedScope ts(timer, "mask_build", s);
        if ((rc = launch_mask_build(genes, P, k, g->n, g->words, g->d_noniso, g->n_noniso, ws.masks.as<uint32_t>(),
                                    ws.alive.as<int32_t>(), flag, s)) != GAPA_OK)
            return rc;
    }
    return eval_masks(g, ws.masks.as<uint32_t>(), ws.alive.as<int32_t>(), P, fitness, mcn, ws, timer, s, nullptr,
                      measure);
}

int eval_masks_unionfind(gapa_graph *g, const uint32_t *masks, int32_t P, int64_t *fitness, int32_t *mcn,
                         FitnessWorkspace &ws, KernelTimer *timer, hipStream_t s, Measure measure)
{
    if (P <= 0) return GAPA_OK;
    const int32_t n = g->n, W = g->words;
    // chunk so that parents + counts stay within ~512 MiB
    int64_t per = (int64_t)n * 8;
    int32_t B = (int32_t)std::max<int64_t>(1, std::min<int64_t>(P, (512ll << 20) / std::max<int64_t>(per, 1)));
    B = std::min(B, 65535);
    int rc;
    if ((rc = ws.parent.reserve((size_t)B * n * 4)) != GAPA_OK) return rc;
    if (ws.count.bytes < (size_t)B * n * 4) {
        if ((rc = ws.count.reserve((size_t)B * n * 4)) != GAPA_OK) return rc;
        if ((rc = launch_fill_u32(ws.count.ptr, 0u, (int64_t)B * n, s)) != GAPA_OK) return rc;
    }
    if ((rc = launch_fill_u32(fitness, 0u, (int64_t)P * 2, s)) != GAPA_OK) return rc;
    if (mcn && (rc = launch_fill_u32(mcn, 0u, P, s)) != GAPA_OK) return rc;
    int32_t *parent = ws.parent.as<int32_t>();
    int32_t *count = ws.count.as<int32_t>();
    for (int32_t c0 = 0; c0 < P; c0 += B) {
        const int32_t nb = std::min(B, P - c0);
        TimedScope pass(timer, "fitness_pass", s, 1);
        const uint32_t *m = masks + (int64_t)c0 * W;
        const dim3 gv((n + kBlock - 1) / kBlock, nb);
        {
            TimedScope ts(timer, "cc_init", s);
            hipLaunchKernelGGL(k_cc_init, gv, dim3(kBlock), 0, s, parent, n);
        }
        if (g->nnz > 0) {
            TimedScope ts(timer, "cc_hook", s);
            const dim3 ge((unsigned)((g->nnz + kBlock - 1) / kBlock), nb);
            hipLaunchKernelGGL(k_cc_hook, ge, dim3(kBlock), 0, s, g->d_src, g->d_col, g->nnz, m, W, parent, n);
        }
        {
            TimedScope ts(timer, "cc_count", s);
            hipLaunchKernelGGL(k_cc_count, gv, dim3(kBlock), 0, s, parent, m, W, count, n);
        }
        {
            TimedScope ts(timer, "cc_reduce", s);
            const int slices = std::max(1, std::min(64, (n + kBlock * 8 - 1) / (kBlock * 8)));
            hipLaunchKernelGGL(k_cc_reduce, dim3(slices, nb), dim3(kBlock), 0, s, count, n,
                               reinterpret_cast<unsigned long long *>(fitness + c0), mcn ? mcn + c0 : nullptr,
                               (int32_t)measure);
        }
        GAPA_HIP(hipGetLastError());
    }
    return GAPA_OK;
}

}  // namespace gapa
