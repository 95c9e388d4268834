// Bit-parallel batched fitness.
//
// A chunk of B individuals (B = 32 * Wd, Wd a power of two <= 32) is
// evaluated together.  For every node v the chunk keeps two rows of Wd 32-bit
// words, node-major so that one row is one contiguous 4*Wd-byte segment:
//   dead[v]  bit i set: v is removed in individual i (the perturbation P^ of
//            eq. 13 applied to the whole chunk at once),
//   reach[v] bit i set: v is known to lie in the component of individual i's
//            root r_i.
// Each individual's root is its highest-degree surviving node.  The root
// components grow by pull sweeps: a node ORs its neighbours' reach rows and
// keeps the bits of individuals in which it survives.  One sweep visits the
// nodes band by band in the breadth-first order of G from its highest-degree
// nodes, so most of G settles in that one sweep; a few sweeps over the nodes
// still pending follow.
//
// Whatever the sweeps leave pending is finished exactly: for every
// (individual, pending node) pair a union-find over the surviving edges
// between pending nodes, with the reached set R_i contracted into r_i (it is
// connected and contains r_i, so an edge into R_i is an edge into r_i).
// Every component other than the root's is then made only of pending nodes
// and is counted directly; the root's component is what remains of the
// surviving non-isolated nodes.  PC = sum |C|(|C|-1)/2 and MCN follow.
// Isolated nodes of G are singletons in every G - S and never enter.
#include <algorithm>
#include <climits>

#include "device_common.h"
#include "internal.h"

namespace gapa {
namespace {

constexpr int kBlk = 256;
constexpr int kSweepGrid = 1024;  // blocks of the grid-stride worklist kernels
constexpr int kSweeps = 6;        // follow-up sweeps over the pending nodes

__device__ __forceinline__ int32_t ld_relaxed(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t ld_relaxed_u(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lanes of a wave are split into groups of Wd consecutive lanes; a group
// handles one node.  Returns the mask of the calling lane's group inside the
// 64-bit ballot.
__device__ __forceinline__ uint64_t group_mask(int Wd)
{
    const int lane = threadIdx.x & 63;
    const uint64_t ones = Wd == 64 ? ~0ull : ((1ull << Wd) - 1ull);
    return ones << (lane & ~(Wd - 1));
}

// dead rows of a chunk start as "padding removes everything": bits of
// individuals past B_real set, the rest clear.
__global__ void k_dead_init(uint32_t *__restrict__ dead, int64_t words, int32_t Wd, int32_t B_real)
{
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < words; x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t w = (int32_t)(x & (Wd - 1));
        const int32_t first = w * 32;
        uint32_t pad = 0;
        if (B_real <= first) pad = 0xFFFFFFFFu;
        else if (B_real < first + 32) pad = ~((1u << (B_real - first)) - 1u);
        dead[x] = pad;
    }
}

// One block per individual i: sets i's bit in the dead row of each of its
// genes (eq. 13's batched perturbation), and counts its distinct removed
// non-isolated nodes: alive_noniso[i] = n_noniso - that count.  Genes outside
// [0, n) raise flag[0] and are skipped.  kDistinct: the caller guarantees
// distinct ids per row (the GA's rows), so each gene counts once.
template <bool kDistinct>
__global__ __launch_bounds__(kBlk) void k_dead_scatter(const int32_t *__restrict__ genes, int32_t k, int32_t n,
                                                       int32_t Wd, const int32_t *__restrict__ row_ptr,
                                                       int32_t n_noniso, uint32_t *__restrict__ dead,
                                                       int32_t *__restrict__ alive_noniso, int32_t *__restrict__ flag)
{
    __shared__ int32_t part[kBlk / 64];
    const int32_t i = blockIdx.x;
    const int32_t w = i >> 5;
    const uint32_t bit = 1u << (i & 31);
    const int32_t *row = genes + (int64_t)i * k;
    int32_t cnt = 0;
    for (int32_t j = threadIdx.x; j < k; j += blockDim.x) {
        const int32_t v = row[j];
        if (v < 0 || v >= n) {
            atomicOr(flag, 1);
            continue;
        }
        if (kDistinct) {
            // rows known to hold distinct ids: no need for the old value
            atomicOr(dead + (int64_t)v * Wd + w, bit);
            if (row_ptr[v + 1] > row_ptr[v]) ++cnt;
        } else {
            const uint32_t old = atomicOr(dead + (int64_t)v * Wd + w, bit);
            if (!(old & bit) && row_ptr[v + 1] > row_ptr[v]) ++cnt;
        }
    }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t s = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += part[q];
        alive_noniso[i] = n_noniso - s;
    }
}

// Root of each individual: the first surviving node in (degree desc, id)
// order; its reach bit is set.  No survivor: root = -1.
__global__ void k_seed(const uint32_t *__restrict__ dead, const int32_t *__restrict__ order, int32_t n, int32_t Wd,
                       int32_t B_real, int32_t *__restrict__ root, uint32_t *__restrict__ reach)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B_real) return;
    const int32_t w = i >> 5;
    const uint32_t bit = 1u << (i & 31);
    int32_t r = -1;
    for (int32_t p = 0; p < n; ++p) {
        const int32_t v = order[p];
        if (!(dead[(int64_t)v * Wd + w] & bit)) {
            r = v;
            break;
        }
    }
    root[i] = r;
    if (r >= 0) atomicOr(reach + (int64_t)r * Wd + w, bit);
}

// Pull for one node by its lane group: OR the neighbours' reach rows (in
// degree-descending order) until every pending bit is covered.  Returns true
// if the node gained bits.
__device__ __forceinline__ bool pull_node(int32_t v, int Wd, int w, uint64_t gmask,
                                          const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ colD,
                                          const uint32_t *__restrict__ dead, uint32_t *__restrict__ reach)
{
    const uint32_t mine = ld_relaxed_u(reach + (int64_t)v * Wd + w);
    const uint32_t pend = ~dead[(int64_t)v * Wd + w] & ~mine;
    if ((__ballot(pend != 0) & gmask) == 0) return false;
    uint32_t acc = 0;
    const int32_t e0 = row_ptr[v], e1 = row_ptr[v + 1];
    for (int32_t e = e0; e < e1; ++e) {
        const int32_t u = colD[e];
        acc |= ld_relaxed_u(reach + (int64_t)u * Wd + w);
        if ((__ballot((acc & pend) != pend) & gmask) == 0) break;
    }
    const uint32_t gain = acc & pend;
    if (gain) __hip_atomic_store(reach + (int64_t)v * Wd + w, mine | gain, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (__ballot(gain != 0) & gmask) != 0;
}

// One band of the ordered sweep: nodes band_v[b0, b1).
__global__ void k_pull_band(const int32_t *__restrict__ band_v, int32_t b0, int32_t b1, int32_t Wd,
                            const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ colD,
                            const uint32_t *__restrict__ dead, uint32_t *__restrict__ reach)
{
    const int lane = threadIdx.x & 63;
    const int w = lane & (Wd - 1);
    const uint64_t gmask = group_mask(Wd);
    const int64_t group = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / Wd;
    const int64_t ngroups = (int64_t)gridDim.x * blockDim.x / Wd;
    // every lane of a wave iterates the same number of times so that ballots
    // see whole groups
    const int32_t count = b1 - b0;
    const int64_t iters = (count + ngroups - 1) / ngroups;
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t idx = group + it * ngroups;
        const bool valid = idx < count;
        const int32_t v = valid ? band_v[b0 + idx] : 0;
        if (__ballot(valid) == 0) continue;
        if (valid) pull_node(v, Wd, w, gmask, row_ptr, colD, dead, reach);
    }
}

// Block-level compaction: every block owns a contiguous range of the input,
// counts its items, reserves room with one global atomic and writes them at
// offsets taken from an LDS counter.  Order inside the output is not fixed,
// and nothing downstream depends on it.
__device__ __forceinline__ int32_t block_reserve(int32_t mine, int32_t *counter, int32_t *s_tot, int32_t *s_base,
                                                 int32_t *s_off)
{
    // returns the block's base slot; *s_off is reset to 0 for the write pass
    if (threadIdx.x == 0) *s_tot = 0;
    __syncthreads();
    int32_t x = mine;
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if ((threadIdx.x & 63) == 0 && x) atomicAdd(s_tot, x);
    __syncthreads();
    if (threadIdx.x == 0) {
        *s_base = *s_tot ? atomicAdd(counter, *s_tot) : 0;
        *s_off = 0;
    }
    __syncthreads();
    return *s_base;
}

constexpr int kCompactRange = 256;  // input items per compaction block

// Nodes still pending after the ordered sweep -> worklist.
__global__ __launch_bounds__(kBlk) void k_collect_pending(const int32_t *__restrict__ band_v, int32_t count,
                                                          int32_t Wd, const uint32_t *__restrict__ dead,
                                                          const uint32_t *__restrict__ reach,
                                                          int32_t *__restrict__ worklist, int32_t *__restrict__ wl_count)
{
    __shared__ int32_t s_tot, s_base, s_off;
    __shared__ int32_t s_list[kCompactRange];
    const int w = threadIdx.x & (Wd - 1);
    const uint64_t gmask = group_mask(Wd);
    const int32_t gpb = blockDim.x / Wd;
    const int32_t r0 = blockIdx.x * kCompactRange, r1 = min(count, r0 + kCompactRange);
    if (threadIdx.x == 0) s_off = 0;
    __syncthreads();
    for (int32_t idx0 = r0; idx0 < r1; idx0 += gpb) {
        const int32_t idx = idx0 + (int32_t)(threadIdx.x / Wd);
        const bool valid = idx < r1;
        const int32_t v = valid ? band_v[idx] : 0;
        const uint32_t pend = valid ? (~dead[(int64_t)v * Wd + w] & ~reach[(int64_t)v * Wd + w]) : 0u;
        const bool any = (__ballot(pend != 0) & gmask) != 0;
        if (valid && any && w == 0) s_list[atomicAdd(&s_off, 1)] = v;
    }
    __syncthreads();
    const int32_t found = s_off;
    const int32_t base = block_reserve(threadIdx.x == 0 ? found : 0, wl_count, &s_tot, &s_base, &s_off);
    for (int32_t q = threadIdx.x; q < found; q += blockDim.x) worklist[base + q] = s_list[q];
}

// Further sweeps over the worklist; sweep s runs only if sweep s - 1 changed
// something (changed[s - 1] != 0; changed[0] is set by the caller).
__global__ void k_pull_worklist(const int32_t *__restrict__ worklist, const int32_t *__restrict__ wl_count,
                                int32_t Wd, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ colD,
                                const uint32_t *__restrict__ dead, uint32_t *__restrict__ reach,
                                int32_t *__restrict__ changed, int32_t s)
{
    if (ld_relaxed(changed + s - 1) == 0) return;
    const int lane = threadIdx.x & 63;
    const int w = lane & (Wd - 1);
    const uint64_t gmask = group_mask(Wd);
    const int64_t group = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / Wd;
    const int64_t ngroups = (int64_t)gridDim.x * blockDim.x / Wd;
    const int32_t count = ld_relaxed(wl_count);
    const int64_t iters = (count + ngroups - 1) / ngroups;
    bool any_gain = false;
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t idx = group + it * ngroups;
        const bool valid = idx < count;
        const int32_t v = valid ? worklist[idx] : 0;
        if (__ballot(valid) == 0) continue;
        if (valid) any_gain |= pull_node(v, Wd, w, gmask, row_ptr, colD, dead, reach);
    }
    if (__ballot(any_gain) != 0 && lane == 0) atomicOr(changed + s, 1);
}

// (individual, node) pairs still pending -> pair list; parent[i][v] = v.
// Padding individuals remove every node, so their bits are never pending.
// Each block owns kCompactRange worklist entries: one pass counts, one global
// atomic reserves, a second pass writes.
__global__ __launch_bounds__(kBlk) void k_collect_pairs(const int32_t *__restrict__ worklist,
                                                        const int32_t *__restrict__ wl_count, int32_t Wd, int32_t n,
                                                        const uint32_t *__restrict__ dead,
                                                        const uint32_t *__restrict__ reach, int64_t *__restrict__ pairs,
                                                        int32_t *__restrict__ pair_count, int32_t *__restrict__ parent)
{
    __shared__ int32_t s_tot, s_base, s_off;
    const int w = threadIdx.x & (Wd - 1);
    const int32_t gpb = blockDim.x / Wd;
    const int32_t count = *wl_count;
    for (int32_t r0 = blockIdx.x * kCompactRange; r0 < count; r0 += gridDim.x * kCompactRange) {
        const int32_t r1 = min(count, r0 + kCompactRange);
        int32_t mine = 0;
        for (int32_t idx = r0 + (int32_t)(threadIdx.x / Wd); idx < r1; idx += gpb) {
            const int32_t v = worklist[idx];
            mine += __popc(~dead[(int64_t)v * Wd + w] & ~reach[(int64_t)v * Wd + w]);
        }
        const int32_t base = block_reserve(mine, pair_count, &s_tot, &s_base, &s_off);
        for (int32_t idx = r0 + (int32_t)(threadIdx.x / Wd); idx < r1; idx += gpb) {
            const int32_t v = worklist[idx];
            uint32_t pend = ~dead[(int64_t)v * Wd + w] & ~reach[(int64_t)v * Wd + w];
            if (!pend) continue;
            int32_t q = base + atomicAdd(&s_off, __popc(pend));
            while (pend) {
                const int t = __ffs(pend) - 1;
                pend &= pend - 1;
                const int64_t key = (int64_t)(w * 32 + t) * n + v;
                pairs[q++] = key;
                parent[key] = v;
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int32_t uf_find(int32_t *parent, int32_t x)
{
    int32_t p = ld_relaxed(parent + x);
    while (p != x) {
        const int32_t gp = ld_relaxed(parent + p);
        if (gp != p) __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = p;
        p = gp;
    }
    return x;
}

__device__ __forceinline__ void uf_unite(int32_t *parent, int32_t a, int32_t b)
{
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    while (a != b) {
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        const int32_t old = atomicCAS(parent + a, a, b);
        if (old == a) return;
        a = uf_find(parent, old);
        b = uf_find(parent, b);
    }
}

__global__ void k_root_init(const int32_t *__restrict__ root, int32_t B_real, int32_t n, int32_t *__restrict__ parent)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B_real && root[i] >= 0) parent[(int64_t)i * n + root[i]] = root[i];
}

// Union over the surviving edges of each pending pair: a surviving neighbour
// that is reached joins the root's set; a pending one (each such edge once,
// from its smaller end) is united with it.
__global__ void k_pairs_hook(const int64_t *__restrict__ pairs, const int32_t *__restrict__ pair_count, int32_t n,
                             int32_t Wd, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                             const uint32_t *__restrict__ dead, const uint32_t *__restrict__ reach,
                             const int32_t *__restrict__ root, int32_t *__restrict__ parent)
{
    const int32_t count = *pair_count;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t key = pairs[q];
        const int32_t i = (int32_t)(key / n);
        const int32_t v = (int32_t)(key - (int64_t)i * n);
        const int32_t w = i >> 5;
        const uint32_t bit = 1u << (i & 31);
        int32_t *pi = parent + (int64_t)i * n;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const int32_t u = col[e];
            if (dead[(int64_t)u * Wd + w] & bit) continue;
            if (reach[(int64_t)u * Wd + w] & bit) uf_unite(pi, v, root[i]);
            else if (v < u) uf_unite(pi, v, u);
        }
    }
}

// Pending nodes counted at the representative of their set.
__global__ void k_pairs_count(const int64_t *__restrict__ pairs, const int32_t *__restrict__ pair_count, int32_t n,
                              int32_t *__restrict__ parent, int32_t *__restrict__ ucount)
{
    const int32_t count = *pair_count;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t key = pairs[q];
        const int32_t i = (int32_t)(key / n);
        const int32_t v = (int32_t)(key - (int64_t)i * n);
        const int32_t r = uf_find(parent + (int64_t)i * n, v);
        atomicAdd(ucount + (int64_t)i * n + r, 1);
    }
}

__global__ void k_root_rep(const int32_t *__restrict__ root, int32_t B_real, int32_t n, int32_t *__restrict__ parent,
                           int32_t *__restrict__ rep)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B_real) return;
    rep[i] = root[i] >= 0 ? uf_find(parent + (int64_t)i * n, root[i]) : -1;
}

__device__ __forceinline__ void add_component(int64_t s, unsigned long long *fit, int32_t *mcn)
{
    if (s > 1) atomicAdd(fit, (unsigned long long)s * (unsigned long long)(s - 1) / 2ull);
    if (mcn && s > 0) atomicMax(mcn, (int32_t)s);
}

// Components made only of pending nodes (set representative is a pending node
// other than the root's representative): counted, and their sizes summed into
// other[i].  Their counters are cleared for reuse.
__global__ void k_pairs_reduce(const int64_t *__restrict__ pairs, const int32_t *__restrict__ pair_count, int32_t n,
                               const int32_t *__restrict__ parent, const int32_t *__restrict__ rep,
                               int32_t *__restrict__ ucount, int32_t *__restrict__ other,
                               unsigned long long *__restrict__ fitness, int32_t *__restrict__ mcn)
{
    const int32_t count = *pair_count;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t key = pairs[q];
        const int32_t i = (int32_t)(key / n);
        const int32_t v = (int32_t)(key - (int64_t)i * n);
        if (parent[key] != v || v == rep[i]) continue;
        const int32_t s = ucount[key];
        ucount[key] = 0;
        atomicAdd(other + i, s);
        add_component(s, fitness + i, mcn ? mcn + i : nullptr);
    }
}

// The root's component: every surviving non-isolated node not in another
// component (an isolated root means every non-isolated node is removed and
// the component is the root alone).
__global__ void k_root_final(const int32_t *__restrict__ root, const int32_t *__restrict__ rep,
                             const int32_t *__restrict__ alive_noniso, const int32_t *__restrict__ other,
                             const int32_t *__restrict__ row_ptr, int32_t B_real, int32_t n,
                             int32_t *__restrict__ ucount, unsigned long long *__restrict__ fitness,
                             int32_t *__restrict__ mcn)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B_real || root[i] < 0) return;
    const int32_t r = root[i];
    ucount[(int64_t)i * n + rep[i]] = 0;
    const int64_t s = row_ptr[r + 1] > row_ptr[r] ? (int64_t)alive_noniso[i] - other[i] : 1;
    add_component(s, fitness + i, mcn ? mcn + i : nullptr);
}

}  // namespace

int eval_genes_bits(gapa_graph *g, const int32_t *genes, int32_t P, int32_t k, bool distinct, int64_t *fitness,
                    int32_t *mcn, int32_t *flag, FitnessWorkspace &ws, KernelTimer *timer, hipStream_t s)
{
    if (P <= 0) return GAPA_OK;
    const int32_t n = g->n;
    // chunk width: 32 * Wd individuals, Wd a power of two <= 32
    int32_t Wd = 1;
    while (Wd < 32 && Wd * 32 < P) Wd <<= 1;
    const int32_t B = Wd * 32;
    int rc;
    if ((rc = ws.dead.reserve((size_t)n * Wd * 4)) != GAPA_OK) return rc;
    if ((rc = ws.reach.reserve((size_t)n * Wd * 4)) != GAPA_OK) return rc;
    if ((rc = ws.parent.reserve((size_t)B * n * 4)) != GAPA_OK) return rc;
    if (ws.ucount.bytes < (size_t)B * n * 4) {
        if ((rc = ws.ucount.reserve((size_t)B * n * 4)) != GAPA_OK) return rc;
        if ((rc = launch_fill_u32(ws.ucount.ptr, 0u, (int64_t)B * n, s)) != GAPA_OK) return rc;
    }
    const int64_t max_pairs = (int64_t)B * std::max(g->n_noniso, 1);
    if ((rc = ws.pairs.reserve((size_t)max_pairs * 8)) != GAPA_OK) return rc;
    if ((rc = ws.worklist.reserve((size_t)std::max(g->n_noniso, 1) * 4)) != GAPA_OK) return rc;
    if ((rc = ws.small.reserve((size_t)(4 * B + 64) * 4)) != GAPA_OK) return rc;
    int32_t *root = ws.small.as<int32_t>();
    int32_t *alive = root + B, *other = root + 2 * B, *rep = root + 3 * B;
    int32_t *ctr = root + 4 * B;  // [0] worklist count, [1] pair count, [2..] changed flags
    int32_t *wl_count = ctr, *pair_count = ctr + 1, *changed = ctr + 2;
    ws.stats_ctr = ctr;
    ws.stats_B = B;
    uint32_t *dead = ws.dead.as<uint32_t>(), *reach = ws.reach.as<uint32_t>();
    int32_t *parent = ws.parent.as<int32_t>(), *ucount = ws.ucount.as<int32_t>();
    int64_t *pairs = ws.pairs.as<int64_t>();
    int32_t *worklist = ws.worklist.as<int32_t>();

    if ((rc = launch_fill_u32(fitness, 0u, (int64_t)P * 2, s)) != GAPA_OK) return rc;
    if (mcn && (rc = launch_fill_u32(mcn, 0u, P, s)) != GAPA_OK) return rc;

    const int32_t nb = (int32_t)g->band_off.size() - 1;
    const int32_t noniso = g->n_noniso;
    const int64_t rows = (int64_t)n * Wd;
    const int row_blocks = (int)std::min<int64_t>((rows + kBlk - 1) / kBlk, 8192);
    for (int32_t c0 = 0; c0 < P; c0 += B) {
        const int32_t Br = std::min(B, P - c0);
        unsigned long long *fit = reinterpret_cast<unsigned long long *>(fitness + c0);
        int32_t *mc = mcn ? mcn + c0 : nullptr;
        {
            TimedScope ts(timer, "k_dead_scatter", s);
            if ((rc = launch_fill_u32(reach, 0u, rows, s)) != GAPA_OK) return rc;
            if ((rc = launch_fill_u32(ctr, 0u, 64, s)) != GAPA_OK) return rc;
            if ((rc = launch_fill_u32(other, 0u, B, s)) != GAPA_OK) return rc;
            if ((rc = launch_fill_u32(changed, 1u, 1, s)) != GAPA_OK) return rc;
            hipLaunchKernelGGL(k_dead_init, dim3(row_blocks), dim3(kBlk), 0, s, dead, rows, Wd, Br);
            if (distinct)
                hipLaunchKernelGGL(k_dead_scatter<true>, dim3(Br), dim3(kBlk), 0, s, genes + (int64_t)c0 * k, k, n, Wd,
                                   g->d_row_ptr, noniso, dead, alive, flag);
            else
                hipLaunchKernelGGL(k_dead_scatter<false>, dim3(Br), dim3(kBlk), 0, s, genes + (int64_t)c0 * k, k, n,
                                   Wd, g->d_row_ptr, noniso, dead, alive, flag);
        }
        {
            TimedScope ts(timer, "k_seed", s);
            hipLaunchKernelGGL(k_seed, dim3((Br + 63) / 64), dim3(64), 0, s, dead, g->d_order, n, Wd, Br, root, reach);
        }
        {
            TimedScope ts(timer, "k_pull_band", s);
            for (int32_t b = 0; b < nb; ++b) {
                const int32_t b0 = g->band_off[b], b1 = g->band_off[b + 1];
                if (b1 <= b0) continue;
                const int64_t threads = (int64_t)(b1 - b0) * Wd;
                const int blocks = (int)std::min<int64_t>((threads + kBlk - 1) / kBlk, 8192);
                hipLaunchKernelGGL(k_pull_band, dim3(blocks), dim3(kBlk), 0, s, g->d_band_v, b0, b1, Wd,
                                   g->d_row_ptr, g->d_colD, dead, reach);
            }
        }
        if (noniso > 0) {
            TimedScope ts(timer, "k_collect_pending", s);
            hipLaunchKernelGGL(k_collect_pending, dim3((unsigned)((noniso + kCompactRange - 1) / kCompactRange)),
                               dim3(kBlk), 0, s, g->d_band_v, noniso, Wd, dead, reach, worklist, wl_count);
        }
        {
            TimedScope ts(timer, "k_pull_worklist", s);
            for (int32_t sw = 1; sw <= kSweeps; ++sw)
                hipLaunchKernelGGL(k_pull_worklist, dim3(kSweepGrid), dim3(kBlk), 0, s, worklist, wl_count, Wd,
                                   g->d_row_ptr, g->d_colD, dead, reach, changed, sw);
        }
        {
            TimedScope ts(timer, "k_collect_pairs", s);
            hipLaunchKernelGGL(k_collect_pairs, dim3(kSweepGrid), dim3(kBlk), 0, s, worklist, wl_count, Wd, n, dead,
                               reach, pairs, pair_count, parent);
            hipLaunchKernelGGL(k_root_init, dim3((Br + 63) / 64), dim3(64), 0, s, root, Br, n, parent);
        }
        {
            TimedScope ts(timer, "k_pairs_hook", s);
            hipLaunchKernelGGL(k_pairs_hook, dim3(kSweepGrid), dim3(kBlk), 0, s, pairs, pair_count, n, Wd,
                               g->d_row_ptr, g->d_col, dead, reach, root, parent);
        }
        {
            TimedScope ts(timer, "k_pairs_count", s);
            hipLaunchKernelGGL(k_pairs_count, dim3(kSweepGrid), dim3(kBlk), 0, s, pairs, pair_count, n, parent, ucount);
            hipLaunchKernelGGL(k_root_rep, dim3((Br + 63) / 64), dim3(64), 0, s, root, Br, n, parent, rep);
        }
        {
            TimedScope ts(timer, "k_pairs_reduce", s);
            hipLaunchKernelGGL(k_pairs_reduce, dim3(kSweepGrid), dim3(kBlk), 0, s, pairs, pair_count, n, parent, rep,
                               ucount, other, fit, mc);
            hipLaunchKernelGGL(k_root_final, dim3((Br + 63) / 64), dim3(64), 0, s, root, rep, alive, other,
                               g->d_row_ptr, Br, n, ucount, fit, mc);
        }
        GAPA_HIP(hipGetLastError());
    }
    return GAPA_OK;
}

}  // namespace gapa
