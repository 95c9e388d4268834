// Bit-parallel batched fitness.
//
// A chunk of B individuals (B = 32 * Wd, Wd a power of two <= 64) is
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
// surviving non-isolated nodes: all of them but the pending nodes outside
// the root's set.  PC = sum |C|(|C|-1)/2 and MCN follow.
// Isolated nodes of G are singletons in every G - S and never enter.
#include <algorithm>
#include <climits>
#include <utility>
#include <vector>

#include "device_common.h"
#include "internal.h"

namespace gapa {
namespace {

constexpr int kBlk = 256;
constexpr int kMaxSlots = 2048;  // individuals of one pass: 64 words a node row

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

}  // namespace

// Instances evaluated in one bit-parallel pass.  Instance b owns the nodes
// [voff(b), voff(b+1)) of the graph (a disjoint union when several graphs are
// batched) and the individual slots [b*bseg, (b+1)*bseg): bit i of a node's
// row belongs to slot b*bseg + i.  live(b) slots are in use; the others are
// padding that removes every node.  Genes and masks of an instance use its
// local node ids (node - voff(b)); the removed-node bit set of its slot i
// starts at word moff(b) + i * W_b of the mask array.  The leftover
// union-find of slot (b, i) works on local ids in the block of n_b entries
// at bseg * voff(b) + i * n_b.  With count == 1 the arrays are unused and the
// one instance is all n1 nodes with live1 slots in use.
struct Insts {
    int32_t count;
    int32_t bseg;              // slots per instance, 32 * Wd
    int32_t n1, live1;         // count == 1
    const int32_t *voff;       // [count + 1]
    const int32_t *live;       // [count]
    const int64_t *moff;       // [count]
    const int32_t *node_inst;  // [n]: instance of each node
    const int32_t *tiles;      // (instance, first node word) of each transpose tile
};

namespace {

__device__ __forceinline__ int32_t i_voff(const Insts &I, int32_t b)
{
    return I.count == 1 ? (b ? I.n1 : 0) : I.voff[b];
}

__device__ __forceinline__ int32_t i_live(const Insts &I, int32_t b)
{
    return I.count == 1 ? I.live1 : I.live[b];
}

__device__ __forceinline__ int32_t inst_of_node(const Insts &I, int32_t v)
{
    return I.count == 1 ? 0 : I.node_inst[v];
}

// Start of the union-find block of slot gi.
__device__ __forceinline__ int64_t uf_block(const Insts &I, int32_t gi)
{
    const int32_t b = gi / I.bseg;
    const int32_t v0 = i_voff(I, b);
    return (int64_t)I.bseg * v0 + (int64_t)(gi - b * I.bseg) * (i_voff(I, b + 1) - v0);
}

// dead rows from per-individual removed-node bit sets masks[B_real][W]: a
// block takes TW node words (32 TW nodes) of every individual of the chunk,
// TW = kTileWords * 32 / Wd so that a tile always holds 1024 kTileWords
// words whatever the chunk width; stages them in LDS (rows of TW words are
// contiguous in global memory), transposes each 32 x 32 bit block with
// lane shuffles, and writes the tile's dead rows, which are one contiguous
// range of the node-major array.  The same range of reach rows is cleared.
// Individuals past B_real are padding and remove every node.
constexpr int kTileWords = kTransposeWords;

// LDS words of the transposer: the input tile [B][TW + 1], then the output
// tile [32 TW][Wd + 1] in the same buffer.
__host__ __device__ constexpr int32_t transpose_lds_words(int32_t log_wd)
{
    return 1024 * kTileWords + ((32 << log_wd) > 32 * ((kTileWords * 32) >> log_wd) ? (32 << log_wd)
                                                                                     : 32 * ((kTileWords * 32) >> log_wd));
}

// 32 x 32 bit-matrix transpose across the 32 lanes of a half-wave: lane r
// holds row r (bit c = entry (r, c)); afterwards lane c holds column c (bit r =
// entry (r, c)).  Five rounds swap the off-diagonal blocks of 16, 8, 4, 2 and 1
// bits between lanes r and r ^ j.
__device__ __forceinline__ uint32_t transpose32(uint32_t x, int l32)
{
    const uint32_t masks[5] = {0x0000FFFFu, 0x00FF00FFu, 0x0F0F0F0Fu, 0x33333333u, 0x55555555u};
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        const int j = 16 >> s;
        const uint32_t m = masks[s];
        const uint32_t y = __shfl_xor(x, j, 64);
        x = (l32 & j) ? (((y >> j) & m) | (x & ~m)) : ((x & m) | ((y & m) << j));
    }
    return x;
}

__global__ __launch_bounds__(kBlk) void k_dead_transpose(const uint32_t *__restrict__ masks, const Insts I,
                                                         int32_t log_wd, uint32_t *__restrict__ dead,
                                                         uint32_t *__restrict__ reach)
{
    extern __shared__ uint32_t tile[];
    const int32_t Wd = 1 << log_wd;
    const int32_t log_tw = 5 - log_wd + (kTileWords == 1 ? 0 : kTileWords == 2 ? 1 : kTileWords == 4 ? 2 : 3);
    const int32_t TW = 1 << log_tw;
    // this tile: instance b, its node words [j0, j0 + TW)
    // tiles side by side read the same 128-byte lines of each mask row
    const int32_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int32_t b = I.count == 1 ? 0 : I.tiles[2 * t];
    const int32_t j0 = I.count == 1 ? t * TW : I.tiles[2 * t + 1];
    const int32_t vb = i_voff(I, b);
    const int32_t nb = i_voff(I, b + 1) - vb;
    const int32_t W = (nb + 31) / 32;
    const int32_t B_real = i_live(I, b);
    const int64_t mstride = W;
    if (I.count > 1) masks += I.moff[b];
    // rows are padded by one word so that column walks spread over the LDS banks
    const int32_t In = TW + 1;
    const int32_t Wo = Wd + 1;
    // all loads of a thread are issued before any LDS store: they are
    // independent, so they are in flight together (B * TW = 1024 kTileWords)
    constexpr int kLoads = 32 * 32 * kTileWords / kBlk;
    uint32_t vals[kLoads];
#pragma unroll
    for (int r = 0; r < kLoads; ++r) {
        const int32_t x = threadIdx.x + r * kBlk;
        const int32_t ind = x >> log_tw, jj = x & (TW - 1);
        vals[r] = (ind < B_real && j0 + jj < W) ? masks[(int64_t)ind * mstride + j0 + jj] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int r = 0; r < kLoads; ++r) {
        const int32_t x = threadIdx.x + r * kBlk;
        tile[(x >> log_tw) * In + (x & (TW - 1))] = vals[r];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    // (node word jj, individual word w) 32 x 32 blocks, one per half-wave
    // pass: TW * Wd = 32 kTileWords of them
    constexpr int kIters = kTileWords * 32 / 8;
    uint32_t res[kIters];
#pragma unroll
    for (int it = 0; it < kIters; ++it) {
        const int32_t cc = (it * nw + wv) * 2 + half;
        const int32_t jj = cc >> log_wd, w = cc & (Wd - 1);
        res[it] = transpose32(tile[(w * 32 + l32) * In + jj], l32);
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kIters; ++it) {
        const int32_t cc = (it * nw + wv) * 2 + half;
        tile[((cc >> log_wd) * 32 + l32) * Wo + (cc & (Wd - 1))] = res[it];
    }
    __syncthreads();
    const int64_t v0 = vb + (int64_t)j0 * 32;
    const int32_t rows = min(32 * TW, nb - j0 * 32);
    for (int32_t x = threadIdx.x; x < (rows << log_wd); x += blockDim.x) {
        dead[v0 * Wd + x] = tile[(x >> log_wd) * Wo + (x & (Wd - 1))];
        if (reach) reach[v0 * Wd + x] = 0u;
    }
}

// Root of each slot: the first surviving node of its instance in (degree
// desc, id) order; its reach bit is set and its union-find entry initialised.
// No survivor (or a padding slot): root = -1.  Also clears the slot's outputs
// and counters and the pass's counters (ctr[2] is the "sweep 0 changed"
// flag, set).  One wave per slot tests 64 candidates of the order at a time
// (the highest-degree nodes are the ones a population removes most).
// With src_band > 0, band 0 holds exactly the sources and is not swept:
// instead the surviving sources next to each root take its bit here.  They
// lead the root's neighbour list, which is by (degree desc, id), so its first
// 64 entries hold them all.  A block's kSeedWaves slots share one word of the
// rows, so their bits for each source are gathered in LDS and each source's
// word gets one atomic OR.  Band 0's pending flags are set for the
// compaction (a source with nothing pending only costs a worklist entry).
constexpr int kSeedWaves = 16;

__global__ __launch_bounds__(64 * kSeedWaves) void k_seed(
    const uint32_t *__restrict__ dead, const int32_t *__restrict__ order, const Insts I, int32_t Wd,
    int32_t *__restrict__ root, uint32_t *__restrict__ reach, int32_t *__restrict__ parent,
    int32_t *__restrict__ other, int32_t *__restrict__ ctr, unsigned long long *__restrict__ fitness,
    int32_t *__restrict__ mcn, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ colD,
    const int8_t *__restrict__ src_idx, uint8_t *__restrict__ pflag, int32_t src_band)
{
    __shared__ uint32_t s_src[64];
    const int lane = threadIdx.x & 63;
    const int32_t S = I.count * I.bseg;
    const int32_t g0 = (int32_t)blockIdx.x * kSeedWaves;
    const int32_t gi = g0 + (int32_t)(threadIdx.x >> 6);
    if (blockIdx.x == 0 && threadIdx.x < 64) ctr[threadIdx.x] = threadIdx.x == 2 ? 1 : 0;
    if (blockIdx.x == 0)
        for (int32_t t = threadIdx.x; t < src_band; t += blockDim.x) pflag[t] = 1;
    if (threadIdx.x < 64) s_src[threadIdx.x] = 0u;
    __syncthreads();
    if (gi < S) {  // uniform over the wave, as is everything below up to the barrier
        const int32_t b = gi / I.bseg, i = gi - b * I.bseg;
        if (i < i_live(I, b)) {
            const int32_t w = i >> 5;
            const uint32_t bit = 1u << (i & 31);
            const int32_t p0 = i_voff(I, b), p1 = i_voff(I, b + 1);
            int32_t r = -1;
            for (int32_t p = p0; p < p1; p += 64) {
                const int32_t v = p + lane < p1 ? order[p + lane] : -1;
                const bool alive = v >= 0 && !(dead[(int64_t)v * Wd + w] & bit);
                const uint64_t hit = __ballot(alive);
                if (hit) {
                    r = __shfl(v, (int)__ffsll((unsigned long long)hit) - 1, 64);
                    break;
                }
            }
            if (src_band > 0 && r >= 0) {
                const int32_t e = row_ptr[r] + lane;
                if (e < row_ptr[r + 1]) {
                    const int32_t u = colD[e];
                    const int32_t t = src_idx[u];
                    if (t >= 0 && !(dead[(int64_t)u * Wd + w] & bit)) atomicOr(&s_src[t], bit);
                }
            }
            if (lane == 0) {
                root[gi] = r;
                other[gi] = 0;
                fitness[gi] = 0ull;
                if (mcn) mcn[gi] = 0;
                if (r >= 0) {
                    atomicOr(reach + (int64_t)r * Wd + w, bit);
                    parent[uf_block(I, gi) + (r - p0)] = r - p0;
                }
            }
        } else if (lane == 0) {
            root[gi] = -1;
            other[gi] = 0;
        }
    }
    if (src_band > 0) {  // uniform over the grid
        __syncthreads();
        // the block's slots lie in one instance and one word (kSeedWaves
        // divides 32, and every instance's slots start at a multiple of 32)
        if (threadIdx.x < 64 && g0 < S && s_src[threadIdx.x]) {
            const int32_t b = g0 / I.bseg, w = (g0 - b * I.bseg) >> 5;
            const int32_t u = order[i_voff(I, b) + (int32_t)threadIdx.x];
            atomicOr(reach + (int64_t)u * Wd + w, s_src[threadIdx.x]);
        }
    }
}

// A node's record for the sweeps: (node, first edge, end of its edges), by
// position in the band order; the worklist holds the records of the nodes
// still pending, so no sweep loads row pointers.
//
// Pull for one node by its lane group: OR the neighbours' reach rows (in
// degree-descending order), four at a time, until every pending bit is
// covered or max_scan neighbours have been read; the node keeps the bits of
// individuals in which it survives.  Whatever stays pending is picked up by
// a later sweep or, in the end, by the union-find pass, so the cap only
// moves work.  A node with nothing pending reads only its own two words.
//
// Reach rows are shared between the XCDs within one kernel: they are read
// and written with agent-scope atomics, which bypass each XCD's own L2, so
// bits another XCD set earlier in the same sweep are seen and spread at once
// (plain loads that hit a stale line in the local L2 leave about 40 % more
// nodes pending at n = 200k and make the pass 20 % slower; plain loads for
// the neighbours in earlier bands only, whose rows are final, were no
// faster).  Loading the next node's record and first neighbour ids while
// the current one pulls was tried too: 10 % slower, most of those loads
// being wasted on nodes with nothing pending.
//
// In the band sweep the group's lanes load the neighbour ids, one id per
// lane (a chunk of WD ids in one coalesced load; several chunks for groups
// narrower than kPullIds lanes), and read them back by shuffle: one load
// round trip per kPullIds or more neighbours instead of one per four.  The
// band kernel is compiled for each group width.  Slower, on the same GPU:
// the first chunk of ids loaded together with the node's own words, the
// next record prefetched, eight neighbours' bits at a time.
constexpr int kPullIds = 8;

// Groups of at least kIdLanes lanes in the worklist sweep and the pending
// split also load a chunk of Wd ids at a time (one per lane) and read them
// back by shuffle; narrower groups load them four at a time (with 8-lane
// groups too: the pass at P = 256, n = 200k took 0.193 ms with chunks of
// eight against 0.176 ms).
constexpr int kIdLanes = 16;

struct PullOut {
    bool gained;   // the node gained bits
    bool pending;  // bits still pending after the pull
};

template <int WD>
__device__ __forceinline__ PullOut pull_node(const int4 r, int w, uint64_t gmask, const int32_t *__restrict__ colD,
                                             const uint32_t *__restrict__ dead, uint32_t *__restrict__ reach,
                                             int32_t max_scan)
{
    constexpr int K = WD >= kPullIds ? 1 : kPullIds / WD;  // id loads per lane per round trip
    constexpr int CH = WD * K;
    const int64_t vo = (int64_t)r.x * WD + w;
    const uint32_t mine = ld_relaxed_u(reach + vo);
    const uint32_t pend = ~dead[vo] & ~mine;
    PullOut out{false, false};
    if ((__ballot(pend != 0) & gmask) == 0) return out;
    uint32_t acc = 0;
    const int32_t e0 = r.y;
    const int32_t e1 = r.z - e0 > max_scan ? e0 + max_scan : r.z;
    const int gb = (threadIdx.x & 63) & ~(WD - 1);
    bool open = true;
    for (int32_t c = e0; open && c < e1; c += CH) {
        // ids c + q WD + w of chunk q in lane w: one coalesced load per chunk
        int32_t ids[K];
#pragma unroll
        for (int q = 0; q < K; ++q) ids[q] = c + q * WD + w < e1 ? colD[c + q * WD + w] : -1;
        // four neighbours' bits at a time, read back by shuffle in the group
        if constexpr (K == 1) {
            const int32_t m = e1 - c < WD ? e1 - c : WD;
#pragma unroll 1
            for (int32_t t = 0; t < m; t += 4) {
                const int32_t u0 = __shfl(ids[0], gb + t, 64), u1 = __shfl(ids[0], gb + t + 1, 64);
                const int32_t u2 = __shfl(ids[0], gb + t + 2, 64), u3 = __shfl(ids[0], gb + t + 3, 64);
                acc |= ld_relaxed_u(reach + (int64_t)u0 * WD + w) |
                       (u1 >= 0 ? ld_relaxed_u(reach + (int64_t)u1 * WD + w) : 0u) |
                       (u2 >= 0 ? ld_relaxed_u(reach + (int64_t)u2 * WD + w) : 0u) |
                       (u3 >= 0 ? ld_relaxed_u(reach + (int64_t)u3 * WD + w) : 0u);
                if ((__ballot((acc & pend) != pend) & gmask) == 0) {
                    open = false;
                    break;
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < CH; t += 4) {
                if (!open || c + t >= e1) break;
                int32_t u[4];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    u[j] = WD == 1 ? ids[t + j] : __shfl(ids[(t + j) / WD], gb + (t + j) % WD, 64);
                uint32_t x = ld_relaxed_u(reach + (int64_t)u[0] * WD + w);
#pragma unroll
                for (int j = 1; j < 4; ++j) x |= u[j] >= 0 ? ld_relaxed_u(reach + (int64_t)u[j] * WD + w) : 0u;
                acc |= x;
                if ((__ballot((acc & pend) != pend) & gmask) == 0) open = false;
            }
        }
    }
    const uint32_t gain = acc & pend;
    if (gain) __hip_atomic_store(reach + vo, mine | gain, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    out.pending = (__ballot((pend & ~gain) != 0) & gmask) != 0;
    out.gained = (__ballot(gain != 0) & gmask) != 0;
    return out;
}

// A sweep over count records (recs[b0 + i]), a group of WD lanes per node.
// Band sweep (pflag given): pflag[b0 + i] records whether node i is still
// pending; a node's reach row is written only by its own pull, so its
// pending bits are final once it has pulled (every non-isolated node has one
// band position, so every flag the compaction reads is written here, and
// consecutive groups write neighbouring bytes).  Returns whether any node of
// the calling wave gained bits.
template <int WD>
__device__ __forceinline__ bool pull_sweep(const int4 *__restrict__ recs, int32_t b0, int32_t count,
                                           const int32_t *__restrict__ colD, const uint32_t *__restrict__ dead,
                                           uint32_t *__restrict__ reach, int32_t max_scan, uint8_t *__restrict__ pflag)
{
    const int lane = threadIdx.x & 63;
    const int w = lane & (WD - 1);
    const uint64_t gmask = group_mask(WD);
    const int64_t group = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WD;
    const int64_t ngroups = (int64_t)gridDim.x * blockDim.x / WD;
    const int64_t iters = (count + ngroups - 1) / ngroups;
    bool any_gain = false;
    for (int64_t it = 0, idx = group; it < iters; ++it, idx += ngroups) {
        if (idx < count) {
            const int4 r = recs[b0 + idx];
            const PullOut o = pull_node<WD>(r, w, gmask, colD, dead, reach, max_scan);
            any_gain |= o.gained;
            if (pflag && w == 0) pflag[b0 + idx] = o.pending ? 1 : 0;
        }
    }
    return __ballot(any_gain) != 0;
}

// The pull of the worklist sweeps, with the group width a run-time value.
// Compiled per width like the band pull (ids in chunks of kPullIds or more
// for every width), the worklist kernel measured slower on hub-heavy
// populations at n = 200k: 63 against 31 us per pass at P = 64, 48 against
// 38 us at P = 1024; equal on the benchmark's own population.  Its long scans
// of hub neighbour lists are where the two differ; no cause was found in
// the generated code.
__device__ __forceinline__ PullOut pull_node_rt(const int4 r, int Wd, int w, uint64_t gmask,
                                                const int32_t *__restrict__ colD, const uint32_t *__restrict__ dead,
                                                uint32_t *__restrict__ reach, int32_t max_scan)
{
    const int64_t vo = (int64_t)r.x * Wd + w;
    const uint32_t mine = ld_relaxed_u(reach + vo);
    const uint32_t pend = ~dead[vo] & ~mine;
    PullOut out{false, false};
    if ((__ballot(pend != 0) & gmask) == 0) return out;
    uint32_t acc = 0;
    const int32_t e0 = r.y;
    const int32_t e1 = r.z - e0 > max_scan ? e0 + max_scan : r.z;
    if (Wd >= kIdLanes) {
        // a chunk of Wd neighbour ids in one load, one id per lane, read back
        // by shuffle within the group; four neighbours' bits at a time
        const int gb = (threadIdx.x & 63) & ~(Wd - 1);
        bool open = true;
        for (int32_t c = e0; open && c < e1; c += Wd) {
            const int32_t ids = c + w < e1 ? colD[c + w] : -1;
            const int32_t m = e1 - c < Wd ? e1 - c : Wd;
            for (int32_t t = 0; t < m; t += 4) {
                const int32_t u0 = __shfl(ids, gb + t, 64), u1 = __shfl(ids, gb + t + 1, 64);
                const int32_t u2 = __shfl(ids, gb + t + 2, 64), u3 = __shfl(ids, gb + t + 3, 64);
                acc |= ld_relaxed_u(reach + (int64_t)u0 * Wd + w) |
                       (u1 >= 0 ? ld_relaxed_u(reach + (int64_t)u1 * Wd + w) : 0u) |
                       (u2 >= 0 ? ld_relaxed_u(reach + (int64_t)u2 * Wd + w) : 0u) |
                       (u3 >= 0 ? ld_relaxed_u(reach + (int64_t)u3 * Wd + w) : 0u);
                if ((__ballot((acc & pend) != pend) & gmask) == 0) {
                    open = false;
                    break;
                }
            }
        }
    } else {
        int32_t e = e0;
        for (; e + 4 <= e1; e += 4) {
            const int32_t u0 = colD[e], u1 = colD[e + 1], u2 = colD[e + 2], u3 = colD[e + 3];
            acc |= ld_relaxed_u(reach + (int64_t)u0 * Wd + w) | ld_relaxed_u(reach + (int64_t)u1 * Wd + w) |
                   ld_relaxed_u(reach + (int64_t)u2 * Wd + w) | ld_relaxed_u(reach + (int64_t)u3 * Wd + w);
            if ((__ballot((acc & pend) != pend) & gmask) == 0) break;
        }
        if ((__ballot((acc & pend) != pend) & gmask) != 0)
            for (; e < e1; ++e) acc |= ld_relaxed_u(reach + (int64_t)colD[e] * Wd + w);
    }
    const uint32_t gain = acc & pend;
    if (gain) __hip_atomic_store(reach + vo, mine | gain, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    out.pending = (__ballot((pend & ~gain) != 0) & gmask) != 0;
    out.gained = (__ballot(gain != 0) & gmask) != 0;
    return out;
}

// The sweep loop of pull_sweep around pull_node_rt, for the worklist.
// pflag[i] (worklist position i; pflag may be NULL): written after each
// pull, 1 while the node has bits pending; read (read_flags) so that settled
// nodes are skipped without loading their rows (a node's reach row changes
// only by its own pull, so a settled node stays settled).
__device__ __forceinline__ bool pull_sweep_rt(const int4 *__restrict__ recs, int32_t count, int32_t Wd,
                                              const int32_t *__restrict__ colD, const uint32_t *__restrict__ dead,
                                              uint32_t *__restrict__ reach, int32_t max_scan,
                                              uint8_t *__restrict__ pflag, bool read_flags)
{
    const int lane = threadIdx.x & 63;
    const int w = lane & (Wd - 1);
    const uint64_t gmask = group_mask(Wd);
    const int64_t group = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / Wd;
    const int64_t ngroups = (int64_t)gridDim.x * blockDim.x / Wd;
    const int64_t iters = (count + ngroups - 1) / ngroups;
    bool any_gain = false;
    for (int64_t it = 0, idx = group; it < iters; ++it, idx += ngroups) {
        if (idx < count) {
            const int4 r = recs[idx];
            if (pflag && read_flags && !pflag[idx]) continue;
            const PullOut o = pull_node_rt(r, Wd, w, gmask, colD, dead, reach, max_scan);
            any_gain |= o.gained;
            if (pflag && w == 0) pflag[idx] = o.pending ? 1 : 0;
        }
    }
    return __ballot(any_gain) != 0;
}

// One band of the ordered sweep: the nodes at band positions [b0, b1).
template <int WD>
__global__ void k_pull_band(const int4 *__restrict__ band_rec, int32_t b0, int32_t b1,
                            const int32_t *__restrict__ colD, const uint32_t *__restrict__ dead,
                            uint32_t *__restrict__ reach, int32_t max_scan, uint8_t *__restrict__ pflag)
{
    (void)pull_sweep<WD>(band_rec, b0, b1 - b0, colD, dead, reach, max_scan, pflag);
}

// Block-level compaction: every block owns a contiguous range of the input,
// counts its items, reserves room with one global atomic and writes them at
// offsets taken from an LDS counter.  Order inside the output is not fixed,
// and nothing downstream depends on it.
// The counter is int32 (worklist: at most n_noniso < 2^31 entries) or
// unsigned 64-bit (pending pairs: up to B * n_noniso, which passes 2^31 on
// graphs of a few million nodes).
template <class C>
__device__ __forceinline__ C block_reserve(int32_t mine, C *counter, int32_t *s_tot, C *s_base, int32_t *s_off)
{
    // returns the block's base slot; *s_off is reset to 0 for the write pass
    if (threadIdx.x == 0) *s_tot = 0;
    __syncthreads();
    int32_t x = mine;
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if ((threadIdx.x & 63) == 0 && x) atomicAdd(s_tot, x);
    __syncthreads();
    if (threadIdx.x == 0) {
        *s_base = *s_tot ? atomicAdd(counter, (C)*s_tot) : (C)0;
        *s_off = 0;
    }
    __syncthreads();
    return *s_base;
}

// Counters of a pass (int32 entries after the per-slot roots and sizes): [0]
// the worklist count, [2 ..] the changed flags of the follow-up sweeps (at
// most 33), [kPairCountSlot, kPairCountSlot + 2) the 64-bit pair count; k_seed
// clears all 64.
constexpr int kPairCountSlot = 36;
static_assert(kPairCountSlot % 2 == 0 && kPairCountSlot >= 2 + 33 && kPairCountSlot + 2 <= 64, "counter layout");

// Nodes still pending after the ordered sweep -> worklist: the compaction of
// the pending flags, which are kept by position in the band order (each band
// writes one contiguous run of them).  A thread reads F flags at once (F =
// 16, or 4 when 16 would leave fewer than kPendBlocks blocks: at n = 200k
// the pass took 0.164 ms with 4 against 0.169 with 16; over the 64 batched
// graphs' 1M nodes 0.305 ms with 16 against 0.313 with 4); a block scans
// its counts and reserves its room in the worklist with one global atomic.
constexpr int kPendBlocks = 128;

template <int F>
__global__ __launch_bounds__(kBlk) void k_collect_pending(const uint8_t *__restrict__ pflag, int32_t n,
                                                          const int4 *__restrict__ band_rec,
                                                          int4 *__restrict__ worklist, int32_t *__restrict__ wl_count)
{
    static_assert(F == 4 || F == 16, "flags a thread");
    __shared__ int32_t s_wave[kBlk / 64];
    __shared__ int32_t s_base;
    const int32_t v0 = (blockIdx.x * kBlk + threadIdx.x) * F;
    // the records of the thread's pending nodes are loaded before the
    // reservation, so their round trip overlaps the scan and the atomic
    uint32_t f[F / 4];
#pragma unroll
    for (int t = 0; t < F / 4; ++t) f[t] = 0u;
    if (v0 + F <= n) {
        if constexpr (F == 16) {
            const uint4 q = *reinterpret_cast<const uint4 *>(pflag + v0);
            f[0] = q.x;
            f[1] = q.y;
            f[2] = q.z;
            f[3] = q.w;
        } else {
            f[0] = *reinterpret_cast<const uint32_t *>(pflag + v0);
        }
    } else {
        for (int t = 0; t < F && v0 + t < n; ++t) f[t >> 2] |= (uint32_t)pflag[v0 + t] << (8 * (t & 3));
    }
    int4 rec[F];
#pragma unroll
    for (int t = 0; t < F; ++t) rec[t] = ((f[t >> 2] >> (8 * (t & 3))) & 1u) ? band_rec[v0 + t] : make_int4(0, 0, 0, 0);
    int32_t mine = 0;
#pragma unroll
    for (int t = 0; t < F / 4; ++t) mine += __popc(f[t] & 0x01010101u);
    // exclusive scan of the counts over the block, then one reservation
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) s_wave[wv] = incl;
    __syncthreads();
    int32_t before = 0, total = 0;
#pragma unroll
    for (int q = 0; q < kBlk / 64; ++q) {
        before += q < wv ? s_wave[q] : 0;
        total += s_wave[q];
    }
    if (threadIdx.x == 0) s_base = total ? atomicAdd(wl_count, total) : 0;
    __syncthreads();
    int32_t pos = s_base + before + incl - mine;
#pragma unroll
    for (int t = 0; t < F; ++t)
        if ((f[t >> 2] >> (8 * (t & 3))) & 1u) worklist[pos++] = rec[t];
}

// Further sweeps over the worklist; sweep s runs only if sweep s - 1 changed
// something (changed[s - 1] != 0; changed[0] is set by the caller).
__global__ void k_pull_worklist(const int4 *__restrict__ worklist, const int32_t *__restrict__ wl_count,
                                int32_t Wd, const int32_t *__restrict__ colD, const uint32_t *__restrict__ dead,
                                uint32_t *__restrict__ reach, int32_t *__restrict__ changed, int32_t s,
                                uint8_t *__restrict__ pflag)
{
    if (ld_relaxed(changed + s - 1) == 0) return;
    const int32_t count = ld_relaxed(wl_count);
    // with flags (pflag not NULL) the first sweep writes every worklist
    // position's flag, later ones skip the nodes it (or they) left settled
    const bool any_gain = pull_sweep_rt(worklist, count, Wd, colD, dead, reach, INT_MAX, pflag, s > 1);
    // one flag for the whole grid: set it with a plain store, and only if no
    // other wave has (same-address atomics from every wave would serialise)
    if (any_gain && (threadIdx.x & 63) == 0 && ld_relaxed(changed + s) == 0)
        __hip_atomic_store(changed + s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Pending (individual, node) pairs.  Every pending node is counted for its
// individual (per block, into one partial row of single_part, which
// k_pairs_count's extra blocks add to other[i]; with several instances
// directly into other[i]).  A pending node with no surviving neighbour is a
// component of its own and stops there; the rest go to the pair list for the
// union-find (parent[i][v] = v).
// Padding individuals remove every node, so their bits are never pending.
// A block takes one worklist entry per group at a time: it splits every
// (node, word) entry, reserves room for the block's pairs with one global
// atomic, then writes them.
constexpr int kSplitChunk = 4;

__device__ __forceinline__ void pending_split(const int4 r, int Wd, int w, uint64_t gmask,
                                              const int32_t *__restrict__ colD, const uint32_t *__restrict__ dead,
                                              const uint32_t *__restrict__ reach, bool valid, uint32_t &single,
                                              uint32_t &multi)
{
    const int64_t vo = (int64_t)r.x * Wd + w;
    const uint32_t dv = valid ? dead[vo] : ~0u;
    const uint32_t rv = valid ? reach[vo] : 0u;
    const int32_t e0 = valid ? r.y : 0, e1 = valid ? r.z : 0;
    const uint32_t pend = ~dv & ~rv;
    uint32_t nb = 0;
    const bool any = (__ballot(pend != 0) & gmask) != 0;
    if (any && Wd >= kIdLanes) {
        // ids a chunk of Wd at a time by lane, read back by shuffle;
        // kSplitChunk neighbours' bits at a time
        const int gb = (threadIdx.x & 63) & ~(Wd - 1);
        bool open = true;
        for (int32_t c = e0; open && c < e1; c += Wd) {
            const int32_t ids = c + w < e1 ? colD[c + w] : -1;
            const int32_t m = e1 - c < Wd ? e1 - c : Wd;
            for (int32_t t = 0; t < m; t += kSplitChunk) {
                int32_t u[kSplitChunk];
#pragma unroll
                for (int q = 0; q < kSplitChunk; ++q) u[q] = __shfl(ids, gb + t + q, 64);
#pragma unroll
                for (int q = 0; q < kSplitChunk; ++q)
                    if (u[q] >= 0) nb |= ~dead[(int64_t)u[q] * Wd + w];
                if ((__ballot((nb & pend) != pend) & gmask) == 0) {
                    open = false;
                    break;
                }
            }
        }
    } else if (any) {
        // kSplitChunk neighbours at a time (their ids, then their bits, each
        // set of loads in flight together); stopping once every pending bit
        // has a surviving neighbour (or at the end of the list) gives the same
        // split
        for (int32_t e = e0; e < e1; e += kSplitChunk) {
            int32_t u[kSplitChunk];
#pragma unroll
            for (int t = 0; t < kSplitChunk; ++t) u[t] = e + t < e1 ? colD[e + t] : -1;
#pragma unroll
            for (int t = 0; t < kSplitChunk; ++t)
                if (u[t] >= 0) nb |= ~dead[(int64_t)u[t] * Wd + w];
            if ((__ballot((nb & pend) != pend) & gmask) == 0) break;
        }
    }
    single = pend & ~nb;
    multi = pend & nb;
}

// A block of k_collect_pairs takes one worklist entry per group of Wd lanes
// (kBlk / Wd entries) at a time.  A range is split with dependent loads (the
// node, its bits, its neighbours' bits), so the ranges one block takes form a
// chain: short ranges spread the worklist over more blocks in flight.  At
// n = 200k, P = 1024 (8 entries per range) the pass took 236 us against 280 us
// with 64-entry ranges.
__device__ __forceinline__ int32_t pair_range(int32_t Wd) { return kBlk / Wd; }

// Ranges a block splits between two reservations of room in the pair list.
constexpr int kPairBatch = 4;

__global__ __launch_bounds__(kBlk) void k_collect_pairs(const int4 *__restrict__ worklist,
                                                        const int32_t *__restrict__ wl_count, int32_t Wd, const Insts I,
                                                        const int32_t *__restrict__ colD,
                                                        const uint32_t *__restrict__ dead,
                                                        const uint32_t *__restrict__ reach, int64_t *__restrict__ pairs,
                                                        unsigned long long *__restrict__ pair_count,
                                                        int32_t *__restrict__ parent,
                                                        int32_t *__restrict__ single_part, int32_t *__restrict__ other,
                                                        const uint8_t *__restrict__ pflag)
{
    __shared__ int32_t s_tot, s_off;
    __shared__ unsigned long long s_base;
    __shared__ int32_t s_single[kMaxSlots];
    const int w = threadIdx.x & (Wd - 1);
    const uint64_t gmask = group_mask(Wd);
    const int32_t range = pair_range(Wd);
    // pending counts: per-block LDS counters written as a partial row when
    // all slots fit (one instance, at most kMaxSlots slots), else global atomics
    const int32_t B = I.count * I.bseg;
    const bool lds_singles = I.count == 1;
    const int32_t count = *wl_count;
    if ((int64_t)blockIdx.x * range >= count) return;  // no range: no partial row (see single_sum)
    if (lds_singles)
        for (int32_t t = threadIdx.x; t < B; t += blockDim.x) s_single[t] = 0;
    __syncthreads();
    // the block's ranges r0, r0 + stride, ... are split kPairBatch at a time,
    // their multi-neighbour bits kept in registers, and written after one
    // reservation for all of them
    const int32_t stride = gridDim.x * range;
    for (int32_t r0 = blockIdx.x * range; r0 < count; r0 += kPairBatch * stride) {
        uint32_t mulk[kPairBatch];
        int32_t vk[kPairBatch];
        int32_t mine = 0;
#pragma unroll
        for (int j = 0; j < kPairBatch; ++j) {
            const int64_t idx = (int64_t)r0 + (int64_t)j * stride + (int32_t)(threadIdx.x / Wd);
            // pflag (the follow-up sweeps' flags by worklist position): a
            // settled node has nothing to split
            const bool valid = idx < count && (!pflag || pflag[idx]);
            const int4 rec = valid ? worklist[idx] : make_int4(0, 0, 0, 0);
            uint32_t single, mul;
            pending_split(rec, Wd, w, gmask, colD, dead, reach, valid, single, mul);
            const int32_t gbase = inst_of_node(I, rec.x) * I.bseg + w * 32;
            // in LDS the pair nodes are counted where their pairs are written
            // (one divergent loop fewer); the global counts take them here
            for (uint32_t cnt = lds_singles ? single : single | mul; cnt; cnt &= cnt - 1) {
                if (lds_singles) atomicAdd(&s_single[w * 32 + __ffs(cnt) - 1], 1);
                else atomicAdd(other + gbase + __ffs(cnt) - 1, 1);
            }
            mulk[j] = mul;
            vk[j] = rec.x;
            mine += __popc(mul);
        }
        const unsigned long long base = block_reserve(mine, pair_count, &s_tot, &s_base, &s_off);
        if (mine) {
            int64_t q = (int64_t)base + atomicAdd(&s_off, mine);
#pragma unroll
            for (int j = 0; j < kPairBatch; ++j) {
                const int32_t v = vk[j];
                const int32_t b = inst_of_node(I, v);
                const int32_t vl = v - i_voff(I, b);
                for (uint32_t mul = mulk[j]; mul; mul &= mul - 1) {
                    const int32_t gi = b * I.bseg + w * 32 + __ffs(mul) - 1;
                    pairs[q++] = ((int64_t)gi << 32) | (uint32_t)v;
                    parent[uf_block(I, gi) + vl] = vl;
                    if (lds_singles) atomicAdd(&s_single[gi], 1);
                }
            }
        }
        __syncthreads();
    }
    // pending counts of this block: one partial row, summed by single_sum
    if (lds_singles)
        for (int32_t t = threadIdx.x; t < B; t += blockDim.x) single_part[(int64_t)blockIdx.x * B + t] = s_single[t];
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


// Union over the surviving edges of each pending pair (key: slot << 32 |
// node): a surviving neighbour that is reached joins the root's set; a
// pending one (each such edge once, from its smaller end) is united with it.
// A pair takes kHookLanes lanes, each walking every kHookLanes-th neighbour,
// so a node's unions run side by side.  (One thread a pair, taking eight
// neighbours' ids and bits at a time and uniting in turn, left most of the
// GPU idle: the pairs of a pass fill about one wave per SIMD.)
constexpr int kHookLanes = 8;

__global__ void k_pairs_hook(const int64_t *__restrict__ pairs, const unsigned long long *__restrict__ pair_count,
                             const Insts I, int32_t Wd, const int32_t *__restrict__ row_ptr,
                             const int32_t *__restrict__ col, const uint32_t *__restrict__ dead,
                             const uint32_t *__restrict__ reach, const int32_t *__restrict__ root,
                             int32_t *__restrict__ parent)
{
    const int64_t count = (int64_t)*pair_count;
    const int32_t sub = threadIdx.x & (kHookLanes - 1);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x / kHookLanes;
    for (int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kHookLanes; q < count; q += stride) {
        const int64_t key = pairs[q];
        const int32_t gi = (int32_t)(key >> 32), v = (int32_t)(uint32_t)key;
        const int32_t b = gi / I.bseg, i = gi - b * I.bseg;
        const int32_t off = i_voff(I, b);
        const int32_t w = i >> 5;
        const uint32_t bit = 1u << (i & 31);
        int32_t *pi = parent + uf_block(I, gi);
        const int32_t e1 = row_ptr[v + 1];
        for (int32_t e = row_ptr[v] + sub; e < e1; e += kHookLanes) {
            const int32_t u = col[e];
            if (dead[(int64_t)u * Wd + w] & bit) continue;
            if (reach[(int64_t)u * Wd + w] & bit) uf_unite(pi, v - off, root[gi] - off);
            else if (v < u) uf_unite(pi, v - off, u - off);
        }
    }
}

// Pending nodes counted at the representative of their set.
// Adds the pending-count partial rows of the collect blocks that owned a range to
// other[i]: block (x, y) sums rows [64 y, 64 y + 64) for individuals
// [kBlk x, kBlk x + kBlk), loads unrolled, then one atomic per individual.
constexpr int kSumRows = 64;

__device__ __forceinline__ void single_sum(int32_t bx, int32_t by, const int32_t *__restrict__ single_part,
                                           const int32_t *__restrict__ wl_count, int32_t nparts, int32_t B,
                                           int32_t Wd, int32_t *__restrict__ other)
{
    const int32_t i = bx * blockDim.x + threadIdx.x;
    const int32_t range = pair_range(Wd);
    const int32_t used = min(nparts, (*wl_count + range - 1) / range);
    const int32_t b0 = by * kSumRows;
    if (i >= B || b0 >= used) return;
    const int32_t b1 = min(used, b0 + kSumRows);
    int32_t acc = 0;
#pragma unroll 16
    for (int32_t b = b0; b < b1; ++b) acc += single_part[(int64_t)b * B + i];
    if (acc) atomicAdd(other + i, acc);
}

// Blocks [0, grid): each pair's node counted at the representative of its
// set.  Blocks from grid on (one instance only; sum_x blocks per row group)
// add the pending-count partial rows: independent work sharing the launch.
__global__ void k_pairs_count(const int64_t *__restrict__ pairs, const unsigned long long *__restrict__ pair_count, const Insts I,
                              int32_t *__restrict__ parent, int32_t *__restrict__ ucount, int32_t grid,
                              const int32_t *__restrict__ single_part, const int32_t *__restrict__ wl_count,
                              int32_t B, int32_t Wd, int32_t sum_x, int32_t *__restrict__ other)
{
    if ((int32_t)blockIdx.x >= grid) {
        const int32_t sb = (int32_t)blockIdx.x - grid;
        single_sum(sb % sum_x, sb / sum_x, single_part, wl_count, grid, B, Wd, other);
        return;
    }
    const int64_t count = (int64_t)*pair_count;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)grid * blockDim.x) {
        const int64_t key = pairs[q];
        const int32_t gi = (int32_t)(key >> 32), v = (int32_t)(uint32_t)key;
        const int64_t blk = uf_block(I, gi);
        const int32_t r = uf_find(parent + blk, v - i_voff(I, gi / I.bseg));
        atomicAdd(ucount + blk + r, 1);
    }
}

// A component of s nodes adds s(s - 1)/2 to PC, or s - 1 with `forest`.
__device__ __forceinline__ void add_component(int64_t s, unsigned long long *fit, int32_t *mcn, int32_t forest)
{
    if (s > 1)
        atomicAdd(fit, forest ? (unsigned long long)(s - 1) : (unsigned long long)s * (unsigned long long)(s - 1) / 2ull);
    if (mcn && s > 0) atomicMax(mcn, (int32_t)s);
}

// Blocks [0, grid): the components made only of pending nodes (set
// representative is a pending node other than the root's representative),
// counted; their counters are cleared for reuse.
// Blocks from grid on, one slot a thread: the root's component, which holds
// every surviving non-isolated node but the pending ones outside the root's
// set: alive - other[gi] (all its pending nodes) + the root set's counter
// (the root alone when it is isolated); that counter is cleared for reuse.
// Neither part reads a value the other changes: the root's counter is skipped
// by the pair part, other[] is final once k_pairs_count has ended, and the
// path compression both do in parent[] only points entries at ancestors with
// the same representative.
__global__ void k_pairs_reduce(const int64_t *__restrict__ pairs, const unsigned long long *__restrict__ pair_count, const Insts I,
                               int32_t grid, int32_t *__restrict__ parent, const int32_t *__restrict__ root,
                               int32_t *__restrict__ ucount, const int32_t *__restrict__ alive_noniso,
                               const int32_t *__restrict__ other, const int32_t *__restrict__ row_ptr,
                               unsigned long long *__restrict__ fitness, int32_t *__restrict__ mcn, int32_t forest)
{
    if ((int32_t)blockIdx.x >= grid) {
        const int32_t gi = ((int32_t)blockIdx.x - grid) * blockDim.x + threadIdx.x;
        if (gi >= I.count * I.bseg || root[gi] < 0) return;
        const int32_t r = root[gi];
        const int32_t off = i_voff(I, gi / I.bseg);
        const int64_t blk = uf_block(I, gi);
        const int32_t rep = uf_find(parent + blk, r - off);
        const int64_t s = row_ptr[r + 1] > row_ptr[r]
                              ? (int64_t)alive_noniso[gi] - other[gi] + ucount[blk + rep]
                              : 1;
        ucount[blk + rep] = 0;
        add_component(s, fitness + gi, mcn ? mcn + gi : nullptr, forest);
        return;
    }
    const int64_t count = (int64_t)*pair_count;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)grid * blockDim.x) {
        const int64_t key = pairs[q];
        const int32_t gi = (int32_t)(key >> 32), v = (int32_t)(uint32_t)key;
        const int32_t off = i_voff(I, gi / I.bseg);
        const int64_t blk = uf_block(I, gi);
        const int32_t vl = v - off;
        if (parent[blk + vl] != vl || vl == uf_find(parent + blk, root[gi] - off)) continue;
        const int32_t s = ucount[blk + vl];
        ucount[blk + vl] = 0;
        add_component(s, fitness + gi, mcn ? mcn + gi : nullptr, forest);
    }
}

}  // namespace

// Launch of KERNEL<WD>, kBlk threads a block, for the group width
// WD = 2^log_wd of a pass (1 to 64 words a node row).
#define GAPA_LAUNCH_WD(KERNEL, log_wd, grid, s, ...)                                       \
    do {                                                                                   \
        switch (log_wd) {                                                                  \
        case 0: hipLaunchKernelGGL(KERNEL<1>, grid, dim3(kBlk), 0, s, __VA_ARGS__); break;  \
        case 1: hipLaunchKernelGGL(KERNEL<2>, grid, dim3(kBlk), 0, s, __VA_ARGS__); break;  \
        case 2: hipLaunchKernelGGL(KERNEL<4>, grid, dim3(kBlk), 0, s, __VA_ARGS__); break;  \
        case 3: hipLaunchKernelGGL(KERNEL<8>, grid, dim3(kBlk), 0, s, __VA_ARGS__); break;  \
        case 4: hipLaunchKernelGGL(KERNEL<16>, grid, dim3(kBlk), 0, s, __VA_ARGS__); break; \
        case 5: hipLaunchKernelGGL(KERNEL<32>, grid, dim3(kBlk), 0, s, __VA_ARGS__); break;  \
        default: hipLaunchKernelGGL(KERNEL<64>, grid, dim3(kBlk), 0, s, __VA_ARGS__); break; \
        }                                                                                  \
    } while (0)

int launch_bits_transpose(const uint32_t *masks, int32_t P, int32_t W, int32_t n, uint32_t *rows, hipStream_t s)
{
    int32_t Wd = P / 32, log_wd = 0;
    if (P % 32 != 0 || Wd < 1 || Wd > 32 || (Wd & (Wd - 1)) != 0) return GAPA_E_INVALID_ARG;
    while ((1 << log_wd) < Wd) ++log_wd;
    const Insts I{1, P, n, P, nullptr, nullptr, nullptr, nullptr, nullptr};
    const int32_t tw = transpose_tile_words(Wd);
    hipLaunchKernelGGL(k_dead_transpose, dim3((W + tw - 1) / tw), dim3(kBlk),
                       (size_t)transpose_lds_words(log_wd) * 4, s, masks, I, log_wd, rows, nullptr);
    GAPA_HIP(hipGetLastError());
    return GAPA_OK;
}

namespace {

// Slot layout of one pass: Wd words per node row, B = 32 Wd slots per
// instance, S slots in all.
struct PassShape {
    int32_t Wd, log_wd, B, S;
    bool multi;
};

int reserve_pass(gapa_graph *g, FitnessWorkspace &ws, const PassShape &sh, hipStream_t s)
{
    const int32_t n = g->n, B = sh.B;
    int rc;
    if ((rc = ws.dead.reserve((size_t)n * sh.Wd * 4)) != GAPA_OK) return rc;
    if ((rc = ws.reach.reserve((size_t)n * sh.Wd * 4)) != GAPA_OK) return rc;
    if ((rc = ws.parent.reserve((size_t)B * n * 4)) != GAPA_OK) return rc;
    if (ws.ucount.bytes < (size_t)B * n * 4) {
        if ((rc = ws.ucount.reserve((size_t)B * n * 4)) != GAPA_OK) return rc;
        if ((rc = launch_fill_u32(ws.ucount.ptr, 0u, (int64_t)B * n, s)) != GAPA_OK) return rc;
    }
    // pending pairs of slot (b, i) are nodes of instance b: at most B per node
    const int64_t max_pairs = (int64_t)B * std::max(g->n_noniso, 1);
    if ((rc = ws.pairs.reserve((size_t)max_pairs * 8)) != GAPA_OK) return rc;
    if ((rc = ws.worklist.reserve((size_t)std::max(g->n_noniso, 1) * 16)) != GAPA_OK) return rc;
    // pending flags by band position: each pass writes every position below
    // n_noniso before the compaction reads it (zeroed once here all the same)
    const size_t flag_bytes = ((size_t)std::max(g->n_noniso, 1) + 15) & ~(size_t)15;
    if (ws.pflag.bytes < flag_bytes || !ws.pflag_clear) {
        if ((rc = ws.pflag.reserve(flag_bytes)) != GAPA_OK) return rc;
        if ((rc = launch_fill_u32(ws.pflag.ptr, 0u, (int64_t)(flag_bytes / 4), s)) != GAPA_OK) return rc;
        ws.pflag_clear = true;
    }
    const size_t nparts = sh.multi ? 0 : (size_t)g->tune.sweep_grid * B;
    if ((rc = ws.small.reserve((size_t)(2 * (size_t)sh.S + 64 + nparts) * 4)) != GAPA_OK) return rc;
    return GAPA_OK;
}

// One pass over the slots [c0, c0 + B) of a single instance, or over every
// instance (multi), with workspace ws on stream s.
int run_pass(gapa_graph *g, FitnessWorkspace &ws, const PassShape &sh, const InstTable *it, const uint32_t *masks,
             const int32_t *alive, int32_t P, int32_t c0, int64_t *fitness, int32_t *mcn, Measure measure,
             KernelTimer *timer, hipStream_t s)
{
    const int32_t n = g->n, W = g->words, Wd = sh.Wd, log_wd = sh.log_wd, B = sh.B, S = sh.S;
    const bool multi = sh.multi;
    const Tuning &tu = g->tune;
    const int32_t grid = tu.sweep_grid;
    int32_t *root = ws.small.as<int32_t>();
    int32_t *other = root + S;
    // [0] worklist count, [2, 2 + sweeps] changed flags, [kPairCountSlot, +2)
    // the 64-bit pair count (8-byte aligned: S is a multiple of 32)
    int32_t *ctr = root + 2 * S;
    int32_t *wl_count = ctr, *changed = ctr + 2;
    unsigned long long *pair_count = reinterpret_cast<unsigned long long *>(ctr + kPairCountSlot);
    int32_t *single_part = ctr + 64;  // [grid][B] singleton counts per collect block (one instance)
    ws.stats_ctr = ctr;
    ws.stats_B = S;
    uint32_t *dead = ws.dead.as<uint32_t>(), *reach = ws.reach.as<uint32_t>();
    int32_t *parent = ws.parent.as<int32_t>(), *ucount = ws.ucount.as<int32_t>();
    int64_t *pairs = ws.pairs.as<int64_t>();
    int4 *worklist = ws.worklist.as<int4>();
    const int32_t nb = (int32_t)g->band_off.size() - 1;
    const int32_t noniso = g->n_noniso;
    {
        Insts I{};
        if (multi) {
            I = Insts{it->count, B, 0, 0, it->voff, it->live, it->moff, it->node_inst, it->tiles};
        } else {
            I = Insts{1, B, n, std::min(B, P - c0), nullptr, nullptr, nullptr, nullptr, nullptr};
        }
        unsigned long long *fit = reinterpret_cast<unsigned long long *>(fitness + c0);
        int32_t *mc = mcn ? mcn + c0 : nullptr;
        const int32_t *al = alive + c0;
        TimedScope pass(timer, "fitness_pass", s, 1);
        {
            TimedScope ts(timer, "k_dead_transpose", s);
            const int32_t tw = transpose_tile_words(Wd);
            const int32_t tiles = multi ? it->ntiles : (W + tw - 1) / tw;
            hipLaunchKernelGGL(k_dead_transpose, dim3(tiles), dim3(kBlk), (size_t)transpose_lds_words(log_wd) * 4, s,
                               masks + (int64_t)c0 * W, I, log_wd, dead, reach);
        }
        {
            TimedScope ts(timer, "k_seed", s);
            // one wave per slot, kSeedWaves slots per block
            hipLaunchKernelGGL(k_seed, dim3((S + kSeedWaves - 1) / kSeedWaves), dim3(64 * kSeedWaves), 0, s, dead,
                               g->d_order, I, Wd, root, reach, parent, other, ctr, fit, mc, g->d_row_ptr, g->d_colD,
                               g->d_src_idx, ws.pflag.as<uint8_t>(), g->src_band);
        }
        {
            TimedScope ts(timer, "k_pull_band", s);
            // band 0, the sources, is taken by k_seed when it holds them alone
            for (int32_t b = g->src_band > 0 ? 1 : 0; b < nb; ++b) {
                const int32_t b0 = g->band_off[b], b1 = g->band_off[b + 1];
                if (b1 <= b0) continue;
                const int64_t threads = (int64_t)(b1 - b0) * Wd;
                const int blocks = (int)std::min<int64_t>((threads + kBlk - 1) / kBlk, tu.band_blocks);
                GAPA_LAUNCH_WD(k_pull_band, log_wd, dim3(blocks), s, g->d_band_rec, b0, b1, g->d_colD, dead, reach,
                               tu.band_scan, ws.pflag.as<uint8_t>());
            }
        }
        if (noniso > 0) {
            TimedScope ts(timer, "k_collect_pending", s);
            const bool wide = (noniso + kBlk * 16 - 1) / (kBlk * 16) >= kPendBlocks;
            const int32_t per_block = kBlk * (wide ? 16 : 4);
            const dim3 grid_p((unsigned)((noniso + per_block - 1) / per_block));
            if (wide)
                hipLaunchKernelGGL(k_collect_pending<16>, grid_p, dim3(kBlk), 0, s, ws.pflag.as<uint8_t>(), noniso,
                                   g->d_band_rec, worklist, wl_count);
            else
                hipLaunchKernelGGL(k_collect_pending<4>, grid_p, dim3(kBlk), 0, s, ws.pflag.as<uint8_t>(), noniso,
                                   g->d_band_rec, worklist, wl_count);
        }
        // Settled-node flags (by worklist position, in the band flags' buffer,
        // consumed by then) pay when later sweeps revisit many settled nodes:
        // with three sweeps over the 64 batched graphs the pass went from 0.305
        // to 0.287 ms; with two at n = 200k, whose worklist nodes mostly stay
        // pending, from 0.162 to 0.164 ms.  So they are kept from three on.
        const bool settled_flags = tu.sweeps >= 3;
        {
            TimedScope ts(timer, "k_pull_worklist", s);
            for (int32_t sw = 1; sw <= tu.sweeps; ++sw)
                hipLaunchKernelGGL(k_pull_worklist, dim3(grid), dim3(kBlk), 0, s, worklist, wl_count, Wd, g->d_colD,
                                   dead, reach, changed, sw, settled_flags ? ws.pflag.as<uint8_t>() : nullptr);
        }
        {
            TimedScope ts(timer, "k_collect_pairs", s);
            hipLaunchKernelGGL(k_collect_pairs, dim3(grid), dim3(kBlk), 0, s, worklist, wl_count, Wd, I, g->d_colD,
                               dead, reach, pairs, pair_count, parent, single_part, other,
                               settled_flags ? ws.pflag.as<uint8_t>() : nullptr);
        }
        {
            TimedScope ts(timer, "k_pairs_hook", s);
            hipLaunchKernelGGL(k_pairs_hook, dim3(grid), dim3(kBlk), 0, s, pairs, pair_count, I, Wd,
                               g->d_row_ptr, g->d_col, dead, reach, root, parent);
        }
        {
            TimedScope ts(timer, "k_pairs_count", s);
            // with one instance, the singleton sums ride in the same launch
            const int32_t sum_x = (B + kBlk - 1) / kBlk;
            const int32_t extra = multi ? 0 : sum_x * ((grid + kSumRows - 1) / kSumRows);
            hipLaunchKernelGGL(k_pairs_count, dim3(grid + extra), dim3(kBlk), 0, s, pairs, pair_count, I, parent,
                               ucount, grid, single_part, wl_count, B, Wd, sum_x, other);
        }
        {
            TimedScope ts(timer, "k_pairs_reduce", s);
            // the root components ride in the same launch as extra blocks
            const int32_t roots = (S + kBlk - 1) / kBlk;
            hipLaunchKernelGGL(k_pairs_reduce, dim3(grid + roots), dim3(kBlk), 0, s, pairs, pair_count, I, grid,
                               parent, root, ucount, al, other, g->d_row_ptr, fit, mc, (int32_t)measure);
        }
        GAPA_HIP(hipGetLastError());
    }
    return GAPA_OK;
}

}  // namespace

namespace {

// Parts of a caller-provided scratch region for chunks of B = 32 Wd
// individuals (byte offsets, each part 256-byte aligned; the sizes are those
// reserve_pass asks for).
struct ScratchLayout {
    size_t flag, masks, alive, dead, reach, parent, ucount, pairs, worklist, pflag, small, total;
};

ScratchLayout scratch_layout(const gapa_graph *g, int32_t Wd)
{
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t B = 32 * (size_t)Wd, n = (size_t)g->n, W = (size_t)g->words;
    const size_t nn = (size_t)std::max(g->n_noniso, 1);
    ScratchLayout l{};
    size_t o = 0;
    l.flag = o;
    o += up(16);
    l.masks = o;
    o += up(B * W * 4);
    l.alive = o;
    o += up(B * 4);
    l.dead = o;
    o += up(n * Wd * 4);
    l.reach = o;
    o += up(n * Wd * 4);
    l.parent = o;
    o += up(B * n * 4);
    l.ucount = o;
    o += up(B * n * 4);
    l.pairs = o;
    o += up(B * nn * 8);
    l.worklist = o;
    o += up(nn * 16);
    l.pflag = o;
    o += up((n + 15) & ~(size_t)15);
    l.small = o;
    o += up((2 * B + 64 + (size_t)g->tune.sweep_grid * B) * 4);
    l.total = o;
    return l;
}

}  // namespace

size_t bits_scratch_bytes(const gapa_graph *g, int32_t Wd)
{
    return scratch_layout(g, Wd).total;
}

int eval_genes_bits_scratch(gapa_graph *g, const int32_t *genes, int32_t P, int32_t k, int64_t *fitness,
                            int32_t *mcn, Measure measure, void *scratch, size_t bytes, int32_t **flag_out,
                            hipStream_t s)
{
    // the widest chunk that fits, and no wider than the population needs
    int32_t Wd = 1;
    while (Wd < 32 && Wd * 32 < P) Wd <<= 1;
    while (Wd >= 1 && scratch_layout(g, Wd).total > bytes) Wd >>= 1;
    if (Wd < 1) {
        set_error("graph too large for the fixed scratch: 32 individuals per pass need %zu bytes, the scratch "
                  "holds %zu",
                  scratch_layout(g, 1).total, bytes);
        return GAPA_E_INVALID_ARG;
    }
    const ScratchLayout l = scratch_layout(g, Wd);
    char *b = static_cast<char *>(scratch);
    FitnessWorkspace ws;  // views of the scratch only: nothing here allocates or frees
    ws.masks.borrow(b + l.masks, l.alive - l.masks);
    ws.alive.borrow(b + l.alive, l.dead - l.alive);
    ws.dead.borrow(b + l.dead, l.reach - l.dead);
    ws.reach.borrow(b + l.reach, l.parent - l.reach);
    ws.parent.borrow(b + l.parent, l.ucount - l.parent);
    ws.ucount.borrow(b + l.ucount, l.pairs - l.ucount);
    ws.pairs.borrow(b + l.pairs, l.worklist - l.pairs);
    ws.worklist.borrow(b + l.worklist, l.pflag - l.worklist);
    ws.pflag.borrow(b + l.pflag, l.small - l.pflag);
    ws.pflag_clear = false;  // cleared by reserve_pass below: the scratch keeps the last call's flags
    ws.small.borrow(b + l.small, l.total - l.small);
    int32_t *flag = reinterpret_cast<int32_t *>(b + l.flag);
    *flag_out = flag;
    PassShape sh{};
    sh.Wd = Wd;
    sh.log_wd = 0;
    while ((1 << sh.log_wd) < Wd) ++sh.log_wd;
    sh.B = sh.S = 32 * Wd;
    sh.multi = false;
    int rc;
    // the scratch keeps whatever the last call left: the gene flag and the
    // leftover union-find's set sizes must start at zero
    if ((rc = launch_fill_u32(flag, 0u, 4, s)) != GAPA_OK) return rc;
    if ((rc = launch_fill_u32(ws.ucount.ptr, 0u, (int64_t)sh.B * g->n, s)) != GAPA_OK) return rc;
    if ((rc = reserve_pass(g, ws, sh, s)) != GAPA_OK) return rc;
    for (int32_t c0 = 0; c0 < P; c0 += sh.B) {
        const int32_t rows = std::min(sh.B, P - c0);
        if ((rc = launch_mask_build(genes ? genes + (int64_t)c0 * k : nullptr, rows, k, g->n, g->words, g->d_noniso,
                                    g->n_noniso, ws.masks.as<uint32_t>(), ws.alive.as<int32_t>(), flag, s)) != GAPA_OK)
            return rc;
        if ((rc = run_pass(g, ws, sh, nullptr, ws.masks.as<uint32_t>(), ws.alive.as<int32_t>(), rows, 0, fitness + c0,
                           mcn ? mcn + c0 : nullptr, measure, nullptr, s)) != GAPA_OK)
            return rc;
    }
    return GAPA_OK;
}

// Extra lanes of a workspace: chunks of a population wider than one pass run
// concurrently on their own streams and workspaces (the pass is bound by its
// chain of dependent kernels, not by bandwidth, so chunks side by side
// overlap well).  Created on first use, before any graph capture.
constexpr int kPassLanes = 4;

int ensure_lanes(FitnessWorkspace &ws, int32_t lanes)
{
    if (!ws.fork) GAPA_HIP(hipEventCreateWithFlags(&ws.fork, hipEventDisableTiming));
    while ((int32_t)ws.lanes.size() < lanes - 1) {
        FitnessWorkspace *w = new (std::nothrow) FitnessWorkspace();
        if (!w) return GAPA_E_OOM;
        ws.lanes.push_back(w);
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        GAPA_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        ws.lane_streams.push_back(st);
        GAPA_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        ws.lane_done.push_back(ev);
    }
    return GAPA_OK;
}

namespace {

// Shape of a pass over chunks of Wd words per node row.
PassShape pass_shape(int32_t Wd, const InstTable *it)
{
    PassShape sh{};
    sh.multi = it && it->count > 1;
    sh.Wd = Wd;
    sh.log_wd = 0;
    while ((1 << sh.log_wd) < sh.Wd) ++sh.log_wd;
    sh.B = sh.Wd * 32;
    sh.S = sh.multi ? it->count * sh.B : sh.B;
    return sh;
}

}  // namespace

int eval_masks_bits(gapa_graph *g, const uint32_t *masks, const int32_t *alive, int32_t P, int64_t *fitness,
                    int32_t *mcn, FitnessWorkspace &ws, KernelTimer *timer, hipStream_t s, const InstTable *it,
                    Measure measure)
{
    const bool multi = it && it->count > 1;
    if (!multi && P <= 0) return GAPA_OK;
    // Chunks of 32 * Wd individuals, Wd a power of two <= 64: full chunks of
    // 2048, then the rest in the narrowest chunk that holds it.  (A pass's
    // cost is mostly per node, whatever its width: splitting a rest of 544 as
    // 512 + 32 on two lanes cut its latency but nearly doubled its work, which
    // a busy GPU pays.)
    std::vector<std::pair<int32_t, int32_t>> plan;  // (first individual, Wd)
    if (multi) {
        plan.emplace_back(0, it->bseg / 32);
    } else {
        int32_t c0 = 0;
        for (; P - c0 >= kMaxSlots; c0 += kMaxSlots) plan.emplace_back(c0, kMaxSlots / 32);
        const int32_t r = P - c0;
        if (r > 0) {
            int32_t wd = 1;
            while (wd * 32 < r) wd <<= 1;
            plan.emplace_back(c0, wd);
        }
    }
    const int32_t chunks = (int32_t)plan.size();
    const int32_t lanes = std::min(chunks, kPassLanes);
    int rc;
    if (lanes <= 1) {
        const PassShape sh = pass_shape(plan[0].second, it);
        if ((rc = reserve_pass(g, ws, sh, s)) != GAPA_OK) return rc;
        for (int32_t c = 0; c < chunks; ++c)
            if ((rc = run_pass(g, ws, sh, it, masks, alive, P, plan[c].first, fitness, mcn, measure, timer, s)) !=
                GAPA_OK)
                return rc;
        return GAPA_OK;
    }
    if ((rc = ensure_lanes(ws, lanes)) != GAPA_OK) return rc;
    auto lane_ws = [&](int32_t i) -> FitnessWorkspace & { return i == 0 ? ws : *ws.lanes[i - 1]; };
    auto lane_stream = [&](int32_t i) { return i == 0 ? s : ws.lane_streams[i - 1]; };
    // fork: every lane starts after the work already on s
    GAPA_HIP(hipEventRecord(ws.fork, s));
    for (int32_t i = 1; i < lanes; ++i) GAPA_HIP(hipStreamWaitEvent(lane_stream(i), ws.fork, 0));
    for (int32_t c = 0; c < chunks; ++c) {
        const int32_t i = c % lanes;
        const PassShape sh = pass_shape(plan[c].second, it);
        if ((rc = reserve_pass(g, lane_ws(i), sh, lane_stream(i))) != GAPA_OK) return rc;
        if ((rc = run_pass(g, lane_ws(i), sh, it, masks, alive, P, plan[c].first, fitness, mcn, measure, timer,
                           lane_stream(i))) != GAPA_OK)
            return rc;
    }
    // join: s continues once every lane is done
    for (int32_t i = 1; i < lanes; ++i) {
        GAPA_HIP(hipEventRecord(ws.lane_done[i - 1], lane_stream(i)));
        GAPA_HIP(hipStreamWaitEvent(s, ws.lane_done[i - 1], 0));
    }
    const PassShape sh0 = pass_shape(plan[0].second, it);
    ws.stats_ctr = ws.small.as<int32_t>() + 2 * sh0.S;
    ws.stats_B = sh0.S;
    return GAPA_OK;
}

}  // namespace gapa
