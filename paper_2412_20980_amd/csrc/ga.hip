// Genetic operators on the device (Section III-B): initial population (eq. 2),
// tournament selection, positional crossover (eq. 3-6) with duplicate repair,
// swap mutation (eq. 7-9) and elitism (eq. 10-11).
//
// One workgroup builds one individual.  Its membership bit set over the nodes
// lives in LDS while the row is built; the finished row is written out sorted
// for the fitness kernels.  Every random decision is a Philox draw keyed by
// (seed, generation, individual, slot), so the result is a pure function of
// the seed and does not depend on the launch geometry.  The parts that are
// sequential by definition (rejection draws that depend on the current
// membership, in ascending slot order) run on one lane over LDS only; their
// first-attempt draws are computed by the whole block beforehand.
#include <algorithm>
#include <climits>

#include "device_common.h"
#include "internal.h"

namespace gapa {
namespace {

constexpr int kOpBlock = 256;
constexpr int kRankTile = 256;

struct OpArgs {
    const int32_t *pop;   // [P][k] current population, rows ascending
    const int64_t *fit;   // [P]   ordered by (PC, position)
    int32_t *children;    // [L][k] out
    int32_t *flag;        // [1]   attempts exhausted
    uint64_t seed, t_pc, t_pm;
    uint32_t gen;
    int32_t P, k, n, W, K2, KW, T;
};

// LDS of one operator block: membership bits over the nodes, the row (padded
// to a power of two for the sort), first-attempt candidates per slot, and
// three bit sets over the slots.
struct OpLds {
    uint32_t *U;          // [W]
    int32_t *row;         // [K2]
    int32_t *cand;        // [k]
    uint32_t *from_donor; // [KW]
    uint32_t *dup;        // [KW]
    uint32_t *mut;        // [KW]
};

__device__ __forceinline__ OpLds carve(uint32_t *smem, const OpArgs &a)
{
    OpLds l;
    l.U = smem;
    l.row = reinterpret_cast<int32_t *>(smem + a.W);
    l.cand = l.row + a.K2;
    l.from_donor = reinterpret_cast<uint32_t *>(l.cand + a.k);
    l.dup = l.from_donor + a.KW;
    l.mut = l.dup + a.KW;
    return l;
}

__device__ __forceinline__ bool lds_test(const uint32_t *U, uint32_t v)
{
    return (U[v >> 5] >> (v & 31)) & 1u;
}

__device__ __forceinline__ void lds_set(uint32_t *U, uint32_t v)
{
    U[v >> 5] |= 1u << (v & 31);
}

// Starting from candidate u (attempt t0), the first attempt of
// (slot, ind, gen, stream | t) that is not a member; -1 if attempts run out.
__device__ int32_t first_non_member(const uint32_t *U, uint32_t u, uint32_t t0, uint64_t seed, uint32_t slot,
                                    uint32_t ind, uint32_t gen, uint32_t stream, uint32_t n)
{
    uint32_t t = t0;
    while (lds_test(U, u)) {
        if (++t >= kMaxAttempts) return -1;
        u = bounded(draw(seed, slot, ind, gen, stream, t).w0, n);
    }
    return (int32_t)u;
}

// Ascending bitonic sort of K2 (a power of two) ints in LDS by the whole block.
__device__ void block_sort(int32_t *a, int32_t K2)
{
    for (int32_t size = 2; size <= K2; size <<= 1) {
        for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int32_t i = threadIdx.x; i < (K2 >> 1); i += blockDim.x) {
                const int32_t lo = 2 * i - (i & (stride - 1));
                const int32_t hi = lo + stride;
                const bool up = (lo & size) == 0;
                const int32_t x = a[lo], y = a[hi];
                if ((x > y) == up) {
                    a[lo] = y;
                    a[hi] = x;
                }
            }
            __syncthreads();
        }
    }
}

__device__ void clear_lds(const OpLds &l, const OpArgs &a)
{
    for (int32_t w = threadIdx.x; w < a.W; w += blockDim.x) l.U[w] = 0u;
    for (int32_t w = threadIdx.x; w < a.KW; w += blockDim.x) l.from_donor[w] = l.dup[w] = l.mut[w] = 0u;
    for (int32_t j = a.k + threadIdx.x; j < a.K2; j += blockDim.x) l.row[j] = INT_MAX;
}

__device__ void sort_and_write(const OpLds &l, const OpArgs &a, int32_t idx)
{
    block_sort(l.row, a.K2);
    int32_t *dst = a.children + (int64_t)idx * a.k;
    for (int32_t j = threadIdx.x; j < a.k; j += blockDim.x) dst[j] = l.row[j];
}

// Initial individual i (eq. 2): slot j takes the first INIT draw that is not
// already in the row; the row is then sorted.
__global__ __launch_bounds__(kOpBlock) void k_init(OpArgs a)
{
    extern __shared__ uint32_t smem[];
    const OpLds l = carve(smem, a);
    const int32_t i = blockIdx.x;
    clear_lds(l, a);
    for (int32_t j = threadIdx.x; j < a.k; j += blockDim.x)
        l.cand[j] = (int32_t)bounded(draw(a.seed, j, i, 0, kStreamInit, 0).w0, a.n);
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int32_t j = 0; j < a.k; ++j) {
            const int32_t u = first_non_member(l.U, l.cand[j], 0, a.seed, j, i, 0, kStreamInit, a.n);
            if (u < 0) {
                atomicOr(a.flag, 1);
                l.row[j] = 0;
                continue;
            }
            lds_set(l.U, u);
            l.row[j] = u;
        }
    }
    __syncthreads();
    sort_and_write(l, a, i);
}

// Offspring o of generation gen >= 1.
//   base  = POP[o mod P]; donor = tournament winner (smallest (PC, position)
//           among T uniform draws with replacement; contestant c is word c mod 4
//           of SELECT draw slot c / 4).
//   eq. 6 gene j = donor[j] where the crossover mask (eq. 4) word-0 coin of
//           XOVER draw j is below floor(pc 2^32), else base[j]; word 1 of the
//           same draw is the mutation coin of eq. 8.
//   repair  a slot whose value already sits at a lower slot gets a uniform
//           non-member (REPAIR draws), slots ascending.
//   eq. 9   each mutated slot, ascending, swaps its gene for a uniform
//           non-member (MUTATE draws).
//   sort    the row ascending.
__global__ __launch_bounds__(kOpBlock) void k_offspring(OpArgs a)
{
    extern __shared__ uint32_t smem[];
    __shared__ int32_t s_donor;
    const OpLds l = carve(smem, a);
    const int32_t o = blockIdx.x;

    if (threadIdx.x == 0) {
        int32_t best = -1;
        Words4 w{0, 0, 0, 0};
        for (int32_t c = 0; c < a.T; ++c) {
            if ((c & 3) == 0) w = draw(a.seed, (uint32_t)(c >> 2), o, a.gen, kStreamSelect, 0);
            const uint32_t word = (c & 3) == 0 ? w.w0 : (c & 3) == 1 ? w.w1 : (c & 3) == 2 ? w.w2 : w.w3;
            const int32_t x = (int32_t)bounded(word, (uint32_t)a.P);
            if (best < 0 || a.fit[x] < a.fit[best] || (a.fit[x] == a.fit[best] && x < best)) best = x;
        }
        s_donor = best;
    }
    clear_lds(l, a);
    __syncthreads();

    const int32_t *base = a.pop + (int64_t)(o % a.P) * a.k;
    const int32_t *donor = a.pop + (int64_t)s_donor * a.k;
    // crossover coins; values taken from the base row enter the membership set
    for (int32_t j = threadIdx.x; j < a.k; j += blockDim.x) {
        const Words4 x = draw(a.seed, j, o, a.gen, kStreamXover, 0);
        const bool take = (uint64_t)x.w0 < a.t_pc;
        const int32_t c = take ? donor[j] : base[j];
        l.row[j] = c;
        if (take) atomicOr(&l.from_donor[j >> 5], 1u << (j & 31));
        else atomicOr(&l.U[c >> 5], 1u << (c & 31));
        if ((uint64_t)x.w1 < a.t_pm) {
            atomicOr(&l.mut[j >> 5], 1u << (j & 31));
            l.cand[j] = (int32_t)bounded(draw(a.seed, j, o, a.gen, kStreamMutate, 0).w0, a.n);
        }
    }
    __syncthreads();

    // Base and donor rows are ascending and distinct, so a value occurs at most
    // twice in the child: once from each row.  A donor value c that is already
    // a member came from the base row at the slot p where base[p] = c; the
    // later of p and j is the copy.  Other donor values join the set.
    for (int32_t j = threadIdx.x; j < a.k; j += blockDim.x) {
        if (!((l.from_donor[j >> 5] >> (j & 31)) & 1u)) continue;
        const int32_t c = l.row[j];
        if (lds_test(l.U, c)) {
            int32_t lo = 0, hi = a.k;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (base[mid] < c) lo = mid + 1;
                else hi = mid;
            }
            const int32_t later = lo < j ? j : lo;
            atomicOr(&l.dup[later >> 5], 1u << (later & 31));
        } else {
            atomicOr(&l.U[c >> 5], 1u << (c & 31));
        }
    }
    __syncthreads();

    if (threadIdx.x == 0) {
        for (int32_t q = 0; q < a.KW; ++q) {
            for (uint32_t bits = l.dup[q]; bits; bits &= bits - 1) {
                const int32_t j = q * 32 + __ffs(bits) - 1;
                const uint32_t u0 = bounded(draw(a.seed, j, o, a.gen, kStreamRepair, 0).w0, a.n);
                const int32_t u = first_non_member(l.U, u0, 0, a.seed, j, o, a.gen, kStreamRepair, a.n);
                if (u < 0) {
                    atomicOr(a.flag, 1);
                    continue;
                }
                lds_set(l.U, u);
                l.row[j] = u;
            }
        }
        for (int32_t q = 0; q < a.KW; ++q) {
            for (uint32_t bits = l.mut[q]; bits; bits &= bits - 1) {
                const int32_t j = q * 32 + __ffs(bits) - 1;
                const int32_t u = first_non_member(l.U, l.cand[j], 0, a.seed, j, o, a.gen, kStreamMutate, a.n);
                if (u < 0) {
                    atomicOr(a.flag, 1);
                    continue;
                }
                const int32_t old = l.row[j];
                l.U[old >> 5] &= ~(1u << (old & 31));
                lds_set(l.U, u);
                l.row[j] = u;
            }
        }
    }
    __syncthreads();
    sort_and_write(l, a, o);
}

// Elitism (eq. 10-11) as a merge by ranks.  Keys: parents (PC, tag r) for the
// npar rows already ordered by (PC, tag), pooled offspring (PC, tag npar + o)
// for o = pool[q] (q < npool; pool NULL: o = q).  A key's output position is
// the number of keys smaller in (PC, tag) order.  k_rank_count adds, per
// (key, tile of pooled offspring), the offspring below the key; k_rank_place
// adds the parents (they are sorted: a binary search) and writes the first
// `keep` positions.
__global__ __launch_bounds__(kRankTile) void k_rank_count(const int64_t *__restrict__ f_par, int32_t npar,
                                                          const int64_t *__restrict__ f_pool,
                                                          const int32_t *__restrict__ pool, int32_t npool,
                                                          int32_t *__restrict__ pos)
{
    __shared__ int64_t tf[kRankTile];
    __shared__ int32_t tt[kRankTile];
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t q0 = blockIdx.y * kRankTile;
    const int32_t q = q0 + threadIdx.x;
    tf[threadIdx.x] = q < npool ? f_pool[q] : INT64_MAX;
    tt[threadIdx.x] = q < npool ? (pool ? pool[q] : q) : INT_MAX;
    __syncthreads();
    if (t >= npar + npool) return;
    const bool is_par = t < npar;
    const int64_t f = is_par ? f_par[t] : f_pool[t - npar];
    const int32_t tag = is_par ? -1 : (pool ? pool[t - npar] : t - npar);
    const int32_t m = min(kRankTile, npool - q0);
    int32_t cnt = 0;
    for (int32_t i = 0; i < m; ++i) {
        const int64_t g = tf[i];
        // pooled offspring tags exceed every parent tag
        cnt += is_par ? (g < f) : (g < f || (g == f && tt[i] < tag));
    }
    if (cnt) atomicAdd(pos + t, cnt);
}

__global__ void k_rank_place(const int64_t *__restrict__ f_par, int32_t npar, const int64_t *__restrict__ f_pool,
                             const int32_t *__restrict__ pool, int32_t npool, int32_t keep,
                             const int32_t *__restrict__ pos, int32_t *__restrict__ src, int64_t *__restrict__ f_out)
{
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npar + npool) return;
    int32_t p = pos[t];
    int64_t f;
    int32_t tag;
    if (t < npar) {
        f = f_par[t];
        p += t;
        tag = t;
    } else {
        f = f_pool[t - npar];
        int32_t lo = 0, hi = npar;  // parents with PC <= f come first
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (f_par[mid] <= f) lo = mid + 1;
            else hi = mid;
        }
        p += lo;
        tag = npar + (pool ? pool[t - npar] : t - npar);
    }
    if (p < keep) {
        src[p] = tag;
        f_out[p] = f;
    }
}

__global__ void k_gather_rows(const int32_t *__restrict__ src, int32_t npar, const int32_t *__restrict__ parents,
                              const int32_t *__restrict__ children, int32_t k, int32_t *__restrict__ out)
{
    const int32_t r = blockIdx.x;
    const int32_t tag = src[r];
    const int32_t *s = tag < npar ? parents + (int64_t)tag * k : children + (int64_t)(tag - npar) * k;
    int32_t *d = out + (int64_t)r * k;
    for (int32_t j = threadIdx.x; j < k; j += blockDim.x) d[j] = s[j];
}

OpArgs make_args(gapa_ga *ga, const int32_t *pop, const int64_t *fit, uint32_t gen)
{
    const gapa_graph *g = ga->graph;
    OpArgs a;
    a.pop = pop;
    a.fit = fit;
    a.children = ga->children.as<int32_t>();
    a.flag = ga->flag.as<int32_t>();
    a.seed = ga->params.seed;
    a.t_pc = ga->t_pc;
    a.t_pm = ga->t_pm;
    a.gen = gen;
    a.P = ga->params.pop;
    a.k = ga->params.k;
    a.n = g->n;
    a.W = g->words;
    int32_t K2 = 1;
    while (K2 < a.k) K2 <<= 1;
    a.K2 = K2;
    a.KW = (a.k + 31) / 32;
    a.T = ga->params.tournament;
    return a;
}

}  // namespace

int ga_rank_and_gather(gapa_ga *ga, const int64_t *f_par, const int32_t *par_rows, int32_t npar,
                       const int64_t *f_pool, const int32_t *pool, int32_t npool, hipStream_t s)
{
    const int nxt = npar ? 1 - ga->cur : ga->cur;
    const int32_t P = ga->params.pop, k = ga->params.k;
    const int32_t total = npar + npool;
    int32_t *pos = ga->rank.as<int32_t>();
    int rc;
    if ((rc = launch_fill_u32(pos, 0u, total, s)) != GAPA_OK) return rc;
    {
        TimedScope ts(&ga->timer, "elitism_rank", s);
        const dim3 grid((total + kRankTile - 1) / kRankTile, (npool + kRankTile - 1) / kRankTile);
        if (npool > 0)
            hipLaunchKernelGGL(k_rank_count, grid, dim3(kRankTile), 0, s, f_par, npar, f_pool, pool, npool, pos);
        hipLaunchKernelGGL(k_rank_place, dim3((total + 255) / 256), dim3(256), 0, s, f_par, npar, f_pool, pool, npool,
                           P, pos, ga->src.as<int32_t>(), ga->fit[nxt].as<int64_t>());
    }
    {
        TimedScope ts(&ga->timer, "gather_rows", s);
        hipLaunchKernelGGL(k_gather_rows, dim3(P), dim3(256), 0, s, ga->src.as<int32_t>(), npar, par_rows,
                           ga->children.as<int32_t>(), k, ga->pop[nxt].as<int32_t>());
    }
    GAPA_HIP(hipGetLastError());
    ga->cur = nxt;
    return GAPA_OK;
}

size_t ga_op_lds_bytes(int32_t n, int32_t k)
{
    const size_t W = ((size_t)n + 31) / 32;
    size_t K2 = 1;
    while (K2 < (size_t)k) K2 <<= 1;
    const size_t KW = ((size_t)k + 31) / 32;
    return 4 * (W + K2 + (size_t)k + 3 * KW);
}

int ga_prepare_kernels(size_t lds)
{
    if (lds > 64 * 1024) {
        GAPA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_init),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        GAPA_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_offspring),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    return GAPA_OK;
}

int ga_launch_init(gapa_ga *ga, hipStream_t s)
{
    OpArgs a = make_args(ga, nullptr, nullptr, 0);
    TimedScope ts(&ga->timer, "ga_init", s);
    hipLaunchKernelGGL(k_init, dim3(ga->params.pop), dim3(kOpBlock), ga->op_lds_bytes, s, a);
    GAPA_HIP(hipGetLastError());
    return GAPA_OK;
}

int ga_launch_offspring(gapa_ga *ga, uint32_t gen, int32_t count, hipStream_t s)
{
    OpArgs a = make_args(ga, ga->pop[ga->cur].as<int32_t>(), ga->fit[ga->cur].as<int64_t>(), gen);
    TimedScope ts(&ga->timer, "ga_offspring", s);
    hipLaunchKernelGGL(k_offspring, dim3(count), dim3(kOpBlock), ga->op_lds_bytes, s, a);
    GAPA_HIP(hipGetLastError());
    return GAPA_OK;
}

int ga_init_population(gapa_ga *ga, hipStream_t s)
{
    const int32_t P = ga->params.pop;
    int rc = ga_launch_init(ga, s);
    if (rc != GAPA_OK) return rc;
    rc = eval_genes(ga->graph, ga->children.as<int32_t>(), P, ga->params.k, true, ga->child_fit.as<int64_t>(),
                    nullptr, ga->flag.as<int32_t>() + 1, ga->ws, &ga->timer, s);
    if (rc != GAPA_OK) return rc;
    return ga_rank_and_gather(ga, nullptr, nullptr, 0, ga->child_fit.as<int64_t>(), nullptr, P, s);
}

int ga_generation(gapa_ga *ga, hipStream_t s)
{
    const int32_t P = ga->params.pop, L = ga->lambda;
    const uint32_t gen = (uint32_t)(ga->generation + 1);
    int rc = ga_launch_offspring(ga, gen, L, s);
    if (rc != GAPA_OK) return rc;
    rc = eval_genes(ga->graph, ga->children.as<int32_t>(), L, ga->params.k, true, ga->child_fit.as<int64_t>(),
                    nullptr, ga->flag.as<int32_t>() + 1, ga->ws, &ga->timer, s);
    if (rc != GAPA_OK) return rc;
    rc = ga_rank_and_gather(ga, ga->fit[ga->cur].as<int64_t>(), ga->pop[ga->cur].as<int32_t>(), P,
                            ga->child_fit.as<int64_t>(), nullptr, L, s);
    if (rc != GAPA_OK) return rc;
    ga->generation += 1;
    return GAPA_OK;
}

}  // namespace gapa
