// Genetic operators on the device (Section III-B): initial population (eq. 2),
// tournament selection, positional crossover (eq. 3-6) with duplicate repair,
// swap mutation (eq. 7-9) and elitism (eq. 10-11).
//
// One workgroup builds one individual; its membership bit set over the nodes
// lives in LDS while the row is built, and the finished row is written out
// sorted for the fitness kernels.  Every random decision is
// a Philox draw keyed by (seed, generation, individual, slot): the result is a
// pure function of the seed and does not depend on the launch geometry.
#include <algorithm>
#include <climits>

#include "device_common.h"
#include "internal.h"

namespace gapa {
namespace {

constexpr int kOpBlock = 256;
constexpr int kRankBlock = 256;

struct OpArgs {
    const int32_t *pop;   // [P][k] current population, rows ascending
    const int64_t *fit;   // [P]   ordered by (PC, position)
    int32_t *children;    // [L][k] out
    int32_t *flag;        // [1]   attempts exhausted
    uint64_t seed, t_pc, t_pm;
    uint32_t gen;
    int32_t P, k, n, W, K2, T;
};

struct OpLds {
    uint32_t *U;     // [W]  membership bit set
    int32_t *row;    // [K2] the row, padded with INT_MAX for the sort
    uint8_t *from_donor, *dup, *mut;  // [k] each
};

__device__ __forceinline__ OpLds carve(uint32_t *smem, int32_t W, int32_t K2, int32_t k)
{
    OpLds l;
    l.U = smem;
    l.row = reinterpret_cast<int32_t *>(smem + W);
    l.from_donor = reinterpret_cast<uint8_t *>(l.row + K2);
    l.dup = l.from_donor + k;
    l.mut = l.dup + k;
    return l;
}

__device__ __forceinline__ bool lds_test(const uint32_t *U, uint32_t v)
{
    return (U[v >> 5] >> (v & 31)) & 1u;
}

// First attempt t = 0, 1, ... of (slot, ind, gen, stream | t) whose bounded
// word 0 is not a member; marks it a member.  -1 if the attempts run out.
__device__ int32_t take_non_member(uint32_t *U, uint64_t seed, uint32_t slot, uint32_t ind, uint32_t gen,
                                   uint32_t stream, uint32_t n)
{
    for (uint32_t t = 0; t < kMaxAttempts; ++t) {
        const uint32_t u = bounded(draw(seed, slot, ind, gen, stream, t).w0, n);
        if (!lds_test(U, u)) {
            U[u >> 5] |= 1u << (u & 31);
            return (int32_t)u;
        }
    }
    return -1;
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

__device__ void write_out(const OpLds &l, const OpArgs &a, int32_t idx)
{
    int32_t *dst = a.children + (int64_t)idx * a.k;
    for (int32_t j = threadIdx.x; j < a.k; j += blockDim.x) dst[j] = l.row[j];
}

// Initial individual i (eq. 2): slot j takes the first INIT draw that is not
// already in the row; the row is then sorted.
__global__ __launch_bounds__(kOpBlock) void k_init(OpArgs a)
{
    extern __shared__ uint32_t smem[];
    const OpLds l = carve(smem, a.W, a.K2, a.k);
    const int32_t i = blockIdx.x;
    for (int32_t w = threadIdx.x; w < a.W; w += blockDim.x) l.U[w] = 0u;
    for (int32_t j = a.k + threadIdx.x; j < a.K2; j += blockDim.x) l.row[j] = INT_MAX;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int32_t j = 0; j < a.k; ++j) {
            const int32_t u = take_non_member(l.U, a.seed, j, i, 0, kStreamInit, a.n);
            if (u < 0) {
                atomicOr(a.flag, 1);
                l.row[j] = 0;
                continue;
            }
            l.row[j] = u;
        }
    }
    __syncthreads();
    block_sort(l.row, a.K2);
    write_out(l, a, i);
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
    const OpLds l = carve(smem, a.W, a.K2, a.k);
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
    for (int32_t w = threadIdx.x; w < a.W; w += blockDim.x) l.U[w] = 0u;
    for (int32_t j = a.k + threadIdx.x; j < a.K2; j += blockDim.x) l.row[j] = INT_MAX;
    __syncthreads();

    const int32_t *base = a.pop + (int64_t)(o % a.P) * a.k;
    const int32_t *donor = a.pop + (int64_t)s_donor * a.k;
    for (int32_t j = threadIdx.x; j < a.k; j += blockDim.x) {
        const Words4 x = draw(a.seed, j, o, a.gen, kStreamXover, 0);
        const bool take = (uint64_t)x.w0 < a.t_pc;
        l.row[j] = take ? donor[j] : base[j];
        l.from_donor[j] = take;
        l.mut[j] = (uint64_t)x.w1 < a.t_pm;
    }
    __syncthreads();

    // Base and donor rows are ascending and distinct, so a value occurs at most
    // twice in the child: once taken from each row.  Slot j's value c came from
    // one row; c is repeated iff the other row holds c at a slot p != j that
    // took its value from that other row.  The later of the two is the copy.
    for (int32_t j = threadIdx.x; j < a.k; j += blockDim.x) {
        const int32_t c = l.row[j];
        const bool take = l.from_donor[j];
        const int32_t *other = take ? base : donor;
        int32_t lo = 0, hi = a.k;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (other[mid] < c) lo = mid + 1;
            else hi = mid;
        }
        const bool repeated = lo < j && other[lo] == c && (bool)l.from_donor[lo] != take;
        l.dup[j] = repeated;
        if (!repeated) atomicOr(&l.U[c >> 5], 1u << (c & 31));
    }
    __syncthreads();

    if (threadIdx.x == 0) {
        for (int32_t j = 0; j < a.k; ++j) {
            if (!l.dup[j]) continue;
            const int32_t u = take_non_member(l.U, a.seed, j, o, a.gen, kStreamRepair, a.n);
            if (u < 0) {
                atomicOr(a.flag, 1);
                continue;
            }
            l.row[j] = u;
        }
        for (int32_t j = 0; j < a.k; ++j) {
            if (!l.mut[j]) continue;
            const int32_t u = take_non_member(l.U, a.seed, j, o, a.gen, kStreamMutate, a.n);
            if (u < 0) {
                atomicOr(a.flag, 1);
                continue;
            }
            const int32_t old = l.row[j];
            l.U[old >> 5] &= ~(1u << (old & 31));
            l.row[j] = u;
        }
    }
    __syncthreads();
    block_sort(l.row, a.K2);
    write_out(l, a, o);
}

// Elitism (eq. 10-11) as a merge by ranks.  Parents (tags 0..npar-1) are
// already ordered by (PC, tag); offspring get tags npar + o.  Each key's
// output position is the number of keys smaller in (PC, tag) order; the
// first `keep` positions are written (source tag and PC).
__global__ __launch_bounds__(kRankBlock) void k_elitism_rank(const int64_t *__restrict__ f_par, int32_t npar,
                                                             const int64_t *__restrict__ f_off, int32_t L,
                                                             int32_t keep, int32_t *__restrict__ src,
                                                             int64_t *__restrict__ f_out)
{
    __shared__ int64_t tile[kRankBlock];
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool is_par = t < npar;
    const bool active = t < npar + L;
    const int32_t o = t - npar;
    const int64_t f = !active ? 0 : is_par ? f_par[t] : f_off[o];
    int32_t pos = is_par ? t : 0;
    for (int32_t base = 0; base < L; base += kRankBlock) {
        const int32_t q = base + threadIdx.x;
        tile[threadIdx.x] = q < L ? f_off[q] : INT64_MAX;
        __syncthreads();
        const int32_t m = min(kRankBlock, L - base);
        if (active) {
            for (int32_t i = 0; i < m; ++i) {
                const int64_t g = tile[i];
                // offspring tags npar + q exceed every parent tag
                pos += is_par ? (g < f) : (g < f || (g == f && base + i < o));
            }
        }
        __syncthreads();
    }
    if (!active) return;
    if (!is_par) {
        int32_t lo = 0, hi = npar;  // parents with PC <= f precede offspring o
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (f_par[mid] <= f) lo = mid + 1;
            else hi = mid;
        }
        pos += lo;
    }
    if (pos < keep) {
        src[pos] = t;
        f_out[pos] = f;
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
    a.T = ga->params.tournament;
    return a;
}

int rank_and_gather(gapa_ga *ga, const int64_t *f_par, const int32_t *par_rows, int32_t npar, int32_t L,
                    hipStream_t s)
{
    const int nxt = npar ? 1 - ga->cur : ga->cur;
    const int32_t P = ga->params.pop, k = ga->params.k;
    const int32_t total = npar + L;
    {
        TimedScope ts(&ga->timer, "elitism_rank", s);
        hipLaunchKernelGGL(k_elitism_rank, dim3((total + kRankBlock - 1) / kRankBlock), dim3(kRankBlock), 0, s,
                           f_par, npar, ga->child_fit.as<int64_t>(), L, P, ga->src.as<int32_t>(),
                           ga->fit[nxt].as<int64_t>());
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

}  // namespace

size_t ga_op_lds_bytes(int32_t n, int32_t k)
{
    const int32_t W = (n + 31) / 32;
    int32_t K2 = 1;
    while (K2 < k) K2 <<= 1;
    return (size_t)W * 4 + (size_t)K2 * 4 + (((size_t)3 * k + 3) & ~(size_t)3);
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

int ga_init_population(gapa_ga *ga, hipStream_t s)
{
    const int32_t P = ga->params.pop;
    OpArgs a = make_args(ga, nullptr, nullptr, 0);
    {
        TimedScope ts(&ga->timer, "ga_init", s);
        hipLaunchKernelGGL(k_init, dim3(P), dim3(kOpBlock), ga->op_lds_bytes, s, a);
    }
    GAPA_HIP(hipGetLastError());
    int rc = eval_genes(ga->graph, ga->children.as<int32_t>(), P, ga->params.k, true, ga->child_fit.as<int64_t>(), nullptr,
                        ga->flag.as<int32_t>() + 1, ga->ws, &ga->timer, s);
    if (rc != GAPA_OK) return rc;
    return rank_and_gather(ga, nullptr, nullptr, 0, P, s);
}

int ga_generation(gapa_ga *ga, hipStream_t s)
{
    const int32_t P = ga->params.pop, L = ga->lambda;
    const uint32_t gen = (uint32_t)(ga->generation + 1);
    const int32_t *pop = ga->pop[ga->cur].as<int32_t>();
    const int64_t *fit = ga->fit[ga->cur].as<int64_t>();
    OpArgs a = make_args(ga, pop, fit, gen);
    {
        TimedScope ts(&ga->timer, "ga_offspring", s);
        hipLaunchKernelGGL(k_offspring, dim3(L), dim3(kOpBlock), ga->op_lds_bytes, s, a);
    }
    GAPA_HIP(hipGetLastError());
    int rc = eval_genes(ga->graph, ga->children.as<int32_t>(), L, ga->params.k, true, ga->child_fit.as<int64_t>(), nullptr,
                        ga->flag.as<int32_t>() + 1, ga->ws, &ga->timer, s);
    if (rc != GAPA_OK) return rc;
    rc = rank_and_gather(ga, fit, pop, P, L, s);
    if (rc != GAPA_OK) return rc;
    ga->generation += 1;
    return GAPA_OK;
}

}  // namespace gapa
