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
//
// A launch serves one GA or a batch of independent GAs (one per instance
// graph): blockIdx.y selects the instance, whose sizes, seed and buffer
// offsets come from a device table, so every instance follows exactly the
// rules (and draws) of a GA run alone.  The generation number is read from
// device memory, which lets a whole generation be captured once and replayed.
#include <algorithm>
#include <climits>

#include "device_common.h"
#include "internal.h"

namespace gapa {
namespace {

constexpr int kOpBlock = 256;

// Launch arguments: buffer bases shared by all instances of the launch.
struct OpArgs {
    const GaInst *inst;       // [instances]
    const int32_t *pop;       // current population rows, ascending
    const int64_t *fit;       // current fitness, ordered by (PC, position)
    const uint32_t *noniso;   // non-isolated node bit sets
    int32_t *children;        // out: child rows, ascending
    uint32_t *masks;          // out: removed-node bit set of each child
    int32_t *alive;           // out: surviving non-isolated nodes of each child
    int32_t *flag;            // [1] attempts exhausted
    const uint32_t *gen_ctr;  // [1] generations completed
    int32_t rows_only;        // emit only the rows (no bit sets, no alive counts)
};

// One instance's view, resolved by each block from the table.
struct Op {
    const int32_t *pop;     // [P][k]
    const int64_t *fit;     // [P]
    const uint32_t *noniso; // [W] bit v set: v has an edge
    int32_t *children;      // [L][k]
    uint32_t *masks;        // [L][W]
    int32_t *alive;         // [L]
    int32_t *flag;
    uint64_t seed, t_pc, t_pm;
    int32_t P, L, k, n, W, KW, T, n_noniso;
    int32_t rows_only;
};

__device__ __forceinline__ Op resolve(const OpArgs &a)
{
    const GaInst &I = a.inst[blockIdx.y];
    Op o;
    o.pop = a.pop ? a.pop + I.pop_off : nullptr;
    o.fit = a.fit ? a.fit + I.fit_off : nullptr;
    o.noniso = a.noniso + I.noniso_off;
    o.children = a.children + I.child_off;
    o.masks = a.masks + I.mask_off;
    o.alive = a.alive + I.slot_off;
    o.flag = a.flag;
    o.seed = I.seed;
    o.t_pc = I.t_pc;
    o.t_pm = I.t_pm;
    o.P = I.P;
    o.L = I.L;
    o.k = I.k;
    o.n = I.n;
    o.W = I.W;
    o.KW = I.KW;
    o.T = I.T;
    o.n_noniso = I.n_noniso;
    o.rows_only = a.rows_only;
    return o;
}

// LDS of one operator block: membership bits over the nodes, the row by slot,
// a list of slots (16-bit: the LDS limit keeps k far below 65536), and three
// bit sets over the slots.  Kept small so that four blocks fit a compute unit
// at n = 200k, k = 2000.
struct OpLds {
    uint32_t *U;          // [W]
    int32_t *row;         // [k]
    uint16_t *list;       // [k, rounded up to even]
    uint32_t *from_donor; // [KW]
    uint32_t *dup;        // [KW]
    uint32_t *mut;        // [KW]
};

__device__ __forceinline__ OpLds carve(uint32_t *smem, const Op &a)
{
    OpLds l;
    l.U = smem;
    l.row = reinterpret_cast<int32_t *>(smem + a.W);
    l.list = reinterpret_cast<uint16_t *>(l.row + a.k);
    l.from_donor = reinterpret_cast<uint32_t *>(l.list + ((a.k + 1) & ~1));
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

// Slots whose bit is set in bits[0 .. ceil(k/32)), ascending, into list[];
// returns how many.  Run by one whole wave.
__device__ int32_t wave_list_slots(const uint32_t *bits, int32_t k, uint16_t *list)
{
    const int lane = threadIdx.x & 63;
    int32_t count = 0;
    for (int32_t j0 = 0; j0 < k; j0 += 64) {
        const int32_t j = j0 + lane;
        const bool on = j < k && ((bits[j >> 5] >> (j & 31)) & 1u);
        const uint64_t mask = __ballot(on);
        if (on) list[count + __popcll(mask & ((1ull << lane) - 1ull))] = (uint16_t)j;
        count += __popcll(mask);
    }
    return count;
}

// The defining rule, in slot order: slot list[a] (a = 0, 1, ...) takes the
// first draw (slot, ind, gen, stream | t), t = 0, 1, ..., that is not in the
// membership set U; U gains it and, with `swap`, loses the slot's previous
// value.  One wave resolves 64 slots at a time: every lane takes its attempt
// 0, and lane l's draw is accepted if it is not a member (checked against U
// as it stood before the batch) and no earlier lane drew the same value.  All
// lanes before the first rejected one are committed at once; the rejected
// one is resolved alone with further attempts from its attempt 0, exactly as
// the sequential rule would given the committed lanes; the next batch starts
// after it.  A draw equal to a value an earlier lane frees (swap) is
// rejected too and then accepted by the lone resolution: the same result.
//
// With `pre` (no swap), slot j's attempt-0 value was computed beforehand by
// the whole block and stored in row[j] (the slot's old value is not needed).
//
// Equal draws within the batch are found through U itself: every candidate
// not yet a member sets its bit with an atomic OR, and a lane that finds its
// bit already set by another lane of the batch marks a collision.  Without
// one (the usual case) no lane is taken; with one the lanes compare values
// directly.  Bits set for lanes that are not committed are cleared again.
__device__ void wave_draw_in_order(const OpLds &l, const Op &a, const uint16_t *list, int32_t count, bool swap,
                                   uint32_t ind, uint32_t gen, uint32_t stream, bool pre = false)
{
    const int lane = threadIdx.x & 63;
    int32_t pos = 0;
    while (pos < count) {
        const int32_t nvalid = min(64, count - pos);
        const bool valid = lane < nvalid;
        const int32_t j = valid ? (list ? list[pos + lane] : pos + lane) : 0;
        // attempt 0 of slot j: drawn here, or (pre, no swap) already in row[j]
        const uint32_t c = !valid ? 0u : pre ? (uint32_t)l.row[j] : bounded(draw(a.seed, j, ind, gen, stream, 0).w0, a.n);
        const int32_t old = (valid && swap) ? l.row[j] : -1;
        const uint32_t w = c >> 5, bit = 1u << (c & 31);
        // membership before the batch: every lane reads before any lane writes
        const bool in_u = valid && (l.U[w] & bit);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        bool mine = false, clash = false;
        if (valid && !in_u) {
            const uint32_t prev = atomicOr(&l.U[w], bit);
            mine = !(prev & bit);
            clash = !mine;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        bool taken = false;
        if (__ballot(clash) != 0) {
            // q is uniform across the wave: lane q's value is read with readlane
            for (int q = 0; q < nvalid; ++q) {
                const uint32_t cq = (uint32_t)__builtin_amdgcn_readlane((int)c, q);
                taken |= q < lane && cq == c;
            }
        }
        const bool reject = valid && (in_u || taken);
        const uint64_t rej = __ballot(reject);
        const int32_t f = rej ? (int32_t)__ffsll((unsigned long long)rej) - 1 : nvalid;
        // lanes from f on are not committed: clear the bits they set
        if (mine && lane >= f) atomicAnd(&l.U[w], ~bit);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (lane < f) {
            // (a committed value whose bit a later, uncommitted lane with the
            // same draw had set and just cleared is set again)
            atomicOr(&l.U[w], bit);
            if (swap) atomicAnd(&l.U[old >> 5], ~(1u << (old & 31)));
            l.row[j] = (int32_t)c;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (f < nvalid) {
            if (lane == f) {
                const int32_t u = first_non_member(l.U, c, 0, a.seed, j, ind, gen, stream, a.n);
                if (u < 0) {
                    atomicOr(a.flag, 1);
                } else {
                    if (swap) l.U[old >> 5] &= ~(1u << (old & 31));
                    lds_set(l.U, u);
                    l.row[j] = u;
                }
            }
            pos += f + 1;
        } else {
            pos += nvalid;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

// Exclusive prefix sum over the block (blockDim.x <= 1024, a multiple of 64);
// also returns the block total.  Every thread must call it.
__device__ int32_t block_exclusive_scan(int32_t x, int32_t *total);

// Slots whose bit is set in bits[0 .. ceil(k/32)), ascending, into list[];
// returns how many.  Whole block: each thread enumerates a contiguous run of
// words at the offset a block scan of their popcounts gives.  The list is
// visible to every thread on return.
__device__ int32_t block_list_slots(const uint32_t *bits, int32_t k, uint16_t *list)
{
    const int32_t KW = (k + 31) / 32;
    const int32_t per = (KW + (int32_t)blockDim.x - 1) / (int32_t)blockDim.x;
    const int32_t w0 = min(KW, (int32_t)threadIdx.x * per), w1 = min(KW, w0 + per);
    int32_t cnt = 0;
    for (int32_t w = w0; w < w1; ++w) cnt += __popc(bits[w]);
    int32_t total = 0;
    int32_t off = block_exclusive_scan(cnt, &total);
    for (int32_t w = w0; w < w1; ++w)
        for (uint32_t x = bits[w]; x; x &= x - 1) list[off++] = (uint16_t)(w * 32 + __ffs(x) - 1);
    __syncthreads();
    return total;
}

__device__ int32_t block_exclusive_scan(int32_t x, int32_t *total)
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

__device__ void clear_lds(const OpLds &l, const Op &a)
{
    for (int32_t w = threadIdx.x; w < a.W; w += blockDim.x) l.U[w] = 0u;
    for (int32_t w = threadIdx.x; w < a.KW; w += blockDim.x) l.from_donor[w] = l.dup[w] = l.mut[w] = 0u;
}

// The finished individual leaves as its membership bit set (the removed-node
// mask the fitness kernels consume), its row in ascending order (the set bits
// enumerated in order: each thread owns a contiguous run of words, a block
// scan of their popcounts gives its output offset) and its count of
// surviving non-isolated nodes (n_noniso minus the genes that have an edge).
__device__ void emit(const OpLds &l, const Op &a, int32_t idx)
{
    // removed non-isolated nodes, counted from the bit set while it is copied
    // out (the set's words and the non-isolated set's are read in the same
    // coalesced order), summed in LDS
    __shared__ int32_t s_gone;
    if (threadIdx.x == 0) s_gone = 0;
    __syncthreads();
    if (!a.rows_only) {
        uint32_t *m = a.masks + (int64_t)idx * a.W;
        int32_t gone = 0;
        int32_t w = threadIdx.x;
        for (; w + 7 * (int32_t)blockDim.x < a.W; w += 8 * blockDim.x) {
            uint32_t x[8], y[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                x[u] = l.U[w + u * blockDim.x];
                y[u] = a.noniso[w + u * blockDim.x];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                m[w + u * blockDim.x] = x[u];
                gone += __popc(x[u] & y[u]);
            }
        }
        for (; w < a.W; w += blockDim.x) {
            const uint32_t x = l.U[w];
            m[w] = x;
            gone += __popc(x & a.noniso[w]);
        }
        for (int off = 32; off > 0; off >>= 1) gone += __shfl_down(gone, off, 64);
        if ((threadIdx.x & 63) == 0 && gone) atomicAdd(&s_gone, gone);
    }
    const int32_t per = (a.W + blockDim.x - 1) / blockDim.x;
    const int32_t w0 = min(a.W, (int32_t)threadIdx.x * per), w1 = min(a.W, w0 + per);
    int32_t cnt = 0;
    for (int32_t w = w0; w < w1; ++w) cnt += __popc(l.U[w]);
    int32_t total = 0;
    int32_t off = block_exclusive_scan(cnt, &total);
    // the sorted row is staged in LDS (the row by slot is no longer needed)
    // and written out coalesced
    for (int32_t w = w0; w < w1; ++w)
        for (uint32_t bits = l.U[w]; bits; bits &= bits - 1)
            if (off < a.k) l.row[off++] = w * 32 + __ffs(bits) - 1;
    __syncthreads();
    int32_t *dst = a.children + (int64_t)idx * a.k;
    for (int32_t j = threadIdx.x; j < a.k; j += blockDim.x) dst[j] = l.row[j];
    if (threadIdx.x == 0) {
        if (!a.rows_only) a.alive[idx] = a.n_noniso - s_gone;
        if (total != a.k) atomicOr(a.flag, 1);
    }
}

// Initial individual i (eq. 2): slot j takes the first INIT draw that is not
// already in the row; the row is then sorted.
__global__ __launch_bounds__(kOpBlock) void k_init(OpArgs args)
{
    extern __shared__ uint32_t smem[];
    const Op a = resolve(args);
    const int32_t i = blockIdx.x;
    if (i >= a.P) return;
    const OpLds l = carve(smem, a);
    clear_lds(l, a);
    __syncthreads();
    if (threadIdx.x < 64) wave_draw_in_order(l, a, nullptr, a.k, false, i, 0, kStreamInit);
    emit(l, a, i);
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
// Position of value c in the ascending base row staged in bs[0, k): galloping
// from slot j (the rows of a converged population differ by small shifts),
// then a binary search inside the bracket.  c must be in the row.
__device__ __forceinline__ int32_t base_position(const int32_t *bs, int32_t k, int32_t j, int32_t c)
{
    int32_t lo, hi;
    if (bs[j] < c) {
        int32_t b = 1;
        while (j + b < k && bs[j + b] < c) b <<= 1;
        lo = j + (b >> 1) + 1;
        hi = min(j + b, k);
    } else {
        int32_t b = 1;
        while (j - b >= 0 && bs[j - b] >= c) b <<= 1;
        lo = max(j - b + 1, 0);
        hi = j - (b >> 1);
    }
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (bs[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Rows up to kOpBlock * kOpSlots genes keep each thread's base and donor
// genes in registers from the crossover to the row fill (slot j = thread +
// kOpBlock i); longer rows read them again from global memory.
constexpr int kOpSlots = 8;

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
__global__ __launch_bounds__(kOpBlock) void k_offspring(OpArgs args)
{
    extern __shared__ uint32_t smem[];
    __shared__ int32_t s_donor;
    const Op a = resolve(args);
    const int32_t o = blockIdx.x;
    if (o >= a.L) return;
    const uint32_t gen = *args.gen_ctr + 1u;
    const OpLds l = carve(smem, a);

    if (threadIdx.x == 0) {
        int32_t best = -1;
        Words4 w{0, 0, 0, 0};
        for (int32_t c = 0; c < a.T; ++c) {
            if ((c & 3) == 0) w = draw(a.seed, (uint32_t)(c >> 2), o, gen, kStreamSelect, 0);
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
    const bool regs = a.k <= kOpBlock * kOpSlots;
    int32_t bv[kOpSlots], dv[kOpSlots];
    uint32_t takes = 0u;  // bit i: slot threadIdx.x + kOpBlock i takes the donor gene
    // Crossover coins; the base row is staged in LDS (row[] holds it while
    // duplicates are located), values taken from it enter the membership set.
    if (regs) {
#pragma unroll
        for (int i = 0; i < kOpSlots; ++i) {
            const int32_t j = threadIdx.x + kOpBlock * i;
            bv[i] = j < a.k ? base[j] : 0;
            dv[i] = j < a.k ? donor[j] : 0;
        }
#pragma unroll
        for (int i = 0; i < kOpSlots; ++i) {
            const int32_t j = threadIdx.x + kOpBlock * i;
            if (j >= a.k) break;
            const Words4 x = draw(a.seed, j, o, gen, kStreamXover, 0);
            const bool take = (uint64_t)x.w0 < a.t_pc;
            l.row[j] = bv[i];
            if (take) takes |= 1u << i;
            else atomicOr(&l.U[bv[i] >> 5], 1u << (bv[i] & 31));
            if ((uint64_t)x.w1 < a.t_pm) atomicOr(&l.mut[j >> 5], 1u << (j & 31));
        }
    } else {
#pragma unroll 4
        for (int32_t j = threadIdx.x; j < a.k; j += blockDim.x) {
            const Words4 x = draw(a.seed, j, o, gen, kStreamXover, 0);
            const bool take = (uint64_t)x.w0 < a.t_pc;
            const int32_t b = base[j];
            l.row[j] = b;
            if (take) atomicOr(&l.from_donor[j >> 5], 1u << (j & 31));
            else atomicOr(&l.U[b >> 5], 1u << (b & 31));
            if ((uint64_t)x.w1 < a.t_pm) atomicOr(&l.mut[j >> 5], 1u << (j & 31));
        }
    }
    __syncthreads();

    // Base and donor rows are ascending and distinct, so a value occurs at most
    // twice in the child: once from each row.  A donor value c that is already
    // a member came from the base row at the slot p where base[p] = c; the
    // later of p and j is the copy.  Other donor values join the set.
    if (regs) {
#pragma unroll
        for (int i = 0; i < kOpSlots; ++i) {
            if (!((takes >> i) & 1u)) continue;
            const int32_t j = threadIdx.x + kOpBlock * i;
            const int32_t c = dv[i];
            if (lds_test(l.U, c)) {
                const int32_t p = base_position(l.row, a.k, j, c);
                const int32_t later = p < j ? j : p;
                atomicOr(&l.dup[later >> 5], 1u << (later & 31));
            } else {
                atomicOr(&l.U[c >> 5], 1u << (c & 31));
            }
        }
    } else {
#pragma unroll 2
        for (int32_t j = threadIdx.x; j < a.k; j += blockDim.x) {
            if (!((l.from_donor[j >> 5] >> (j & 31)) & 1u)) continue;
            const int32_t c = donor[j];
            if (lds_test(l.U, c)) {
                const int32_t p = base_position(l.row, a.k, j, c);
                const int32_t later = p < j ? j : p;
                atomicOr(&l.dup[later >> 5], 1u << (later & 31));
            } else {
                atomicOr(&l.U[c >> 5], 1u << (c & 31));
            }
        }
    }
    __syncthreads();
    // the child's row by slot: donor values where the coin took the donor
    if (regs) {
#pragma unroll
        for (int i = 0; i < kOpSlots; ++i)
            if ((takes >> i) & 1u) l.row[threadIdx.x + kOpBlock * i] = dv[i];
    } else {
        for (int32_t j = threadIdx.x; j < a.k; j += blockDim.x)
            if ((l.from_donor[j >> 5] >> (j & 31)) & 1u) l.row[j] = donor[j];
    }
    __syncthreads();

    // Repair, then mutation, each in ascending slot order by one wave.  The
    // slot lists are built by the whole block, and so are the repair slots'
    // attempt-0 draws (a repaired slot's duplicate value is not needed, so the
    // draw takes its place in row[]).
    const int32_t nd = block_list_slots(l.dup, a.k, l.list);
    for (int32_t q = threadIdx.x; q < nd; q += blockDim.x) {
        const int32_t j = l.list[q];
        l.row[j] = (int32_t)bounded(draw(a.seed, j, o, gen, kStreamRepair, 0).w0, a.n);
    }
    __syncthreads();
    if (threadIdx.x < 64) wave_draw_in_order(l, a, l.list, nd, false, o, gen, kStreamRepair, true);
    __syncthreads();
    const int32_t nm = block_list_slots(l.mut, a.k, l.list);
    if (threadIdx.x < 64) wave_draw_in_order(l, a, l.list, nm, true, o, gen, kStreamMutate);
    emit(l, a, o);
}

// Fitness of every slot from the pass's MCN (GAPA_MINIMISE_MCN).
__global__ void k_mcn_objective(const int32_t *__restrict__ mcn, int64_t *__restrict__ fit, int32_t count)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) fit[i] = mcn[i];
}

// Elitism (eq. 10-11) as a merge by ranks, per instance (blockIdx.y).
// Keys: parents (PC, tag r) for the npar rows already ordered by (PC, tag),
// pooled offspring (PC, tag npar + o) for o = pool[q] (q < npool; pool NULL:
// o = q).  At generation 0 there are no parents and the P initial
// individuals are the pool.  A key's output position is the number of keys
// smaller in (PC, tag) order: the pooled offspring below it plus the
// parents below it (they are sorted: its own index, or a binary search for
// an offspring).  The first P positions are written.
//
// A block takes kRankKeys keys.  Each of its waves holds a 64-entry slice of
// the pool, one entry per lane, and compares it with one key at a time: a
// ballot and a bit count give the slice's entries below the key.  The waves'
// counts meet in LDS, and the block places its keys in the same launch.  At
// P = lambda = 1024 elitism (ranks and the row gather) takes 13.9 us per
// generation with 8 keys a block, against 15.1 with 16 and 20.0 with 64
// (the keys' loop is a chain of LDS reads; more blocks share it), and 22 us
// for a tile-by-tile count into atomic counters plus a second launch placing
// the keys.
// Slower: counting the parents by ballot too, and the comparison loop
// written without branches, eight keys a batch.
struct RankArgs {
    const GaInst *inst;
    const int64_t *f_par;   // current fitness (instance base fit_off)
    const int64_t *f_pool;  // pooled offspring fitness (instance base slot_off)
    const int32_t *pool;    // NULL, or [npool] offspring of each pooled entry (one instance)
    int32_t npool;          // with pool
    int32_t init;           // generation 0: no parents
    int32_t *src;           // [P] source tag of each kept row (instance base fit_off)
    int64_t *f_out;         // next fitness (instance base fit_off)
};

struct RankView {
    const int64_t *f_par, *f_pool;
    int32_t npar, npool;
};

__device__ __forceinline__ RankView rank_view(const RankArgs &a, int32_t b)
{
    const GaInst &I = a.inst[b];
    RankView v;
    v.npar = a.init ? 0 : I.P;
    v.npool = a.init ? I.P : (a.pool ? a.npool : I.L);
    v.f_par = a.f_par + I.fit_off;
    v.f_pool = a.f_pool + I.slot_off;
    return v;
}

constexpr int kRankKeys = 8;    // keys per block
constexpr int kRankWaves = 16;  // waves per block

__global__ __launch_bounds__(64 * kRankWaves) void k_rank_place(RankArgs a)
{
    __shared__ int64_t kf[kRankKeys];
    __shared__ int32_t kt[kRankKeys], kc[kRankKeys];
    const GaInst &I = a.inst[blockIdx.y];
    const RankView r = rank_view(a, blockIdx.y);
    const int32_t total = r.npar + r.npool;
    const int32_t k0 = blockIdx.x * kRankKeys;
    if (k0 >= total) return;  // uniform over the block
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x < kRankKeys) {
        const int32_t t = k0 + threadIdx.x;
        int64_t f = INT64_MAX;
        int32_t tag = INT_MAX;
        if (t < total) {
            f = t < r.npar ? r.f_par[t] : r.f_pool[t - r.npar];
            tag = t < r.npar ? -1 : (a.pool ? a.pool[t - r.npar] : t - r.npar);
        }
        kf[threadIdx.x] = f;
        kt[threadIdx.x] = tag;
        kc[threadIdx.x] = 0;
    }
    __syncthreads();
    int32_t mine = 0;
    for (int32_t q0 = wv * 64; q0 < r.npool; q0 += 64 * kRankWaves) {
        const int32_t q = q0 + lane;
        const bool in = q < r.npool;
        const int64_t g = in ? r.f_pool[q] : 0;
        const int32_t gt = in ? (a.pool ? a.pool[q] : q) : 0;
#pragma unroll 8
        for (int k = 0; k < kRankKeys; ++k) {
            const int64_t f = kf[k];
            const int32_t tag = kt[k];
            const int32_t c = __popcll(__ballot(in && (g < f || (g == f && gt < tag))));
            mine += lane == k ? c : 0;
        }
    }
    if (mine) atomicAdd(&kc[lane], mine);
    __syncthreads();
    const int32_t t = k0 + threadIdx.x;
    if (threadIdx.x >= kRankKeys || t >= total) return;
    const int64_t f = kf[threadIdx.x];
    int32_t p = kc[threadIdx.x], tag;
    if (t < r.npar) {
        p += t;
        tag = t;
    } else {
        int32_t lo = 0, hi = r.npar;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (r.f_par[mid] <= f) lo = mid + 1;
            else hi = mid;
        }
        p += lo;
        tag = r.npar + kt[threadIdx.x];
    }
    if (p < I.P) {
        a.src[I.fit_off + p] = tag;
        a.f_out[I.fit_off + p] = f;
    }
}

// Row r of the next population from its source tag; after generation 0 the
// first block also advances the device generation counter (every reader of
// it in this generation has finished: stream order).
__global__ void k_gather_rows(const GaInst *__restrict__ inst, const int32_t *__restrict__ src, int32_t init,
                              const int32_t *__restrict__ parents, const int32_t *__restrict__ children,
                              int32_t *__restrict__ out, uint32_t *__restrict__ gen_ctr)
{
    const GaInst &I = inst[blockIdx.y];
    const int32_t r = blockIdx.x;
    if (!init && r == 0 && blockIdx.y == 0 && threadIdx.x == 0) gen_ctr[0] += 1u;
    if (r >= I.P) return;
    const int32_t npar = init ? 0 : I.P;
    const int32_t tag = src[I.fit_off + r];
    const int32_t k = I.k;
    const int32_t *s = tag < npar ? parents + I.pop_off + (int64_t)tag * k
                                  : children + I.child_off + (int64_t)(tag - npar) * k;
    int32_t *d = out + I.pop_off + (int64_t)r * k;
    for (int32_t j = threadIdx.x; j < k; j += blockDim.x) d[j] = s[j];
}

OpArgs make_args(gapa_ga *ga, const int32_t *pop, const int64_t *fit)
{
    OpArgs a;
    a.inst = ga->inst.as<GaInst>();
    a.pop = pop;
    a.fit = fit;
    a.noniso = ga->noniso ? ga->noniso : ga->graph->d_noniso;
    a.children = ga->children.as<int32_t>();
    a.masks = ga->masks.as<uint32_t>();
    a.alive = ga->alive.as<int32_t>();
    a.flag = ga->flag.as<int32_t>();
    a.gen_ctr = ga->gen_ctr.as<uint32_t>();
    a.rows_only = 0;
    return a;
}

}  // namespace

int ga_rank_and_gather(gapa_ga *ga, bool init, const int64_t *f_pool, const int32_t *pool, int32_t npool,
                       hipStream_t s)
{
    const int nxt = init ? ga->cur : 1 - ga->cur;
    const int32_t count = ga->count;
    RankArgs a;
    a.inst = ga->inst.as<GaInst>();
    a.f_par = ga->fit[ga->cur].as<int64_t>();
    a.f_pool = f_pool;
    a.pool = pool;
    a.npool = npool;
    a.init = init ? 1 : 0;
    a.src = ga->src.as<int32_t>();
    a.f_out = ga->fit[nxt].as<int64_t>();
    // launch extents: the largest instance
    const int32_t max_total = init ? ga->max_pop : (pool ? ga->max_pop + npool : ga->max_pop_lambda);
    TimedScope pass(&ga->timer, "elitism", s, 1);
    {
        TimedScope ts(&ga->timer, "elitism_rank", s);
        hipLaunchKernelGGL(k_rank_place, dim3((max_total + kRankKeys - 1) / kRankKeys, count), dim3(64 * kRankWaves),
                           0, s, a);
    }
    {
        TimedScope ts(&ga->timer, "gather_rows", s);
        hipLaunchKernelGGL(k_gather_rows, dim3(ga->max_pop, count), dim3(256), 0, s, ga->inst.as<GaInst>(),
                           ga->src.as<int32_t>(), a.init, ga->pop[ga->cur].as<int32_t>(), ga->children.as<int32_t>(),
                           ga->pop[nxt].as<int32_t>(), ga->gen_ctr.as<uint32_t>());
    }
    GAPA_HIP(hipGetLastError());
    ga->cur = nxt;
    return GAPA_OK;
}

size_t ga_op_lds_bytes(int32_t n, int32_t k)
{
    const size_t W = ((size_t)n + 31) / 32;
    const size_t KW = ((size_t)k + 31) / 32;
    return 4 * (W + (size_t)k + 3 * KW) + 2 * (((size_t)k + 1) & ~(size_t)1);
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
    OpArgs a = make_args(ga, nullptr, nullptr);
    TimedScope ts(&ga->timer, "ga_init", s, 1);
    hipLaunchKernelGGL(k_init, dim3(ga->max_pop, ga->count), dim3(kOpBlock), ga->op_lds_bytes, s, a);
    GAPA_HIP(hipGetLastError());
    return GAPA_OK;
}

int ga_launch_offspring(gapa_ga *ga, hipStream_t s, bool rows_only)
{
    OpArgs a = make_args(ga, ga->pop[ga->cur].as<int32_t>(), ga->fit[ga->cur].as<int64_t>());
    a.rows_only = rows_only ? 1 : 0;
    TimedScope ts(&ga->timer, "ga_offspring", s, 1);
    hipLaunchKernelGGL(k_offspring, dim3(ga->max_lambda, ga->count), dim3(kOpBlock), ga->op_lds_bytes, s, a);
    GAPA_HIP(hipGetLastError());
    return GAPA_OK;
}

int ga_eval_children(gapa_ga *ga, bool init, hipStream_t s)
{
    int32_t *mcn = ga->objective_mcn ? ga->child_mcn.as<int32_t>() : nullptr;
    const Measure measure = ga->objective_forest ? kMeasureForest : kMeasurePC;
    int rc;
    if (ga->count > 1)
        rc = eval_masks(ga->graph, ga->masks.as<uint32_t>(), ga->alive.as<int32_t>(), 0, ga->child_fit.as<int64_t>(),
                        mcn, ga->ws, &ga->timer, s, init ? &ga->tab_init : &ga->tab_gen, measure);
    else
        rc = eval_masks(ga->graph, ga->masks.as<uint32_t>(), ga->alive.as<int32_t>(),
                        init ? ga->params.pop : ga->lambda, ga->child_fit.as<int64_t>(), mcn, ga->ws, &ga->timer, s,
                        nullptr, measure);
    if (rc != GAPA_OK || !mcn) return rc;
    // the objective is MCN: it replaces PC as the fitness of every slot
    hipLaunchKernelGGL(k_mcn_objective, dim3((ga->slots + 255) / 256), dim3(256), 0, s, mcn,
                       ga->child_fit.as<int64_t>(), ga->slots);
    GAPA_HIP(hipGetLastError());
    return GAPA_OK;
}

int ga_init_population(gapa_ga *ga, hipStream_t s)
{
    int rc = launch_fill_u32(ga->gen_ctr.ptr, 0u, 1, s);
    if (rc == GAPA_OK) rc = ga_launch_init(ga, s);
    if (rc == GAPA_OK) rc = ga_eval_children(ga, true, s);
    if (rc == GAPA_OK) rc = ga_rank_and_gather(ga, true, ga->child_fit.as<int64_t>(), nullptr, 0, s);
    return rc;
}

int ga_generation(gapa_ga *ga, hipStream_t s)
{
    int rc = ga_launch_offspring(ga, s);
    if (rc == GAPA_OK) rc = ga_eval_children(ga, false, s);
    if (rc == GAPA_OK) rc = ga_rank_and_gather(ga, false, ga->child_fit.as<int64_t>(), nullptr, 0, s);
    if (rc != GAPA_OK) return rc;
    ga->generation += 1;
    return GAPA_OK;
}

}  // namespace gapa
