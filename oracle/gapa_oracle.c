/*
 * CPU oracle for GA-based critical node detection (CND).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link
 * or call this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code with the HIP path.
 *
 * What it computes, in plain and slow form:
 *
 *  - pairwise connectivity PC(S) = sum over connected components C of G - S of
 *    |C|(|C|-1)/2, as int64, and the largest component size MCN.  Removing a
 *    node removes all of its incident edges (Section III-C, the perturbation
 *    update over the adjacency matrix); PC(G) is the CND quality measure of
 *    Section IV-C and Table III, read as unordered pairs of still-connected
 *    nodes.  Two independent routes: breadth-first search (primary) and
 *    union-find by size with path halving (cross-check).
 *
 *  - the genetic algorithm of Section III-B on a population of k-node removal
 *    sets: random initialisation (eq. 2), per-gene crossover mask (eq. 3-4)
 *    with a tournament-selected partner (replacing the roulette wheel of
 *    eq. 5) blended as in eq. 6, per-gene mutation mask (eq. 7-8) with
 *    replacement genes as in eq. 9, and elitism over parents and offspring
 *    (eq. 10-11), minimising PC.  Where the paper is silent (duplicate genes,
 *    distribution of replacement genes, tie-breaks) the reading used here is
 *    the one written next to each step below.
 *
 *  - the Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
 *    "Parallel Random Numbers: As Easy as 1, 2, 3", SC 2011) keyed by
 *    (seed, generation, individual, slot), the only source of randomness.
 *
 * Parity status: PC/MCN are pinned by closed forms, library connected
 * components, the paper's reachability identity eq. 17 and brute force.
 * Philox is pinned by rocRAND's independent implementation.  The GA trajectory
 * is defined by the readings written here (the paper fixes no random stream);
 * it is pinned by invariants and special cases, not by printed values.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10                                                            */
/* ------------------------------------------------------------------------ */

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

/* One round: two 32x32->64 products; the outputs swap and mix with the other
 * two counter words and the round key (SC'11, Section 4). */
static void philox_round(uint32_t c[4], const uint32_t key[2])
{
    uint64_t p0 = (uint64_t)PHILOX_M0 * c[0];
    uint64_t p1 = (uint64_t)PHILOX_M1 * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t r0 = hi1 ^ c[1] ^ key[0];
    uint32_t r1 = lo1;
    uint32_t r2 = hi0 ^ c[3] ^ key[1];
    uint32_t r3 = lo0;
    c[0] = r0; c[1] = r1; c[2] = r2; c[3] = r3;
}

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        philox_round(c, k);
        k[0] += PHILOX_W0;   /* Weyl key schedule between rounds */
        k[1] += PHILOX_W1;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* Random streams: one per kind of decision, in the top byte of counter word 3;
 * the low 24 bits of that word count rejection attempts. */
enum { ST_INIT = 0, ST_SELECT = 1, ST_XOVER = 2, ST_REPAIR = 3, ST_MUTATE = 4 };
#define MAX_ATTEMPTS (1u << 24)

/* counter = (slot, individual, generation, stream<<24 | attempt),
 * key = (seed low word, seed high word). */
static void draw(uint64_t seed, uint32_t slot, uint32_t ind, uint32_t gen,
                 uint32_t stream, uint32_t attempt, uint32_t out[4])
{
    uint32_t ctr[4] = {slot, ind, gen, (stream << 24) | attempt};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

void oracle_draw(uint64_t seed, uint32_t slot, uint32_t ind, uint32_t gen,
                 uint32_t stream, uint32_t attempt, uint32_t out[4])
{
    draw(seed, slot, ind, gen, stream, attempt, out);
}

/* Learned-screening extension (not in the paper): initial weights.  Element
 * (r, c) of parameter tensor t is bound * (2u - 1) with u = (w + 1/2) / 2^32,
 * w the first word of the draw (slot c, individual r, generation t, stream
 * SURR_INIT = 5): a uniform value in (-bound, bound), computed in double. */
void oracle_uniform_sym(uint64_t seed, uint32_t tensor, int64_t rows, int32_t cols, double bound, double *out)
{
    for (int64_t r = 0; r < rows; ++r)
        for (int32_t c = 0; c < cols; ++c) {
            uint32_t w[4];
            draw(seed, (uint32_t)c, (uint32_t)r, tensor, 5u, 0u, w);
            const double u = ((double)w[0] + 0.5) * (1.0 / 4294967296.0);
            out[r * cols + c] = bound * (2.0 * u - 1.0);
        }
}

/* Integer in [0, m): the high word of w*m (multiply-shift, no rejection). */
uint32_t oracle_bounded(uint32_t w, uint32_t m)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)m) >> 32);
}

/* Bernoulli(p) is decided as w < floor(p * 2^32) on the 32-bit word w; the
 * threshold is an exact integer (p = 1 gives 2^32, always true). */
uint64_t oracle_threshold(double p)
{
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return 1ull << 32;
    return (uint64_t)(p * 4294967296.0);   /* scaling by 2^32 is exact */
}

/* ------------------------------------------------------------------------ */
/* Pairwise connectivity                                                    */
/* ------------------------------------------------------------------------ */

/* PC and MCN of G - S by breadth-first search from every unvisited survivor.
 * genes: k node ids (any order; repeated ids are one removal).
 * Returns -1 if a gene is out of range. */
int64_t oracle_pc_bfs(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                      const int32_t *genes, int32_t k, int32_t *mcn_out)
{
    uint8_t *removed = (uint8_t *)calloc((size_t)n, 1);
    uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int64_t pc = 0;
    int32_t mcn = 0;
    for (int32_t j = 0; j < k; ++j) {
        if (genes[j] < 0 || genes[j] >= n) { pc = -1; goto done; }
        removed[genes[j]] = 1;
    }
    for (int32_t s = 0; s < n; ++s) {
        if (removed[s] || seen[s]) continue;
        int32_t head = 0, tail = 0;
        queue[tail++] = s;
        seen[s] = 1;
        while (head < tail) {
            int32_t v = queue[head++];
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                int32_t u = col_idx[e];
                if (!removed[u] && !seen[u]) {
                    seen[u] = 1;
                    queue[tail++] = u;
                }
            }
        }
        int64_t size = tail;                 /* component of s */
        pc += size * (size - 1) / 2;
        if (size > mcn) mcn = (int32_t)size;
    }
done:
    if (mcn_out) *mcn_out = mcn;
    free(removed); free(seen); free(queue);
    return pc;
}

/* Number of connected components of G - S (every surviving node, isolated
 * ones included, lies in exactly one), by breadth-first search from every
 * unvisited survivor; *survivors_out receives |V minus S|.  genes: k node ids
 * (repeated ids are one removal).  Returns -1 if a gene is out of range. */
int64_t oracle_components(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                          const int32_t *genes, int32_t k, int32_t *survivors_out)
{
    uint8_t *removed = (uint8_t *)calloc((size_t)n, 1);
    uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int64_t count = 0;
    int32_t survivors = n;
    for (int32_t j = 0; j < k; ++j) {
        if (genes[j] < 0 || genes[j] >= n) { count = -1; goto done; }
        if (!removed[genes[j]]) --survivors;
        removed[genes[j]] = 1;
    }
    for (int32_t s = 0; s < n; ++s) {
        if (removed[s] || seen[s]) continue;
        int32_t head = 0, tail = 0;
        queue[tail++] = s;
        seen[s] = 1;
        while (head < tail) {
            int32_t v = queue[head++];
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                int32_t u = col_idx[e];
                if (!removed[u] && !seen[u]) {
                    seen[u] = 1;
                    queue[tail++] = u;
                }
            }
        }
        ++count;
    }
done:
    if (survivors_out) *survivors_out = survivors;
    free(removed); free(seen); free(queue);
    return count;
}

static int32_t uf_find(int32_t *parent, int32_t x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];      /* path halving */
        x = parent[x];
    }
    return x;
}

/* Same quantity by union-find over the surviving edges (cross-check). */
int64_t oracle_pc_unionfind(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                            const int32_t *genes, int32_t k, int32_t *mcn_out)
{
    uint8_t *removed = (uint8_t *)calloc((size_t)n, 1);
    int32_t *parent = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int64_t *size = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int64_t pc = 0;
    int32_t mcn = 0;
    for (int32_t j = 0; j < k; ++j) {
        if (genes[j] < 0 || genes[j] >= n) { pc = -1; goto done; }
        removed[genes[j]] = 1;
    }
    for (int32_t v = 0; v < n; ++v) { parent[v] = v; size[v] = 1; }
    for (int32_t v = 0; v < n; ++v) {
        if (removed[v]) continue;
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int32_t u = col_idx[e];
            if (u <= v || removed[u]) continue;
            int32_t a = uf_find(parent, v), b = uf_find(parent, u);
            if (a == b) continue;
            if (size[a] < size[b]) { int32_t t = a; a = b; b = t; }
            parent[b] = a;
            size[a] += size[b];
        }
    }
    for (int32_t v = 0; v < n; ++v) {
        if (removed[v] || parent[v] != v) continue;
        pc += size[v] * (size[v] - 1) / 2;
        if (size[v] > mcn) mcn = (int32_t)size[v];
    }
done:
    if (mcn_out) *mcn_out = mcn;
    free(removed); free(parent); free(size);
    return pc;
}

/* PC of every row of a P x k gene matrix.  Rows are independent; OpenMP
 * spreads them over host threads when nthreads > 1.  Returns 0, or the index
 * + 1 of the first row holding an out-of-range gene. */
int64_t oracle_eval_population(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                               const int32_t *genes, int32_t P, int32_t k,
                               int64_t *fitness, int32_t *mcn, int32_t nthreads)
{
    int64_t bad = 0;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(max : bad)
#endif
    for (int32_t i = 0; i < P; ++i) {
        int32_t m = 0;
        int64_t f = oracle_pc_bfs(n, row_ptr, col_idx, genes + (int64_t)i * k, k, &m);
        fitness[i] = f;
        if (mcn) mcn[i] = m;
        if (f < 0 && (int64_t)i + 1 > bad) bad = (int64_t)i + 1;
    }
    (void)nthreads;
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Genetic operators                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n;          /* nodes */
    int32_t k;          /* budget: genes per individual */
    int32_t pop;        /* P: parents kept by elitism */
    int32_t offspring;  /* lambda: children made per generation */
    int32_t tournament; /* T: contestants per tournament */
    int32_t objective;  /* 0: minimise PC; 1: minimise MCN (the CND fitness of Sec. III-D);
                           2: maximise the number of components NC, as minimising
                           |V minus S| - NC */
    uint64_t seed;
    uint64_t t_pc;      /* crossover threshold, floor(pc * 2^32) */
    uint64_t t_pm;      /* mutation threshold, floor(pm * 2^32) */
} oracle_params;

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Uniform node outside `member` (a byte per node): attempt t draws from
 * (slot, ind, gen, stream | t) until it hits a non-member.  Returns -1 when
 * the attempt counter is exhausted. */
static int32_t draw_non_member(const oracle_params *p, const uint8_t *member,
                               uint32_t slot, uint32_t ind, uint32_t gen, uint32_t stream)
{
    for (uint32_t t = 0; t < MAX_ATTEMPTS; ++t) {
        uint32_t w[4];
        draw(p->seed, slot, ind, gen, stream, t, w);
        uint32_t u = oracle_bounded(w[0], (uint32_t)p->n);
        if (!member[u]) return (int32_t)u;
    }
    return -1;
}

/* Initial individual i (eq. 2): slot j takes the first uniform draw
 * (INIT stream, attempts t = 0, 1, ...) that is not already in the row.
 * The row is then sorted ascending.  Returns 0 or -1. */
int oracle_init_individual(const oracle_params *p, int32_t i, int32_t *row)
{
    uint8_t *member = (uint8_t *)calloc((size_t)p->n, 1);
    int rc = 0;
    for (int32_t j = 0; j < p->k; ++j) {
        int32_t u = draw_non_member(p, member, (uint32_t)j, (uint32_t)i, 0, ST_INIT);
        if (u < 0) { rc = -1; break; }
        row[j] = u;
        member[u] = 1;
    }
    free(member);
    if (rc == 0) qsort(row, (size_t)p->k, sizeof(int32_t), cmp_i32);
    return rc;
}

/* (F, tag) order: smaller pairwise connectivity first, ties by tag. */
static int better_or_equal(int64_t fa, int64_t ta, int64_t fb, int64_t tb)
{
    return fa < fb || (fa == fb && ta <= tb);
}

/* Tournament (replacing the roulette wheel of eq. 5): T contestants drawn
 * uniformly with replacement, contestant c from word c mod 4 of draw
 * (slot c / 4, offspring o, generation g, SELECT); the winner has the smallest
 * (F, position). */
int32_t oracle_tournament(const oracle_params *p, int32_t gen, int32_t o, const int64_t *F)
{
    int32_t best = -1;
    uint32_t w[4];
    for (int32_t c = 0; c < p->tournament; ++c) {
        if (c % 4 == 0) draw(p->seed, (uint32_t)(c / 4), (uint32_t)o, (uint32_t)gen, ST_SELECT, 0, w);
        int32_t a = (int32_t)oracle_bounded(w[c % 4], (uint32_t)p->pop);
        if (best < 0 || !better_or_equal(F[best], best, F[a], a)) best = a;
    }
    return best;
}

/* Offspring o of generation g >= 1, from the current population (rows sorted,
 * population ordered by (F, tag)).  Steps:
 *  1. base = POP[o mod P]; donor = tournament winner.
 *  2. crossover, eq. 6: gene j comes from the donor where the crossover mask
 *     TC_j = [w0 < T_pc] (eq. 4) is 1, else from the base; w0 is word 0 of
 *     draw (j, o, g, XOVER).
 *  3. repair (not in the paper: eq. 6 can repeat a node id): a slot holding a
 *     value already seen at a lower slot gets a uniform non-member (REPAIR
 *     stream, attempts), slots in ascending order.
 *  4. mutation, eq. 9: where TM_j = [w1 < T_pm] (eq. 8; w1 is word 1 of the
 *     same XOVER draw), slots ascending, the gene is replaced by a uniform
 *     node not currently in the row (MUTATE stream, attempts).
 *  5. the row is sorted ascending.
 * pre_repair (optional, k ints) receives the row after step 2, and
 * pre_mutation after step 3, both unsorted.  Returns 0 or -1. */
int oracle_make_child(const oracle_params *p, int32_t gen, int32_t o,
                      const int32_t *pop_rows, const int64_t *F, int32_t *child,
                      int32_t *pre_repair, int32_t *pre_mutation, int32_t *donor_out)
{
    const int32_t k = p->k;
    const int32_t *base = pop_rows + (int64_t)(o % p->pop) * k;
    int32_t d = oracle_tournament(p, gen, o, F);
    const int32_t *donor = pop_rows + (int64_t)d * k;
    if (donor_out) *donor_out = d;
    uint8_t *mutate = (uint8_t *)malloc((size_t)k);
    uint8_t *member = (uint8_t *)calloc((size_t)p->n, 1);
    int rc = 0;

    for (int32_t j = 0; j < k; ++j) {
        uint32_t w[4];
        draw(p->seed, (uint32_t)j, (uint32_t)o, (uint32_t)gen, ST_XOVER, 0, w);
        child[j] = ((uint64_t)w[0] < p->t_pc) ? donor[j] : base[j];
        mutate[j] = (uint64_t)w[1] < p->t_pm;
    }
    if (pre_repair) memcpy(pre_repair, child, (size_t)k * sizeof(int32_t));

    /* membership of the distinct values; later copies are duplicates */
    uint8_t *dup = (uint8_t *)calloc((size_t)k, 1);
    for (int32_t j = 0; j < k; ++j) {
        if (member[child[j]]) dup[j] = 1;
        else member[child[j]] = 1;
    }
    for (int32_t j = 0; j < k && rc == 0; ++j) {
        if (!dup[j]) continue;
        int32_t u = draw_non_member(p, member, (uint32_t)j, (uint32_t)o, (uint32_t)gen, ST_REPAIR);
        if (u < 0) { rc = -1; break; }
        child[j] = u;
        member[u] = 1;
    }
    free(dup);
    if (pre_mutation) memcpy(pre_mutation, child, (size_t)k * sizeof(int32_t));

    for (int32_t j = 0; j < k && rc == 0; ++j) {
        if (!mutate[j]) continue;
        int32_t u = draw_non_member(p, member, (uint32_t)j, (uint32_t)o, (uint32_t)gen, ST_MUTATE);
        if (u < 0) { rc = -1; break; }
        member[child[j]] = 0;
        member[u] = 1;
        child[j] = u;
    }
    free(mutate);
    free(member);
    if (rc == 0) qsort(child, (size_t)k, sizeof(int32_t), cmp_i32);
    return rc;
}

typedef struct {
    int64_t f;
    int64_t tag;
} fkey;

static int cmp_fkey(const void *a, const void *b)
{
    const fkey *x = (const fkey *)a, *y = (const fkey *)b;
    if (x->f != y->f) return (x->f > y->f) - (x->f < y->f);
    return (x->tag > y->tag) - (x->tag < y->tag);
}

/* The GA's fitness of P rows: PC; with objective 1 the largest surviving
 * component (MCN); with objective 2 the survivors minus the number of
 * components (smallest when G - S falls into the most pieces). */
static int eval_objective(const oracle_params *p, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                          const int32_t *rows, int32_t P, int32_t k, int64_t *f, int32_t nthreads)
{
    if (p->objective == 2) {
        int bad = 0;
        for (int32_t i = 0; i < P; ++i) {
            int32_t alive = 0;
            const int64_t nc = oracle_components(n, row_ptr, col_idx, rows + (int64_t)i * k, k, &alive);
            if (nc < 0) bad = 1;
            f[i] = alive - nc;
        }
        (void)nthreads;
        return bad ? -1 : 0;
    }
    if (p->objective != 1) return oracle_eval_population(n, row_ptr, col_idx, rows, P, k, f, NULL, nthreads);
    int32_t *mcn = (int32_t *)malloc((size_t)(P > 0 ? P : 1) * sizeof(int32_t));
    if (!mcn) return -1;
    const int rc = oracle_eval_population(n, row_ptr, col_idx, rows, P, k, f, mcn, nthreads);
    for (int32_t i = 0; i < P; ++i) f[i] = mcn[i];
    free(mcn);
    return rc;
}

/* Population at generation 0: P initial rows, evaluated, ordered by (F, i). */
int oracle_ga_init(const oracle_params *p, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                   int32_t *pop_rows, int64_t *F, int32_t nthreads)
{
    const int32_t P = p->pop, k = p->k;
    int32_t *rows = (int32_t *)calloc((size_t)P * k, sizeof(int32_t));
    int64_t *f = (int64_t *)malloc((size_t)P * sizeof(int64_t));
    fkey *keys = (fkey *)malloc((size_t)P * sizeof(fkey));
    int rc = 0;
    for (int32_t i = 0; i < P && rc == 0; ++i)
        rc = oracle_init_individual(p, i, rows + (int64_t)i * k);
    if (rc == 0 && eval_objective(p, n, row_ptr, col_idx, rows, P, k, f, nthreads) != 0) rc = -1;
    if (rc == 0) {
        for (int32_t i = 0; i < P; ++i) { keys[i].f = f[i]; keys[i].tag = i; }
        qsort(keys, (size_t)P, sizeof(fkey), cmp_fkey);
        for (int32_t r = 0; r < P; ++r) {
            memcpy(pop_rows + (int64_t)r * k, rows + keys[r].tag * k, (size_t)k * sizeof(int32_t));
            F[r] = keys[r].f;
        }
    }
    free(rows); free(f); free(keys);
    return rc;
}

/* One generation g >= 1 (eq. 3-11): lambda offspring, each evaluated, then
 * elitism keeps the P smallest (F, tag) of parents (tags 0..P-1, in their
 * current order) and pooled offspring (tag P + o).  The paper's elitism text
 * sorts descending and keeps one half "if the algorithm requires high
 * fitness"; CND minimises PC, so the lower half is kept.
 *
 * pool_idx (optional, n_pool entries, ascending offspring indices) restricts
 * which offspring are evaluated and pooled (all lambda when NULL).
 * children/child_F (optional) receive the lambda offspring rows and their
 * fitness (-1 for offspring outside the pool).  Returns 0 or -1. */
int oracle_ga_step(const oracle_params *p, int32_t gen, int32_t n, const int32_t *row_ptr,
                   const int32_t *col_idx, int32_t *pop_rows, int64_t *F,
                   const int32_t *pool_idx, int32_t n_pool,
                   int32_t *children, int64_t *child_F, int32_t nthreads)
{
    const int32_t P = p->pop, k = p->k, L = p->offspring;
    int32_t *kids = (int32_t *)malloc((size_t)L * k * sizeof(int32_t));
    int64_t *kf = (int64_t *)malloc((size_t)L * sizeof(int64_t));
    int32_t *pooled = (int32_t *)malloc((size_t)L * sizeof(int32_t));
    fkey *keys = (fkey *)malloc((size_t)(P + L) * sizeof(fkey));
    int32_t *next = (int32_t *)malloc((size_t)P * k * sizeof(int32_t));
    int64_t *nextF = (int64_t *)malloc((size_t)P * sizeof(int64_t));
    int rc = 0;

    for (int32_t o = 0; o < L && rc == 0; ++o)
        rc = oracle_make_child(p, gen, o, pop_rows, F, kids + (int64_t)o * k, NULL, NULL, NULL);

    int32_t np = 0;
    if (pool_idx) {
        for (int32_t q = 0; q < n_pool; ++q) pooled[np++] = pool_idx[q];
    } else {
        for (int32_t o = 0; o < L; ++o) pooled[np++] = o;
    }
    for (int32_t o = 0; o < L; ++o) kf[o] = -1;
    if (rc == 0) {
        int32_t *rows = (int32_t *)malloc((size_t)(np > 0 ? np : 1) * k * sizeof(int32_t));
        int64_t *f = (int64_t *)malloc((size_t)(np > 0 ? np : 1) * sizeof(int64_t));
        for (int32_t q = 0; q < np; ++q)
            memcpy(rows + (int64_t)q * k, kids + (int64_t)pooled[q] * k, (size_t)k * sizeof(int32_t));
        if (eval_objective(p, n, row_ptr, col_idx, rows, np, k, f, nthreads) != 0) rc = -1;
        for (int32_t q = 0; q < np; ++q) kf[pooled[q]] = f[q];
        free(rows); free(f);
    }
    if (rc == 0) {
        int32_t nk = 0;
        for (int32_t r = 0; r < P; ++r) { keys[nk].f = F[r]; keys[nk].tag = r; ++nk; }
        for (int32_t q = 0; q < np; ++q) { keys[nk].f = kf[pooled[q]]; keys[nk].tag = (int64_t)P + pooled[q]; ++nk; }
        qsort(keys, (size_t)nk, sizeof(fkey), cmp_fkey);
        for (int32_t r = 0; r < P; ++r) {
            int64_t t = keys[r].tag;
            const int32_t *src = t < P ? pop_rows + t * k : kids + (t - P) * k;
            memcpy(next + (int64_t)r * k, src, (size_t)k * sizeof(int32_t));
            nextF[r] = keys[r].f;
        }
        memcpy(pop_rows, next, (size_t)P * k * sizeof(int32_t));
        memcpy(F, nextF, (size_t)P * sizeof(int64_t));
    }
    if (children) memcpy(children, kids, (size_t)L * k * sizeof(int32_t));
    if (child_F) memcpy(child_F, kf, (size_t)L * sizeof(int64_t));
    free(kids); free(kf); free(pooled); free(keys); free(next); free(nextF);
    return rc;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
