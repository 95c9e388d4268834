/*
 * gapa.h -- C ABI of the MI355X population-fitness engine for GA-based
 * critical node detection (CND), the perturbed-substructure-optimisation
 * problem of "Efficient Parallel Genetic Algorithm for Perturbed Substructure
 * Optimization in Complex Network" (Section III).
 *
 * The library evaluates and evolves populations of k-node removal sets S over
 * one undirected, unweighted graph G = (V, E) (Section III-A).  The fitness of
 * an individual is the pairwise connectivity of G - S,
 *
 *     PC(S) = sum over connected components C of G - S of |C| (|C| - 1) / 2,
 *
 * the CND measure PC(G) of Section IV-C / Table III, which the GA minimises
 * under the budget |S| = k (the cost constraint C(p) of eq. 1).  Removing a
 * node removes all of its edges (Section III-C, eq. 13).  PC is computed
 * exactly (the components of G - S), not with the six-hop truncation of
 * eq. 15; MCN is the size of the largest component.
 *
 * Conventions for every entry point
 *   - Return value: GAPA_OK or a gapa_status code; the message of the last
 *     failure on the calling thread is gapa_last_error().  No C++ exception
 *     crosses the ABI.  Outputs are unspecified when a call fails.
 *   - Ownership: input arrays are borrowed for the duration of the call (and
 *     copied where kept); outputs are caller-allocated; handles are owned by
 *     the library until their *_destroy call.  *_destroy(NULL) is GAPA_OK.
 *   - Devices and streams: a handle lives on the HIP device that was current
 *     when it was created.  `stream` is a hipStream_t (NULL: the device's null
 *     stream).  Host-pointer calls return after their results are on the
 *     host; GAPA_DEVICE_PTRS calls only enqueue work on `stream`.
 *   - A device error (GAPA_E_DEVICE) is sticky on the handle it happened on:
 *     destroy the handle.
 *   - Threading: calls on one handle must not overlap; distinct handles may be
 *     used from distinct threads.
 *   - Results never depend on the stream, the launch geometry or how the
 *     population is split into chunks.
 */
#ifndef GAPA_H
#define GAPA_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define GAPA_API __attribute__((visibility("default")))
#else
#define GAPA_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gapa_graph gapa_graph;
typedef struct gapa_ga gapa_ga;
typedef struct gapa_batch gapa_batch;

typedef enum gapa_status {
    GAPA_OK = 0,
    GAPA_E_INVALID_ARG = 1, /* a size, pointer or parameter is out of range     */
    GAPA_E_BAD_GRAPH = 2,   /* the CSR is not a symmetric simple sorted graph   */
    GAPA_E_BAD_GENE = 3,    /* a gene is not a node id in [0, n)                */
    GAPA_E_NO_DEVICE = 4,   /* no usable HIP device                             */
    GAPA_E_DEVICE = 5,      /* a HIP call or kernel failed (sticky)             */
    GAPA_E_OOM = 6,         /* device or host allocation failed                 */
    GAPA_E_STATE = 7        /* the handle is unusable (earlier failure, or a
                               random draw exhausted its 2^24 attempts)          */
} gapa_status;

enum {
    GAPA_DEVICE_PTRS = 1u << 0, /* genes/fitness/mcn are device pointers; the call
                                   is asynchronous on `stream`                  */
    GAPA_TRUST_INPUT = 1u << 1, /* skip host-side validation                    */
    GAPA_WANT_MCN = 1u << 2,    /* also compute the largest component size      */
    GAPA_UNIONFIND = 1u << 3,   /* gapa_graph_create: evaluate with edge-parallel
                                   union-find instead of bit-parallel sweeps
                                   (same results, slower; a cross-check)        */
    GAPA_GRAPH_REPLAY = 1u << 4, /* gapa_params.flags: record one generation's
                                   launches as a HIP graph once and replay it
                                   (same results; fewer launch gaps).  Kernel
                                   timing, when enabled, runs generations
                                   eagerly instead.                             */
    GAPA_MINIMISE_MCN = 1u << 5, /* gapa_params.flags: the GA minimises the
                                   largest surviving component (MCN, the CND
                                   fitness of Section III-D) instead of PC: the
                                   fitness arrays then hold MCN.  Not with a
                                   surrogate.                                   */
    GAPA_MAXIMISE_COMPONENTS = 1u << 6 /* gapa_params.flags, and the flags of
                                   gapa_eval_population: the objective is the
                                   number NC of connected components of G - S,
                                   read off the same partition as PC and MCN
                                   (an extension; the paper reports PC and MCN).
                                   Fitness values then hold |V minus S| - NC =
                                   sum over components of (|C| - 1), the size
                                   of a spanning forest of G - S, which the GA
                                   minimises (most components first).  Not with
                                   GAPA_MINIMISE_MCN nor a surrogate.           */
};

/* ---------------------------------------------------------------------------
 * Graph (Section III-A: undirected, unweighted G = (V, E), |V| = n).
 *
 * row_ptr: int32 [n + 1], col_idx: int32 [nnz], host memory, the symmetric
 * CSR of G: every undirected edge {u, v} appears as v in row u and u in row v;
 * neighbour lists strictly ascending (no repeated edges), no self-loops,
 * row_ptr[0] = 0, row_ptr[n] = nnz.  Both arrays are copied to the device.
 * Validation (skipped with GAPA_TRUST_INPUT) fails with GAPA_E_BAD_GRAPH.
 * Limits: 1 <= n <= 2^30, 0 <= nnz < 2^31.
 * ------------------------------------------------------------------------- */
GAPA_API int gapa_graph_create(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                      uint32_t flags, gapa_graph **out);
/* Releases the caller's handle.  GAs and batches created on the graph hold
 * their own references: its device memory is freed once the last of them is
 * destroyed too, so handles may be destroyed in any order.  NULL is OK. */
GAPA_API int gapa_graph_destroy(gapa_graph *g);

/* ---------------------------------------------------------------------------
 * Batched fitness (Section III-C, eq. 13: the perturbation of a whole
 * population applied to G at once, then evaluated).
 *
 * genes:   int32 [P][k] row-major node ids, any order within a row; a repeated
 *          id in a row is one removal (set semantics).
 * fitness: int64 [P] out, PC of each row (with GAPA_MAXIMISE_COMPONENTS:
 *          the row's survivors minus the components of G - S).
 * mcn:     int32 [P] out or NULL; written only with GAPA_WANT_MCN.
 * An id outside [0, n) gives GAPA_E_BAD_GENE (with GAPA_DEVICE_PTRS the check
 * runs on the device and the call waits for it unless GAPA_TRUST_INPUT).
 * P >= 0 (P = 0 is a no-op), 0 <= k <= n.
 * ------------------------------------------------------------------------- */
GAPA_API int gapa_eval_population(gapa_graph *g, const int32_t *genes, int32_t P, int32_t k,
                         int64_t *fitness, int32_t *mcn, uint32_t flags, void *stream);

/* ---------------------------------------------------------------------------
 * Batched fitness that allocates nothing, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, results and gene semantics as
 * gapa_eval_population with GAPA_DEVICE_PTRS, which `flags` must include
 * (besides it only GAPA_TRUST_INPUT, GAPA_WANT_MCN and
 * GAPA_MAXIMISE_COMPONENTS): genes, fitness and mcn are device pointers and
 * the call enqueues its work on `stream`; without GAPA_TRUST_INPUT it waits
 * for the device's gene check (pass GAPA_TRUST_INPUT under graph capture).
 * The graph's bit-parallel algorithm is used whatever it was created with.
 *
 * Every buffer the evaluation needs comes from a fixed scratch array of
 * GAPA_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * from the library's load to the end of the process.  The population is
 * evaluated in chunks of 32 Wd individuals, Wd the largest power of two <= 32
 * whose buffers fit: about 32 Wd (8.25 n + 8 n_noniso + 4 W + 4 sweep_grid)
 * bytes for n nodes, n_noniso of them with an edge, W = ceil(n / 32) and the
 * graph's sweep_grid (gapa_tuning); a graph on which not even 32 individuals
 * fit (n above about 250 000 at the default launch shapes) gives
 * GAPA_E_INVALID_ARG before any work is enqueued.  All calls on one GPU
 * share its scratch, which keeps the last call's contents (each call clears
 * what must start at zero): calls that overlap on one GPU (several streams or
 * host threads at once) race and must be serialised by the caller.
 * ------------------------------------------------------------------------- */
#define GAPA_NOALLOC_SCRATCH_BYTES (128ull << 20)
GAPA_API int gapa_eval_population_noalloc(gapa_graph *g, const int32_t *genes, int32_t P, int32_t k,
                                          int64_t *fitness, int32_t *mcn, uint32_t flags, void *stream);

/* ---------------------------------------------------------------------------
 * The paper's dense reachability fitness (Section III-D, eq. 13-17, the
 * "SixDST" function), on the matrix cores.
 *
 * For each row S of genes: M = Normalizer((A_S + I)^hops), A_S the
 * adjacency matrix with every edge of a removed node deleted (eq. 13), the
 * power by repeated squaring with every product normalised (entries > 0
 * become 1); row v of M marks the nodes within `hops` hops of v.
 * pc:  int64 [P] out, (sum of M - n) / 2: the pairs of surviving nodes within
 *      `hops` hops of each other.
 * mcn: int32 [P] out, the largest row sum over surviving nodes (0 if none).
 * With hops >= the diameter of every component these are PC and MCN of
 * gapa_eval_population exactly; the paper uses hops = 6 (eq. 15).
 * Dense n x n int8 matrices (three per individual in flight, within a 2 GiB
 * workspace): n <= GAPA_SIXDST_MAX_N, hops >= 1, else GAPA_E_INVALID_ARG.
 * Genes, flags (GAPA_DEVICE_PTRS, GAPA_TRUST_INPUT), stream and errors as for
 * gapa_eval_population; results are exact integers.
 * ------------------------------------------------------------------------- */
#define GAPA_SIXDST_MAX_N 8192
GAPA_API int gapa_sixdst_eval(gapa_graph *g, const int32_t *genes, int32_t P, int32_t k, int32_t hops,
                              int64_t *pc, int32_t *mcn, uint32_t flags, void *stream);

/* ---------------------------------------------------------------------------
 * Genetic algorithm (Section III-B, Fig. 1 single-GPU "S" mode).
 *
 * k          budget: genes per individual (1 <= k <= n / 2)
 * pop        P: population kept by elitism (eq. 10-11), >= 1
 * tournament T: contestants per tournament, 1..64 (replaces the roulette
 *            wheel of eq. 5; winner = smallest (PC, position))
 * offspring  lambda: children per generation, 0 means P
 * seed       Philox4x32-10 key; all randomness is a pure function of
 *            (seed, generation, individual, slot)
 * pc, pm     per-gene crossover (eq. 4) and mutation (eq. 8) probabilities,
 *            in [0, 1]
 * ------------------------------------------------------------------------- */
typedef struct gapa_params {
    int32_t k;
    int32_t pop;
    int32_t tournament;
    int32_t offspring;
    uint64_t seed;
    double pc;
    double pm;
    uint32_t flags;   /* 0 or GAPA_GRAPH_REPLAY, with at most one of
                         GAPA_MINIMISE_MCN and GAPA_MAXIMISE_COMPONENTS */
    int32_t reserved; /* 0 */
} gapa_params;

/* Creates the GA on graph g (the GA holds a reference to g): draws the
 * initial population (eq. 2), evaluates it and orders it by (fitness,
 * index): generation 0.  The work is enqueued on `stream`; the call returns
 * once it is enqueued. */
GAPA_API int gapa_ga_create(gapa_graph *g, const gapa_params *p, void *stream, gapa_ga **out);

/* Runs n_generations >= 0 further generations, each: tournament selection,
 * crossover (eq. 3-6) with duplicate repair, mutation (eq. 7-9), batched
 * fitness of the offspring, elitism (eq. 10-11) keeping the P best of parents
 * and offspring.  Enqueues only; no host synchronisation. */
GAPA_API int gapa_generation_step(gapa_ga *ga, int32_t n_generations, void *stream);

/* With GAPA_GRAPH_REPLAY: records n_generations (1..4096) generations, from
 * the current state's buffer parity, as one HIP graph, without running them;
 * a later gapa_generation_step of exactly n_generations from the same parity
 * is then one graph launch.  Needs one generation run since creation or the
 * last tuning change (buffers sized); GAPA_E_STATE otherwise, or with a
 * surrogate attached.  Results are those of running the generations
 * eagerly. */
GAPA_API int gapa_ga_record(gapa_ga *ga, int32_t n_generations);

/* Checkpoint and resume of a single GA without a surrogate.  gapa_ga_save
 * writes the GA's parameters, its graph's identity (n, nnz and a hash of the
 * CSR), the generation number, the population rows in order and their
 * fitness to the file at `path` (synchronous; GAPA_E_STATE for a batch or
 * with a surrogate, GAPA_E_INVALID_ARG if the file cannot be written).
 * gapa_ga_load creates a GA on graph g from such a file: since every random
 * draw is keyed by (seed, generation, individual, slot), stepping it gives
 * exactly the generations the saved GA would have run.  A file that is not a
 * checkpoint, is truncated or fails its checksum, or was taken on another
 * graph gives GAPA_E_INVALID_ARG.  The new GA is owned by the caller
 * (gapa_ga_destroy). */
GAPA_API int gapa_ga_save(gapa_ga *ga, const char *path);
/* The GA's parameters and the number of generations enqueued so far (either
 * output may be NULL). */
GAPA_API int gapa_ga_params(gapa_ga *ga, gapa_params *params_out, int64_t *generation_out);
GAPA_API int gapa_ga_load(gapa_graph *g, const char *path, void *stream, gapa_ga **out);

/* Best individual after the last enqueued generation (eq. 1's arg max): its k
 * genes ascending (genes_out, k int32, may be NULL), PC (may be NULL) and the
 * generation count (may be NULL).  Host pointers; waits for the GA's work. */
GAPA_API int gapa_best(gapa_ga *ga, int32_t *genes_out, int64_t *fitness_out, int64_t *generation_out);

/* The best fitness after the last enqueued generation, copied to
 * fitness_out (8 bytes of device memory or of pinned, mapped host memory)
 * by work enqueued on `stream` -- the stream the generations were enqueued
 * on -- without waiting for it: a caller can follow the best value
 * generation by generation without synchronising the host. */
GAPA_API int gapa_best_async(gapa_ga *ga, int64_t *fitness_out, void *stream);

/* Whole population, ordered by (PC, tag): genes_out int32 [P][k], fitness_out
 * int64 [P] (either may be NULL).  Host pointers; waits for the GA's work. */
GAPA_API int gapa_get_population(gapa_ga *ga, int32_t *genes_out, int64_t *fitness_out);

GAPA_API int gapa_ga_destroy(gapa_ga *ga);

/* ---------------------------------------------------------------------------
 * Learned screening surrogate (an extension; not in the paper).  The paper
 * evaluates every offspring exactly (Section III-C).  With a surrogate
 * attached, each generation still makes `offspring` children with the same
 * operators, but a small network predicts their fitness and only the
 * `screen` children with the lowest predictions are evaluated exactly and
 * enter elitism; exact fitness stays the only value the population holds.
 *
 *   x(S) = sum over v in S of E[v]           E: n x 64 node embeddings
 *   yhat = w3 . relu(W2 relu(W1 x + b1) + b2) + b3      (64 -> 256 -> 256 -> 1)
 *
 * FP32 master weights, bfloat16 copies for the products (matrix-core
 * kernels, FP32 accumulation).  Trained online on (S, ln(1 + PC(S))) pairs of
 * the exactly evaluated offspring, kept in a ring buffer: labels are
 * standardised by the buffer's mean and spread sqrt(variance + 1e-12); mean squared
 * error; Adam (Kingma and Ba 2015) with beta = (0.9, 0.999), eps = 1e-8, lazy
 * on E (rows of nodes absent from the batch keep weights and moments);
 * `train_steps` steps per generation on batches drawn with Philox stream 6
 * (slot j, individual step, generation).  Initial weights from Philox stream
 * 5: E uniform in +-0.05, W1 and W2 uniform in +-sqrt(6 / fan_in), w3 in
 * +-sqrt(3 / fan_in), biases 0.
 *
 * Generations 1..warmup_gens evaluate every child (and train).  Later
 * generations screen; a screened generation also evaluates min(32, offspring
 * - screen) of the other children, drawn uniformly with Philox stream 7, for
 * the judge only (they join the training buffer, not elitism).  The judge is
 * the Spearman correlation between predictions and exact fitness over the
 * evaluated children (at most 1024 of them, evenly spaced).  Generation g is
 * screened or evaluated in full as decided from the judge of generation g - 2
 * (so a call never waits for the generation before it): after `fallback_gens`
 * consecutive judged screened generations with a correlation below min_rho,
 * generation g evaluates every child, and generation g - 1, launched before
 * that decision, does not count towards the next one.
 * ------------------------------------------------------------------------- */
enum {
    GAPA_SCREEN_RANDOM = 1u << 0 /* gapa_surrogate_params.flags: screen a uniformly
                                    random subset instead (Philox stream 7); no
                                    training -- the ablation baseline             */
};

typedef struct gapa_surrogate_params {
    int32_t emb_dim;       /* 64 (the only supported value)                       */
    int32_t hidden;        /* 256 (the only supported value)                      */
    int32_t screen;        /* children evaluated exactly per screened generation,
                              1 <= screen <= offspring                            */
    int32_t batch;         /* training batch: 32, 64, 128, 256, 512 or 1024        */
    int32_t train_steps;   /* Adam steps per generation, >= 0                      */
    int32_t warmup_gens;   /* full generations before screening starts, >= 0       */
    int32_t buffer;        /* ring buffer capacity in pairs, >= batch             */
    int32_t fallback_gens; /* consecutive low-correlation generations that trigger
                              one full generation; 0 never                        */
    float lr;              /* Adam step size, > 0                                  */
    float min_rho;         /* judge threshold                                     */
    uint32_t flags;        /* 0 or GAPA_SCREEN_RANDOM                              */
    int32_t reserved;      /* 0                                                   */
} gapa_surrogate_params;

/* Attaches a surrogate to a GA at generation 0 (one instance, offspring <=
 * 8192, n * 64 embeddings and a buffer of `buffer` rows of k genes in device
 * memory).  Later gapa_generation_step calls run screened generations
 * (eagerly: GAPA_GRAPH_REPLAY does not apply). */
GAPA_API int gapa_surrogate_attach(gapa_ga *ga, const gapa_surrogate_params *sp, void *stream);

typedef struct gapa_surrogate_report {
    int64_t generation;  /* generation the figures belong to                      */
    int32_t evaluated;   /* children evaluated exactly in it                       */
    int32_t pooled;      /* of which entered elitism                              */
    int32_t screened;    /* 1 if it was screened, 0 if every child was evaluated  */
    int32_t reserved;
    double spearman;     /* judge correlation (0 when no prediction was made)     */
    double rel_err;      /* mean |expm1(prediction) - PC| / max(PC, 1)             */
    double loss;         /* mean squared error of the last step of the training
                            on generation g - 2's labels (generation g - 1's
                            training still runs beside generation g; after
                            gapa_surrogate_train_batch: that step's)          */
    int32_t fallbacks;   /* full generations forced by the judge so far            */
    int32_t train_steps; /* Adam steps taken so far                               */
    double label_mean;   /* the label standardisation the generation's predictions */
    double label_spread; /* were made in (0 when it made none): a standardised
                            prediction y stands for ln(1 + PC) = y spread + mean */
} gapa_surrogate_report;

/* Figures of the last generation (host pointer; waits for the GA's work). */
GAPA_API int gapa_surrogate_stats(gapa_ga *ga, gapa_surrogate_report *out);

/* The judge's statistics on explicit data (the computation behind the
 * spearman and rel_err of gapa_surrogate_report).  Device pointers: yhat
 * float predictions (standardised scale), indexed by pool[q] (int32 [m]; NULL:
 * by q), fitness int64 [m] the exact PC of the same children.  Over J =
 * min(m, 1024) entries, entry i being q = floor(i m / J): out[0] Spearman's
 * rank correlation between yhat and fitness (average ranks for ties, 0 when
 * either side is constant), out[1] the mean over them of
 * |expm1(yhat label_spread + label_mean) - PC| / max(PC, 1).  out is host
 * double [2]; the call waits on `stream`.  m >= 1, label_spread > 0, else
 * GAPA_E_INVALID_ARG; pool entries must index yhat (not checked). */
GAPA_API int gapa_surrogate_judge(const float *yhat, const int32_t *pool, const int64_t *fitness, int32_t m,
                                  double label_mean, double label_spread, double *out, void *stream);

/* Children evaluated exactly in the last generation (host; waits): the pooled
 * ones ascending, then the judge's extra sample ascending; up to `cap`
 * indices into pool_out, the number through *count. */
GAPA_API int gapa_surrogate_last_pool(gapa_ga *ga, int32_t *pool_out, int32_t cap, int32_t *count);

/* Predictions made in the last generation for all of its children, in child
 * order (0 entries when that generation made none: warm-up, or random
 * screening); host pointer, waits.  They precede that generation's training. */
GAPA_API int gapa_surrogate_last_predictions(gapa_ga *ga, float *yhat_out, int32_t cap, int32_t *count);

/* Predictions (standardised scale) of the current model for P gene rows:
 * genes int32 [P][k] and yhat float [P], device pointers, enqueued on
 * `stream`.  Genes must be node ids in [0, n) (not checked). */
GAPA_API int gapa_surrogate_predict(gapa_ga *ga, const int32_t *genes, int32_t P, float *yhat, void *stream);

/* One Adam step on an explicit batch: genes int32 [B][k] (rows of distinct
 * node ids), target float [B] (standardised labels), device pointers, B a
 * supported batch size.  With keep_grads the step's gradients are kept for
 * gapa_surrogate_tensor(kind 1). */
GAPA_API int gapa_surrogate_train_batch(gapa_ga *ga, const int32_t *genes, const float *target, int32_t B,
                                        int32_t keep_grads, void *stream);

/* Copies a tensor between the model and host memory: which 0 E [n][64],
 * 1 W1 [256][64], 2 b1 [256], 3 W2 [256][256], 4 b2 [256], 5 w3 [256], 6 b3 [1];
 * kind 0 the FP32 weights, 1 the last kept gradient; set = 1 writes the
 * weights (kind 0 only; the bfloat16 copies follow).  count must equal the
 * tensor's size.  Waits for the GA's work. */
GAPA_API int gapa_surrogate_tensor(gapa_ga *ga, int32_t which, int32_t kind, float *host, int64_t count,
                                   int32_t set);

/* ---------------------------------------------------------------------------
 * Batch of independent GAs (Section III-D runs several GA processes side by
 * side in its M and MNM modes; here many independent instances share each
 * device pass instead).
 *
 * count      1 <= count <= 4096 instances
 * graphs     [count] graph handles on the current device (the same handle may
 *            appear several times).  Their disjoint union is built once on
 *            the device (sum of n <= 2^30); the batch keeps its own
 *            reference, so the handles may be destroyed before it.
 * params     [count] parameters as for gapa_ga_create, per instance
 *            (max(pop, offspring) <= 1024 for each; flags from
 *            GAPA_GRAPH_REPLAY | GAPA_MINIMISE_MCN | GAPA_MAXIMISE_COMPONENTS,
 *            the same for every instance)
 *
 * Instance b evolves exactly as gapa_ga_create(graphs[b], &params[b]) and
 * its generation steps would alone: same draws, same populations, same
 * fitness, generation by generation.  One generation of the batch is one
 * operator launch over all instances' offspring, one bit-parallel fitness
 * pass over all of them and one elitism launch.  Enqueue semantics and
 * host-pointer waits are those of the single-GA calls (gapa_batch_record as
 * gapa_ga_record); idx selects an instance (0 <= idx < count).
 * ------------------------------------------------------------------------- */
GAPA_API int gapa_batch_create(int32_t count, gapa_graph *const *graphs, const gapa_params *params, void *stream,
                               gapa_batch **out);
GAPA_API int gapa_batch_step(gapa_batch *b, int32_t n_generations, void *stream);
GAPA_API int gapa_batch_record(gapa_batch *b, int32_t n_generations);
GAPA_API int gapa_batch_best(gapa_batch *b, int32_t idx, int32_t *genes_out, int64_t *fitness_out,
                             int64_t *generation_out);
GAPA_API int gapa_batch_get_population(gapa_batch *b, int32_t idx, int32_t *genes_out, int64_t *fitness_out);
GAPA_API int gapa_batch_destroy(gapa_batch *b);

/* ---------------------------------------------------------------------------
 * Diagnostics
 * ------------------------------------------------------------------------- */

/* Kernel timing: `enable` 1 brackets whole passes with HIP events on their
 * launch stream ("fitness_pass": the batched fitness of one chunk of up to
 * 2048 individuals; "ga_offspring", "ga_init": the operator kernel;
 * "elitism"); 2 also brackets every kernel launch inside them (the extra
 * events add gaps, so pass totals are exact only at 1); 0 disables.
 * gapa_*_kernel_times fills up to `cap` entries with the scope name, count
 * and summed milliseconds (it waits for outstanding work) and returns the
 * number of entries through *count.  Names stay valid until the handle is
 * destroyed. */
typedef struct gapa_kernel_time {
    const char *name;
    int64_t launches;
    double total_ms;
} gapa_kernel_time;

GAPA_API int gapa_graph_set_timing(gapa_graph *g, int32_t enable);
GAPA_API int gapa_graph_kernel_times(gapa_graph *g, gapa_kernel_time *out, int32_t cap, int32_t *count);
GAPA_API int gapa_ga_set_timing(gapa_ga *ga, int32_t enable);
GAPA_API int gapa_ga_kernel_times(gapa_ga *ga, gapa_kernel_time *out, int32_t cap, int32_t *count);
GAPA_API int gapa_batch_set_timing(gapa_batch *b, int32_t enable);
GAPA_API int gapa_batch_kernel_times(gapa_batch *b, gapa_kernel_time *out, int32_t cap, int32_t *count);

/* Counters of the last chunk the bit-parallel fitness evaluated on a handle
 * (waits for outstanding work): out[0] individuals per chunk, out[1] nodes
 * still pending after the ordered sweep, out[2] (individual, node) pairs left
 * to the union-find pass, out[3] follow-up sweeps that still changed
 * something.  All zero before the first evaluation. */
GAPA_API int gapa_graph_fitness_stats(gapa_graph *g, int64_t out[4]);
GAPA_API int gapa_ga_fitness_stats(gapa_ga *ga, int64_t out[4]);

/* Launch shapes of the bit-parallel fitness pass.  They change speed only:
 * results never depend on them.
 *   sweep_grid   blocks of the worklist, pair and union-find kernels, 1..65535
 *   band_scan    neighbours a node reads in the ordered sweep, >= 1
 *   sweeps       follow-up sweeps over the nodes still pending, 0..32
 *   band_blocks  block cap of one band launch, 1..65535
 * Defaults 4096, 32, 3, 8192.  A change also applies to GAs and batches on
 * the graph (recorded generations are re-recorded). */
typedef struct gapa_tuning {
    int32_t sweep_grid;
    int32_t band_scan;
    int32_t sweeps;
    int32_t band_blocks;
} gapa_tuning;

GAPA_API int gapa_graph_get_tuning(gapa_graph *g, gapa_tuning *out);
GAPA_API int gapa_graph_set_tuning(gapa_graph *g, const gapa_tuning *t);

/* Autotuner: times `reps` >= 1 fitness passes over the children the GA (or
 * batch) currently holds for each launch shape of a fixed candidate grid
 * (sweep_grid 1024/2048/4096/8192, band_scan 8/16/32/64, sweeps 2/3/4,
 * band_blocks 2048/4096/16384; timed with events on the stream), keeps the
 * fastest on the evaluating graph and returns it
 * through best_out (may be NULL).  Work is enqueued on `stream` and waited
 * for.  It overwrites only scratch fitness values; the GA state is
 * untouched. */
GAPA_API int gapa_ga_autotune(gapa_ga *ga, int32_t reps, void *stream, gapa_tuning *best_out);
GAPA_API int gapa_batch_autotune(gapa_batch *b, int32_t reps, void *stream, gapa_tuning *best_out);
/* Launch shapes of a batch's fitness pass (its disjoint-union graph), as
 * gapa_graph_get_tuning / gapa_graph_set_tuning; NULL gives
 * GAPA_E_INVALID_ARG. */
GAPA_API int gapa_batch_get_tuning(gapa_batch *b, gapa_tuning *out);
GAPA_API int gapa_batch_set_tuning(gapa_batch *b, const gapa_tuning *t);

/* Message of the last failed call on this thread ("" if none). */
GAPA_API const char *gapa_last_error(void);
GAPA_API const char *gapa_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GAPA_H */
