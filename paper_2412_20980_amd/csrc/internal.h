// Host-side internals of the HIP library: handle layouts, device buffers,
// kernel-timing bookkeeping and the launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <map>
#include <string>
#include <vector>

#include "gapa.h"

namespace gapa {

// ---------------------------------------------------------------- errors ----

void set_error(const char *fmt, ...);

struct Status {
    int code = GAPA_OK;
    bool ok() const { return code == GAPA_OK; }
};

// ------------------------------------------------------- device buffers -----

// Grow-only device allocation (contents not preserved on growth).  A
// borrowed buffer is a view of memory owned elsewhere: reserve() never
// allocates for it (a request beyond its size is an error) and release()
// only forgets it.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    bool borrowed = false;
    int reserve(size_t want);  // GAPA_OK, GAPA_E_OOM, or GAPA_E_INVALID_ARG for a borrowed view too small
    void release();
    void borrow(void *p, size_t n)
    {
        ptr = p;
        bytes = n;
        borrowed = true;
    }
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// ---------------------------------------------------------------- timing ----

// While enabled, named scopes are bracketed by a pair of HIP events recorded
// on their stream; totals are folded in on collect().  Level 1 times whole
// passes (the batched fitness of a chunk, the operator kernel, elitism);
// level 2 also times every kernel launch inside them (the extra events add
// gaps between kernels, so pass totals are only exact at level 1).
class KernelTimer {
public:
    int level = 0;
    void begin(const char *name, hipStream_t s);
    void end(hipStream_t s);
    int collect(gapa_kernel_time *out, int cap, int *count);
    ~KernelTimer();

private:
    struct Pending {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending_;
    std::vector<hipEvent_t> free_;
    std::map<std::string, std::pair<int64_t, double>> totals_;
    std::vector<std::string> names_;  // stable storage for returned names
    std::vector<size_t> open_;        // indices into pending_ of open scopes
    hipEvent_t take();
};

struct TimedScope {
    KernelTimer *t;
    hipStream_t s;
    bool on;
    TimedScope(KernelTimer *timer, const char *name, hipStream_t stream, int level = 2)
        : t(timer), s(stream), on(timer && timer->level >= level)
    {
        if (on) t->begin(name, s);
    }
    ~TimedScope()
    {
        if (on) t->end(s);
    }
};

// ----------------------------------------------------------------- graph ----

// Scratch for the batched fitness of one chunk of individuals.
struct FitnessWorkspace {
    DevBuf parent;   // int32 [B][n]  union-find parents
    DevBuf count;    // int32 [B][n]  component sizes at roots (union-find path)
    DevBuf dead;     // uint32 [n][Wd] removed bits, node-major (bit-parallel path)
    DevBuf reach;    // uint32 [n][Wd] root-component bits
    DevBuf ucount;   // int32 [B][n]  set sizes of the leftover union-find, kept zero
    DevBuf pairs;    // int64 [B * n_noniso] pending (individual, node) keys
    DevBuf worklist; // int4 [n_noniso] records (node, first edge, edge end) of the nodes still pending after the ordered sweep
    DevBuf pflag;    // uint8 [n_noniso] 1: the node at this band position is still pending after the ordered sweep (then: at this worklist position, after the last follow-up sweep)
    bool pflag_clear = false;  // pflag zeroed since it was (re)allocated
    DevBuf small;    // int32 roots, root-set sizes, counters, count partials
    int32_t *stats_ctr = nullptr;  // device counters of the last bit-parallel chunk
    int32_t stats_B = 0;
    DevBuf masks;    // uint32 [P][W] removed-node bit sets (eval_population)
    DevBuf alive;    // int32 [P]    surviving non-isolated nodes (eval_population)
    DevBuf genes;    // int32 [P][k]  staged host genes
    DevBuf fitness;  // int64 [P]
    DevBuf mcn;      // int32 [P]
    DevBuf flag;     // int32 [4]     device error flags
    DevBuf six_mats; // int8 [3][chunk][n_pad][n_pad] dense reachability matrices
    DevBuf six_tot;  // uint64 [chunk] their entry sums
    // extra lanes (owned): chunks of a population wider than one pass run
    // side by side, each with its own workspace and stream
    std::vector<FitnessWorkspace *> lanes;
    std::vector<hipStream_t> lane_streams;
    std::vector<hipEvent_t> lane_done;
    hipEvent_t fork = nullptr;
};

// Launch shapes of the bit-parallel fitness pass (results do not depend on
// them; only speed does).
struct Tuning {
    int32_t sweep_grid = 4096;   // blocks of the worklist, pair and union-find kernels
    int32_t band_scan = 32;      // neighbours read per node in the ordered sweep
    int32_t sweeps = 3;          // follow-up sweeps over the pending nodes
    int32_t band_blocks = 8192;  // block cap of one band launch
};

}  // namespace gapa

struct gapa_graph {
    std::atomic<int32_t> refs{1};  // the caller's handle, plus one per GA or batch using the graph
    int device = 0;
    uint64_t content_hash = 0;     // FNV-1a of n, row_ptr and col_idx (checkpoints name their graph by it)
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t words = 0;          // ceil(n / 32): words of a node bit set
    int32_t *d_row_ptr = nullptr;
    int32_t *d_col = nullptr;
    int32_t *d_src = nullptr;   // source node of every CSR entry (COO rows)
    int32_t *d_order = nullptr; // [n] nodes by (degree desc, id)
    int32_t *d_colD = nullptr;  // [nnz] each neighbour list by (degree desc, id)
    int4 *d_band_rec = nullptr;   // [n_noniso] non-isolated nodes by (BFS level, id) as records
                                  // (node, row_ptr[node], row_ptr[node + 1], 0)
    uint32_t *d_noniso = nullptr; // [words] bit v set: v has at least one edge
    int8_t *d_src_idx = nullptr;  // [n] index of a band source among its instance's (order[voff + t]), else -1
    std::vector<int32_t> band_off;  // host: band b is d_band_rec[band_off[b], band_off[b+1])
    int32_t src_band = 0;       // size of band 0 when it holds exactly the sources, else 0
    int32_t n_noniso = 0;       // nodes with at least one edge
    int32_t algorithm = 0;      // 0: bit-parallel sweeps, 1: edge-parallel union-find
    gapa::Tuning tune;
    int32_t tune_version = 0;   // bumped by every tuning change (recorded graphs are re-recorded)
    gapa::FitnessWorkspace ws;
    gapa::KernelTimer timer;
    bool failed = false;
};

namespace gapa {

// Node words per tile of the dead-row transpose (32 nodes each); the tile
// lists of instance tables step by it.
constexpr int kTransposeWords = 4;

// Node words per transposer tile for chunks of Wd words per node row (Wd a
// power of two <= 32): kTransposeWords * 32 / Wd.
inline int32_t transpose_tile_words(int32_t Wd)
{
    return kTransposeWords * 32 / Wd;
}

// Several instances (disjoint node ranges of one graph, each with its own
// individuals) evaluated in one bit-parallel fitness pass.  All arrays are on
// the device.  Slot i of instance b is entry b * bseg + i of the alive,
// fitness and mcn arrays; its removed-node bit set (local node ids, W_b =
// ceil(n_b / 32) words) starts at word moff[b] + i * W_b of the mask array.
struct InstTable {
    int32_t count = 0;
    int32_t bseg = 0;                    // slots per instance: 32 * Wd, Wd a power of two <= 32
    const int32_t *voff = nullptr;       // [count + 1] first node of each instance
    const int32_t *live = nullptr;       // [count] slots in use
    const int64_t *moff = nullptr;       // [count]
    const int32_t *node_inst = nullptr;  // [n] instance of each node
    const int32_t *tiles = nullptr;      // [2 * ntiles] (instance, first node word) of each 8-word tile
    int32_t ntiles = 0;
};

// What the fitness sums over the components C of G - S: |C|(|C| - 1)/2
// (pairwise connectivity), or |C| - 1, whose sum is |V minus S| minus the
// number of components (the size of a spanning forest of G - S).
enum Measure : int32_t { kMeasurePC = 0, kMeasureForest = 1 };

// Fitness of P individuals given as removed-node bit sets masks[P][W]
// (device) with alive[P] = surviving non-isolated nodes of each.  Writes
// fitness[P] (int64, the sum selected by `measure`) and, if mcn != nullptr,
// mcn[P] (int32).  Runs the graph's selected algorithm.
// With an instance table of count > 1 (bit-parallel algorithm only), P is
// ignored and all slots of all instances are evaluated in one pass.
int eval_masks(gapa_graph *g, const uint32_t *masks, const int32_t *alive, int32_t P, int64_t *fitness, int32_t *mcn,
               FitnessWorkspace &ws, KernelTimer *timer, hipStream_t s, const InstTable *it = nullptr,
               Measure measure = kMeasurePC);
int eval_masks_bits(gapa_graph *g, const uint32_t *masks, const int32_t *alive, int32_t P, int64_t *fitness,
                    int32_t *mcn, FitnessWorkspace &ws, KernelTimer *timer, hipStream_t s,
                    const InstTable *it = nullptr, Measure measure = kMeasurePC);
// Bytes of scratch the bit-parallel fitness needs for chunks of 32 * Wd
// individuals on graph g (every buffer of one pass plus the chunk's bit sets,
// each part 256-byte aligned).
size_t bits_scratch_bytes(const gapa_graph *g, int32_t Wd);
// Bit-parallel fitness of P gene rows (device, [P][k]) with every buffer
// carved from `scratch` (`bytes` long): chunks of 32 * Wd rows, Wd the widest
// power of two <= 32 that fits, one after another on stream s; a gene outside
// [0, n) sets flag[0] (flag: 4 int32 in the scratch, cleared here).  Nothing
// is allocated; GAPA_E_INVALID_ARG if not even 32 rows fit.
int eval_genes_bits_scratch(gapa_graph *g, const int32_t *genes, int32_t P, int32_t k, int64_t *fitness,
                            int32_t *mcn, Measure measure, void *scratch, size_t bytes, int32_t **flag_out,
                            hipStream_t s);
int eval_masks_unionfind(gapa_graph *g, const uint32_t *masks, int32_t P, int64_t *fitness, int32_t *mcn,
                         FitnessWorkspace &ws, KernelTimer *timer, hipStream_t s, Measure measure = kMeasurePC);
// Same from gene rows genes[P][k] (device node ids; a repeated id in a row is
// one removal); a gene outside [0, n) sets flag[0] and is ignored.
int eval_genes(gapa_graph *g, const int32_t *genes, int32_t P, int32_t k, int64_t *fitness, int32_t *mcn,
               int32_t *flag, FitnessWorkspace &ws, KernelTimer *timer, hipStream_t s, Measure measure = kMeasurePC);

// Removed-node bit sets masks[P][W] of P = 32 Wd individuals (Wd a power of
// two <= 32) to node-major rows rows[n][Wd]: bit i of row v is set when
// individual i removes v.
int launch_bits_transpose(const uint32_t *masks, int32_t P, int32_t W, int32_t n, uint32_t *rows, hipStream_t s);

// Fills count 32-bit words at p with value (a kernel, not a memset node).
int launch_fill_u32(void *p, uint32_t value, int64_t count, hipStream_t s);
size_t sixdst_bytes_per_individual(int32_t n);
int sixdst_eval_masks(gapa_graph *g, const uint32_t *masks, int32_t P, int32_t hops, int32_t chunk, uint8_t *mats,
                      unsigned long long *tot, int64_t *pc, int32_t *mcn, hipStream_t s);

// genes[P][k] (device) -> masks[P][W] and alive[P]; out-of-range genes
// raise flag[0].
int launch_mask_build(const int32_t *genes, int32_t P, int32_t k, int32_t n, int32_t W, const uint32_t *noniso,
                      int32_t n_noniso, uint32_t *masks, int32_t *alive, int32_t *flag, hipStream_t s);

// ------------------------------------------------------------------- GA -----

// Dynamic LDS of the operator kernels for n nodes and budget k, and the
// function attributes they need when it exceeds the default 64 KiB.
size_t ga_op_lds_bytes(int32_t n, int32_t k);
int ga_prepare_kernels(size_t lds);

// Device table entry of one GA instance: where its rows live in the shared
// buffers, its sizes and its random-stream parameters.  A single GA is a
// one-entry table with every offset 0.
struct GaInst {
    int64_t pop_off;    // first element of its rows in pop[*] (row stride k)
    int64_t child_off;  // first element of its rows in children (row stride k)
    int64_t mask_off;   // first word of its child masks (row stride W)
    int32_t fit_off;    // first entry in fit[*] and src
    int32_t slot_off;   // first entry in child_fit and alive
    int32_t noniso_off; // first word of its non-isolated node bit set
    uint64_t seed, t_pc, t_pm;
    int32_t P, L, k, n, W, KW, T, n_noniso;
};

int ga_init_population(gapa_ga *ga, hipStream_t s);
// One generation of every instance; the generation number is read on the
// device, so the launches can be captured into a graph and replayed.
int ga_generation(gapa_ga *ga, hipStream_t s);
int ga_launch_init(gapa_ga *ga, hipStream_t s);
// rows_only: the children's rows only; their bit sets and alive counts are
// left for the caller to build (for the few it evaluates).
int ga_launch_offspring(gapa_ga *ga, hipStream_t s, bool rows_only = false);
// Elitism of every instance over its current parents (none at generation 0,
// `init`) and its evaluated offspring (f_pool[q] is the fitness of child
// pool[q], or of child q when pool is NULL; a pool only with one instance);
// writes the next population buffer and, after generation 0, advances the
// device generation counter.
int ga_rank_and_gather(gapa_ga *ga, bool init, const int64_t *f_pool, const int32_t *pool, int32_t npool,
                       hipStream_t s);
// Exact fitness of the children currently held (the initial population at
// generation 0) into child_fit.
int ga_eval_children(gapa_ga *ga, bool init, hipStream_t s);

// ------------------------------------------------------------ surrogate -----

struct SurrogateState;
// Allocates and initialises the learned screening model of a one-instance GA.
int surrogate_attach(gapa_ga *ga, const gapa_surrogate_params *sp, hipStream_t s);
void surrogate_release(SurrogateState *st);
// One generation with screening (or a full one during warm-up / fallback).
int surrogate_generation(gapa_ga *ga, hipStream_t s);
int surrogate_predict(gapa_ga *ga, const int32_t *genes, int32_t P, float *yhat, hipStream_t s);
int surrogate_train_batch(gapa_ga *ga, const int32_t *genes, const float *target, int32_t B, bool keep_grads,
                          hipStream_t s);
int surrogate_tensor(gapa_ga *ga, int32_t which, int32_t kind, float *host, int64_t count, bool set);
int surrogate_stats(gapa_ga *ga, gapa_surrogate_report *out);
int surrogate_last_pool(gapa_ga *ga, int32_t *pool, int32_t cap, int32_t *count);
int surrogate_last_predictions(gapa_ga *ga, float *yhat, int32_t cap, int32_t *count);
// The judge's statistics of m predictions against exact fitness (device
// arrays), written to host out[2]; waits on s.
int surrogate_judge(const float *yhat, const int32_t *pool, const int64_t *F, int32_t m, double mu, double sd,
                    double *out, hipStream_t s);

// Error reporting for HIP calls.
int hip_fail(hipError_t e, const char *what);
#define GAPA_HIP(call)                                                  \
    do {                                                                \
        hipError_t _e = (call);                                         \
        if (_e != hipSuccess) return ::gapa::hip_fail(_e, #call);       \
    } while (0)

}  // namespace gapa

struct gapa_ga {
    gapa_graph *graph = nullptr;  // for a batch: the disjoint union of the instance graphs
    gapa_params params{};         // first instance's parameters
    int32_t lambda = 0;
    uint64_t t_pc = 0, t_pm = 0;  // Bernoulli thresholds floor(p * 2^32)
    int64_t generation = 0;
    int cur = 0;                  // which population buffer is current
    int32_t count = 1;            // instances
    std::vector<gapa::GaInst> hinst;
    gapa::DevBuf inst;            // GaInst [count]
    int32_t max_pop = 0, max_lambda = 0, max_pop_lambda = 0;
    gapa::DevBuf pop[2];          // int32 rows of every instance
    gapa::DevBuf fit[2];          // int64 [sum P]
    gapa::DevBuf children;        // int32 rows
    gapa::DevBuf child_fit;       // int64 slots
    gapa::DevBuf child_mcn;       // int32 slots (GAPA_MINIMISE_MCN: the pass's MCN, copied into child_fit)
    int32_t slots = 0;
    bool objective_mcn = false;
    bool objective_forest = false;  // GAPA_MAXIMISE_COMPONENTS: fitness = |V minus S| - components
    gapa::DevBuf masks;           // uint32 removed-node bit sets of the children
    gapa::DevBuf alive;           // int32 slots: surviving non-isolated nodes
    gapa::DevBuf src;             // int32 [sum P] elitism: source tag of each kept row
    gapa::DevBuf flag;            // int32 [4] device error flags
    gapa::DevBuf gen_ctr;         // uint32 [1] generations completed (read by the operator kernel)
    uint32_t *noniso = nullptr;   // batch: per-instance non-isolated bit sets (else the graph's)
    gapa::DevBuf noniso_buf;
    // batch: instance tables of the fitness pass at generation 0 and later
    gapa::InstTable tab_init, tab_gen;
    gapa::DevBuf tab_voff, tab_live_init, tab_live_gen, tab_moff, tab_node_inst, tab_tiles;
    gapa::FitnessWorkspace ws;
    gapa::KernelTimer timer;
    hipStream_t last_stream = nullptr;
    size_t op_lds_bytes = 0;      // dynamic LDS of the operator kernels
    bool failed = false;
    // graph replay of one generation (one per current-buffer parity)
    bool use_graph = false;
    bool warm = false;            // a generation has run eagerly: buffers are sized
    int32_t captured_version = -1;  // graph tuning the recorded generations were made with
    hipStream_t cap_stream = nullptr;
    struct Replay {
        int parity;        // current population buffer the recording starts from
        int32_t gens;      // generations it runs
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<Replay> replays;
    gapa::SurrogateState *surr = nullptr;  // learned screening, when attached
};

struct gapa_batch {
    gapa_ga *ga = nullptr;
    gapa_graph *super = nullptr;  // owned
};
