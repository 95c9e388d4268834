// Host-side internals of the HIP library: handle layouts, device buffers,
// kernel-timing bookkeeping and the launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Grow-only device allocation (contents not preserved on growth).
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int reserve(size_t want);  // GAPA_OK or GAPA_E_OOM
    void release();
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
    DevBuf worklist; // int32 [n_noniso] nodes still pending after the ordered sweep
    DevBuf small;    // int32 roots, root-set sizes, counters, count partials
    int32_t *stats_ctr = nullptr;  // device counters of the last bit-parallel chunk
    int32_t stats_B = 0;
    DevBuf masks;    // uint32 [P][W] removed-node bit sets (eval_population)
    DevBuf alive;    // int32 [P]    surviving non-isolated nodes (eval_population)
    DevBuf genes;    // int32 [P][k]  staged host genes
    DevBuf fitness;  // int64 [P]
    DevBuf mcn;      // int32 [P]
    DevBuf flag;     // int32 [4]     device error flags
};

}  // namespace gapa

struct gapa_graph {
    int device = 0;
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t words = 0;          // ceil(n / 32): words of a node bit set
    int32_t *d_row_ptr = nullptr;
    int32_t *d_col = nullptr;
    int32_t *d_src = nullptr;   // source node of every CSR entry (COO rows)
    int32_t *d_order = nullptr; // [n] nodes by (degree desc, id)
    int32_t *d_colD = nullptr;  // [nnz] each neighbour list by (degree desc, id)
    int32_t *d_band_v = nullptr;  // [n_noniso] non-isolated nodes by (BFS level, id)
    uint32_t *d_noniso = nullptr; // [words] bit v set: v has at least one edge
    std::vector<int32_t> band_off;  // host: band b is d_band_v[band_off[b], band_off[b+1])
    int32_t n_noniso = 0;       // nodes with at least one edge
    int32_t algorithm = 0;      // 0: bit-parallel sweeps, 1: edge-parallel union-find
    gapa::FitnessWorkspace ws;
    gapa::KernelTimer timer;
    bool failed = false;
};

namespace gapa {

// Fitness of P individuals given as removed-node bit sets masks[P][W]
// (device) with alive[P] = surviving non-isolated nodes of each.  Writes
// fitness[P] (int64) and, if mcn != nullptr, mcn[P] (int32).  Runs the graph's
// selected algorithm.
int eval_masks(gapa_graph *g, const uint32_t *masks, const int32_t *alive, int32_t P, int64_t *fitness, int32_t *mcn,
               FitnessWorkspace &ws, KernelTimer *timer, hipStream_t s);
int eval_masks_bits(gapa_graph *g, const uint32_t *masks, const int32_t *alive, int32_t P, int64_t *fitness,
                    int32_t *mcn, FitnessWorkspace &ws, KernelTimer *timer, hipStream_t s);
int eval_masks_unionfind(gapa_graph *g, const uint32_t *masks, int32_t P, int64_t *fitness, int32_t *mcn,
                         FitnessWorkspace &ws, KernelTimer *timer, hipStream_t s);
// Same from gene rows genes[P][k] (device node ids; a repeated id in a row is
// one removal); a gene outside [0, n) sets flag[0] and is ignored.
int eval_genes(gapa_graph *g, const int32_t *genes, int32_t P, int32_t k, int64_t *fitness, int32_t *mcn,
               int32_t *flag, FitnessWorkspace &ws, KernelTimer *timer, hipStream_t s);

// Fills count 32-bit words at p with value (a kernel, not a memset node).
int launch_fill_u32(void *p, uint32_t value, int64_t count, hipStream_t s);

// genes[P][k] (device) -> masks[P][W] and alive[P]; out-of-range genes
// raise flag[0].
int launch_mask_build(const int32_t *genes, int32_t P, int32_t k, int32_t n, int32_t W, const uint32_t *noniso,
                      int32_t n_noniso, uint32_t *masks, int32_t *alive, int32_t *flag, hipStream_t s);

// ------------------------------------------------------------------- GA -----

// Dynamic LDS of the operator kernels for n nodes and budget k, and the
// function attributes they need when it exceeds the default 64 KiB.
size_t ga_op_lds_bytes(int32_t n, int32_t k);
int ga_prepare_kernels(size_t lds);

int ga_init_population(gapa_ga *ga, hipStream_t s);
int ga_generation(gapa_ga *ga, hipStream_t s);
int ga_launch_init(gapa_ga *ga, hipStream_t s);
int ga_launch_offspring(gapa_ga *ga, uint32_t gen, int32_t count, hipStream_t s);
// Elitism over the npar current parents (f_par / par_rows; 0 at generation 0)
// and npool evaluated offspring (f_pool[q] is the fitness of child pool[q], or
// of child q when pool is NULL); writes the next population buffer.
int ga_rank_and_gather(gapa_ga *ga, const int64_t *f_par, const int32_t *par_rows, int32_t npar,
                       const int64_t *f_pool, const int32_t *pool, int32_t npool, hipStream_t s);

// Error reporting for HIP calls.
int hip_fail(hipError_t e, const char *what);
#define GAPA_HIP(call)                                                  \
    do {                                                                \
        hipError_t _e = (call);                                         \
        if (_e != hipSuccess) return ::gapa::hip_fail(_e, #call);       \
    } while (0)

}  // namespace gapa

struct gapa_ga {
    gapa_graph *graph = nullptr;
    gapa_params params{};
    int32_t lambda = 0;
    uint64_t t_pc = 0, t_pm = 0;  // Bernoulli thresholds floor(p * 2^32)
    int64_t generation = 0;
    int cur = 0;                  // which population buffer is current
    gapa::DevBuf pop[2];          // int32 [P][k]
    gapa::DevBuf fit[2];          // int64 [P]
    gapa::DevBuf children;        // int32 [lambda][k]
    gapa::DevBuf child_fit;       // int64 [lambda]
    gapa::DevBuf masks;           // uint32 [max(P, lambda)][W] removed-node bit sets
    gapa::DevBuf alive;           // int32 [max(P, lambda)] surviving non-isolated nodes
    gapa::DevBuf src;             // int32 [P] elitism: source tag of each kept row
    gapa::DevBuf rank;            // int32 [P + lambda] elitism: offspring below each key
    gapa::DevBuf flag;            // int32 [4] device error flags
    gapa::FitnessWorkspace ws;
    gapa::KernelTimer timer;
    hipStream_t last_stream = nullptr;
    size_t op_lds_bytes = 0;      // dynamic LDS of the operator kernels
    bool failed = false;
};
