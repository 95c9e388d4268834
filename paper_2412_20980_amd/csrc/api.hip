// The C ABI of the library (include/gapa.h): argument and graph validation,
// device buffers, streams, error reporting and kernel timing around the
// fitness and genetic-operator kernels.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace gapa {

namespace {
thread_local std::string g_last_error;
}

void set_error(const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

int hip_fail(hipError_t e, const char *what)
{
    set_error("HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
    return e == hipErrorOutOfMemory ? GAPA_E_OOM : GAPA_E_DEVICE;
}

int DevBuf::reserve(size_t want)
{
    if (want <= bytes && ptr) return GAPA_OK;
    if (borrowed) {
        set_error("a borrowed scratch buffer of %zu bytes cannot hold %zu", bytes, want);
        return GAPA_E_INVALID_ARG;
    }
    release();
    if (want == 0) want = 4;
    hipError_t e = hipMalloc(&ptr, want);
    if (e != hipSuccess) {
        ptr = nullptr;
        bytes = 0;
        (void)hipGetLastError();
        set_error("device allocation of %zu bytes failed: %s", want, hipGetErrorString(e));
        return GAPA_E_OOM;
    }
    bytes = want;
    return GAPA_OK;
}

void DevBuf::release()
{
    if (ptr && !borrowed) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
    borrowed = false;
}

// ------------------------------------------------------------------ timer ----

hipEvent_t KernelTimer::take()
{
    if (!free_.empty()) {
        hipEvent_t e = free_.back();
        free_.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void KernelTimer::begin(const char *name, hipStream_t s)
{
    Pending p;
    p.name = name;
    p.a = take();
    p.b = take();
    if (!p.a || !p.b) {
        open_.push_back(SIZE_MAX);
        return;
    }
    (void)hipEventRecord(p.a, s);
    pending_.push_back(p);
    open_.push_back(pending_.size() - 1);
}

void KernelTimer::end(hipStream_t s)
{
    if (open_.empty()) return;
    const size_t i = open_.back();
    open_.pop_back();
    if (i != SIZE_MAX) (void)hipEventRecord(pending_[i].b, s);
}

int KernelTimer::collect(gapa_kernel_time *out, int cap, int *count)
{
    for (auto &p : pending_) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(p.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        auto &t = totals_[p.name];
        t.first += 1;
        t.second += ms;
        free_.push_back(p.a);
        free_.push_back(p.b);
    }
    pending_.clear();
    names_.clear();
    for (auto &kv : totals_) names_.push_back(kv.first);
    int i = 0;
    for (auto &kv : totals_) {
        if (i < cap && out) {
            out[i].name = names_[i].c_str();
            out[i].launches = kv.second.first;
            out[i].total_ms = kv.second.second;
        }
        ++i;
    }
    if (count) *count = (int)totals_.size();
    return GAPA_OK;
}


KernelTimer::~KernelTimer()
{
    for (auto &p : pending_) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : free_) (void)hipEventDestroy(e);
}

namespace {

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int check_device(int *dev)
{
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        set_error("no HIP device available");
        return GAPA_E_NO_DEVICE;
    }
    if (hipGetDevice(dev) != hipSuccess) {
        set_error("hipGetDevice failed");
        return GAPA_E_NO_DEVICE;
    }
    return GAPA_OK;
}

uint64_t bernoulli_threshold(double p)
{
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return 1ull << 32;
    return (uint64_t)std::floor(std::ldexp(p, 32));
}

int validate_graph(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci)
{
    if (rp[0] != 0) {
        set_error("row_ptr[0] = %d, expected 0", rp[0]);
        return GAPA_E_BAD_GRAPH;
    }
    for (int32_t v = 0; v < n; ++v) {
        if (rp[v + 1] < rp[v]) {
            set_error("row_ptr decreases at node %d", v);
            return GAPA_E_BAD_GRAPH;
        }
    }
    if ((int64_t)rp[n] != nnz) {
        set_error("row_ptr[n] = %d but nnz = %lld", rp[n], (long long)nnz);
        return GAPA_E_BAD_GRAPH;
    }
    for (int32_t v = 0; v < n; ++v) {
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
            const int32_t u = ci[e];
            if (u < 0 || u >= n) {
                set_error("neighbour %d of node %d is out of range", u, v);
                return GAPA_E_BAD_GRAPH;
            }
            if (u == v) {
                set_error("self-loop at node %d", v);
                return GAPA_E_BAD_GRAPH;
            }
            if (e > rp[v] && ci[e - 1] >= u) {
                set_error("neighbours of node %d are not strictly ascending", v);
                return GAPA_E_BAD_GRAPH;
            }
            // symmetric: v must appear in u's (ascending) list
            if (!std::binary_search(ci + rp[u], ci + rp[u + 1], v)) {
                set_error("edge (%d, %d) has no reverse entry", v, u);
                return GAPA_E_BAD_GRAPH;
            }
        }
    }
    return GAPA_OK;
}

// Host-side orderings used by the bit-parallel fitness kernels.  The graph
// may be a disjoint union of instances (node ranges [voff[b], voff[b+1]));
// everything is computed per instance and only the bands are shared.
//   order  - the nodes of each instance by (degree desc, id): root candidates;
//   colD   - each neighbour list by (degree desc, id): hubs are read first;
//   bands  - non-isolated nodes by breadth-first level from the kSources
//            highest-degree nodes of their instance (multi-source); level l
//            of every instance falls in the same band; levels are merged
//            into at most kMaxBands bands; nodes no source reaches take the
//            level after their instance's last one.
constexpr int kSources = 64;
constexpr int kMaxBands = 24;
constexpr int kMinBand = 16384;  // at n = 200k the 8.9k nodes of BFS levels 3+ join level 2's band: 2 % faster

// Also returns each source's index among its instance's sources (the t-th
// source is order[voff[b] + t]; -1 for every other node) and, when band 0
// holds exactly the sources (no merge took them into band 1), its size in
// src_band (else 0).
void graph_orderings(int32_t n, const int32_t *rp, const int32_t *ci, const std::vector<int32_t> &voff,
                     std::vector<int32_t> &order, std::vector<int32_t> &colD, std::vector<int32_t> &band_v,
                     std::vector<int32_t> &band_off, std::vector<int8_t> &src_idx, int32_t &src_band)
{
    std::vector<int32_t> deg(n);
    for (int32_t v = 0; v < n; ++v) deg[v] = rp[v + 1] - rp[v];
    auto by_degree = [&](int32_t a, int32_t b) { return deg[a] != deg[b] ? deg[a] > deg[b] : a < b; };
    order.resize(n);
    for (int32_t v = 0; v < n; ++v) order[v] = v;
    colD.assign(ci, ci + rp[n]);
    for (int32_t v = 0; v < n; ++v) std::sort(colD.begin() + rp[v], colD.begin() + rp[v + 1], by_degree);

    std::vector<int32_t> level(n, -1);
    std::vector<int32_t> frontier, next;
    std::vector<std::pair<int32_t, int8_t>> sources;
    int32_t nlev = 1;
    for (size_t b = 0; b + 1 < voff.size(); ++b) {
        const int32_t v0 = voff[b], v1 = voff[b + 1];
        std::sort(order.begin() + v0, order.begin() + v1, by_degree);
        frontier.clear();
        for (int32_t p = v0; p < v1 && (int)frontier.size() < kSources; ++p) {
            const int32_t v = order[p];
            if (deg[v] == 0) break;
            level[v] = 0;
            frontier.push_back(v);
        }
        for (size_t t = 0; t < frontier.size(); ++t) sources.emplace_back(frontier[t], (int8_t)t);
        int32_t lv = 0;
        while (!frontier.empty()) {
            next.clear();
            for (int32_t v : frontier)
                for (int32_t e = rp[v]; e < rp[v + 1]; ++e)
                    if (level[ci[e]] < 0) {
                        level[ci[e]] = lv + 1;
                        next.push_back(ci[e]);
                    }
            frontier.swap(next);
            ++lv;
        }
        for (int32_t v = v0; v < v1; ++v)  // non-isolated nodes no source reaches
            if (deg[v] > 0 && level[v] < 0) level[v] = lv;
        nlev = std::max(nlev, lv + 1);
    }
    band_v.clear();
    for (int32_t v = 0; v < n; ++v)
        if (deg[v] > 0) band_v.push_back(v);
    std::sort(band_v.begin(), band_v.end(),
              [&](int32_t a, int32_t b) { return level[a] != level[b] ? level[a] < level[b] : a < b; });
    // Bands: level 0 (the sources) alone; later levels joined until a band
    // holds kMinBand nodes, so that sparse tail levels do not each cost a
    // launch (a last remainder below kMinBand joins the band before it); at
    // most kMaxBands bands.
    std::vector<int32_t> lev_count(nlev, 0);
    for (int32_t v : band_v) ++lev_count[level[v]];
    band_off.assign(1, 0);
    int32_t acc = 0, cur = 0;
    for (int32_t lv2 = 0; lv2 < nlev; ++lv2) {
        acc += lev_count[lv2];
        cur += lev_count[lv2];
        if (lv2 == 0 || cur >= kMinBand) {
            band_off.push_back(acc);
            cur = 0;
        }
    }
    if (band_off.back() != acc) {
        // a sparse tail joins the band before it (unless that is the sources)
        if (band_off.size() > 2 && cur < kMinBand) band_off.back() = acc;
        else band_off.push_back(acc);
    }
    while ((int32_t)band_off.size() - 1 > kMaxBands) {  // merge the two smallest neighbours
        size_t best = 1;
        int32_t best_size = INT32_MAX;
        for (size_t b = 1; b + 1 < band_off.size(); ++b) {
            const int32_t sz = band_off[b + 1] - band_off[b - 1];
            if (sz < best_size) {
                best_size = sz;
                best = b;
            }
        }
        band_off.erase(band_off.begin() + best);
    }
    src_idx.assign((size_t)std::max(n, 1), (int8_t)-1);
    for (const auto &st : sources) src_idx[st.first] = st.second;
    src_band = band_off.size() > 1 && band_off[1] == (int32_t)sources.size() ? (int32_t)sources.size() : 0;
}

#define API_TRY(expr)                  \
    do {                               \
        int _rc = (expr);              \
        if (_rc != GAPA_OK) return _rc; \
    } while (0)

void release_workspace(FitnessWorkspace &w)
{
    for (DevBuf *b : {&w.parent, &w.count, &w.dead, &w.reach, &w.ucount, &w.pairs, &w.worklist, &w.pflag, &w.small,
                      &w.masks,
                      &w.alive, &w.genes, &w.fitness, &w.mcn, &w.flag, &w.six_mats, &w.six_tot})
        b->release();
    for (FitnessWorkspace *l : w.lanes) {
        release_workspace(*l);
        delete l;
    }
    w.lanes.clear();
    for (hipStream_t st : w.lane_streams) (void)hipStreamDestroy(st);
    w.lane_streams.clear();
    for (hipEvent_t ev : w.lane_done) (void)hipEventDestroy(ev);
    w.lane_done.clear();
    if (w.fork) (void)hipEventDestroy(w.fork);
    w.fork = nullptr;
    w.stats_ctr = nullptr;
    w.pflag_clear = false;
}

int fitness_stats(FitnessWorkspace &w, int64_t out[4])
{
    for (int i = 0; i < 4; ++i) out[i] = 0;
    if (!w.stats_ctr) return GAPA_OK;
    // the pass's counters: [0] worklist count, [2..] changed flags (the first is
    // set by the pass itself), [36, 38) the 64-bit pair count
    int32_t h[40] = {0};
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(h, w.stats_ctr, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "fitness stats");
    out[0] = w.stats_B;
    out[1] = h[0];
    uint64_t pairs = 0;
    std::memcpy(&pairs, h + 36, 8);
    out[2] = (int64_t)pairs;
    for (int i = 3; i < 36; ++i) out[3] += h[i] != 0;  // changed flags of sweeps 1..
    return GAPA_OK;
}

int fail_handle(bool *failed, int rc)
{
    if (rc == GAPA_E_DEVICE) *failed = true;
    return rc;
}

// Device copy of a validated CSR and its orderings; voff splits the nodes
// into instances (a single graph: {0, n}).
constexpr uint64_t kFnvBasis = 0xcbf29ce484222325ull;

// FNV-1a, 64-bit (Fowler, Noll, Vo), continuing from h.
uint64_t fnv1a(const void *data, size_t bytes, uint64_t h)
{
    const unsigned char *p = static_cast<const unsigned char *>(data);
    for (size_t i = 0; i < bytes; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

int graph_build(int dev, int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                const std::vector<int32_t> &voff, int algorithm, gapa_graph **out)
{
    gapa_graph *g = new (std::nothrow) gapa_graph();
    if (!g) {
        set_error("host allocation failed");
        return GAPA_E_OOM;
    }
    g->device = dev;
    g->n = n;
    g->nnz = nnz;
    g->content_hash = fnv1a(&n, 4, kFnvBasis);
    g->content_hash = fnv1a(row_ptr, (size_t)(n + 1) * 4, g->content_hash);
    g->content_hash = fnv1a(col_idx, (size_t)nnz * 4, g->content_hash);
    g->words = (n + 31) / 32;
    g->algorithm = algorithm;
    std::vector<int32_t> src((size_t)std::max<int64_t>(nnz, 1));
    for (int32_t v = 0; v < n; ++v)
        for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) src[e] = v;
    std::vector<int32_t> order, colD, band_v;
    std::vector<int8_t> src_idx;
    graph_orderings(n, row_ptr, col_idx, voff, order, colD, band_v, g->band_off, src_idx, g->src_band);
    g->n_noniso = (int32_t)band_v.size();
    std::vector<uint32_t> noniso_bits((size_t)g->words, 0u);
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] > row_ptr[v]) noniso_bits[v >> 5] |= 1u << (v & 31);
    auto fail = [&](int rc) {
        gapa_graph_destroy(g);
        return rc;
    };
    hipError_t e;
    if ((e = hipMalloc(&g->d_row_ptr, (size_t)(n + 1) * 4)) != hipSuccess) return fail(hip_fail(e, "hipMalloc"));
    if ((e = hipMalloc(&g->d_col, (size_t)std::max<int64_t>(nnz, 1) * 4)) != hipSuccess)
        return fail(hip_fail(e, "hipMalloc"));
    if ((e = hipMalloc(&g->d_src, (size_t)std::max<int64_t>(nnz, 1) * 4)) != hipSuccess)
        return fail(hip_fail(e, "hipMalloc"));
    if ((e = hipMemcpy(g->d_row_ptr, row_ptr, (size_t)(n + 1) * 4, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(hip_fail(e, "hipMemcpy"));
    if ((e = hipMalloc(&g->d_colD, (size_t)std::max<int64_t>(nnz, 1) * 4)) != hipSuccess)
        return fail(hip_fail(e, "hipMalloc"));
    if ((e = hipMalloc(&g->d_order, (size_t)n * 4)) != hipSuccess) return fail(hip_fail(e, "hipMalloc"));
    if (nnz > 0) {
        if ((e = hipMemcpy(g->d_col, col_idx, (size_t)nnz * 4, hipMemcpyHostToDevice)) != hipSuccess)
            return fail(hip_fail(e, "hipMemcpy"));
        if ((e = hipMemcpy(g->d_src, src.data(), (size_t)nnz * 4, hipMemcpyHostToDevice)) != hipSuccess)
            return fail(hip_fail(e, "hipMemcpy"));
        if ((e = hipMemcpy(g->d_colD, colD.data(), (size_t)nnz * 4, hipMemcpyHostToDevice)) != hipSuccess)
            return fail(hip_fail(e, "hipMemcpy"));
    }
    if ((e = hipMemcpy(g->d_order, order.data(), (size_t)n * 4, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(hip_fail(e, "hipMemcpy"));
    if ((e = hipMalloc(&g->d_noniso, (size_t)g->words * 4)) != hipSuccess) return fail(hip_fail(e, "hipMalloc"));
    if ((e = hipMemcpy(g->d_noniso, noniso_bits.data(), (size_t)g->words * 4, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(hip_fail(e, "hipMemcpy"));
    if ((e = hipMalloc(&g->d_src_idx, src_idx.size())) != hipSuccess) return fail(hip_fail(e, "hipMalloc"));
    if ((e = hipMemcpy(g->d_src_idx, src_idx.data(), src_idx.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(hip_fail(e, "hipMemcpy"));
    {
        std::vector<int4> rec(std::max<size_t>(band_v.size(), 1), make_int4(0, 0, 0, 0));
        for (size_t i = 0; i < band_v.size(); ++i) {
            const int32_t v = band_v[i];
            rec[i] = make_int4(v, row_ptr[v], row_ptr[v + 1], 0);
        }
        if ((e = hipMalloc(&g->d_band_rec, rec.size() * sizeof(int4))) != hipSuccess)
            return fail(hip_fail(e, "hipMalloc"));
        if ((e = hipMemcpy(g->d_band_rec, rec.data(), rec.size() * sizeof(int4), hipMemcpyHostToDevice)) != hipSuccess)
            return fail(hip_fail(e, "hipMemcpy"));
    }
    *out = g;
    return GAPA_OK;
}

void graph_retain(gapa_graph *g)
{
    g->refs.fetch_add(1);
}

// Drops one reference; the last one frees the graph.
void graph_release(gapa_graph *g)
{
    if (g->refs.fetch_sub(1) != 1) return;
    {
        DeviceGuard dg(g->device);
        (void)hipDeviceSynchronize();
        if (g->d_row_ptr) (void)hipFree(g->d_row_ptr);
        if (g->d_col) (void)hipFree(g->d_col);
        for (int32_t *p : {g->d_src, g->d_colD, g->d_order})
            if (p) (void)hipFree(p);
        if (g->d_noniso) (void)hipFree(g->d_noniso);
        if (g->d_src_idx) (void)hipFree(g->d_src_idx);
        if (g->d_band_rec) (void)hipFree(g->d_band_rec);
        release_workspace(g->ws);
    }
    delete g;
}

}  // namespace
}  // namespace gapa

using namespace gapa;

extern "C" {

const char *gapa_last_error(void)
{
    return g_last_error.c_str();
}

const char *gapa_version(void)
{
    return "gapa-mi355x 0.1 (gfx950)";
}

int gapa_graph_create(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, uint32_t flags,
                      gapa_graph **out)
{
    g_last_error.clear();
    if (!out) {
        set_error("out is NULL");
        return GAPA_E_INVALID_ARG;
    }
    *out = nullptr;
    if (n < 1 || n > (1 << 30) || nnz < 0 || nnz >= (1ll << 31) || !row_ptr || (nnz > 0 && !col_idx)) {
        set_error("invalid graph sizes or pointers (n=%d, nnz=%lld)", n, (long long)nnz);
        return GAPA_E_INVALID_ARG;
    }
    if (!(flags & GAPA_TRUST_INPUT)) API_TRY(validate_graph(n, nnz, row_ptr, col_idx));
    int dev = 0;
    API_TRY(check_device(&dev));
    return graph_build(dev, n, nnz, row_ptr, col_idx, std::vector<int32_t>{0, n}, (flags & GAPA_UNIONFIND) ? 1 : 0,
                       out);
}

int gapa_graph_destroy(gapa_graph *g)
{
    if (g) graph_release(g);
    return GAPA_OK;
}

int gapa_eval_population(gapa_graph *g, const int32_t *genes, int32_t P, int32_t k, int64_t *fitness,
                         int32_t *mcn, uint32_t flags, void *stream)
{
    g_last_error.clear();
    if (!g) {
        set_error("graph is NULL");
        return GAPA_E_INVALID_ARG;
    }
    if (g->failed) {
        set_error("graph handle is in a failed state");
        return GAPA_E_STATE;
    }
    if (P < 0 || k < 0 || k > g->n || (P > 0 && ((k > 0 && !genes) || !fitness))) {
        set_error("invalid population arguments (P=%d, k=%d)", P, k);
        return GAPA_E_INVALID_ARG;
    }
    if (P == 0) return GAPA_OK;
    const bool dev_ptrs = flags & GAPA_DEVICE_PTRS;
    const bool trust = flags & GAPA_TRUST_INPUT;
    const bool want_mcn = (flags & GAPA_WANT_MCN) && mcn;
    const Measure measure = (flags & GAPA_MAXIMISE_COMPONENTS) ? kMeasureForest : kMeasurePC;
    if (!dev_ptrs && !trust) {
        for (int64_t i = 0; i < (int64_t)P * k; ++i) {
            if (genes[i] < 0 || genes[i] >= g->n) {
                set_error("gene %d (row %lld) is not a node id in [0, %d)", genes[i], (long long)(i / std::max(k, 1)),
                          g->n);
                return GAPA_E_BAD_GENE;
            }
        }
    }
    DeviceGuard dg(g->device);
    if (!dg.ok) {
        set_error("cannot select device %d", g->device);
        return GAPA_E_DEVICE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    FitnessWorkspace &w = g->ws;
    int rc;
    if ((rc = w.flag.reserve(16)) != GAPA_OK) return rc;
    const int32_t *d_genes = genes;
    int64_t *d_fit = fitness;
    int32_t *d_mcn = want_mcn ? mcn : nullptr;
    if (!dev_ptrs) {
        if ((rc = w.genes.reserve((size_t)std::max<int64_t>((int64_t)P * k, 1) * 4)) != GAPA_OK) return rc;
        if ((rc = w.fitness.reserve((size_t)P * 8)) != GAPA_OK) return rc;
        if (want_mcn && (rc = w.mcn.reserve((size_t)P * 4)) != GAPA_OK) return rc;
        if (k > 0)
            GAPA_HIP(hipMemcpyAsync(w.genes.ptr, genes, (size_t)P * k * 4, hipMemcpyHostToDevice, s));
        d_genes = w.genes.as<int32_t>();
        d_fit = w.fitness.as<int64_t>();
        d_mcn = want_mcn ? w.mcn.as<int32_t>() : nullptr;
    }
    if ((rc = launch_fill_u32(w.flag.ptr, 0u, 4, s)) != GAPA_OK) return fail_handle(&g->failed, rc);
    if ((rc = eval_genes(g, d_genes, P, k, d_fit, d_mcn, w.flag.as<int32_t>(), w, &g->timer, s, measure)) !=
        GAPA_OK)
        return fail_handle(&g->failed, rc);
    if (dev_ptrs && trust) return GAPA_OK;
    int32_t hflag[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(hflag, w.flag.ptr, 16, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && !dev_ptrs) e = hipMemcpyAsync(fitness, d_fit, (size_t)P * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && !dev_ptrs && want_mcn)
        e = hipMemcpyAsync(mcn, d_mcn, (size_t)P * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_handle(&g->failed, hip_fail(e, "eval_population copy-back"));
    if (hflag[0]) {
        set_error("a gene is not a node id in [0, %d)", g->n);
        return GAPA_E_BAD_GENE;
    }
    return GAPA_OK;
}

}  // extern "C"

namespace gapa {
namespace {

// The scratch of gapa_eval_population_noalloc: a fixed device array that
// every GPU the library runs on holds from module load to the end of the
// process.  In host code its name is only a stand-in for the symbol: the
// device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device with that device current and kept in g_scratch.
constexpr size_t kNoAllocBytes = GAPA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// The calling thread's current device must be `dev`.
int scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d is beyond the %d devices the fixed scratch serves", dev, kMaxDevices);
        return GAPA_E_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        GAPA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("hipGetSymbolAddress gave no address for the fixed scratch on device %d", dev);
            return GAPA_E_DEVICE;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return GAPA_OK;
}

}  // namespace
}  // namespace gapa

extern "C" {

int gapa_eval_population_noalloc(gapa_graph *g, const int32_t *genes, int32_t P, int32_t k, int64_t *fitness,
                                 int32_t *mcn, uint32_t flags, void *stream)
{
    g_last_error.clear();
    if (!g) {
        set_error("graph is NULL");
        return GAPA_E_INVALID_ARG;
    }
    if (g->failed) {
        set_error("graph handle is in a failed state");
        return GAPA_E_STATE;
    }
    const uint32_t allowed = GAPA_DEVICE_PTRS | GAPA_TRUST_INPUT | GAPA_WANT_MCN | GAPA_MAXIMISE_COMPONENTS;
    if (!(flags & GAPA_DEVICE_PTRS) || (flags & ~allowed) != 0) {
        set_error("gapa_eval_population_noalloc takes device pointers (GAPA_DEVICE_PTRS) and only "
                  "GAPA_TRUST_INPUT, GAPA_WANT_MCN or GAPA_MAXIMISE_COMPONENTS besides");
        return GAPA_E_INVALID_ARG;
    }
    if (P < 0 || k < 0 || k > g->n || (P > 0 && ((k > 0 && !genes) || !fitness))) {
        set_error("invalid population arguments (P=%d, k=%d)", P, k);
        return GAPA_E_INVALID_ARG;
    }
    if (P == 0) return GAPA_OK;
    const bool want_mcn = (flags & GAPA_WANT_MCN) && mcn;
    const Measure measure = (flags & GAPA_MAXIMISE_COMPONENTS) ? kMeasureForest : kMeasurePC;
    DeviceGuard dg(g->device);
    if (!dg.ok) {
        set_error("cannot select device %d", g->device);
        return GAPA_E_DEVICE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *scr = nullptr;
    int rc = scratch_address(g->device, &scr);
    if (rc != GAPA_OK) return fail_handle(&g->failed, rc);
    int32_t *flag = nullptr;
    rc = eval_genes_bits_scratch(g, genes, P, k, fitness, want_mcn ? mcn : nullptr, measure, scr, kNoAllocBytes,
                                 &flag, s);
    if (rc != GAPA_OK) return fail_handle(&g->failed, rc);
    if (flags & GAPA_TRUST_INPUT) return GAPA_OK;
    int32_t hflag[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(hflag, flag, 16, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_handle(&g->failed, hip_fail(e, "eval_population_noalloc gene check"));
    if (hflag[0]) {
        set_error("a gene is not a node id in [0, %d)", g->n);
        return GAPA_E_BAD_GENE;
    }
    return GAPA_OK;
}

int gapa_sixdst_eval(gapa_graph *g, const int32_t *genes, int32_t P, int32_t k, int32_t hops, int64_t *pc,
                     int32_t *mcn, uint32_t flags, void *stream)
{
    g_last_error.clear();
    if (!g) {
        set_error("graph is NULL");
        return GAPA_E_INVALID_ARG;
    }
    if (g->failed) {
        set_error("graph handle is in a failed state");
        return GAPA_E_STATE;
    }
    if (g->n > GAPA_SIXDST_MAX_N || hops < 1) {
        set_error("dense reachability needs n <= %d (n = %d) and hops >= 1 (hops = %d)", GAPA_SIXDST_MAX_N, g->n,
                  hops);
        return GAPA_E_INVALID_ARG;
    }
    if (P < 0 || k < 0 || k > g->n || (P > 0 && ((k > 0 && !genes) || !pc || !mcn))) {
        set_error("invalid population arguments (P=%d, k=%d)", P, k);
        return GAPA_E_INVALID_ARG;
    }
    if (P == 0) return GAPA_OK;
    const bool dev_ptrs = flags & GAPA_DEVICE_PTRS;
    const bool trust = flags & GAPA_TRUST_INPUT;
    if (!dev_ptrs && !trust) {
        for (int64_t i = 0; i < (int64_t)P * k; ++i) {
            if (genes[i] < 0 || genes[i] >= g->n) {
                set_error("gene %d (row %lld) is not a node id in [0, %d)", genes[i], (long long)(i / std::max(k, 1)),
                          g->n);
                return GAPA_E_BAD_GENE;
            }
        }
    }
    DeviceGuard dg(g->device);
    if (!dg.ok) {
        set_error("cannot select device %d", g->device);
        return GAPA_E_DEVICE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    FitnessWorkspace &w = g->ws;
    // individuals in flight: three dense matrices each, within a 2 GiB workspace
    const size_t per = sixdst_bytes_per_individual(g->n);
    const int32_t chunk = (int32_t)std::max<size_t>(1, std::min<size_t>((size_t)P, ((size_t)2 << 30) / per));
    int rc;
    if ((rc = w.flag.reserve(16)) != GAPA_OK || (rc = w.masks.reserve((size_t)P * g->words * 4)) != GAPA_OK ||
        (rc = w.alive.reserve((size_t)P * 4)) != GAPA_OK || (rc = w.six_mats.reserve((size_t)chunk * per)) != GAPA_OK ||
        (rc = w.six_tot.reserve((size_t)chunk * 8)) != GAPA_OK)
        return rc;
    const int32_t *d_genes = genes;
    int64_t *d_pc = pc;
    int32_t *d_mcn = mcn;
    if (!dev_ptrs) {
        if ((rc = w.genes.reserve((size_t)std::max<int64_t>((int64_t)P * k, 1) * 4)) != GAPA_OK ||
            (rc = w.fitness.reserve((size_t)P * 8)) != GAPA_OK || (rc = w.mcn.reserve((size_t)P * 4)) != GAPA_OK)
            return rc;
        if (k > 0)
            GAPA_HIP(hipMemcpyAsync(w.genes.ptr, genes, (size_t)P * k * 4, hipMemcpyHostToDevice, s));
        d_genes = w.genes.as<int32_t>();
        d_pc = w.fitness.as<int64_t>();
        d_mcn = w.mcn.as<int32_t>();
    }
    if ((rc = launch_fill_u32(w.flag.ptr, 0u, 4, s)) != GAPA_OK) return fail_handle(&g->failed, rc);
    if ((rc = launch_mask_build(d_genes, P, k, g->n, g->words, g->d_noniso, g->n_noniso, w.masks.as<uint32_t>(),
                                w.alive.as<int32_t>(), w.flag.as<int32_t>(), s)) != GAPA_OK)
        return fail_handle(&g->failed, rc);
    if ((rc = sixdst_eval_masks(g, w.masks.as<uint32_t>(), P, hops, chunk, w.six_mats.as<uint8_t>(),
                                w.six_tot.as<unsigned long long>(), d_pc, d_mcn, s)) != GAPA_OK)
        return fail_handle(&g->failed, rc);
    if (dev_ptrs && trust) return GAPA_OK;
    int32_t hflag[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(hflag, w.flag.ptr, 16, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && !dev_ptrs) e = hipMemcpyAsync(pc, d_pc, (size_t)P * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && !dev_ptrs) e = hipMemcpyAsync(mcn, d_mcn, (size_t)P * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_handle(&g->failed, hip_fail(e, "sixdst_eval copy-back"));
    if (hflag[0]) {
        set_error("a gene is not a node id in [0, %d)", g->n);
        return GAPA_E_BAD_GENE;
    }
    return GAPA_OK;
}

int gapa_graph_fitness_stats(gapa_graph *g, int64_t out[4])
{
    if (!g || !out) return GAPA_E_INVALID_ARG;
    DeviceGuard dg(g->device);
    return fitness_stats(g->ws, out);
}

int gapa_ga_fitness_stats(gapa_ga *ga, int64_t out[4])
{
    if (!ga || !out) return GAPA_E_INVALID_ARG;
    DeviceGuard dg(ga->graph->device);
    return fitness_stats(ga->ws, out);
}

int gapa_graph_set_timing(gapa_graph *g, int32_t enable)
{
    if (!g) return GAPA_E_INVALID_ARG;
    if (enable < 0 || enable > 2) return GAPA_E_INVALID_ARG;
    g->timer.level = enable;
    return GAPA_OK;
}

int gapa_graph_kernel_times(gapa_graph *g, gapa_kernel_time *out, int32_t cap, int32_t *count)
{
    if (!g) return GAPA_E_INVALID_ARG;
    DeviceGuard dg(g->device);
    int c = 0;
    int rc = g->timer.collect(out, cap, &c);
    if (count) *count = c;
    return rc;
}

// ---------------------------------------------------------------------- GA ---

}  // extern "C"

namespace gapa {
namespace {

bool params_ok(const gapa_params *p, int32_t n)
{
    return p->k >= 1 && p->k <= n / 2 && p->pop >= 1 && p->tournament >= 1 && p->tournament <= 64 &&
           p->offspring >= 0 && p->pc >= 0.0 && p->pc <= 1.0 && p->pm >= 0.0 && p->pm <= 1.0 &&
           (p->flags & ~(uint32_t)(GAPA_GRAPH_REPLAY | GAPA_MINIMISE_MCN | GAPA_MAXIMISE_COMPONENTS)) == 0 &&
           (p->flags & (GAPA_MINIMISE_MCN | GAPA_MAXIMISE_COMPONENTS)) !=
               (uint32_t)(GAPA_MINIMISE_MCN | GAPA_MAXIMISE_COMPONENTS) &&
           p->reserved == 0;
}

// Fills the instance table and sizes every buffer of a GA over `count`
// instances; instance b has parameters p[b], n[b] nodes, n_noniso[b]
// non-isolated nodes; slot_stride > 0 puts instance b's slots at
// b * slot_stride (a batch), 0 keeps them contiguous from 0 (one GA).
int ga_allocate(gapa_ga *ga, int32_t count, const gapa_params *p, const int32_t *n, const int32_t *n_noniso,
                int32_t slot_stride)
{
    ga->count = count;
    ga->params = p[0];
    ga->lambda = p[0].offspring > 0 ? p[0].offspring : p[0].pop;
    ga->t_pc = bernoulli_threshold(p[0].pc);
    ga->t_pm = bernoulli_threshold(p[0].pm);
    ga->use_graph = (p[0].flags & GAPA_GRAPH_REPLAY) != 0;
    ga->hinst.assign(count, GaInst{});
    int64_t pop_el = 0, child_el = 0, mask_w = 0;
    int32_t fit_n = 0, noniso_w = 0, slots = 0;
    size_t lds = 0;
    for (int32_t b = 0; b < count; ++b) {
        GaInst &I = ga->hinst[b];
        const int32_t L = p[b].offspring > 0 ? p[b].offspring : p[b].pop;
        const int32_t R = std::max(p[b].pop, L);
        I.P = p[b].pop;
        I.L = L;
        I.k = p[b].k;
        I.n = n[b];
        I.W = (n[b] + 31) / 32;
        I.KW = (p[b].k + 31) / 32;
        I.T = p[b].tournament;
        I.n_noniso = n_noniso[b];
        I.seed = p[b].seed;
        I.t_pc = bernoulli_threshold(p[b].pc);
        I.t_pm = bernoulli_threshold(p[b].pm);
        I.pop_off = pop_el;
        I.child_off = child_el;
        I.mask_off = mask_w;
        I.fit_off = fit_n;
        I.slot_off = slot_stride > 0 ? b * slot_stride : slots;
        I.noniso_off = noniso_w;
        pop_el += (int64_t)I.P * I.k;
        child_el += (int64_t)R * I.k;
        mask_w += (int64_t)R * I.W;
        fit_n += I.P;
        noniso_w += I.W;
        slots += R;
        ga->max_pop = std::max(ga->max_pop, I.P);
        ga->max_lambda = std::max(ga->max_lambda, L);
        ga->max_pop_lambda = std::max(ga->max_pop_lambda, I.P + L);
        lds = std::max(lds, ga_op_lds_bytes(n[b], p[b].k));
    }
    if (slot_stride > 0) slots = count * slot_stride;
    ga->op_lds_bytes = lds;
    if (pop_el >= (1ll << 31) || child_el >= (1ll << 31)) {
        set_error("population too large");
        return GAPA_E_INVALID_ARG;
    }
    if (lds > 160 * 1024) {
        set_error("n and k need %zu bytes of LDS for the operator kernels (limit 160 KiB)", lds);
        return GAPA_E_INVALID_ARG;
    }
    int rc = GAPA_OK;
    for (int i = 0; i < 2 && rc == GAPA_OK; ++i) {
        rc = ga->pop[i].reserve((size_t)pop_el * 4);
        if (rc == GAPA_OK) rc = ga->fit[i].reserve((size_t)fit_n * 8);
    }
    if (rc == GAPA_OK) rc = ga->children.reserve((size_t)child_el * 4);
    if (rc == GAPA_OK) rc = ga->child_fit.reserve((size_t)slots * 8);
    ga->slots = slots;
    ga->objective_mcn = (p[0].flags & GAPA_MINIMISE_MCN) != 0;
    ga->objective_forest = (p[0].flags & GAPA_MAXIMISE_COMPONENTS) != 0;
    if (rc == GAPA_OK && ga->objective_mcn) rc = ga->child_mcn.reserve((size_t)slots * 4);
    if (rc == GAPA_OK) rc = ga->masks.reserve((size_t)mask_w * 4);
    if (rc == GAPA_OK) rc = ga->alive.reserve((size_t)slots * 4);
    if (rc == GAPA_OK) rc = ga->src.reserve((size_t)fit_n * 4);
    if (rc == GAPA_OK) rc = ga->flag.reserve(16);
    if (rc == GAPA_OK) rc = ga->gen_ctr.reserve(16);
    if (rc == GAPA_OK) rc = ga->inst.reserve(sizeof(GaInst) * count);
    if (rc != GAPA_OK) return rc;
    GAPA_HIP(hipMemcpy(ga->inst.ptr, ga->hinst.data(), sizeof(GaInst) * count, hipMemcpyHostToDevice));
    return ga_prepare_kernels(lds);
}

template <class T> int upload(DevBuf &buf, const std::vector<T> &v)
{
    int rc = buf.reserve(std::max<size_t>(v.size(), 1) * sizeof(T));
    if (rc != GAPA_OK) return rc;
    if (!v.empty()) GAPA_HIP(hipMemcpy(buf.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return GAPA_OK;
}

void release_graphs(gapa_ga *ga)
{
    for (auto &r : ga->replays) {
        if (r.exec) (void)hipGraphExecDestroy(r.exec);
        if (r.graph) (void)hipGraphDestroy(r.graph);
    }
    ga->replays.clear();
}

gapa_ga::Replay *find_replay(gapa_ga *ga, int parity, int32_t gens)
{
    for (auto &r : ga->replays)
        if (r.parity == parity && r.gens == gens) return &r;
    return nullptr;
}

// Records `gens` generations starting from population buffer c as one HIP
// graph.  The host-side counters are restored afterwards: nothing ran.
int capture_generations(gapa_ga *ga, int c, int32_t gens)
{
    if (!ga->cap_stream) GAPA_HIP(hipStreamCreateWithFlags(&ga->cap_stream, hipStreamNonBlocking));
    const int64_t gen = ga->generation;
    GAPA_HIP(hipStreamBeginCapture(ga->cap_stream, hipStreamCaptureModeRelaxed));
    int rc = GAPA_OK;
    for (int32_t i = 0; i < gens && rc == GAPA_OK; ++i) rc = ga_generation(ga, ga->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(ga->cap_stream, &graph);
    ga->cur = c;
    ga->generation = gen;
    if (rc != GAPA_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc != GAPA_OK ? rc : hip_fail(e, "hipStreamEndCapture");
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e2 != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e2, "hipGraphInstantiate");
    }
    if (ga->replays.size() >= 8) {  // keep the one-generation recordings, drop the oldest longer one
        for (size_t i = 0; i < ga->replays.size(); ++i)
            if (ga->replays[i].gens > 1) {
                (void)hipGraphExecDestroy(ga->replays[i].exec);
                (void)hipGraphDestroy(ga->replays[i].graph);
                ga->replays.erase(ga->replays.begin() + i);
                break;
            }
    }
    ga->replays.push_back(gapa_ga::Replay{c, gens, graph, exec});
    return GAPA_OK;
}

void check_tuning_version(gapa_ga *ga)
{
    if (ga->captured_version != ga->graph->tune_version) {
        // launch shapes changed: record again, after one eager generation
        release_graphs(ga);
        ga->warm = false;
        ga->captured_version = ga->graph->tune_version;
    }
}

int ga_run(gapa_ga *ga, int32_t n_generations, hipStream_t s)
{
    check_tuning_version(ga);
    for (int32_t i = 0; i < n_generations;) {
        if (ga->surr) {
            const int rc = surrogate_generation(ga, s);
            if (rc != GAPA_OK) return rc;
            ++i;
            continue;
        }
        if (!(ga->use_graph && ga->warm && ga->timer.level == 0)) {
            const int rc = ga_generation(ga, s);
            if (rc != GAPA_OK) return rc;
            ga->warm = true;  // every buffer of a generation has its final size
            ++i;
            continue;
        }
        const int c = ga->cur;
        // a recording of all remaining generations (made by gapa_ga_record), else one generation
        gapa_ga::Replay *r = find_replay(ga, c, n_generations - i);
        if (!r) {
            r = find_replay(ga, c, 1);
            if (!r) {
                const int rc = capture_generations(ga, c, 1);
                if (rc != GAPA_OK) return rc;
                r = find_replay(ga, c, 1);
            }
        }
        const int32_t gens = r->gens;
        GAPA_HIP(hipGraphLaunch(r->exec, s));
        ga->cur = (gens & 1) ? 1 - c : c;
        ga->generation += gens;
        i += gens;
    }
    return GAPA_OK;
}

int ga_record(gapa_ga *ga, int32_t n_generations)
{
    check_tuning_version(ga);
    if (!ga->use_graph || ga->surr || !ga->warm) {
        set_error("recording needs GAPA_GRAPH_REPLAY, no surrogate, and one generation run since the last "
                  "tuning change");
        return GAPA_E_STATE;
    }
    if (n_generations < 1 || n_generations > 4096) {
        set_error("n_generations must be in [1, 4096]");
        return GAPA_E_INVALID_ARG;
    }
    if (find_replay(ga, ga->cur, n_generations)) return GAPA_OK;
    return capture_generations(ga, ga->cur, n_generations);
}

int ga_step_checked(gapa_ga *ga, int32_t n_generations, hipStream_t s)
{
    if (ga->failed) {
        set_error("GA handle is in a failed state");
        return GAPA_E_STATE;
    }
    if (n_generations < 0 || ga->generation + n_generations >= (1ll << 32) - 1) {
        set_error("invalid generation count (the counter must stay below 2^32 - 1)");
        return GAPA_E_INVALID_ARG;
    }
    DeviceGuard dg(ga->graph->device);
    if (s != ga->last_stream) {
        // order this call after work enqueued earlier on another stream
        hipError_t e = hipStreamSynchronize(ga->last_stream);
        if (e != hipSuccess) return fail_handle(&ga->failed, hip_fail(e, "hipStreamSynchronize"));
        ga->last_stream = s;
    }
    const int rc = ga_run(ga, n_generations, s);
    return rc == GAPA_OK ? rc : fail_handle(&ga->failed, rc);
}

int ga_sync_check(gapa_ga *ga)
{
    int32_t hflag[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(hflag, ga->flag.ptr, 16, hipMemcpyDeviceToHost, ga->last_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ga->last_stream);
    if (e != hipSuccess) return fail_handle(&ga->failed, hip_fail(e, "GA synchronisation"));
    if (hflag[0]) {
        ga->failed = true;
        set_error("a random draw exhausted its 2^24 attempts");
        return GAPA_E_STATE;
    }
    return GAPA_OK;
}

// Rows of instance b (all P, or only the best with best_only) to the host.
int ga_copy_out(gapa_ga *ga, int32_t b, bool best_only, int32_t *genes_out, int64_t *fitness_out)
{
    if (ga->failed) {
        set_error("GA handle is in a failed state");
        return GAPA_E_STATE;
    }
    DeviceGuard dg(ga->graph->device);
    const GaInst &I = ga->hinst[b];
    const int32_t rows = best_only ? 1 : I.P;
    hipStream_t s = ga->last_stream;
    hipError_t e = hipSuccess;
    if (genes_out)
        e = hipMemcpyAsync(genes_out, ga->pop[ga->cur].as<int32_t>() + I.pop_off, (size_t)rows * I.k * 4,
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && fitness_out)
        e = hipMemcpyAsync(fitness_out, ga->fit[ga->cur].as<int64_t>() + I.fit_off, (size_t)rows * 8,
                           hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return fail_handle(&ga->failed, hip_fail(e, "population copy"));
    return ga_sync_check(ga);
}

void ga_release(gapa_ga *ga)
{
    (void)hipDeviceSynchronize();
    release_graphs(ga);
    surrogate_release(ga->surr);
    ga->surr = nullptr;
    if (ga->cap_stream) (void)hipStreamDestroy(ga->cap_stream);
    ga->cap_stream = nullptr;
    for (auto *b : {&ga->pop[0], &ga->pop[1], &ga->fit[0], &ga->fit[1], &ga->children, &ga->child_fit, &ga->child_mcn, &ga->masks,
                    &ga->alive, &ga->src, &ga->flag, &ga->gen_ctr, &ga->inst, &ga->noniso_buf,
                    &ga->tab_voff, &ga->tab_live_init, &ga->tab_live_gen, &ga->tab_moff, &ga->tab_node_inst,
                    &ga->tab_tiles})
        b->release();
    release_workspace(ga->ws);
}

int ga_collect_times(gapa_ga *ga, gapa_kernel_time *out, int32_t cap, int32_t *count)
{
    DeviceGuard dg(ga->graph->device);
    int c = 0;
    int rc = ga->timer.collect(out, cap, &c);
    if (count) *count = c;
    return rc;
}

}  // namespace
}  // namespace gapa

extern "C" {

int gapa_ga_create(gapa_graph *g, const gapa_params *p, void *stream, gapa_ga **out)
{
    g_last_error.clear();
    if (!out || !g || !p) {
        set_error("NULL argument");
        return GAPA_E_INVALID_ARG;
    }
    *out = nullptr;
    if (g->failed) {
        set_error("graph handle is in a failed state");
        return GAPA_E_STATE;
    }
    if (!params_ok(p, g->n)) {
        set_error("invalid GA parameters (need 1 <= k <= n/2, pop >= 1, 1 <= T <= 64, pc, pm in [0, 1], "
                  "flags from GAPA_GRAPH_REPLAY | GAPA_MINIMISE_MCN | GAPA_MAXIMISE_COMPONENTS, at most one "
                  "objective)");
        return GAPA_E_INVALID_ARG;
    }
    DeviceGuard dg(g->device);
    gapa_ga *ga = new (std::nothrow) gapa_ga();
    if (!ga) {
        set_error("host allocation failed");
        return GAPA_E_OOM;
    }
    ga->graph = g;
    graph_retain(g);
    auto fail = [&](int code) {
        gapa_ga_destroy(ga);
        return code;
    };
    int rc = ga_allocate(ga, 1, p, &g->n, &g->n_noniso, 0);
    if (rc != GAPA_OK) return fail(rc);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = launch_fill_u32(ga->flag.ptr, 0u, 4, s)) != GAPA_OK) return fail(rc);
    if ((rc = ga_init_population(ga, s)) != GAPA_OK) return fail(rc);
    ga->last_stream = s;
    *out = ga;
    return GAPA_OK;
}

int gapa_generation_step(gapa_ga *ga, int32_t n_generations, void *stream)
{
    g_last_error.clear();
    if (!ga) {
        set_error("GA is NULL");
        return GAPA_E_INVALID_ARG;
    }
    return ga_step_checked(ga, n_generations, static_cast<hipStream_t>(stream));
}

int gapa_ga_record(gapa_ga *ga, int32_t n_generations)
{
    g_last_error.clear();
    if (!ga) {
        set_error("GA is NULL");
        return GAPA_E_INVALID_ARG;
    }
    if (ga->failed) {
        set_error("GA handle is in a failed state");
        return GAPA_E_STATE;
    }
    DeviceGuard dg(ga->graph->device);
    const int rc = ga_record(ga, n_generations);
    return rc == GAPA_E_DEVICE ? fail_handle(&ga->failed, rc) : rc;
}

int gapa_best(gapa_ga *ga, int32_t *genes_out, int64_t *fitness_out, int64_t *generation_out)
{
    g_last_error.clear();
    if (!ga) {
        set_error("GA is NULL");
        return GAPA_E_INVALID_ARG;
    }
    const int rc = ga_copy_out(ga, 0, true, genes_out, fitness_out);
    if (rc == GAPA_OK && generation_out) *generation_out = ga->generation;
    return rc;
}

int gapa_best_async(gapa_ga *ga, int64_t *fitness_out, void *stream)
{
    g_last_error.clear();
    if (!ga || !fitness_out) {
        set_error("NULL argument");
        return GAPA_E_INVALID_ARG;
    }
    if (ga->failed) {
        set_error("GA handle is in a failed state");
        return GAPA_E_STATE;
    }
    DeviceGuard dg(ga->graph->device);
    // the buffer the last enqueued generation's elitism writes
    const int64_t *src = ga->fit[ga->cur].as<int64_t>() + ga->hinst[0].fit_off;
    GAPA_HIP(hipMemcpyAsync(fitness_out, src, 8, hipMemcpyDefault, static_cast<hipStream_t>(stream)));
    return GAPA_OK;
}

int gapa_get_population(gapa_ga *ga, int32_t *genes_out, int64_t *fitness_out)
{
    g_last_error.clear();
    if (!ga) {
        set_error("GA is NULL");
        return GAPA_E_INVALID_ARG;
    }
    return ga_copy_out(ga, 0, false, genes_out, fitness_out);
}

// Checkpoint file: magic, version, the GA parameters, the graph (n, nnz,
// content hash), the generation, then the population rows [P][k] and their
// fitness [P] in order, and an FNV-1a checksum of everything before it.
static const char kCkptMagic[8] = {'G', 'A', 'P', 'A', 'C', 'K', 'P', 'T'};
constexpr uint32_t kCkptVersion = 1;

struct CkptHeader {
    char magic[8];
    uint32_t version;
    uint32_t pad;
    gapa_params params;
    int32_t n;
    int32_t P;
    int64_t nnz;
    uint64_t graph_hash;
    int64_t generation;
};

int gapa_ga_save(gapa_ga *ga, const char *path)
{
    g_last_error.clear();
    if (!ga || !path) {
        set_error("NULL argument");
        return GAPA_E_INVALID_ARG;
    }
    if (ga->count != 1 || ga->surr) {
        set_error("checkpoints cover a single GA without a surrogate");
        return GAPA_E_STATE;
    }
    const int32_t P = ga->params.pop, k = ga->params.k;
    std::vector<int32_t> rows((size_t)P * k);
    std::vector<int64_t> fit((size_t)P);
    int rc = ga_copy_out(ga, 0, false, rows.data(), fit.data());
    if (rc != GAPA_OK) return rc;
    CkptHeader h{};
    std::memcpy(h.magic, kCkptMagic, 8);
    h.version = kCkptVersion;
    h.params = ga->params;
    h.n = ga->graph->n;
    h.P = P;
    h.nnz = ga->graph->nnz;
    h.graph_hash = ga->graph->content_hash;
    h.generation = ga->generation;
    uint64_t sum = fnv1a(&h, sizeof h, kFnvBasis);
    sum = fnv1a(rows.data(), rows.size() * 4, sum);
    sum = fnv1a(fit.data(), fit.size() * 8, sum);
    FILE *f = std::fopen(path, "wb");
    if (!f) {
        set_error("cannot open %s for writing", path);
        return GAPA_E_INVALID_ARG;
    }
    bool ok = std::fwrite(&h, sizeof h, 1, f) == 1 && std::fwrite(rows.data(), 4, rows.size(), f) == rows.size() &&
              std::fwrite(fit.data(), 8, fit.size(), f) == fit.size() && std::fwrite(&sum, 8, 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) {
        set_error("writing %s failed", path);
        return GAPA_E_INVALID_ARG;
    }
    return GAPA_OK;
}

int gapa_ga_params(gapa_ga *ga, gapa_params *params_out, int64_t *generation_out)
{
    g_last_error.clear();
    if (!ga) {
        set_error("GA is NULL");
        return GAPA_E_INVALID_ARG;
    }
    if (params_out) *params_out = ga->params;
    if (generation_out) *generation_out = ga->generation;
    return GAPA_OK;
}

int gapa_ga_load(gapa_graph *g, const char *path, void *stream, gapa_ga **out)
{
    g_last_error.clear();
    if (!g || !path || !out) {
        set_error("NULL argument");
        return GAPA_E_INVALID_ARG;
    }
    *out = nullptr;
    if (g->failed) {
        set_error("graph handle is in a failed state");
        return GAPA_E_STATE;
    }
    FILE *f = std::fopen(path, "rb");
    if (!f) {
        set_error("cannot open %s", path);
        return GAPA_E_INVALID_ARG;
    }
    CkptHeader h{};
    std::vector<int32_t> rows;
    std::vector<int64_t> fit;
    uint64_t sum = 0;
    bool ok = std::fread(&h, sizeof h, 1, f) == 1 && std::memcmp(h.magic, kCkptMagic, 8) == 0 &&
              h.version == kCkptVersion && h.P == h.params.pop && h.P >= 1 && h.params.k >= 1 && h.P <= (1 << 20) &&
              h.params.k <= (1 << 24) && (int64_t)h.P * h.params.k <= (1ll << 31);
    if (ok) {
        rows.resize((size_t)h.P * h.params.k);
        fit.resize((size_t)h.P);
        ok = std::fread(rows.data(), 4, rows.size(), f) == rows.size() &&
             std::fread(fit.data(), 8, fit.size(), f) == fit.size() && std::fread(&sum, 8, 1, f) == 1;
    }
    std::fclose(f);
    if (ok) {
        uint64_t s2 = fnv1a(&h, sizeof h, kFnvBasis);
        s2 = fnv1a(rows.data(), rows.size() * 4, s2);
        s2 = fnv1a(fit.data(), fit.size() * 8, s2);
        ok = s2 == sum;
    }
    if (!ok) {
        set_error("%s is not a GA checkpoint of this version, or is corrupt", path);
        return GAPA_E_INVALID_ARG;
    }
    if (h.n != g->n || h.nnz != g->nnz || h.graph_hash != g->content_hash) {
        set_error("the checkpoint was taken on a different graph");
        return GAPA_E_INVALID_ARG;
    }
    if (!params_ok(&h.params, g->n) || h.generation < 0 || h.generation >= (1ll << 32)) {
        set_error("invalid parameters in the checkpoint");
        return GAPA_E_INVALID_ARG;
    }
    for (int32_t v : rows)
        if (v < 0 || v >= g->n) {
            set_error("gene %d of the checkpoint is not a node id", v);
            return GAPA_E_BAD_GENE;
        }
    // The kernels rely on the GA's invariants, which the checksum alone does not
    // guarantee (anyone can recompute it): every row strictly ascending (the
    // operators' duplicate search) and the fitness non-decreasing down the
    // population (the elitism merge's binary search).
    const int32_t k = h.params.k;
    for (int32_t r = 0; r < h.P; ++r) {
        const int32_t *row = rows.data() + (size_t)r * k;
        for (int32_t j = 1; j < k; ++j)
            if (row[j] <= row[j - 1]) {
                set_error("row %d of the checkpoint is not strictly ascending", r);
                return GAPA_E_INVALID_ARG;
            }
        if (fit[r] < 0 || (r > 0 && fit[r] < fit[r - 1])) {
            set_error("the checkpoint's fitness is not non-negative and non-decreasing (row %d)", r);
            return GAPA_E_INVALID_ARG;
        }
    }
    DeviceGuard dg(g->device);
    gapa_ga *ga = new (std::nothrow) gapa_ga();
    if (!ga) {
        set_error("host allocation failed");
        return GAPA_E_OOM;
    }
    ga->graph = g;
    graph_retain(g);
    auto fail = [&](int code) {
        gapa_ga_destroy(ga);
        return code;
    };
    int rc = ga_allocate(ga, 1, &h.params, &g->n, &g->n_noniso, 0);
    if (rc != GAPA_OK) return fail(rc);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = launch_fill_u32(ga->flag.ptr, 0u, 4, s)) != GAPA_OK) return fail(rc);
    if ((rc = launch_fill_u32(ga->gen_ctr.ptr, (uint32_t)h.generation, 1, s)) != GAPA_OK) return fail(rc);
    hipError_t e = hipMemcpyAsync(ga->pop[0].ptr, rows.data(), rows.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ga->fit[0].ptr, fit.data(), fit.size() * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(hip_fail(e, "checkpoint upload"));
    ga->cur = 0;
    ga->generation = h.generation;
    ga->last_stream = s;
    *out = ga;
    return GAPA_OK;
}

int gapa_ga_destroy(gapa_ga *ga)
{
    if (!ga) return GAPA_OK;
    gapa_graph *g = ga->graph;
    {
        DeviceGuard dg(g->device);
        ga_release(ga);
    }
    delete ga;
    graph_release(g);
    return GAPA_OK;
}

int gapa_ga_set_timing(gapa_ga *ga, int32_t enable)
{
    if (!ga) return GAPA_E_INVALID_ARG;
    if (enable < 0 || enable > 2) return GAPA_E_INVALID_ARG;
    ga->timer.level = enable;
    return GAPA_OK;
}

int gapa_ga_kernel_times(gapa_ga *ga, gapa_kernel_time *out, int32_t cap, int32_t *count)
{
    if (!ga) return GAPA_E_INVALID_ARG;
    return ga_collect_times(ga, out, cap, count);
}

// ------------------------------------------------------------------ tuning ---

static bool tuning_ok(const gapa_tuning *t)
{
    return t && t->sweep_grid >= 1 && t->sweep_grid <= 65535 && t->band_scan >= 1 && t->sweeps >= 0 &&
           t->sweeps <= 32 && t->band_blocks >= 1 && t->band_blocks <= 65535;
}

int gapa_graph_get_tuning(gapa_graph *g, gapa_tuning *out)
{
    if (!g || !out) return GAPA_E_INVALID_ARG;
    out->sweep_grid = g->tune.sweep_grid;
    out->band_scan = g->tune.band_scan;
    out->sweeps = g->tune.sweeps;
    out->band_blocks = g->tune.band_blocks;
    return GAPA_OK;
}

int gapa_graph_set_tuning(gapa_graph *g, const gapa_tuning *t)
{
    g_last_error.clear();
    if (!g || !tuning_ok(t)) {
        set_error("invalid tuning (sweep_grid and band_blocks 1..65535, band_scan >= 1, sweeps 0..32)");
        return GAPA_E_INVALID_ARG;
    }
    DeviceGuard dg(g->device);
    (void)hipDeviceSynchronize();  // passes in flight keep the shapes they were launched with
    g->tune.sweep_grid = t->sweep_grid;
    g->tune.band_scan = t->band_scan;
    g->tune.sweeps = t->sweeps;
    g->tune.band_blocks = t->band_blocks;
    g->tune_version += 1;
    return GAPA_OK;
}

int gapa_ga_autotune(gapa_ga *ga, int32_t reps, void *stream, gapa_tuning *best_out)
{
    g_last_error.clear();
    if (!ga || reps < 1) {
        set_error("invalid arguments");
        return GAPA_E_INVALID_ARG;
    }
    if (ga->failed) {
        set_error("GA handle is in a failed state");
        return GAPA_E_STATE;
    }
    DeviceGuard dg(ga->graph->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    gapa_graph *g = ga->graph;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail_handle(&ga->failed, hip_fail(e, "hipDeviceSynchronize"));
    const bool init = ga->generation == 0;
    const Tuning saved = g->tune;
    Tuning best = saved;
    double best_t = 1e300;
    const int32_t grids[4] = {1024, 2048, 4096, 8192}, scans[4] = {8, 16, 32, 64}, sweeps[3] = {2, 3, 4};
    const int32_t bands[3] = {2048, 4096, 16384};
    // candidates are timed with events on the stream (no host launch time in the figure)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if ((e = hipEventCreate(&ev0)) != hipSuccess || (e = hipEventCreate(&ev1)) != hipSuccess) {
        if (ev0) (void)hipEventDestroy(ev0);
        return fail_handle(&ga->failed, hip_fail(e, "hipEventCreate"));
    }
    struct EventPair {
        hipEvent_t a, b;
        ~EventPair()
        {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } events{ev0, ev1};
    int rc = GAPA_OK;
    for (int32_t gi : grids)
        for (int32_t sc : scans)
            for (int32_t sw : sweeps)
                for (int32_t bb : bands) {
                    g->tune = Tuning{gi, sc, sw, bb};
                    // one untimed pass sizes the buffers for this shape
                    rc = ga_eval_children(ga, init, s);
                    if (rc == GAPA_OK && (e = hipStreamSynchronize(s)) != hipSuccess) rc = hip_fail(e, "sync");
                    if (rc != GAPA_OK) {
                        g->tune = saved;
                        return fail_handle(&ga->failed, rc);
                    }
                    if ((e = hipEventRecord(ev0, s)) != hipSuccess) rc = hip_fail(e, "hipEventRecord");
                    for (int32_t r = 0; r < reps && rc == GAPA_OK; ++r) rc = ga_eval_children(ga, init, s);
                    if (rc == GAPA_OK && (e = hipEventRecord(ev1, s)) != hipSuccess) rc = hip_fail(e, "hipEventRecord");
                    if (rc == GAPA_OK && (e = hipEventSynchronize(ev1)) != hipSuccess) rc = hip_fail(e, "sync");
                    float ms = 0.f;
                    if (rc == GAPA_OK && (e = hipEventElapsedTime(&ms, ev0, ev1)) != hipSuccess)
                        rc = hip_fail(e, "hipEventElapsedTime");
                    if (rc != GAPA_OK) {
                        g->tune = saved;
                        return fail_handle(&ga->failed, rc);
                    }
                    const double t = ms;
                    if (t < best_t) {
                        best_t = t;
                        best = g->tune;
                    }
                }
    g->tune = best;
    g->tune_version += 1;
    if (best_out) {
        best_out->sweep_grid = best.sweep_grid;
        best_out->band_scan = best.band_scan;
        best_out->sweeps = best.sweeps;
        best_out->band_blocks = best.band_blocks;
    }
    return GAPA_OK;
}

int gapa_batch_autotune(gapa_batch *b, int32_t reps, void *stream, gapa_tuning *best_out)
{
    if (!b) return GAPA_E_INVALID_ARG;
    return gapa_ga_autotune(b->ga, reps, stream, best_out);
}

int gapa_batch_get_tuning(gapa_batch *b, gapa_tuning *out)
{
    if (!b) return GAPA_E_INVALID_ARG;
    return gapa_graph_get_tuning(b->ga->graph, out);
}

int gapa_batch_set_tuning(gapa_batch *b, const gapa_tuning *t)
{
    if (!b) {
        set_error("batch is NULL");
        return GAPA_E_INVALID_ARG;
    }
    return gapa_graph_set_tuning(b->ga->graph, t);
}

// --------------------------------------------------------------- surrogate ---

static int surr_check(gapa_ga *ga)
{
    g_last_error.clear();
    if (!ga) {
        set_error("GA is NULL");
        return GAPA_E_INVALID_ARG;
    }
    if (ga->failed) {
        set_error("GA handle is in a failed state");
        return GAPA_E_STATE;
    }
    if (!ga->surr) {
        set_error("no surrogate attached");
        return GAPA_E_STATE;
    }
    return GAPA_OK;
}

int gapa_surrogate_attach(gapa_ga *ga, const gapa_surrogate_params *sp, void *stream)
{
    g_last_error.clear();
    if (!ga || !sp) {
        set_error("NULL argument");
        return GAPA_E_INVALID_ARG;
    }
    if (ga->failed) {
        set_error("GA handle is in a failed state");
        return GAPA_E_STATE;
    }
    DeviceGuard dg(ga->graph->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (s != ga->last_stream) {
        hipError_t e = hipStreamSynchronize(ga->last_stream);
        if (e != hipSuccess) return fail_handle(&ga->failed, hip_fail(e, "hipStreamSynchronize"));
        ga->last_stream = s;
    }
    const int rc = surrogate_attach(ga, sp, s);
    if (rc != GAPA_OK && ga->surr) {
        (void)hipDeviceSynchronize();
        surrogate_release(ga->surr);
        ga->surr = nullptr;
    }
    return rc == GAPA_E_DEVICE ? fail_handle(&ga->failed, rc) : rc;
}

int gapa_surrogate_stats(gapa_ga *ga, gapa_surrogate_report *out)
{
    int rc = surr_check(ga);
    if (rc != GAPA_OK) return rc;
    if (!out) return GAPA_E_INVALID_ARG;
    DeviceGuard dg(ga->graph->device);
    return fail_handle(&ga->failed, surrogate_stats(ga, out));
}

int gapa_surrogate_judge(const float *yhat, const int32_t *pool, const int64_t *fitness, int32_t m,
                         double label_mean, double label_spread, double *out, void *stream)
{
    g_last_error.clear();
    if (!yhat || !fitness || !out || m < 1 || !(label_spread > 0.0) || !std::isfinite(label_mean)) {
        set_error("invalid judge arguments (m = %d)", m);
        return GAPA_E_INVALID_ARG;
    }
    int dev = 0;
    int rc = check_device(&dev);
    if (rc != GAPA_OK) return rc;
    return surrogate_judge(yhat, pool, fitness, m, label_mean, label_spread, out, static_cast<hipStream_t>(stream));
}

int gapa_surrogate_last_pool(gapa_ga *ga, int32_t *pool_out, int32_t cap, int32_t *count)
{
    int rc = surr_check(ga);
    if (rc != GAPA_OK) return rc;
    if (cap < 0) return GAPA_E_INVALID_ARG;
    DeviceGuard dg(ga->graph->device);
    return fail_handle(&ga->failed, surrogate_last_pool(ga, pool_out, cap, count));
}

int gapa_surrogate_last_predictions(gapa_ga *ga, float *yhat_out, int32_t cap, int32_t *count)
{
    int rc = surr_check(ga);
    if (rc != GAPA_OK) return rc;
    if (cap < 0) return GAPA_E_INVALID_ARG;
    DeviceGuard dg(ga->graph->device);
    return fail_handle(&ga->failed, surrogate_last_predictions(ga, yhat_out, cap, count));
}

int gapa_surrogate_predict(gapa_ga *ga, const int32_t *genes, int32_t P, float *yhat, void *stream)
{
    int rc = surr_check(ga);
    if (rc != GAPA_OK) return rc;
    if (P < 0 || (P > 0 && (!genes || !yhat))) {
        set_error("invalid arguments");
        return GAPA_E_INVALID_ARG;
    }
    DeviceGuard dg(ga->graph->device);
    return fail_handle(&ga->failed, surrogate_predict(ga, genes, P, yhat, static_cast<hipStream_t>(stream)));
}

int gapa_surrogate_train_batch(gapa_ga *ga, const int32_t *genes, const float *target, int32_t B, int32_t keep_grads,
                               void *stream)
{
    int rc = surr_check(ga);
    if (rc != GAPA_OK) return rc;
    if (!genes || !target) {
        set_error("invalid arguments");
        return GAPA_E_INVALID_ARG;
    }
    DeviceGuard dg(ga->graph->device);
    return fail_handle(&ga->failed,
                       surrogate_train_batch(ga, genes, target, B, keep_grads != 0, static_cast<hipStream_t>(stream)));
}

int gapa_surrogate_tensor(gapa_ga *ga, int32_t which, int32_t kind, float *host, int64_t count, int32_t set)
{
    int rc = surr_check(ga);
    if (rc != GAPA_OK) return rc;
    DeviceGuard dg(ga->graph->device);
    return fail_handle(&ga->failed, surrogate_tensor(ga, which, kind, host, count, set != 0));
}

// ------------------------------------------------------------------- batch ---

int gapa_batch_create(int32_t count, gapa_graph *const *graphs, const gapa_params *params, void *stream,
                      gapa_batch **out)
{
    g_last_error.clear();
    if (!out || !graphs || !params) {
        set_error("NULL argument");
        return GAPA_E_INVALID_ARG;
    }
    *out = nullptr;
    if (count < 1 || count > 4096) {
        set_error("count = %d, need 1 <= count <= 4096", count);
        return GAPA_E_INVALID_ARG;
    }
    std::vector<int32_t> ns(count), nonisos(count), voff(count + 1, 0);
    std::vector<int64_t> eoff(count + 1, 0);
    int32_t slots_needed = 1;
    for (int32_t b = 0; b < count; ++b) {
        const gapa_graph *g = graphs[b];
        if (!g || g->failed || g->device != graphs[0]->device) {
            set_error("graph %d is NULL, failed or on another device", b);
            return GAPA_E_INVALID_ARG;
        }
        const gapa_params &p = params[b];
        if (!params_ok(&p, g->n) || p.flags != params[0].flags) {
            set_error("invalid GA parameters of instance %d", b);
            return GAPA_E_INVALID_ARG;
        }
        const int32_t L = p.offspring > 0 ? p.offspring : p.pop;
        if (std::max(p.pop, L) > 1024) {
            set_error("instance %d: max(pop, offspring) = %d exceeds 1024", b, std::max(p.pop, L));
            return GAPA_E_INVALID_ARG;
        }
        slots_needed = std::max(slots_needed, std::max(p.pop, L));
        ns[b] = g->n;
        nonisos[b] = g->n_noniso;
        if ((int64_t)voff[b] + g->n > (1 << 30) || eoff[b] + g->nnz >= (1ll << 31)) {
            set_error("the union of the instance graphs is too large");
            return GAPA_E_INVALID_ARG;
        }
        voff[b + 1] = voff[b] + g->n;
        eoff[b + 1] = eoff[b] + g->nnz;
    }
    int32_t bseg = 32;
    while (bseg < slots_needed) bseg <<= 1;
    DeviceGuard dg(graphs[0]->device);
    gapa_batch *bt = new (std::nothrow) gapa_batch();
    if (!bt || !(bt->ga = new (std::nothrow) gapa_ga())) {
        delete bt;
        set_error("host allocation failed");
        return GAPA_E_OOM;
    }
    auto fail = [&](int code) {
        gapa_batch_destroy(bt);
        return code;
    };
    gapa_ga *ga = bt->ga;
    hipError_t e;
    int rc;
    if (count == 1) {
        ga->graph = graphs[0];
        graph_retain(ga->graph);
    } else {
        // the disjoint union of the instance graphs: instance b's node v is
        // node voff[b] + v
        const int32_t N = voff[count];
        const int64_t M = eoff[count];
        std::vector<int32_t> rp((size_t)N + 1), ci((size_t)std::max<int64_t>(M, 1)), tmp_rp;
        for (int32_t b = 0; b < count; ++b) {
            const gapa_graph *g = graphs[b];
            tmp_rp.resize((size_t)g->n + 1);
            if ((e = hipMemcpy(tmp_rp.data(), g->d_row_ptr, ((size_t)g->n + 1) * 4, hipMemcpyDeviceToHost)) !=
                hipSuccess)
                return fail(hip_fail(e, "hipMemcpy"));
            for (int32_t v = 0; v < g->n; ++v) rp[voff[b] + v] = (int32_t)(eoff[b] + tmp_rp[v]);
            if (g->nnz > 0) {
                int32_t *dst = ci.data() + eoff[b];
                if ((e = hipMemcpy(dst, g->d_col, (size_t)g->nnz * 4, hipMemcpyDeviceToHost)) != hipSuccess)
                    return fail(hip_fail(e, "hipMemcpy"));
                for (int64_t q = 0; q < g->nnz; ++q) dst[q] += voff[b];
            }
        }
        rp[N] = (int32_t)M;
        if ((rc = graph_build(graphs[0]->device, N, M, rp.data(), ci.data(), voff, 0, &bt->super)) != GAPA_OK)
            return fail(rc);
        ga->graph = bt->super;
        graph_retain(ga->graph);
    }
    if ((rc = ga_allocate(ga, count, params, ns.data(), nonisos.data(), count > 1 ? bseg : 0)) != GAPA_OK)
        return fail(rc);
    if (count > 1) {
        // per-instance non-isolated bit sets, in local ids
        int64_t words = 0;
        for (int32_t b = 0; b < count; ++b) words += (ns[b] + 31) / 32;
        if ((rc = ga->noniso_buf.reserve((size_t)words * 4)) != GAPA_OK) return fail(rc);
        ga->noniso = ga->noniso_buf.as<uint32_t>();
        for (int32_t b = 0; b < count; ++b)
            if ((e = hipMemcpy(ga->noniso + ga->hinst[b].noniso_off, graphs[b]->d_noniso,
                               (size_t)((ns[b] + 31) / 32) * 4, hipMemcpyDeviceToDevice)) != hipSuccess)
                return fail(hip_fail(e, "hipMemcpy"));
        // instance tables of the fitness pass
        std::vector<int32_t> live_init(count), live_gen(count), node_inst((size_t)voff[count]), tiles;
        std::vector<int64_t> moff(count);
        for (int32_t b = 0; b < count; ++b) {
            const GaInst &I = ga->hinst[b];
            live_init[b] = I.P;
            live_gen[b] = I.L;
            moff[b] = I.mask_off;
            for (int32_t v = voff[b]; v < voff[b + 1]; ++v) node_inst[v] = b;
            for (int32_t j0 = 0; j0 < I.W; j0 += transpose_tile_words(bseg / 32)) {
                tiles.push_back(b);
                tiles.push_back(j0);
            }
        }
        if ((rc = upload(ga->tab_voff, voff)) != GAPA_OK || (rc = upload(ga->tab_live_init, live_init)) != GAPA_OK ||
            (rc = upload(ga->tab_live_gen, live_gen)) != GAPA_OK || (rc = upload(ga->tab_moff, moff)) != GAPA_OK ||
            (rc = upload(ga->tab_node_inst, node_inst)) != GAPA_OK || (rc = upload(ga->tab_tiles, tiles)) != GAPA_OK)
            return fail(rc);
        InstTable t;
        t.count = count;
        t.bseg = bseg;
        t.voff = ga->tab_voff.as<int32_t>();
        t.moff = ga->tab_moff.as<int64_t>();
        t.node_inst = ga->tab_node_inst.as<int32_t>();
        t.tiles = ga->tab_tiles.as<int32_t>();
        t.ntiles = (int32_t)(tiles.size() / 2);
        ga->tab_init = t;
        ga->tab_init.live = ga->tab_live_init.as<int32_t>();
        ga->tab_gen = t;
        ga->tab_gen.live = ga->tab_live_gen.as<int32_t>();
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = launch_fill_u32(ga->flag.ptr, 0u, 4, s)) != GAPA_OK) return fail(rc);
    if ((rc = ga_init_population(ga, s)) != GAPA_OK) return fail(rc);
    ga->last_stream = s;
    *out = bt;
    return GAPA_OK;
}

int gapa_batch_step(gapa_batch *b, int32_t n_generations, void *stream)
{
    g_last_error.clear();
    if (!b) {
        set_error("batch is NULL");
        return GAPA_E_INVALID_ARG;
    }
    return ga_step_checked(b->ga, n_generations, static_cast<hipStream_t>(stream));
}

int gapa_batch_record(gapa_batch *b, int32_t n_generations)
{
    if (!b) return GAPA_E_INVALID_ARG;
    return gapa_ga_record(b->ga, n_generations);
}

int gapa_batch_best(gapa_batch *b, int32_t idx, int32_t *genes_out, int64_t *fitness_out, int64_t *generation_out)
{
    g_last_error.clear();
    if (!b || idx < 0 || idx >= b->ga->count) {
        set_error("batch is NULL or index out of range");
        return GAPA_E_INVALID_ARG;
    }
    const int rc = ga_copy_out(b->ga, idx, true, genes_out, fitness_out);
    if (rc == GAPA_OK && generation_out) *generation_out = b->ga->generation;
    return rc;
}

int gapa_batch_get_population(gapa_batch *b, int32_t idx, int32_t *genes_out, int64_t *fitness_out)
{
    g_last_error.clear();
    if (!b || idx < 0 || idx >= b->ga->count) {
        set_error("batch is NULL or index out of range");
        return GAPA_E_INVALID_ARG;
    }
    return ga_copy_out(b->ga, idx, false, genes_out, fitness_out);
}

int gapa_batch_set_timing(gapa_batch *b, int32_t enable)
{
    if (!b) return GAPA_E_INVALID_ARG;
    return gapa_ga_set_timing(b->ga, enable);
}

int gapa_batch_kernel_times(gapa_batch *b, gapa_kernel_time *out, int32_t cap, int32_t *count)
{
    if (!b) return GAPA_E_INVALID_ARG;
    return ga_collect_times(b->ga, out, cap, count);
}

int gapa_batch_destroy(gapa_batch *b)
{
    if (!b) return GAPA_OK;
    if (b->ga) {
        gapa_graph *g = b->ga->graph;
        if (g) {
            DeviceGuard dg(g->device);
            ga_release(b->ga);
        }
        delete b->ga;
        if (g) graph_release(g);
    }
    gapa_graph_destroy(b->super);
    delete b;
    return GAPA_OK;
}

}  // extern "C"
