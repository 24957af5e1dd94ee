// C interface of the propagation library: argument checks, graph
// construction, run state and the round driver.  Every device step is a
// kernel in pp_kernels.hip (or pp_csr.hip for the graph build).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>
#include <string>
#include <chrono>
#include <thread>
#include <utility>
#include <vector>

#include "pp_internal.h"
#include "pp_build.h"

using pp::Chunk;
using pp::Ctrl;
using pp::GraphDev;
using pp::RunDev;
using pp::Tile;

namespace {

thread_local std::string g_err;

constexpr int32_t kNaNBits = 0x7fc00000;   // quiet NaN (unset cost-model weights)

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return fail(PP_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// The caller's device allocator (pp_set_allocator), and every block it gave
// the library with the allocator and stream it came from, so that a block
// goes back where it came from even after the allocator is changed.
struct Allocator {
    void *(*alloc)(size_t, void *, void *);
    void (*release)(void *, void *, void *);
    void *ctx;
};
struct OwnedBlock {
    Allocator from;
    void *stream;
};
// The lock and the ledger live until the process ends (never destroyed), so
// a handle freed late in the process's exit still finds them.
std::mutex &alloc_mu() {
    static std::mutex *m = new std::mutex();
    return *m;
}
std::unordered_map<void *, OwnedBlock> &owned_blocks() {
    static auto *m = new std::unordered_map<void *, OwnedBlock>();
    return *m;
}
Allocator g_alloc{nullptr, nullptr, nullptr};
thread_local void *t_alloc_stream = nullptr;

template <typename T> int dev_alloc(T **p, int64_t count) {
    if (count <= 0) count = 1;
    *p = (T *)pp::dev_malloc(sizeof(T) * (size_t)count);
    if (!*p)
        return fail(PP_ENOMEM, "device allocation of %lld bytes failed (or the caller's allocator gave a block "
                               "that is not 256-byte aligned)", (long long)(sizeof(T) * count));
    return PP_OK;
}

template <typename T> void dev_free(T *&p) {
    pp::dev_release((void *)p);
    p = nullptr;
}

unsigned hw_threads() {
    unsigned t = std::thread::hardware_concurrency();
    return t == 0 ? 1 : (t > 32 ? 32 : t);
}

template <typename F> void parallel_for(int64_t n, F f) {
    unsigned T = hw_threads();
    if (n < 1 << 16 || T == 1) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    for (unsigned t = 0; t < T; ++t) {
        int64_t a = n * t / T, b = n * (t + 1) / T;
        th.emplace_back([=] { f(a, b); });
    }
    for (auto &x : th) x.join();
}

struct TileSet {
    Tile *tiles = nullptr;
    int32_t ntiles = 0;
    int32_t *hub_node = nullptr;   // node of each high-degree entry
    int32_t nhubs = 0;
    bool short_lists = false;      // no hubs and no node above PULL_NPL successors
    int64_t dead = 0;              // nodes without successors
    std::vector<int32_t> gtile;    // [G+1] first tile of each graph
    std::vector<int32_t> ghub;     // [G+1] first hub of each graph
};

}  // namespace

struct pp_graph_s {
    int64_t n = 0, m = 0;
    int32_t G = 1;
    uint32_t flags = 0;
    hipStream_t stream = nullptr;
    std::vector<int64_t> node_offsets;
    std::vector<int64_t> rp_host;   // kept for tiling at each signature width
    int64_t *rp = nullptr, *trp = nullptr;
    int32_t *col = nullptr, *tcol = nullptr;
    int32_t *node_graph = nullptr;
    int64_t *node_off = nullptr;
    std::map<int, TileSet> tiles;   // by pull arc budget
    std::vector<int32_t> perm;      // stored id of each input node (empty: identity)
    int32_t *perm_d = nullptr;      // the same on the device
    std::vector<uint64_t> pred_bits;  // bit u (stored id): node u has a predecessor
    int32_t *seq_heavy = nullptr;   // PROPAGATE-S: nodes with more than SEQ_LIGHT successors
    int64_t nseq_heavy = 0;
};

struct pp_run_s {
    pp_graph g = nullptr;
    int32_t s = 0, W = 0, cap = 0, G = 1;   // s: seeds per graph; W: row words of one seed group
    int32_t k = 1, sg = 0, Wout = 0;        // seed groups, seeds per group, row words reported
    bool grouped = false;                   // groups or a seed order: internal seed list and positions
    int32_t *iseeds = nullptr;              // [G*s] stored ids in internal order
    int32_t *dpos = nullptr;                // [G*s] internal position of each caller seed
    int32_t *dcur = nullptr;                // [k] current signature buffer of each group
    pp_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    RunDev dev{};
    Ctrl host_ctrl{};
    std::map<int, hipGraphExec_t> graphs;   // captured batches by round count
    std::map<int, hipGraph_t> graph_defs;
    int32_t *dseeds = nullptr;              // [G*s] mapped device seeds for the clustered engine
    // a single graph without seed groups on the per-round engine: dseeds holds
    // the stored ids of the seeds the last initialisation placed
    bool seeds_kept = false;
    bool timing = false;
    bool graph_events = true;               // events recorded inside captured graphs work
    std::vector<hipEvent_t> ev;             // 2 per round slot of a batch
    std::vector<float> pull_ms;             // [cap]
    int pgrid = 0;                          // blocks of the persistent round loop (0: not used)
    std::vector<pp::Cluster> clusters;      // persistent engine: block ranges per graph
    pp::Cluster *dclusters = nullptr;
    std::vector<int> cur;                   // signature buffer of Sig_{round-1}, per control block
    double clock_khz = 100000.0;            // device wall clock rate
    hipEvent_t tev[2] = {nullptr, nullptr}; // events of pp_time_round
    // what the host knows of the device's logs: counts rows [0, staged) and D,
    // refreshed by the same wait that reads the control blocks back
    void *pinned = nullptr;                 // staging: control blocks, D, count rows
    Ctrl *h_ctrl = nullptr;
    int32_t *h_D = nullptr;
    int64_t *h_rows = nullptr;
    void *h_ctrl_dev = nullptr;             // the same three, as the device addresses them
    int32_t *h_D_dev = nullptr;
    int64_t *h_rows_dev = nullptr;
    int32_t *h_seeds = nullptr;             // host seed list, read in place by the initialisation
    int32_t *h_seeds_dev = nullptr;         // the same, as the device addresses it
    hipEvent_t seeds_sent = nullptr;        // its copy has been read
    std::vector<int64_t> counts_host;       // [staged][k][G] as the device logs them
    std::vector<int32_t> D_host;            // [k][G]
    int staged = 0;
    // The push accumulator is all zero between rounds (every round clears
    // what it set), so a reset leaves it alone -- unless a launch failed
    // part-way through a round, or it was never cleared.
    bool acc_clean = false;
};

// count rows copied back per wait at most
constexpr int STAGE_ROWS = 128;

extern "C" {

const char *pp_last_error(void) { return g_err.c_str(); }

void pp_options_default(pp_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->scheduler = PP_SCHED_HEURISTIC;
    opt->use_graph = 1;
    opt->push_div = 8;
}

int64_t pp_graph_arcs(pp_graph g) { return g ? g->m : -1; }
int64_t pp_graph_nodes(pp_graph g) { return g ? g->n : -1; }
int32_t pp_graph_count(pp_graph g) { return g ? g->G : -1; }

}  // extern "C"

// --------------------------------------------------------------------------
// graph construction (host adjacency build, then one upload)
// --------------------------------------------------------------------------

namespace {

// rows[u] = sorted, distinct heads v of arcs u -> v in the propagation
// direction (u ORs in v's signature), self-loops removed.
// Runs f(t) for t in [0, T) on T host threads.
template <typename F> void on_threads(int T, F f) {
    if (T <= 1) {
        f(0);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t) th.emplace_back([=] { f(t); });
    for (auto &x : th) x.join();
}

// Runs f(i) for i in [0, count) on every host thread, each taking the next
// index from a shared counter (uneven items balance themselves).
template <typename F> void on_items(int64_t count, F f) {
    std::atomic<int64_t> next{0};
    on_threads((int)hw_threads(), [&](int) {
        for (int64_t i; (i = next.fetch_add(1)) < count;) f(i);
    });
}

// CSR of the arcs that gen(lo, hi, emit) emits for input items [lo, hi)
// (emit(row, column) per arc), rows sorted, repeated arcs merged.  Parallel
// without atomics on the data: each thread counts its slice's arcs per
// bucket of consecutive rows, the arcs are scattered bucket by bucket as
// 64-bit keys (row, column), and the buckets (many more than threads, taken
// from a shared counter, since degree-skewed graphs fill some far more than
// others) are sorted and deduplicated one per thread at a time.
template <typename Gen>
void build_csr(int64_t n, int64_t items, Gen gen, std::vector<int64_t> &rp, std::vector<int32_t> &col) {
    const int T = (int)hw_threads();
    const int NB = (int)std::min<int64_t>(4096, std::max<int64_t>(1, n / 64));
    const int64_t per = (n + NB - 1) / NB;   // rows per bucket
    std::vector<int64_t> cnt((size_t)T * NB, 0);   // [thread][bucket]
    on_threads(T, [&](int t) {
        int64_t *c = cnt.data() + (size_t)t * NB;
        gen(items * t / T, items * (t + 1) / T, [&](int64_t r, int32_t) { c[r / per]++; });
    });
    std::vector<int64_t> off((size_t)T * NB), bstart((size_t)NB + 1);
    int64_t total = 0;
    for (int bk = 0; bk < NB; ++bk) {
        bstart[(size_t)bk] = total;
        for (int t = 0; t < T; ++t) {
            off[(size_t)t * NB + bk] = total;
            total += cnt[(size_t)t * NB + bk];
        }
    }
    bstart[(size_t)NB] = total;
    std::vector<uint64_t> keys((size_t)total);
    on_threads(T, [&](int t) {
        int64_t *pos = off.data() + (size_t)t * NB;
        gen(items * t / T, items * (t + 1) / T,
            [&](int64_t r, int32_t c) { keys[(size_t)pos[r / per]++] = ((uint64_t)r << 32) | (uint32_t)c; });
    });
    std::vector<int64_t> len((size_t)n, 0), uniq((size_t)NB, 0);
    on_items(NB, [&](int64_t bk) {
        uint64_t *p = keys.data() + bstart[(size_t)bk], *q = keys.data() + bstart[(size_t)bk + 1];
        std::sort(p, q);
        uint64_t *e = std::unique(p, q);
        uniq[(size_t)bk] = e - p;
        for (uint64_t *k = p; k < e; ++k) len[(size_t)(*k >> 32)]++;
    });
    rp.assign((size_t)n + 1, 0);
    for (int64_t u = 0; u < n; ++u) rp[(size_t)u + 1] = rp[(size_t)u] + len[(size_t)u];
    col.resize((size_t)rp[(size_t)n]);
    on_items(NB, [&](int64_t bk) {
        const int64_t first_row = std::min<int64_t>(bk * per, n);
        const uint64_t *p = keys.data() + bstart[(size_t)bk];
        int32_t *out = col.data() + rp[(size_t)first_row];
        for (int64_t k = 0; k < uniq[(size_t)bk]; ++k) out[k] = (int32_t)(p[k] & 0xFFFFFFFFull);
    });
}

// Successor rows of the input arcs: u -> v for pair (src, dst) (reversed
// with `transpose`, both directions with `undirected`), self-loops dropped.
void build_rows(int64_t n, int64_t m, const int32_t *a, const int32_t *b, bool undirected,
                std::vector<int64_t> &rp, std::vector<int32_t> &col) {
    build_csr(n, m, [&](int64_t lo, int64_t hi, auto emit) {
        for (int64_t k = lo; k < hi; ++k) {
            if (a[k] == b[k]) continue;
            emit(a[k], b[k]);
            if (undirected) emit(b[k], a[k]);
        }
    }, rp, col);
}

// Transpose of a CSR: trow[v] = sorted {u : v in row u}.
void transpose_rows(int64_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &col,
                    std::vector<int64_t> &trp, std::vector<int32_t> &tcol) {
    build_csr(n, n, [&](int64_t lo, int64_t hi, auto emit) {
        for (int64_t u = lo; u < hi; ++u)
            for (int64_t e = rp[(size_t)u]; e < rp[(size_t)u + 1]; ++e) emit(col[(size_t)e], (int32_t)u);
    }, trp, tcol);
}

// Storage order of the nodes, graph by graph within a batch (perm[x] is the
// stored id of input node x; returns false when the order is the identity):
// * first the nodes whose rows many arcs gather (at least max(8, twice the
//   graph's mean) predecessors), by decreasing predecessor count: packed
//   into few cache lines, the most-gathered rows raise the caches' hit rate
//   in the pull;
// * then every other node in breadth-first order: searches over the
//   successor lists (col, by input id), rooted first at those nodes in their
//   order and then at each unnumbered node in input order, number the nodes
//   as they reach them.  Nodes near each other in the graph get near ids, so
//   the rows a round touches together share cache lines: a tile's
//   successors in the pull, a frontier's predecessors in a push (on a
//   lattice they lie along rings).  Against input order for the rest: the
//   4096^2 lattice 135.5 -> 124.8 ms per propagation, R-MAT scale 26 with
//   512 seeds 53.5 -> 52.3 ms with seed groups.  The searches run on one
//   host thread (R-MAT 26: about 7 s of the build); searches = false
//   (PP_HUBS_ONLY) leaves the rest in input order.
bool storage_order(const std::vector<int64_t> &noff, int G, const std::vector<int64_t> &rp,
                   const std::vector<int64_t> &trp, const std::function<const int32_t *()> &col_of, bool searches,
                   std::vector<int32_t> &perm) {
    const int64_t n = (int64_t)rp.size() - 1;
    perm.resize((size_t)n);
    const int32_t *col = searches && n > 0 && rp[(size_t)n] > 0 ? col_of() : nullptr;
    bool moved = false;
    for (int g = 0; g < G; ++g) {
        const int64_t a = noff[(size_t)g], b = noff[(size_t)g + 1];
        if (b <= a) continue;
        const double mean = (double)(rp[(size_t)b] - rp[(size_t)a]) / (double)(b - a);
        const double thr = std::max(8.0, 2.0 * mean);
        auto indeg = [&](int64_t x) { return trp[(size_t)x + 1] - trp[(size_t)x]; };
        std::vector<int32_t> hot;
        for (int64_t x = a; x < b; ++x)
            if ((double)indeg(x) >= thr) hot.push_back((int32_t)x);
        std::stable_sort(hot.begin(), hot.end(), [&](int32_t x, int32_t y) { return indeg(x) > indeg(y); });
        int64_t pos = a;
        std::vector<char> seen((size_t)(b - a), 0);   // numbered or queued
        for (int32_t x : hot) {
            seen[(size_t)(x - a)] = 1;
            moved |= pos != x;
            perm[(size_t)x] = (int32_t)pos++;
        }
        std::vector<int32_t> queue((size_t)(b - a) + hot.size());
        int64_t head = 0, tail = 0;
        auto search = [&](int32_t root) {   // root: numbered already
            head = tail = 0;
            queue[(size_t)tail++] = root;
            while (head < tail) {
                const int32_t u = queue[(size_t)head++];
                if (u != root) {
                    moved |= pos != u;
                    perm[(size_t)u] = (int32_t)pos++;
                }
                for (int64_t e = rp[(size_t)u]; e < rp[(size_t)u + 1]; ++e) {
                    const int32_t v = col[(size_t)e];
                    if (!seen[(size_t)(v - a)]) {
                        seen[(size_t)(v - a)] = 1;
                        queue[(size_t)tail++] = v;
                    }
                }
            }
        };
        if (searches && col)
            for (int32_t x : hot) search(x);
        for (int64_t x = a; x < b; ++x) {
            if (seen[(size_t)(x - a)]) continue;
            seen[(size_t)(x - a)] = 1;
            moved |= pos != x;
            perm[(size_t)x] = (int32_t)pos++;
            if (searches && col) search((int32_t)x);
        }
    }
    return moved;
}

// Rows of a CSR under a node renumbering: row perm[u] of the result holds
// perm[v] for every v in row u of the input, sorted.
void relabel_rows(const std::vector<int32_t> &perm, std::vector<int64_t> &rp, std::vector<int32_t> &col) {
    const int64_t n = (int64_t)rp.size() - 1;
    std::vector<int32_t> inv((size_t)n);
    for (int64_t x = 0; x < n; ++x) inv[(size_t)perm[(size_t)x]] = (int32_t)x;
    std::vector<int64_t> rp2((size_t)n + 1, 0);
    for (int64_t y = 0; y < n; ++y) rp2[(size_t)y + 1] = rp2[(size_t)y] + (rp[(size_t)inv[(size_t)y] + 1] - rp[(size_t)inv[(size_t)y]]);
    std::vector<int32_t> col2(col.size());
    constexpr int64_t CH = 1024;   // rows per work item (hub rows come first and are long)
    on_items((n + CH - 1) / CH, [&](int64_t c) {
        const int64_t lo = c * CH, hi = std::min(n, lo + CH);
        for (int64_t y = lo; y < hi; ++y) {
            const int64_t u = inv[(size_t)y];
            int32_t *out = col2.data() + rp2[(size_t)y];
            const int64_t len = rp[(size_t)u + 1] - rp[(size_t)u];
            for (int64_t k = 0; k < len; ++k) out[k] = perm[(size_t)col[(size_t)(rp[(size_t)u] + k)]];
            std::sort(out, out + len);
        }
    });
    rp.swap(rp2);
    col.swap(col2);
}

// Pull tiles: runs of consecutive nodes with at most `edges` arcs and
// pp::TILE_NODES nodes; a node with more than `edges` arcs is split into
// chunks whose partial rows meet in the accumulator (hub_node lists those
// nodes).  Runs without arcs are dropped: their nodes have no successor and
// never gain a bit after initialisation.  Tiles are grouped by graph
// (gtile/ghub give each graph's first tile and hub); within a graph, hub
// chunks come first so the longest-latency work starts early.
void build_tiles(const std::vector<int64_t> &rp, const std::vector<int64_t> &noff, int G, int edges,
                 std::vector<Tile> &tiles, std::vector<int32_t> &hub_node, std::vector<int32_t> &gtile,
                 std::vector<int32_t> &ghub) {
    gtile.assign((size_t)G + 1, 0);
    ghub.assign((size_t)G + 1, 0);
    for (int g = 0; g < G; ++g) {
        std::vector<Tile> hubs, runs;
        gtile[(size_t)g] = (int32_t)tiles.size();
        ghub[(size_t)g] = (int32_t)hub_node.size();
        int64_t u = noff[(size_t)g];
        const int64_t end = noff[(size_t)g + 1];
        while (u < end) {
            const int64_t deg = rp[(size_t)u + 1] - rp[(size_t)u];
            if (deg > edges) {
                const int32_t h = (int32_t)hub_node.size();
                const int32_t nch = (int32_t)((deg + edges - 1) / edges);
                hub_node.push_back((int32_t)u);
                for (int32_t j = 0; j < nch; ++j) {
                    const int64_t e0 = rp[(size_t)u] + (int64_t)j * edges;
                    const int64_t e1 = std::min(rp[(size_t)u + 1], e0 + edges);
                    hubs.push_back(Tile{(int32_t)u, (int32_t)u + 1, e0, e1, h, g});
                }
                ++u;
                continue;
            }
            const int64_t s = u;
            while (u < end && u - s < pp::TILE_NODES) {
                const int64_t d = rp[(size_t)u + 1] - rp[(size_t)u];
                if (d > edges || rp[(size_t)u + 1] - rp[(size_t)s] > edges) break;
                ++u;
            }
            if (rp[(size_t)u] > rp[(size_t)s]) runs.push_back(Tile{(int32_t)s, (int32_t)u, rp[(size_t)s], rp[(size_t)u], -1, g});
        }
        tiles.insert(tiles.end(), hubs.begin(), hubs.end());
        tiles.insert(tiles.end(), runs.begin(), runs.end());
    }
    gtile[(size_t)G] = (int32_t)tiles.size();
    ghub[(size_t)G] = (int32_t)hub_node.size();
}

// arc budget of a pull tile: K arcs per lane (0: the width's default)
int pull_edges(int W, int K) {
    if (K > 0) return K * 64;
    switch (W) {
        case 1: return pp::PullShape<1>::EDGES;
        case 2: return pp::PullShape<2>::EDGES;
        case 4: return pp::PullShape<4>::EDGES;
        default: return pp::PullShape<8>::EDGES;
    }
}

int ensure_tiles(pp_graph g, int W, int K, TileSet **out) {
    const int edges = pull_edges(W, K);
    auto it = g->tiles.find(edges);
    if (it != g->tiles.end()) {
        *out = &it->second;
        return PP_OK;
    }
    std::vector<Tile> tiles;
    std::vector<int32_t> hubs;
    TileSet ts;
    build_tiles(g->rp_host, g->node_offsets, g->G, edges, tiles, hubs, ts.gtile, ts.ghub);
    int rc;
    if ((rc = dev_alloc(&ts.tiles, (int64_t)tiles.size())) != PP_OK) return rc;
    if ((rc = dev_alloc(&ts.hub_node, (int64_t)hubs.size())) != PP_OK) {
        dev_free(ts.tiles);
        return rc;
    }
    ts.ntiles = (int32_t)tiles.size();
    ts.nhubs = (int32_t)hubs.size();
    int64_t dmax = 0;
    for (int64_t u = 0; u < g->n; ++u) {
        const int64_t d = g->rp_host[u + 1] - g->rp_host[u];
        dmax = std::max(dmax, d);
        ts.dead += d == 0;
    }
    ts.short_lists = hubs.empty() && dmax <= pp::PULL_NPL;
    hipError_t e = hipSuccess;
    if (!tiles.empty()) e = hipMemcpy(ts.tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !hubs.empty())
        e = hipMemcpy(ts.hub_node, hubs.data(), sizeof(int32_t) * hubs.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        dev_free(ts.tiles);
        dev_free(ts.hub_node);
        return fail(PP_EDEVICE, "tile upload: %s", hipGetErrorString(e));
    }
    g->tiles[edges] = ts;
    *out = &g->tiles[edges];
    return PP_OK;
}

void free_graph(pp_graph g) {
    if (!g) return;
    dev_free(g->rp);
    dev_free(g->trp);
    dev_free(g->col);
    dev_free(g->tcol);
    dev_free(g->node_graph);
    dev_free(g->node_off);
    dev_free(g->perm_d);
    dev_free(g->seq_heavy);
    for (auto &kv : g->tiles) {
        dev_free(kv.second.tiles);
        dev_free(kv.second.hub_node);
    }
    delete g;
}

// W: the run's row width (sets the pull launch's width; 0 for a view without
// pull tiles)
GraphDev graph_view(pp_graph g, const TileSet *ts, int W) {
    GraphDev d{};
    d.n = g->n;
    d.m = g->m;
    d.rp = g->rp;
    d.col = g->col;
    d.trp = g->trp;
    d.tcol = g->tcol;
    d.tiles = ts ? ts->tiles : nullptr;
    d.ntiles = ts ? ts->ntiles : 0;
    d.nhubs = ts ? ts->nhubs : 0;
    d.hub_node = ts ? ts->hub_node : nullptr;
    d.node_graph = g->node_graph;
    d.node_off = g->node_off;
    d.G = g->G;
    d.pull_grid = pp::pull_grid_for(d.ntiles, W);
    d.short_lists = ts && ts->short_lists ? 1 : 0;
    // rows of nodes without successors are skipped by the pull when there are
    // many (a quarter of the nodes or more) and the two signature buffers
    // exceed the 256 MB last-level cache: the copy would go to HBM; a graph
    // whose rows stay in the cache loses more to the test than it saves
    d.skip_dead = ts && ts->dead * 4 >= g->n && 16.0 * W * (double)g->n > 256.0 * 1048576.0 ? 1 : 0;
    return d;
}

}  // namespace

extern "C" int pp_csr_build(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, uint32_t flags,
                            const int64_t *node_offsets, int32_t num_graphs, void *stream, pp_graph *out) {
    if (!out) return fail(PP_EINVAL, "out is NULL");
    pp::AllocStream as(stream);
    if (n < 1 || n > INT32_MAX - 1) return fail(PP_EINVAL, "n = %lld outside [1, 2^31-2]", (long long)n);
    if (m < 0) return fail(PP_EINVAL, "m < 0");
    if (m > 0 && (!src || !dst)) return fail(PP_EINVAL, "src/dst NULL with m > 0");
    if (flags & ~(uint32_t)(PP_UNDIRECTED | PP_INPUT_ON_DEVICE | PP_TRANSPOSE | PP_KEEP_ORDER | PP_BUILD_ON_HOST |
                            PP_BUILD_ON_DEVICE | PP_HUBS_ONLY))
        return fail(PP_EINVAL, "unknown flag bits");
    if ((flags & PP_BUILD_ON_HOST) && (flags & PP_BUILD_ON_DEVICE))
        return fail(PP_EINVAL, "PP_BUILD_ON_HOST and PP_BUILD_ON_DEVICE together");
    const int G = (num_graphs <= 1 && !node_offsets) ? 1 : num_graphs;
    if (G < 1) return fail(PP_EINVAL, "num_graphs < 1");
    std::vector<int64_t> noff((size_t)G + 1);
    if (node_offsets && G >= 1) {
        for (int g = 0; g <= G; ++g) noff[(size_t)g] = node_offsets[g];
        if (noff[0] != 0 || noff[(size_t)G] != n) return fail(PP_EINVAL, "node_offsets must start at 0 and end at n");
        for (int g = 0; g < G; ++g)
            if (noff[(size_t)g + 1] < noff[(size_t)g]) return fail(PP_EINVAL, "node_offsets not non-decreasing");
    } else {
        noff[0] = 0;
        noff[1] = n;
    }
    const bool und = flags & PP_UNDIRECTED;
    const bool tr = flags & PP_TRANSPOSE;
    const bool on_device = (flags & PP_BUILD_ON_DEVICE) || (!(flags & PP_BUILD_ON_HOST) && m >= PP_DEVICE_BUILD_MIN);
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> ng;
    if (G > 1) {
        ng.resize((size_t)n);
        for (int g = 0; g < G; ++g)
            for (int64_t u = noff[(size_t)g]; u < noff[(size_t)g + 1]; ++u) ng[(size_t)u] = g;
    }
    // arcs outside [0, n) or across graphs: host arrays are checked here,
    // before any device work; device arrays on the device, or after their copy
    auto check_host_arcs = [&](const int32_t *ps, const int32_t *pd) -> int64_t {
        std::atomic<int64_t> bad{-1};
        parallel_for(m, [&](int64_t lo, int64_t hi) {
            for (int64_t k = lo; k < hi; ++k) {
                const int32_t a = ps[k], b = pd[k];
                if (a < 0 || a >= n || b < 0 || b >= n || (G > 1 && ng[(size_t)a] != ng[(size_t)b])) {
                    bad.store(k);
                    return;
                }
            }
        });
        return bad.load();
    };
    if (!(flags & PP_INPUT_ON_DEVICE) && m > 0) {
        const int64_t k = check_host_arcs(src, dst);
        if (k >= 0)
            return fail(PP_ERANGE, "arc %lld (%d -> %d) outside [0, n) or across graphs", (long long)k, src[k], dst[k]);
    }
    pp_graph g = new (std::nothrow) pp_graph_s();
    if (!g) return fail(PP_ENOMEM, "graph handle");
    g->n = n;
    g->G = G;
    g->flags = flags;
    g->stream = st;
    g->node_offsets = noff;
    int rc;
    if ((G > 1 && (rc = dev_alloc(&g->node_graph, n))) || (rc = dev_alloc(&g->node_off, (int64_t)G + 1))) {
        free_graph(g);
        return rc;
    }
    hipError_t e = hipSuccess;
    if (G > 1) e = hipMemcpyAsync(g->node_graph, ng.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(g->node_off, noff.data(), sizeof(int64_t) * (size_t)(G + 1), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(st);
        free_graph(g);
        return fail(PP_EDEVICE, "graph upload: %s", hipGetErrorString(e));
    }
    // the storage order (hub-first or breadth-first per graph) unless the
    // caller keeps the input order
    auto order = [&](const std::vector<int64_t> &rp_, const std::vector<int64_t> &trp_,
                     const std::function<const int32_t *()> &col_, std::vector<int32_t> &perm_) {
        return !(flags & PP_KEEP_ORDER) && storage_order(noff, G, rp_, trp_, col_, !(flags & PP_HUBS_ONLY), perm_);
    };
    // propagation rows: u ORs in v for arc u -> v (or v -> u transposed)
    std::vector<int64_t> rp, trp;
    std::vector<int32_t> perm;
    if (on_device) {
        // the arcs on the device: the caller's, or a copy of the host arrays
        int32_t *da = nullptr, *db = nullptr;
        const int32_t *a = src, *b = dst;
        auto drop_input = [&]() {
            dev_free(da);
            dev_free(db);
        };
        if (!(flags & PP_INPUT_ON_DEVICE) && m > 0) {
            if ((rc = dev_alloc(&da, m)) || (rc = dev_alloc(&db, m))) {
                drop_input();
                free_graph(g);
                return rc;
            }
            e = hipMemcpyAsync(da, src, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipMemcpyAsync(db, dst, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, st);
            if (e != hipSuccess) {
                (void)hipStreamSynchronize(st);
                drop_input();
                free_graph(g);
                return fail(PP_EDEVICE, "arc upload: %s", hipGetErrorString(e));
            }
            a = da;
            b = db;
        }
        int64_t bad = -1;
        if ((flags & PP_INPUT_ON_DEVICE) && (rc = pp::device_check_arcs(a, b, m, n, g->node_graph, &bad, st))) {
            drop_input();
            free_graph(g);
            return rc;
        }
        if (bad >= 0) {
            int32_t ends[2] = {0, 0};
            if (hipMemcpy(&ends[0], a + bad, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(&ends[1], b + bad, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
                (void)hipGetLastError();
            drop_input();
            free_graph(g);
            return fail(PP_ERANGE, "arc %lld (%d -> %d) outside [0, n) or across graphs", (long long)bad, ends[0], ends[1]);
        }
        pp::DevRows rows, trows;
        if (tr) std::swap(a, b);
        rc = pp::device_build(n, m, a, b, und, order, rows, trows, perm, st);
        drop_input();   // device_build has synchronised the stream
        g->rp = rows.rp;
        g->col = rows.col;
        g->trp = trows.rp;
        g->tcol = trows.col;
        g->m = rows.m;
        if (rc) {
            free_graph(g);
            return rc;
        }
        // host copies of the offsets (tiles, the long-list table, predecessor bits)
        try {
            rp.resize((size_t)n + 1);
            trp.resize((size_t)n + 1);
        } catch (const std::bad_alloc &) {
            free_graph(g);
            return fail(PP_ENOMEM, "host memory for the offsets");
        }
        e = hipMemcpyAsync(rp.data(), g->rp, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(trp.data(), g->trp, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(st);
            free_graph(g);
            return fail(PP_EDEVICE, "offset download: %s", hipGetErrorString(e));
        }
    } else {
        // input arcs on the host
        std::vector<int32_t> hs, hd, col, tcol;
        const int32_t *ps = src, *pd = dst;
        if ((flags & PP_INPUT_ON_DEVICE) && m > 0) {
            try {
                hs.resize((size_t)m);
                hd.resize((size_t)m);
            } catch (const std::bad_alloc &) {
                free_graph(g);
                return fail(PP_ENOMEM, "host memory for the arcs");
            }
            e = hipMemcpyAsync(hs.data(), src, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipMemcpyAsync(hd.data(), dst, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                (void)hipStreamSynchronize(st);
                free_graph(g);
                return fail(PP_EDEVICE, "arc download: %s", hipGetErrorString(e));
            }
            ps = hs.data();
            pd = hd.data();
        }
        if ((flags & PP_INPUT_ON_DEVICE) && m > 0) {
            const int64_t k = check_host_arcs(ps, pd);
            if (k >= 0) {
                free_graph(g);
                return fail(PP_ERANGE, "arc %lld (%d -> %d) outside [0, n) or across graphs", (long long)k, ps[k], pd[k]);
            }
        }
        try {
            if (tr) build_rows(n, m, pd, ps, und, rp, col);
            else build_rows(n, m, ps, pd, und, rp, col);
            transpose_rows(n, rp, col, trp, tcol);
            if (order(rp, trp, [&]() { return col.data(); }, perm)) {
                relabel_rows(perm, rp, col);
                relabel_rows(perm, trp, tcol);
            } else {
                perm.clear();
            }
        } catch (const std::bad_alloc &) {
            free_graph(g);
            return fail(PP_ENOMEM, "host memory for the adjacency build");
        }
        g->m = (int64_t)col.size();
        if ((rc = dev_alloc(&g->rp, n + 1)) || (rc = dev_alloc(&g->trp, n + 1)) || (rc = dev_alloc(&g->col, g->m)) ||
            (rc = dev_alloc(&g->tcol, g->m))) {
            free_graph(g);
            return rc;
        }
        e = hipMemcpyAsync(g->rp, rp.data(), sizeof(int64_t) * (size_t)(n + 1), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(g->trp, trp.data(), sizeof(int64_t) * (size_t)(n + 1), hipMemcpyHostToDevice, st);
        if (e == hipSuccess && g->m) e = hipMemcpyAsync(g->col, col.data(), sizeof(int32_t) * (size_t)g->m, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && g->m) e = hipMemcpyAsync(g->tcol, tcol.data(), sizeof(int32_t) * (size_t)g->m, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(st);
            free_graph(g);
            return fail(PP_EDEVICE, "graph upload: %s", hipGetErrorString(e));
        }
    }
    if (!perm.empty()) {
        if ((rc = dev_alloc(&g->perm_d, n))) {
            free_graph(g);
            return rc;
        }
        e = hipMemcpyAsync(g->perm_d, perm.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(st);
            free_graph(g);
            return fail(PP_EDEVICE, "order upload: %s", hipGetErrorString(e));
        }
    }
    // PROPAGATE-S: the nodes whose successor lists go to the group-per-node
    // launch, listed once with the graph (stored ids)
    {
        std::vector<int32_t> hv;
        for (int64_t u = 0; u < n; ++u)
            if (rp[(size_t)u + 1] - rp[(size_t)u] > pp::SEQ_LIGHT) hv.push_back((int32_t)u);
        if ((rc = dev_alloc(&g->seq_heavy, (int64_t)hv.size()))) {
            free_graph(g);
            return rc;
        }
        if (!hv.empty() && (e = hipMemcpy(g->seq_heavy, hv.data(), sizeof(int32_t) * hv.size(),
                                          hipMemcpyHostToDevice)) != hipSuccess) {
            free_graph(g);
            return fail(PP_EDEVICE, "long-list table upload: %s", hipGetErrorString(e));
        }
        g->nseq_heavy = (int64_t)hv.size();
    }
    // which nodes have a predecessor (a seed there can pass its bit on)
    g->pred_bits.assign((size_t)((n + 63) / 64), 0ull);
    for (int64_t u = 0; u < n; ++u)
        if (trp[(size_t)u + 1] > trp[(size_t)u]) g->pred_bits[(size_t)(u >> 6)] |= 1ull << (u & 63);
    g->rp_host = std::move(rp);
    g->perm = std::move(perm);
    *out = g;
    return PP_OK;
}

extern "C" void pp_graph_free(pp_graph g) { free_graph(g); }

extern "C" int pp_graph_get_csr(pp_graph g, int64_t *rp, int32_t *col, int64_t *trp, int32_t *tcol, int32_t *perm) {
    if (!g) return fail(PP_EINVAL, "graph is NULL");
    const size_t n = (size_t)g->n, m = (size_t)g->m;
    hipError_t e = hipSuccess;
    if (rp) e = hipMemcpy(rp, g->rp, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost);
    if (e == hipSuccess && col && m) e = hipMemcpy(col, g->col, sizeof(int32_t) * m, hipMemcpyDeviceToHost);
    if (e == hipSuccess && trp) e = hipMemcpy(trp, g->trp, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost);
    if (e == hipSuccess && tcol && m) e = hipMemcpy(tcol, g->tcol, sizeof(int32_t) * m, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(PP_EDEVICE, "adjacency download: %s", hipGetErrorString(e));
    if (perm)
        for (size_t x = 0; x < n; ++x) perm[x] = g->perm.empty() ? (int32_t)x : g->perm[x];
    return PP_OK;
}

// --------------------------------------------------------------------------
// runs
// --------------------------------------------------------------------------

namespace {

int words_for(int s) {
    const int w = (s + 63) / 64;
    int p = 1;
    while (p < w) p <<= 1;
    return p;
}

void free_run_dev(RunDev &d) {
    // each pair is one allocation owned by member 0
    dev_free(d.sig[0]);
    dev_free(d.acc);
    dev_free(d.stamp);
    dev_free(d.f_ids[0]);
    dev_free(d.f_delta[0]);
    dev_free(d.chunks[0]);
    d.sig[1] = nullptr;
    d.f_ids[1] = nullptr;
    d.f_delta[1] = nullptr;
    d.chunks[1] = nullptr;
    dev_free(d.blk_cnt);
    dev_free(d.blk_nodes);
    dev_free(d.blk_arcs);
    dev_free(d.blk_pulled);
    dev_free(d.counts);
    dev_free(d.seed_counts);
    dev_free(d.D);
    dev_free(d.gconv);
    dev_free(d.mode_log);
    dev_free(d.arcs_log);
    dev_free(d.ctrl);
    dev_free(d.bar);
    dev_free(d.phase_log);
    dev_free(d.feat_log);
    dev_free(d.tickets);
    dev_free(d.post_part);
    dev_free(d.mlp);
    dev_free(d.plan);
    dev_free(d.node_acc);
}

void drop_graphs(pp_run r) {
    for (auto &kv : r->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto &kv : r->graph_defs) (void)hipGraphDestroy(kv.second);
    r->graphs.clear();
    r->graph_defs.clear();
}

void free_run(pp_run r) {
    if (!r) return;
    if (r->stream) (void)hipStreamSynchronize(r->stream);
    drop_graphs(r);
    free_run_dev(r->dev);
    dev_free(r->dseeds);
    dev_free(r->dclusters);
    dev_free(r->iseeds);
    dev_free(r->dpos);
    dev_free(r->dcur);
    for (hipEvent_t e : r->ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : r->tev)
        if (e) (void)hipEventDestroy(e);
    if (r->seeds_sent) (void)hipEventDestroy(r->seeds_sent);
    if (r->pinned) (void)hipHostFree(r->pinned);
    if (r->own_stream && r->stream) (void)hipStreamDestroy(r->stream);
    delete r;
}

// push chunks: at most one per listed entry plus one per chunk of arcs, in a
// region of its own for each graph of a batch
int64_t chunk_capacity(pp_graph g) { return g->n + g->m / pp::PUSH_CHUNK_MIN + 2 * (int64_t)g->G + 2; }

// Allocates every device buffer of a run with the sizes fixed by (g, seeds,
// groups, cap): one copy of each per-group array for every seed group, the
// groups one after another (group_view in the kernels), counts and per-seed
// counts as rows of [groups][graphs] per round.
int alloc_run_dev(pp_graph g, RunDev &d, int s_all, int k, int sg, int W, int cap, bool seed_counts, int pull_grid) {
    const int64_t n = g->n;
    const int G = g->G;
    const int64_t KG = (int64_t)k * G;
    int rc;
    d.s = sg;
    d.sg = sg;
    d.s_last = s_all - (k - 1) * sg;
    d.s_all = s_all;
    d.ngroups = k;
    d.W = W;
    d.cap = cap;
    d.G = G;
    d.cstride = (int32_t)KG;
    d.sstride = (int32_t)(KG * sg);
    d.nn = n;
    d.pgrid = pull_grid;
    // the double buffers come in pairs, each pair one allocation (the kernels
    // pick a member by pointer arithmetic)
    const int64_t cc = chunk_capacity(g);
    d.cc = cc;
    if ((rc = dev_alloc(&d.sig[0], 2 * k * n * W)) || (rc = dev_alloc(&d.acc, k * n * W)) ||
        (rc = dev_alloc(&d.stamp, k * n)) || (rc = dev_alloc(&d.f_ids[0], 2 * k * n)) ||
        (rc = dev_alloc(&d.f_delta[0], 2 * k * n * W)) || (rc = dev_alloc(&d.chunks[0], 2 * k * cc)) ||
        (rc = dev_alloc(&d.blk_cnt, (int64_t)k * pull_grid)) || (rc = dev_alloc(&d.blk_nodes, (int64_t)k * pull_grid)) ||
        (rc = dev_alloc(&d.blk_arcs, (int64_t)k * pull_grid)) || (rc = dev_alloc(&d.blk_pulled, (int64_t)k * pull_grid)) ||
        (rc = dev_alloc(&d.counts, (int64_t)cap * KG)) || (rc = dev_alloc(&d.D, KG)) || (rc = dev_alloc(&d.gconv, KG)) ||
        (rc = dev_alloc(&d.mode_log, (int64_t)cap * KG)) || (rc = dev_alloc(&d.arcs_log, (int64_t)cap * KG)) ||
        (rc = dev_alloc(&d.ctrl, KG)) || (rc = dev_alloc(&d.bar, KG)) ||
        (rc = dev_alloc(&d.phase_log, (int64_t)cap * 3 * KG)) ||
        (rc = dev_alloc(&d.feat_log, (int64_t)cap * pp::MLP_IN * KG)) || (rc = dev_alloc(&d.mlp, pp::MLP_PARAMS)) ||
        (rc = dev_alloc(&d.plan, cap)) ||
        (rc = dev_alloc(&d.tickets, (int64_t)k * pp::TICKET_INTS)) ||
        (rc = dev_alloc(&d.post_part, (int64_t)k * 3 * pp::POST_MAX)))
        return rc;
    d.sig[1] = d.sig[0] + n * W;
    d.f_ids[1] = d.f_ids[0] + n;
    d.f_delta[1] = d.f_delta[0] + n * W;
    d.chunks[1] = d.chunks[0] + cc;
    if (seed_counts && (rc = dev_alloc(&d.seed_counts, (int64_t)cap * KG * sg))) return rc;
    if (!seed_counts) d.seed_counts = nullptr;
    return PP_OK;
}

// clean: per seed group, whether only its seeds' rows (prev_seeds, stored
// ids, sg per group) can hold bits; those groups clear just those rows.
// stale1: the other groups clear their first buffer in full and, in the
// second, only those rows.  That is enough because the second buffer is
// read only after a pull has made it current, and a pull writes every row
// there except those of nodes without successors, which no round changes:
// such a row holds nothing but its node's seed bits from the initialisation.
hipError_t clear_run_dev(pp_graph g, RunDev &d, hipStream_t st, bool with_acc,
                         const std::vector<char> &clean = {}, const int32_t *prev_seeds = nullptr,
                         bool stale1 = false) {
    const int64_t n = g->n;
    const int64_t k = d.ngroups;
    const int64_t KG = k * d.G;
    const int64_t cap = d.cap;
    auto seg = [](void *p, int64_t bytes, uint32_t v) { return pp::FillSeg{(uint32_t *)p, bytes / 4, v}; };
    std::vector<pp::FillSeg> rows;   // signature rows and stamps, then the rest: one fill launch
    bool some_clean = false;
    for (char c : clean) some_clean |= c != 0;
    if (!prev_seeds || (!some_clean && !stale1)) {
        rows.push_back(seg(d.sig[0], 2 * 8 * k * n * d.W, 0u));  // both signature buffers of every group
        rows.push_back(seg(d.stamp, 4 * k * n, 0xFFFFFFFFu));    // -1: never queued
    } else {
        for (int64_t j = 0; j < k; ++j) {
            uint64_t *sj = d.sig[0] + j * 2 * n * d.W;
            const bool cj = (size_t)j < clean.size() && clean[(size_t)j];
            if (cj || stale1) {   // the seeds' rows in both buffers (the fill below runs after)
                const int cnt = j == k - 1 ? d.s_last : d.sg;
                const hipError_t e = pp::launch_clear_seed_rows(prev_seeds + j * d.sg, cnt, n, d.W, sj, d.stamp + j * n, st);
                if (e != hipSuccess) return e;
            }
            if (!cj) {
                rows.push_back(seg(sj, (stale1 ? 1 : 2) * 8 * n * d.W, 0u));
                rows.push_back(seg(d.stamp + j * n, 4 * n, 0xFFFFFFFFu));
            }
        }
    }
    const pp::FillSeg rest[] = {
        seg(d.acc, with_acc ? 8 * k * n * d.W : 0, 0u),
        seg(d.counts, 8 * cap * KG, 0u),
        seg(d.seed_counts, d.seed_counts ? 4 * cap * KG * d.sg : 0, 0u),
        seg(d.D, 4 * KG, 0u),
        seg(d.gconv, 4 * KG, 0u),
        seg(d.mode_log, 4 * cap * KG, 0xFFFFFFFFu),
        seg(d.arcs_log, 8 * cap * KG, 0u),
        seg(d.bar, (int64_t)sizeof(pp::GridBar) * KG, 0u),
        seg(d.phase_log, 8 * cap * 3 * KG, 0u),
        seg(d.feat_log, 4 * cap * pp::MLP_IN * KG, 0u),
        seg(d.ctrl, (int64_t)sizeof(Ctrl) * KG, 0u),
        seg(d.tickets, 4 * pp::TICKET_INTS * k, 0u),
        seg(d.node_acc, d.node_acc ? 8 * n : 0, 0u),
    };
    rows.insert(rows.end(), std::begin(rest), std::end(rest));
    return pp::launch_fills(rows.data(), (int)rows.size(), st);
}

TileSet *run_tiles(pp_run r) { return &r->g->tiles[pull_edges(r->W, r->dev.pull_k)]; }

// Host copy of the control state.  The clustered engine keeps one control
// block per graph: the summary has the largest round, converged when every
// graph has, and the flags of any.
// Pinned host staging of a run: G control blocks, G values of D,
// STAGE_ROWS rows of G counts and a seed list of G s ids.
int alloc_staging(pp_run r) {
    const size_t KG = (size_t)r->k * (size_t)r->G;   // control blocks, D values and counts per row
    const size_t G = KG;
    const size_t bytes = sizeof(Ctrl) * KG + 8 * ((KG + 1) / 2) + sizeof(int64_t) * STAGE_ROWS * KG +
                         sizeof(int32_t) * (size_t)r->G * (size_t)r->s;
    // coherent and mapped: the staging kernel stores into it directly
    if (hipHostMalloc(&r->pinned, bytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        r->pinned = nullptr;
        (void)hipGetLastError();
        return fail(PP_ENOMEM, "pinned host staging of %zu bytes", bytes);
    }
    r->h_ctrl = (Ctrl *)r->pinned;
    r->h_D = (int32_t *)(r->h_ctrl + G);
    r->h_rows = (int64_t *)((char *)r->h_D + 8 * ((G + 1) / 2));
    r->h_seeds = (int32_t *)(r->h_rows + STAGE_ROWS * KG);
    void *dev = nullptr;
    if (hipHostGetDevicePointer(&dev, r->pinned, 0) != hipSuccess || !dev) {
        (void)hipGetLastError();
        return fail(PP_EDEVICE, "pinned host staging is not mapped for the device");
    }
    r->h_ctrl_dev = dev;
    r->h_D_dev = (int32_t *)((char *)dev + ((char *)r->h_D - (char *)r->pinned));
    r->h_rows_dev = (int64_t *)((char *)dev + ((char *)r->h_rows - (char *)r->pinned));
    r->h_seeds_dev = (int32_t *)((char *)dev + ((char *)r->h_seeds - (char *)r->pinned));
    r->D_host.assign(KG, 0);
    if (hipEventCreateWithFlags(&r->seeds_sent, hipEventDisableTiming) != hipSuccess) {
        r->seeds_sent = nullptr;
        return fail(PP_EDEVICE, "event creation");
    }
    return PP_OK;
}

int reset_run(pp_run r, const int32_t *seeds, const int32_t *map);

// Host seeds (already checked): input ids -> stored ids in the pinned list
// (once the initialisation that read the last list has run), then the
// initialisation, which reads the list in place; the event marks when it has.
int reset_with_host_seeds(pp_run r, const int32_t *seeds) {
    const int64_t total = (int64_t)r->G * r->s;
    HIP_TRY(hipEventSynchronize(r->seeds_sent));
    const std::vector<int32_t> &perm = r->g->perm;
    for (int64_t j = 0; j < total; ++j) r->h_seeds[j] = perm.empty() ? seeds[j] : perm[(size_t)seeds[j]];
    int rc = reset_run(r, r->h_seeds_dev, nullptr);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(r->seeds_sent, r->stream));
    return PP_OK;
}

// One wait for the host copy of the control state: the control blocks, D,
// and the count rows [staged, upto) (at most STAGE_ROWS of them).  The
// clustered engine keeps one control block per graph: the summary has the
// largest round, converged when every graph has, and the flags of any.  A
// seed outside its graph (device seed lists are checked by the device) is
// reported here.
int sync_state(pp_run r, int upto) {
    // control blocks staged: one per graph (clustered engine), one per seed
    // group (the per-round engine: group j's at j * G), one otherwise
    const int G = r->G;
    const int KG = r->k * G;
    const int nstage = r->pgrid ? G : (r->k > 1 ? KG : 1);
    const int rows = std::max(0, std::min({upto, r->cap, r->staged + STAGE_ROWS}) - r->staged);
    HIP_TRY(pp::launch_stage(r->dev.ctrl, (int64_t)sizeof(Ctrl) * nstage, r->dev.D, KG,
                             r->dev.counts + (int64_t)r->staged * KG, (int64_t)rows * KG, r->h_ctrl_dev, r->h_D_dev,
                             r->h_rows_dev, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    const int nc = r->pgrid ? G : r->k;          // live control blocks
    const int cstep = r->pgrid ? 1 : G;
    r->host_ctrl = r->h_ctrl[0];
    r->cur.assign((size_t)nc, 0);
    for (int j = 0; j < nc; ++j) {
        const Ctrl &c = r->h_ctrl[(size_t)j * cstep];
        r->cur[(size_t)j] = c.cur & 1;
        if (j == 0) continue;
        r->host_ctrl.round = std::max(r->host_ctrl.round, c.round);
        r->host_ctrl.converged = r->host_ctrl.converged && c.converged;
        r->host_ctrl.overflow |= c.overflow;
        r->host_ctrl.bad_seed |= c.bad_seed;
    }
    r->D_host.assign(r->h_D, r->h_D + KG);
    if (rows > 0) {
        r->counts_host.insert(r->counts_host.end(), r->h_rows, r->h_rows + (size_t)rows * KG);
        r->staged += rows;
    }
    if (r->host_ctrl.bad_seed) return fail(PP_ERANGE, "a seed id lies outside its graph's node range");
    return PP_OK;
}

int sync_ctrl(pp_run r) { return sync_state(r, 0); }

// Count rows [0, upto) on the host (a wait only for rows not copied yet;
// many rows at once go straight into the host array).
int ensure_staged(pp_run r, int upto) {
    upto = std::min(upto, r->cap);
    if (r->staged >= upto) return PP_OK;
    if (upto - r->staged <= STAGE_ROWS) return sync_state(r, upto);
    const size_t G = (size_t)r->k * (size_t)r->G;   // values per round row
    const size_t have = r->counts_host.size();
    r->counts_host.resize((size_t)upto * G);
    HIP_TRY(hipMemcpyAsync(r->counts_host.data() + have, r->dev.counts + have, sizeof(int64_t) * ((size_t)upto * G - have),
                           hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    r->staged = upto;
    return PP_OK;
}

// c_g[row] of graph gi, summed over the seed groups (rows already staged).
int64_t staged_count(pp_run r, int row, int gi) {
    int64_t c = 0;
    const size_t base = (size_t)row * r->k * r->G;
    for (int j = 0; j < r->k; ++j) c += r->counts_host[base + (size_t)j * r->G + gi];
    return c;
}

// D of graph gi: the largest over its seed groups.
int32_t staged_D(pp_run r, int gi) {
    int32_t d = 0;
    for (int j = 0; j < r->k; ++j) d = std::max(d, r->D_host[(size_t)j * r->G + gi]);
    return d;
}

}  // namespace

void *pp::dev_malloc(size_t bytes) {
    Allocator a;
    {
        std::lock_guard<std::mutex> lk(alloc_mu());
        a = g_alloc;
    }
    if (!a.alloc) {
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void *p = a.alloc(bytes, t_alloc_stream, a.ctx);
    if (p && (reinterpret_cast<uintptr_t>(p) & 255u) != 0) {   // the kernels' vector accesses need the alignment
        a.release(p, t_alloc_stream, a.ctx);
        return nullptr;
    }
    if (p) {
        std::lock_guard<std::mutex> lk(alloc_mu());
        owned_blocks()[p] = OwnedBlock{a, t_alloc_stream};
    }
    return p;
}

void pp::dev_release(void *p) {
    if (!p) return;
    OwnedBlock o{};
    bool owned = false;
    {
        std::lock_guard<std::mutex> lk(alloc_mu());
        auto it = owned_blocks().find(p);
        if (it != owned_blocks().end()) {
            o = it->second;
            owned_blocks().erase(it);
            owned = true;
        }
    }
    if (!owned) {
        (void)hipFree(p);
        return;
    }
    // Stream-ordered: every caller of dev_release has waited for the streams
    // its work on the block ran on (a run's stream, a call's stream), so the
    // allocator may hand the block out again at once.
    o.from.release(p, o.stream, o.from.ctx);
}

pp::AllocStream::AllocStream(void *stream) : prev(t_alloc_stream) { t_alloc_stream = stream; }
pp::AllocStream::~AllocStream() { t_alloc_stream = prev; }

extern "C" int pp_set_allocator(void *(*alloc)(size_t, void *, void *), void (*release)(void *, void *, void *),
                                void *ctx) {
    if ((alloc == nullptr) != (release == nullptr)) return fail(PP_EINVAL, "alloc and release: both or neither");
    std::lock_guard<std::mutex> lk(alloc_mu());
    g_alloc = Allocator{alloc, release, alloc ? ctx : nullptr};
    return PP_OK;
}

int pp::set_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

namespace {

// A failed round launch may have stopped part-way through a round.
hipError_t noted(pp_run r, hipError_t e) {
    if (e != hipSuccess) r->acc_clean = false;
    return e;
}

int launch_clusters(pp_run r, int max_round) {
    GraphDev gv = graph_view(r->g, run_tiles(r), r->W);
    HIP_TRY(noted(r, pp::launch_batch_persistent(gv, r->dev, r->dclusters, (int)r->clusters.size(), r->pgrid,
                                                 max_round, r->stream)));
    return PP_OK;
}

// Algorithm 1's initialisation on an allocated run: clear every buffer, place
// the seed bits, run the round-0 commit.  seeds: device-readable input ids,
// mapped to stored ids by map when it is given (ids outside [0, n) become
// -1, which the seed placement reports).  The clustered engine synchronises;
// the per-round engine does not wait.
int reset_run(pp_run r, const int32_t *seeds, const int32_t *map) {
    pp_graph g = r->g;
    TileSet *ts = run_tiles(r);
    GraphDev gv = graph_view(g, ts, r->W);
    // Seed groups whose rows hold nothing but their seeds' bits: the last
    // propagation converged without a new bit in the group after round 0 (a
    // group of seeds without predecessors, as grouping by reach places them
    // last).  Their reset clears only their seeds' rows.
    std::vector<char> clean;
    if (r->grouped && r->G == 1 && r->acc_clean && r->host_ctrl.converged && !r->host_ctrl.bad_seed &&
        !r->host_ctrl.overflow && (int)r->D_host.size() == r->k) {
        clean.assign((size_t)r->k, 0);
        for (int j = 0; j < r->k; ++j) clean[(size_t)j] = r->D_host[(size_t)j] == 0;
    }
    // The other groups' second buffers keep their rows except the seeds'
    // (the stored seed list of the last initialisation names them); so does
    // the second buffer of a single graph without groups once its seeds are
    // kept.
    const bool plain1 = !r->grouped && !r->pgrid && r->G == 1;
    const bool stale1 = r->acc_clean && r->G == 1 && (r->grouped || (plain1 && r->seeds_kept));
    hipError_t e = clear_run_dev(g, r->dev, r->stream, !r->acc_clean, clean, r->grouped ? r->iseeds : r->dseeds,
                                 stale1);
    r->seeds_kept = false;
    if (e == hipSuccess) {
        r->acc_clean = true;
        if (r->grouped) {
            // the seed list in internal order (stored ids), then the groups' seed bits
            e = pp::launch_seed_order(gv, seeds, map, r->G, r->s, r->opt.seed_order == PP_ORDER_BY_REACH, r->iseeds,
                                      r->dpos, r->stream);
            if (e == hipSuccess) e = pp::launch_seed_init(gv, r->dev, r->iseeds, nullptr, r->stream);
        } else if (r->pgrid) {
            if (map) {
                e = pp::launch_map_ids(r->dseeds, seeds, map, (int64_t)r->G * r->s, g->n, r->stream);
                seeds = r->dseeds;
            }
            if (e == hipSuccess) e = pp::launch_seed_scatter_batch(gv, r->dev, seeds, r->stream);
        } else {
            e = pp::launch_seed_init(gv, r->dev, seeds, map, r->stream);
            if (e == hipSuccess && plain1) {
                e = map ? pp::launch_map_ids(r->dseeds, seeds, map, r->s, g->n, r->stream)
                        : hipMemcpyAsync(r->dseeds, seeds, sizeof(int32_t) * (size_t)r->s, hipMemcpyDefault, r->stream);
                r->seeds_kept = e == hipSuccess;
            }
        }
    }
    if (e != hipSuccess) return fail(PP_EDEVICE, "seed initialisation: %s", hipGetErrorString(e));
    r->staged = 0;
    r->counts_host.clear();
    r->D_host.assign((size_t)r->k * r->G, 0);
    if (r->pgrid) {
        int rc = launch_clusters(r, 0);   // round 0 of every graph only
        if (rc) return rc;
        return sync_ctrl(r);
    }
    // The per-round engine does not wait: after the initialisation every
    // graph has c[0] = s > 0, so the state is known -- round 1 next, not
    // converged, signatures in buffer 0.  A device seed outside its graph is
    // reported by the next call that waits.
    r->host_ctrl = Ctrl{};
    r->host_ctrl.round = 1;
    r->cur.assign((size_t)r->k, 0);
    return PP_OK;
}

// Splits the persistent grid among the graphs of a batch, in proportion to
// their arcs plus nodes, at least one block each and at most one per 64 Ki
// arcs plus nodes (blocks beyond every cap stay idle); graph order is kept.
std::vector<pp::Cluster> make_clusters(pp_graph g, const TileSet *ts, int grid) {
    const int G = g->G;
    std::vector<double> w((size_t)G);
    double tot = 0.0;
    for (int k = 0; k < G; ++k) {
        const int64_t n0 = g->node_offsets[(size_t)k], n1 = g->node_offsets[(size_t)k + 1];
        w[(size_t)k] = (double)(g->rp_host[(size_t)n1] - g->rp_host[(size_t)n0]) + (double)(n1 - n0) + 1.0;
        tot += w[(size_t)k];
    }
    // a graph gets at most one block per CLUSTER_ITEMS arcs plus nodes: small
    // graphs run many cheap rounds, where a barrier among a few blocks costs
    // more than the work it spreads (one block synchronises with its own
    // barrier only)
    constexpr double CLUSTER_ITEMS = 65536.0;
    std::vector<int> nb((size_t)G, 1), cap((size_t)G);
    int used = G;
    for (int k = 0; k < G; ++k) {
        cap[(size_t)k] = (int)std::max(1.0, std::ceil(w[(size_t)k] / CLUSTER_ITEMS));
        const int extra = std::min((int)((double)(grid - G) * w[(size_t)k] / tot), cap[(size_t)k] - 1);
        nb[(size_t)k] += extra;
        used += extra;
    }
    for (bool grew = true; used < grid && grew;) {   // leftovers, round robin, up to each cap
        grew = false;
        for (int k = 0; k < G && used < grid; ++k)
            if (nb[(size_t)k] < cap[(size_t)k]) {
                ++nb[(size_t)k];
                ++used;
                grew = true;
            }
    }
    std::vector<pp::Cluster> cl((size_t)G);
    int b0 = 0;
    int64_t ch0 = 0;
    for (int k = 0; k < G; ++k) {
        pp::Cluster &c = cl[(size_t)k];
        const int64_t n0 = g->node_offsets[(size_t)k], n1 = g->node_offsets[(size_t)k + 1];
        c.g = k;
        c.b0 = b0;
        c.nb = nb[(size_t)k];
        c.t0 = ts->gtile[(size_t)k];
        c.t1 = ts->gtile[(size_t)k + 1];
        c.h0 = ts->ghub[(size_t)k];
        c.h1 = ts->ghub[(size_t)k + 1];
        c.pad = 0;
        c.n0 = n0;
        c.n1 = n1;
        c.m = g->rp_host[(size_t)n1] - g->rp_host[(size_t)n0];
        c.ch0 = ch0;
        b0 += c.nb;
        ch0 += (n1 - n0) + c.m / pp::PUSH_CHUNK_MIN + 2;
    }
    return cl;
}

int check_host_seeds(pp_graph g, const int32_t *seeds, int s) {
    for (int gi = 0; gi < g->G; ++gi)
        for (int i = 0; i < s; ++i) {
            const int64_t x = seeds[(int64_t)gi * s + i];
            if (x < g->node_offsets[(size_t)gi] || x >= g->node_offsets[(size_t)gi + 1])
                return fail(PP_ERANGE, "seed %d of graph %d (%lld) outside the graph's nodes", i, gi, (long long)x);
        }
    return PP_OK;
}

}  // namespace

extern "C" int pp_seeds_init(pp_graph g, const int32_t *seeds, int32_t s, const pp_options *opt, void *stream,
                             pp_run *out) {
    if (!g || !out) return fail(PP_EINVAL, "graph or out is NULL");
    pp::AllocStream as(stream);
    if (s < 1 || s > 4096) return fail(PP_EINVAL, "s = %d outside [1, 4096]", s);
    if (!seeds) return fail(PP_EINVAL, "seeds is NULL");
    pp_options o;
    pp_options_default(&o);
    if (opt) o = *opt;
    if (o.push_div <= 0) o.push_div = 8;
    if (o.pull_k == 0) o.pull_k = 4;
    if (o.pull_k != 2 && o.pull_k != 4) return fail(PP_EINVAL, "pull_k = %d: 2 or 4 arcs per lane", o.pull_k);
    if (o.persistent && o.pull_k != 4) return fail(PP_EINVAL, "the persistent engine pulls with 4 arcs per lane");
    if (o.node_stats && o.persistent) return fail(PP_EINVAL, "per-node statistics need the per-round engine");
    if (o.node_stats != 0 && o.node_stats != 1) return fail(PP_EINVAL, "node_stats must be 0 or 1");
    if (o.sparse_pull < 0 || o.sparse_pull > 2) return fail(PP_EINVAL, "sparse_pull = %d: 0, 1 or 2", o.sparse_pull);
    if (o.sparse_pull && o.persistent) return fail(PP_EINVAL, "sparse pulls need the per-round engine");
    if (o.scheduler < PP_SCHED_HEURISTIC || o.scheduler > PP_SCHED_PLAN) return fail(PP_EINVAL, "unknown scheduler %d", o.scheduler);
    if (o.max_rounds < 0 || o.rounds_per_sync < 0) return fail(PP_EINVAL, "negative max_rounds / rounds_per_sync");
    if (o.seed_order != 0 && o.seed_order != PP_ORDER_BY_REACH) return fail(PP_EINVAL, "seed_order = %d: 0 or 1", o.seed_order);
    if (o.seed_groups < PP_GROUPS_BY_REACH || o.seed_groups > 64)
        return fail(PP_EINVAL, "seed_groups = %d outside [-1, 64]", o.seed_groups);
    const int G = g->G;
    int rc = check_host_seeds(g, seeds, s);
    if (rc) return rc;
    // seed groups: k groups of sg seeds (the last may hold fewer), rows of W words each
    if (o.seed_groups == PP_GROUPS_BY_REACH) o.seed_order = PP_ORDER_BY_REACH;
    int k = o.seed_groups > 0 ? o.seed_groups : (s + 511) / 512;
    if (o.seed_groups == PP_GROUPS_BY_REACH) {
        // one group wide enough for the seeds with a predecessor (the most of any graph)
        int live = 1;
        for (int gi = 0; gi < G; ++gi) {
            int c = 0;
            for (int i = 0; i < s; ++i) {
                const int32_t x = seeds[(int64_t)gi * s + i];
                const size_t u = g->perm.empty() ? (size_t)x : (size_t)g->perm[(size_t)x];
                c += (int)((g->pred_bits[u >> 6] >> (u & 63)) & 1ull);
            }
            live = std::max(live, c);
        }
        const int sg0 = std::min(512, 64 * words_for(live));
        k = (s + sg0 - 1) / sg0;
    }
    const int sg = (s + k - 1) / k;
    if (sg > 512) return fail(PP_EINVAL, "%d seeds in %d groups: more than 512 per group", s, k);
    if ((int64_t)(k - 1) * sg >= s) return fail(PP_EINVAL, "%d seeds do not fill %d groups of %d", s, k, sg);
    if (k > 1 && o.persistent) return fail(PP_EINVAL, "seed groups need the per-round engine");
    if (k > 1 && o.node_stats) return fail(PP_EINVAL, "per-node statistics need a single seed group");
    if (o.seed_order && o.persistent) return fail(PP_EINVAL, "a seed order needs the per-round engine");
    int64_t cap = o.max_rounds > 0 ? (int64_t)o.max_rounds + 1 : std::min<int64_t>(g->n + 1, 1 << 20);
    if (cap < 2) cap = 2;
    if (o.seed_counts && cap * G * (int64_t)k * sg * 4 > (int64_t)1 << 31)
        return fail(PP_EINVAL, "per-seed count log of %lld bytes: lower max_rounds",
                    (long long)(cap * G * (int64_t)k * sg * 4));
    const int W = words_for(sg);

    pp_run r = new (std::nothrow) pp_run_s();
    if (!r) return fail(PP_ENOMEM, "run handle");
    r->g = g;
    r->s = s;
    r->W = W;
    r->k = k;
    r->sg = sg;
    r->Wout = words_for(s);
    r->grouped = k > 1 || o.seed_order != 0;
    r->cap = (int32_t)cap;
    r->G = G;
    r->opt = o;
    r->dev.pull_k = o.pull_k;
    r->timing = o.time_kernels != 0;
    if (o.persistent) {
        r->pgrid = pp::persistent_grid(words_for(s));
        if (r->pgrid < 1) {
            delete r;
            return fail(PP_EDEVICE, "no co-resident grid for the persistent round loop");
        }
        if (G > r->pgrid) {
            const int p = r->pgrid;
            delete r;
            return fail(PP_EINVAL, "%d graphs but only %d co-resident blocks: use the per-round engine", G, p);
        }
    }
    {
        int dev = 0, khz = 0;   // the device clock of the per-round stamps
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            r->clock_khz = khz;
    }
    if (stream) {
        r->stream = (hipStream_t)stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete r;
            return fail(PP_EDEVICE, "stream: %s", hipGetErrorString(e));
        }
        r->own_stream = true;
    }
    pp::AllocStream run_as(r->stream);   // the run's blocks are used on its stream
    TileSet *ts = nullptr;
    rc = ensure_tiles(g, W, r->dev.pull_k, &ts);
    if (rc == PP_OK)
        rc = alloc_run_dev(g, r->dev, s, k, sg, W, (int)cap, o.seed_counts != 0,
                           std::max(pp::pull_grid_for(ts->ntiles, W), r->pgrid));
    if (rc == PP_OK) rc = dev_alloc(&r->dseeds, (int64_t)G * s);
    if (rc == PP_OK && r->grouped && ((rc = dev_alloc(&r->iseeds, (int64_t)G * s)) == PP_OK))
        if ((rc = dev_alloc(&r->dpos, (int64_t)G * s)) == PP_OK) rc = dev_alloc(&r->dcur, k);
    if (rc == PP_OK && o.node_stats) rc = dev_alloc(&r->dev.node_acc, g->n);
    if (rc == PP_OK && r->pgrid) {
        r->clusters = make_clusters(g, ts, r->pgrid);
        rc = dev_alloc(&r->dclusters, (int64_t)r->clusters.size());
        if (rc == PP_OK && hipMemcpy(r->dclusters, r->clusters.data(), sizeof(pp::Cluster) * r->clusters.size(),
                                     hipMemcpyHostToDevice) != hipSuccess)
            rc = fail(PP_EDEVICE, "cluster upload");
    }
    if (rc == PP_OK && r->timing) {
        r->pull_ms.assign((size_t)cap, 0.0f);
        r->ev.resize(2 * 64, nullptr);
        for (auto &e : r->ev)
            if (hipEventCreate(&e) != hipSuccess) {
                rc = fail(PP_EDEVICE, "event creation");
                break;
            }
    }
    if (rc != PP_OK) {
        free_run(r);
        return rc;
    }
    r->dev.sched = o.scheduler;
    r->dev.push_div = o.push_div;
    r->dev.sparse_pull = o.sparse_pull;
    r->dev.fuzz_seed = o.fuzz_seed;
    // cost-model weights start as NaN: the heuristic decides until they are set
    hipError_t e = pp::launch_fill_i32((int32_t *)r->dev.mlp, kNaNBits, pp::MLP_PARAMS, r->stream);
    if (e == hipSuccess) e = pp::launch_fill_i32(r->dev.plan, -1, cap, r->stream);   // no plan: the heuristic
    if (e != hipSuccess) {
        free_run(r);
        return fail(PP_EDEVICE, "cost-model reset: %s", hipGetErrorString(e));
    }
    if ((rc = alloc_staging(r)) != PP_OK || (rc = reset_with_host_seeds(r, seeds)) != PP_OK) {
        free_run(r);
        return rc;
    }
    *out = r;
    return PP_OK;
}

extern "C" int pp_seeds_reset(pp_run r, const int32_t *seeds, int32_t seeds_on_device) {
    if (!r || !seeds) return fail(PP_EINVAL, "run or seeds is NULL");
    if (!seeds_on_device) {
        int rc = check_host_seeds(r->g, seeds, r->s);
        if (rc) return rc;
        return reset_with_host_seeds(r, seeds);
    }
    return reset_run(r, seeds, r->g->perm_d);
}

extern "C" void pp_run_free(pp_run r) { free_run(r); }

namespace {

// Rounds up to max_round in one cooperative launch; synchronises.  The
// per-round device-clock stamps of the launch feed the kernel times.
int run_persistent(pp_run r, int max_round) {
    const int before = r->host_ctrl.round;
    int rc = launch_clusters(r, max_round);
    if (rc) return rc;
    if ((rc = sync_ctrl(r))) return rc;
    std::vector<pp::GridBar> bars((size_t)r->G);
    HIP_TRY(hipMemcpy(bars.data(), r->dev.bar, sizeof(pp::GridBar) * bars.size(), hipMemcpyDeviceToHost));
    for (const pp::GridBar &b : bars)
        if (b.abort) {
            r->acc_clean = false;
            return fail(PP_EDEVICE, "persistent round loop: a cluster barrier timed out");
        }
    if (r->timing) {
        const int last = std::min(r->host_ctrl.converged ? r->host_ctrl.round : r->host_ctrl.round - 1, r->cap - 1);
        if (last >= before) {
            std::vector<int64_t> st((size_t)(last - before + 1) * 3);
            HIP_TRY(hipMemcpy(st.data(), r->dev.phase_log + (int64_t)before * 3, sizeof(int64_t) * st.size(),
                              hipMemcpyDeviceToHost));
            for (int k = before; k <= last; ++k) {
                const int64_t *s = st.data() + (size_t)(k - before) * 3;
                if (s[1] > s[0]) r->pull_ms[(size_t)k] += (float)((double)(s[1] - s[0]) / r->clock_khz);
            }
        }
    }
    return PP_OK;
}

}  // namespace
extern "C" int32_t pp_run_round(pp_run r) { return r ? r->host_ctrl.round : -1; }
extern "C" int32_t pp_run_words(pp_run r) { return r ? r->Wout : -1; }
extern "C" int32_t pp_run_groups(pp_run r) { return r ? r->k : -1; }
extern "C" int32_t pp_run_group_words(pp_run r) { return r ? r->W : -1; }

extern "C" int pp_propagate_round(pp_run r, int64_t *new_bits, int32_t *all_converged) {
    if (!r) return fail(PP_EINVAL, "run is NULL");
    const int G = r->G;
    if (r->host_ctrl.converged) {
        if (new_bits) std::memset(new_bits, 0, sizeof(int64_t) * (size_t)G);
        if (all_converged) *all_converged = 1;
        return r->host_ctrl.overflow ? fail(PP_ENOTCONV, "round log full (max_rounds)") : PP_OK;
    }
    const int rr = r->host_ctrl.round;
    int rc;
    if (r->pgrid) {
        if ((rc = run_persistent(r, rr))) return rc;
    } else {
        GraphDev gv = graph_view(r->g, run_tiles(r), r->W);
        hipEvent_t e0 = r->timing ? r->ev[0] : nullptr, e1 = r->timing ? r->ev[1] : nullptr;
        HIP_TRY(noted(r, pp::launch_round(gv, r->dev, r->stream, e0, e1)));
        if ((rc = sync_state(r, rr + 1))) return rc;
        if (r->timing) {
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            r->pull_ms[(size_t)rr] += ms;
        }
    }
    if (new_bits) {
        if (rr < r->cap) {
            if ((rc = ensure_staged(r, rr + 1))) return rc;
            for (int gi = 0; gi < G; ++gi) new_bits[gi] = staged_count(r, rr, gi);
        } else {
            std::memset(new_bits, 0, sizeof(int64_t) * (size_t)G);
        }
    }
    if (all_converged) *all_converged = r->host_ctrl.converged;
    if (r->host_ctrl.overflow) return fail(PP_ENOTCONV, "round log full (max_rounds)");
    return PP_OK;
}

namespace {

hipEvent_t slot_event(pp_run r, int i, int which) { return r->timing ? r->ev[(size_t)(2 * i + which)] : nullptr; }

int launch_batch(pp_run r, int k) {
    GraphDev gv = graph_view(r->g, run_tiles(r), r->W);
    if (!r->opt.use_graph || (r->timing && !r->graph_events)) {
        for (int i = 0; i < k; ++i)
            HIP_TRY(noted(r, pp::launch_round(gv, r->dev, r->stream, slot_event(r, i, 0), slot_event(r, i, 1))));
        return PP_OK;
    }
    auto it = r->graphs.find(k);
    if (it == r->graphs.end()) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        HIP_TRY(hipStreamBeginCapture(r->stream, hipStreamCaptureModeThreadLocal));
        hipError_t le = hipSuccess;
        for (int i = 0; i < k && le == hipSuccess; ++i)
            le = pp::launch_round(gv, r->dev, r->stream, slot_event(r, i, 0), slot_event(r, i, 1));
        hipError_t ce = hipStreamEndCapture(r->stream, &graph);
        if (le != hipSuccess && r->timing) {
            // events inside a capture are not supported here: time direct launches instead
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            r->graph_events = false;
            return launch_batch(r, k);
        }
        if (le != hipSuccess) return fail(PP_EDEVICE, "round capture: %s", hipGetErrorString(le));
        if (ce != hipSuccess) return fail(PP_EDEVICE, "end capture: %s", hipGetErrorString(ce));
        HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        r->graph_defs[k] = graph;
        r->graphs[k] = exec;
        it = r->graphs.find(k);
    }
    HIP_TRY(noted(r, hipGraphLaunch(it->second, r->stream)));
    return PP_OK;
}

}  // namespace

extern "C" int pp_propagate_until_converged(pp_run r, int32_t max_rounds, int64_t *counts, int32_t cap_rounds,
                                            int32_t *D) {
    if (!r) return fail(PP_EINVAL, "run is NULL");
    if (counts && cap_rounds < 1) return fail(PP_EINVAL, "cap_rounds < 1");
    const int G = r->G;
    const int limit = (max_rounds > 0 && max_rounds < r->cap - 1) ? max_rounds : r->cap - 1;
    // adaptive batches: 8 rounds, then as many rounds as have run so far (at
    // most 64) -- a host check costs about as much as a few replayed rounds
    // that find the run converged and return at once
    const int start = r->host_ctrl.round;
    int K = r->opt.rounds_per_sync > 0 ? r->opt.rounds_per_sync : 8;
    if (r->pgrid && !r->host_ctrl.converged && r->host_ctrl.round <= limit) {
        int rc = run_persistent(r, limit);
        if (rc) return rc;
    }
    while (!r->pgrid && !r->host_ctrl.converged && r->host_ctrl.round <= limit) {
        const int left = limit - r->host_ctrl.round + 1;
        int k = std::min(K, left);
        // replayed batches come in powers of two so few graphs are captured
        if (r->opt.use_graph) {
            int p = 1;
            while (p * 2 <= k) p *= 2;
            k = p;
        }
        const int before = r->host_ctrl.round;
        int rc = launch_batch(r, k);
        if (rc) return rc;
        if ((rc = sync_state(r, before + k))) return rc;
        if (r->timing) {
            // rounds before..last ran; launches after convergence returned at once
            const int last = r->host_ctrl.converged ? r->host_ctrl.round : before + k - 1;
            for (int i = 0; i < k && before + i <= last && before + i < r->cap; ++i) {
                float ms = 0.0f;
                const hipError_t te = hipEventElapsedTime(&ms, slot_event(r, i, 0), slot_event(r, i, 1));
                if (te != hipSuccess && r->opt.use_graph && r->graph_events) {
                    // no timing from events replayed in a graph: time direct launches from now on
                    (void)hipGetLastError();
                    r->graph_events = false;
                    break;
                }
                if (te != hipSuccess) return fail(PP_EDEVICE, "event timing: %s", hipGetErrorString(te));
                r->pull_ms[(size_t)(before + i)] += ms;
            }
        }
        if (r->opt.rounds_per_sync <= 0) K = std::min(std::max(8, r->host_ctrl.round - start), 64);
    }
    // results, from what the waits above copied back
    const int last = std::min(r->host_ctrl.round, r->cap - 1);
    if (counts) {
        int rc = ensure_staged(r, last + 1);
        if (rc) return rc;
        std::memset(counts, 0, sizeof(int64_t) * (size_t)G * cap_rounds);
        for (int g = 0; g < G; ++g)
            for (int k = 0; k <= last && k < cap_rounds; ++k) counts[(int64_t)g * cap_rounds + k] = staged_count(r, k, g);
    }
    if (D)
        for (int g = 0; g < G; ++g) D[g] = staged_D(r, g);
    if (!r->host_ctrl.converged || r->host_ctrl.overflow) return fail(PP_ENOTCONV, "stopped after %d rounds without convergence", r->host_ctrl.round);
    return PP_OK;
}

namespace {
int copy_signatures(pp_run r, uint64_t *dst, hipMemcpyKind kind);
}  // namespace

extern "C" int pp_get_signatures(pp_run r, uint64_t *dst, int32_t dst_on_device) {
    if (!r || !dst) return fail(PP_EINVAL, "run or dst is NULL");
    if (r->grouped) {
        // the groups' rows in the caller's bit order (stored node order), then by input id
        int rc = sync_ctrl(r);   // each group's current buffer
        if (rc) return rc;
        const int64_t n = r->g->n, words = n * r->Wout;
        std::vector<int32_t> cur(r->cur.begin(), r->cur.end());
        uint64_t *tmp = nullptr, *out = nullptr;
        const bool direct = dst_on_device && !r->g->perm_d;
        if (!direct) rc = dev_alloc(&tmp, words);
        if (!rc && !dst_on_device && r->g->perm_d) rc = dev_alloc(&out, words);
        hipError_t e = hipSuccess;
        if (!rc) e = hipMemcpyAsync(r->dcur, cur.data(), sizeof(int32_t) * cur.size(), hipMemcpyHostToDevice, r->stream);
        uint64_t *rows = direct ? dst : tmp;
        if (!rc && !e)
            e = pp::launch_sig_regroup(r->dev.sig[0], n, r->W, r->Wout, r->s, r->sg, r->dcur, r->dpos, r->g->node_graph,
                                       rows, r->stream);
        if (!rc && !e && r->g->perm_d) {
            uint64_t *by_id = dst_on_device ? dst : out;
            e = pp::launch_gather_rows(by_id, rows, r->g->perm_d, n, r->Wout, r->stream);
            rows = by_id;
        }
        if (!rc && !e && !dst_on_device)
            e = hipMemcpyAsync(dst, rows, sizeof(uint64_t) * (size_t)words, hipMemcpyDeviceToHost, r->stream);
        if (!rc && !e) e = hipStreamSynchronize(r->stream);
        if (rc || e) (void)hipStreamSynchronize(r->stream);   // queued work done before the blocks go back
        dev_free(tmp);
        dev_free(out);
        if (rc) return rc;
        if (e) return fail(PP_EDEVICE, "signature regroup: %s", hipGetErrorString(e));
        return PP_OK;
    }
    if (r->g->perm_d) {
        // stored order -> input order: assemble the rows, then gather them by id
        const int64_t words = r->g->n * r->W;
        uint64_t *tmp = nullptr, *out = nullptr;
        int rc = dev_alloc(&tmp, words);
        if (!rc && !dst_on_device) rc = dev_alloc(&out, words);
        if (!rc) rc = copy_signatures(r, tmp, hipMemcpyDeviceToDevice);
        hipError_t e = hipSuccess;
        if (!rc) e = pp::launch_gather_rows(dst_on_device ? dst : out, tmp, r->g->perm_d, r->g->n, r->W, r->stream);
        if (!rc && !e && !dst_on_device)
            e = hipMemcpyAsync(dst, out, sizeof(uint64_t) * (size_t)words, hipMemcpyDeviceToHost, r->stream);
        if (!rc && !e) e = hipStreamSynchronize(r->stream);
        if (rc || e) (void)hipStreamSynchronize(r->stream);   // queued work done before the blocks go back
        dev_free(tmp);
        dev_free(out);
        if (rc) return rc;
        if (e) return fail(PP_EDEVICE, "signature gather: %s", hipGetErrorString(e));
        return PP_OK;
    }
    int rc = copy_signatures(r, dst, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(r->stream));
    return PP_OK;
}

namespace {

// The current signature rows in stored order into dst (not synchronised).
int copy_signatures(pp_run r, uint64_t *dst, hipMemcpyKind kind) {
    if (r->cur.size() <= 1) {
        HIP_TRY(hipMemcpyAsync(dst, r->dev.sig[r->host_ctrl.cur & 1], sizeof(uint64_t) * (size_t)r->g->n * r->W, kind,
                               r->stream));
    } else {
        // clustered batch: each graph's rows sit in the buffer its own round count selects
        for (int k = 0; k < r->G; ++k) {
            const int64_t n0 = r->g->node_offsets[(size_t)k], n1 = r->g->node_offsets[(size_t)k + 1];
            if (n1 == n0) continue;
            HIP_TRY(hipMemcpyAsync(dst + n0 * r->W, r->dev.sig[r->cur[(size_t)k]] + n0 * r->W,
                                   sizeof(uint64_t) * (size_t)(n1 - n0) * r->W, kind, r->stream));
        }
    }
    return PP_OK;
}

}  // namespace

extern "C" int pp_get_seed_counts(pp_run r, uint32_t *dst, int32_t cap_rounds) {
    if (!r || !dst) return fail(PP_EINVAL, "run or dst is NULL");
    if (!r->dev.seed_counts) return fail(PP_ESTATE, "run was created without seed_counts");
    if (cap_rounds < 1) return fail(PP_EINVAL, "cap_rounds < 1");
    const int G = r->G, s = r->s, k = r->k, sg = r->sg;
    const int rows = std::min(cap_rounds, r->cap);
    // device layout [round][group][graph][sg]; the caller's seed i of graph g is
    // internal position pos[g s + i]: group pos / sg, column pos % sg
    std::vector<uint32_t> buf((size_t)rows * k * G * sg);
    std::vector<int32_t> pos((size_t)G * s);
    HIP_TRY(hipMemcpyAsync(buf.data(), r->dev.seed_counts, sizeof(uint32_t) * buf.size(), hipMemcpyDeviceToHost, r->stream));
    if (r->grouped)
        HIP_TRY(hipMemcpyAsync(pos.data(), r->dpos, sizeof(int32_t) * pos.size(), hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    if (!r->grouped)
        for (size_t j = 0; j < pos.size(); ++j) pos[j] = (int32_t)(j % (size_t)s);
    std::memset(dst, 0, sizeof(uint32_t) * (size_t)G * cap_rounds * s);
    for (int g = 0; g < G; ++g)
        for (int q = 0; q < rows; ++q) {
            uint32_t *o = dst + ((int64_t)g * cap_rounds + q) * s;
            for (int i = 0; i < s; ++i) {
                const int p = pos[(size_t)g * s + i], grp = p / sg;
                o[i] = buf[(((size_t)q * k + grp) * G + g) * sg + (p - grp * sg)];
            }
        }
    return PP_OK;
}

extern "C" int pp_get_group_log(pp_run r, int32_t group, int32_t *mode, int64_t *arcs, int32_t cap) {
    if (!r) return fail(PP_EINVAL, "run is NULL");
    if (group < 0 || group >= r->k) return fail(PP_EINVAL, "group %d outside [0, %d)", group, r->k);
    const int rows = std::min(cap, r->cap);
    if (rows < 1) return fail(PP_EINVAL, "cap < 1");
    const int64_t off = (int64_t)group * r->G * r->cap;   // group j's logs (row 0 of its graphs)
    if (mode)
        HIP_TRY(hipMemcpyAsync(mode, r->dev.mode_log + off, sizeof(int32_t) * rows, hipMemcpyDeviceToHost, r->stream));
    if (arcs)
        HIP_TRY(hipMemcpyAsync(arcs, r->dev.arcs_log + off, sizeof(int64_t) * rows, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return PP_OK;
}

extern "C" int pp_get_round_log(pp_run r, int32_t *mode, int64_t *arcs, int32_t cap) {
    if (!r) return fail(PP_EINVAL, "run is NULL");
    const int rows = std::min(cap, r->cap);
    if (rows < 1) return fail(PP_EINVAL, "cap < 1");
    int rc = pp_get_group_log(r, 0, mode, arcs, cap);
    if (rc || !arcs) return rc;
    std::vector<int64_t> more((size_t)rows);
    for (int j = 1; j < r->k; ++j) {
        if ((rc = pp_get_group_log(r, j, nullptr, more.data(), cap))) return rc;
        for (int q = 0; q < rows; ++q) arcs[q] += more[(size_t)q];
    }
    return PP_OK;
}

extern "C" int pp_run_snapshot(pp_run r, pp_run *copy) {
    if (!r || !copy) return fail(PP_EINVAL, "run or copy is NULL");
    pp::AllocStream as(r->stream);
    pp_run c = new (std::nothrow) pp_run_s();
    if (!c) return fail(PP_ENOMEM, "run handle");
    c->g = r->g;
    c->s = r->s;
    c->W = r->W;
    c->k = r->k;
    c->sg = r->sg;
    c->Wout = r->Wout;
    c->grouped = r->grouped;
    c->cap = r->cap;
    c->G = r->G;
    c->opt = r->opt;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return fail(PP_EDEVICE, "snapshot stream");
    }
    c->own_stream = true;
    pp::AllocStream copy_as(c->stream);   // the copy's blocks are used on its own stream
    TileSet *ts = run_tiles(r);
    c->pgrid = r->pgrid;
    c->clock_khz = r->clock_khz;
    c->clusters = r->clusters;
    if (r->pgrid) {
        if (dev_alloc(&c->dclusters, (int64_t)c->clusters.size()) != PP_OK ||
            hipMemcpy(c->dclusters, c->clusters.data(), sizeof(pp::Cluster) * c->clusters.size(),
                      hipMemcpyHostToDevice) != hipSuccess) {
            free_run(c);
            return fail(PP_ENOMEM, "snapshot clusters");
        }
    }
    int rc = alloc_run_dev(r->g, c->dev, r->s, r->k, r->sg, r->W, r->cap, r->dev.seed_counts != nullptr,
                           std::max(pp::pull_grid_for(ts->ntiles, r->W), r->pgrid));
    if (!rc && c->grouped && (rc = dev_alloc(&c->iseeds, (int64_t)c->G * c->s)) == PP_OK &&
        (rc = dev_alloc(&c->dpos, (int64_t)c->G * c->s)) == PP_OK)
        rc = dev_alloc(&c->dcur, c->k);
    if (!rc) rc = alloc_staging(c);
    if (rc) {
        free_run(c);
        return rc;
    }
    c->dev.sched = r->dev.sched;
    c->dev.push_div = r->dev.push_div;
    c->dev.pull_k = r->dev.pull_k;
    c->dev.sparse_pull = r->dev.sparse_pull;
    c->dev.fuzz_seed = r->dev.fuzz_seed;
    rc = pp_run_restore(c, r);
    if (rc) {
        free_run(c);
        return rc;
    }
    *copy = c;
    return PP_OK;
}

extern "C" int pp_run_restore(pp_run r, pp_run from) {
    if (!r || !from) return fail(PP_EINVAL, "run is NULL");
    if (r->g != from->g || r->s != from->s || r->cap != from->cap || r->k != from->k ||
        r->grouped != from->grouped || (r->dev.seed_counts == nullptr) != (from->dev.seed_counts == nullptr))
        return fail(PP_EINVAL, "runs differ in graph, s, seed groups, max_rounds or seed_counts");
    if (r == from) return PP_OK;
    if (from->stream != r->stream) HIP_TRY(hipStreamSynchronize(from->stream));
    const int64_t n = r->g->n, W = r->W, k = r->k, KG = (int64_t)r->k * r->G, cap = r->cap;
    hipStream_t st = r->stream;
    auto cp = [&](void *d, const void *s, size_t bytes) { return hipMemcpyAsync(d, s, bytes, hipMemcpyDeviceToDevice, st); };
    const RunDev &a = from->dev;
    RunDev &b = r->dev;
    // every group's arrays, each one allocation (pairs included)
    hipError_t e = cp(b.sig[0], a.sig[0], 8 * 2 * k * n * W);
    if (!e) e = cp(b.acc, a.acc, 8 * k * n * W);
    if (!e) e = cp(b.stamp, a.stamp, 4 * k * n);
    if (!e) e = cp(b.f_ids[0], a.f_ids[0], 4 * 2 * k * n);
    if (!e) e = cp(b.f_delta[0], a.f_delta[0], 8 * 2 * k * n * W);
    if (!e) e = cp(b.chunks[0], a.chunks[0], sizeof(Chunk) * 2 * k * chunk_capacity(r->g));
    if (!e) e = cp(b.counts, a.counts, 8 * cap * KG);
    if (!e && b.seed_counts) e = cp(b.seed_counts, a.seed_counts, 4 * cap * KG * r->sg);
    if (!e) e = cp(b.D, a.D, 4 * KG);
    if (!e) e = cp(b.gconv, a.gconv, 4 * KG);
    if (!e) e = cp(b.mode_log, a.mode_log, 4 * cap * KG);
    if (!e) e = cp(b.arcs_log, a.arcs_log, 8 * cap * KG);
    if (!e) e = cp(b.phase_log, a.phase_log, 8 * cap * 3 * KG);
    if (!e) e = cp(b.feat_log, a.feat_log, sizeof(float) * pp::MLP_IN * cap * KG);
    if (!e) e = cp(b.mlp, a.mlp, sizeof(float) * pp::MLP_PARAMS);
    if (!e) e = cp(b.plan, a.plan, sizeof(int32_t) * cap);
    if (!e) e = cp(b.tickets, a.tickets, sizeof(int32_t) * pp::TICKET_INTS * k);
    if (!e && b.node_acc && a.node_acc) e = cp(b.node_acc, a.node_acc, sizeof(int64_t) * n);
    if (!e) e = cp(b.ctrl, a.ctrl, sizeof(Ctrl) * KG);
    if (!e) e = cp(b.bar, a.bar, sizeof(pp::GridBar) * KG);
    if (!e && r->grouped) e = cp(r->iseeds, from->iseeds, sizeof(int32_t) * (size_t)r->G * r->s);
    if (!e && r->grouped) e = cp(r->dpos, from->dpos, sizeof(int32_t) * (size_t)r->G * r->s);
    if (!e) e = hipStreamSynchronize(st);
    if (e) {
        r->acc_clean = false;
        return fail(PP_EDEVICE, "restore: %s", hipGetErrorString(e));
    }
    r->host_ctrl = from->host_ctrl;
    r->cur = from->cur;
    r->staged = from->staged;
    r->counts_host = from->counts_host;
    r->D_host = from->D_host;
    r->acc_clean = from->acc_clean;
    r->seeds_kept = false;   // the restored rows' seeds are not in this run's list: the next reset clears all
    return PP_OK;
}

extern "C" int pp_get_node_stats(pp_run r, int32_t *reached, int64_t *dist_sum) {
    if (!r || !reached || !dist_sum) return fail(PP_EINVAL, "run, reached or dist_sum is NULL");
    if (!r->dev.node_acc) return fail(PP_ESTATE, "run created without node_stats");
    int rc = sync_ctrl(r);
    if (rc) return rc;
    // states accumulated: the initialisation and every round run
    const int64_t K = (int64_t)r->host_ctrl.round + (r->host_ctrl.converged ? 1 : 0);
    const int64_t n = r->g->n;
    int32_t *dr = nullptr;
    int64_t *dd = nullptr;
    if ((rc = dev_alloc(&dr, n)) || (rc = dev_alloc(&dd, n))) {
        dev_free(dr);
        return rc;
    }
    std::vector<int32_t> hr((size_t)n);
    std::vector<int64_t> hd((size_t)n);
    // the per-round engine (node_stats excludes the clustered one) keeps Sig in one buffer
    hipError_t e = pp::launch_node_stats(r->dev.sig[r->host_ctrl.cur & 1], r->dev.node_acc, n, r->W, K, dr, dd,
                                         r->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hr.data(), dr, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, r->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hd.data(), dd, sizeof(int64_t) * (size_t)n, hipMemcpyDeviceToHost, r->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) (void)hipStreamSynchronize(r->stream);
    dev_free(dr);
    dev_free(dd);
    if (e != hipSuccess) return fail(PP_EDEVICE, "node statistics: %s", hipGetErrorString(e));
    const std::vector<int32_t> &perm = r->g->perm;
    for (int64_t u = 0; u < n; ++u) {
        const size_t x = perm.empty() ? (size_t)u : (size_t)perm[(size_t)u];
        reached[u] = hr[x];
        dist_sum[u] = hd[x];
    }
    return PP_OK;
}

extern "C" int pp_get_kernel_times(pp_run r, float *pull_ms, int32_t cap) {
    if (!r || !pull_ms) return fail(PP_EINVAL, "run or pull_ms is NULL");
    if (!r->timing) return fail(PP_ESTATE, "run was created without time_kernels");
    for (int32_t k = 0; k < cap; ++k) pull_ms[k] = k < r->cap ? r->pull_ms[(size_t)k] : 0.0f;
    return PP_OK;
}

extern "C" int pp_run_set_mlp(pp_run r, const float *params) {
    if (!r) return fail(PP_EINVAL, "run is NULL");
    if (params) {
        HIP_TRY(hipMemcpyAsync(r->dev.mlp, params, sizeof(float) * pp::MLP_PARAMS, hipMemcpyHostToDevice, r->stream));
    } else {
        HIP_TRY(pp::launch_fill_i32((int32_t *)r->dev.mlp, kNaNBits, pp::MLP_PARAMS, r->stream));
    }
    // the next round's direction was taken with the old weights
    // live control blocks: one per graph (clustered engine), one per seed group otherwise
    if (params) HIP_TRY(pp::launch_redecide(r->dev, r->pgrid ? r->G : r->k, r->pgrid ? 1 : r->G, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return sync_ctrl(r);
}

extern "C" int pp_get_round_features(pp_run r, float *feat, int32_t cap) {
    if (!r || !feat) return fail(PP_EINVAL, "run or feat is NULL");
    const int rows = std::min(cap, r->cap);
    if (rows < 1) return fail(PP_EINVAL, "cap < 1");
    HIP_TRY(hipMemcpyAsync(feat, r->dev.feat_log, sizeof(float) * pp::MLP_IN * rows, hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return PP_OK;
}

extern "C" int pp_run_set_plan(pp_run r, const int32_t *plan, int32_t len) {
    if (!r) return fail(PP_EINVAL, "run is NULL");
    if (len < 0 || (len > 0 && !plan)) return fail(PP_EINVAL, "plan is NULL with len > 0");
    const int n = std::min(len, r->cap);
    HIP_TRY(pp::launch_fill_i32(r->dev.plan, -1, r->cap, r->stream));
    if (n > 0) HIP_TRY(hipMemcpyAsync(r->dev.plan, plan, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    return PP_OK;
}

extern "C" int pp_get_round_times(pp_run r, float *ms, int32_t cap) {
    if (!r || !ms) return fail(PP_EINVAL, "run or ms is NULL");
    if (cap < 1) return fail(PP_EINVAL, "cap < 1");
    if (r->pgrid) return fail(PP_ESTATE, "round times are kept by the per-round engine");
    const int rows = std::min(cap, r->cap);
    std::vector<int64_t> st((size_t)rows * 3);
    HIP_TRY(hipMemcpyAsync(st.data(), r->dev.phase_log, sizeof(int64_t) * st.size(), hipMemcpyDeviceToHost, r->stream));
    HIP_TRY(hipStreamSynchronize(r->stream));
    for (int q = 0; q < cap; ++q) {
        const int64_t a = q < rows ? st[(size_t)q * 3] : 0, b = q < rows ? st[(size_t)q * 3 + 2] : 0;
        ms[q] = (q >= 1 && a > 0 && b > a) ? (float)((double)(b - a) / r->clock_khz) : 0.0f;
    }
    return PP_OK;
}

extern "C" int pp_time_round(pp_run r, int32_t mode, float *features, float *ms) {
    if (!r || !ms) return fail(PP_EINVAL, "run or ms is NULL");
    if (mode != pp::MODE_PULL && mode != pp::MODE_PUSH && mode != pp::MODE_SPULL && mode != pp::MODE_PUSH_FLAT)
        return fail(PP_EINVAL, "mode %d is none of pull (0), push (1), sparse pull (3), flattened push (4)", mode);
    if (mode == pp::MODE_PUSH && r->dev.sparse_pull == 1) mode = pp::MODE_SPULL;   // the run's sparse direction
    if (r->pgrid) return fail(PP_ESTATE, "timing of single rounds needs the per-round engine");
    int rc = sync_ctrl(r);
    if (rc) return rc;
    if (r->host_ctrl.converged) return fail(PP_ESTATE, "run has converged");
    if (r->host_ctrl.round >= r->cap - 1) return fail(PP_ENOTCONV, "round log full (max_rounds)");
    if (features)
        for (int i = 0; i < pp::MLP_IN; ++i) features[i] = r->host_ctrl.feat[i];
    for (auto &e : r->tev)
        if (!e) HIP_TRY(hipEventCreate(&e));
    GraphDev gv = graph_view(r->g, run_tiles(r), r->W);
    // every direction is valid in every round: forcing one changes the work
    // done, never the result
    // every seed group's control block: the direction, and the frontier's
    // tiling (bit 0; a sparse pull keeps the fixed threshold's, bit 1)
    std::vector<int32_t> fw((size_t)r->k * 2);
    for (int j = 0; j < r->k; ++j) {
        const int32_t hf = (r->h_ctrl[(size_t)j * (r->k > 1 ? r->G : 1)].flat >> 1) & 1;
        const int32_t b0 = mode == pp::MODE_PUSH_FLAT ? 1 : (mode == pp::MODE_PUSH ? 0 : hf);
        fw[(size_t)2 * j] = mode == pp::MODE_PUSH_FLAT ? pp::MODE_PUSH : mode;
        fw[(size_t)2 * j + 1] = b0 | (hf << 1);
        HIP_TRY(hipMemcpyAsync(&r->dev.ctrl[(size_t)j * r->G].mode, &fw[(size_t)2 * j], sizeof(int32_t),
                               hipMemcpyHostToDevice, r->stream));
        HIP_TRY(hipMemcpyAsync(&r->dev.ctrl[(size_t)j * r->G].flat, &fw[(size_t)2 * j + 1], sizeof(int32_t),
                               hipMemcpyHostToDevice, r->stream));
    }
    HIP_TRY(hipEventRecord(r->tev[0], r->stream));
    // the sparse kernel of the forced direction (a pull round launches the run's own)
    const int kinds = (mode == pp::MODE_PUSH || mode == pp::MODE_PUSH_FLAT)
                          ? pp::SPARSE_PUSH
                          : (mode == pp::MODE_SPULL ? pp::SPARSE_PULL : pp::SPARSE_BY_RUN);
    HIP_TRY(noted(r, pp::launch_round(gv, r->dev, r->stream, nullptr, nullptr, kinds)));
    HIP_TRY(hipEventRecord(r->tev[1], r->stream));
    HIP_TRY(hipEventSynchronize(r->tev[1]));
    HIP_TRY(hipEventElapsedTime(ms, r->tev[0], r->tev[1]));
    return sync_ctrl(r);
}

extern "C" int pp_autotune(pp_graph g, const int32_t *seeds, int32_t s, const pp_options *base, int32_t reps,
                           pp_options *best, pp_tune_entry *table, int32_t cap, int32_t *ntried) {
    if (!g || !seeds || !best) return fail(PP_EINVAL, "graph, seeds or best is NULL");
    if (reps < 1) return fail(PP_EINVAL, "reps < 1");
    if (cap < 0 || (cap > 0 && !table)) return fail(PP_EINVAL, "table is NULL with cap > 0");
    int rc = check_host_seeds(g, seeds, s);
    if (rc) return rc;
    pp_options o0;
    pp_options_default(&o0);
    if (base) o0 = *base;
    o0.time_kernels = 0;
    // candidates: tile shape (arcs per lane, hence the high-degree threshold)
    // x push threshold on the per-round engine, the thresholds again with
    // sparse pulls, then the persistent engine
    std::vector<pp_options> cands;
    for (int k : {4, 2})
        for (int d : {8, 4, 16, 32}) {
            pp_options o = o0;
            o.persistent = 0;
            o.pull_k = k;
            o.push_div = d;
            o.sparse_pull = 0;
            cands.push_back(o);
        }
    for (int d : {8, 4, 16, 32}) {
        pp_options o = o0;
        o.persistent = 0;
        o.pull_k = 4;
        o.push_div = d;
        o.sparse_pull = 1;
        cands.push_back(o);
    }
    {
        pp_options o = o0;
        o.persistent = 1;
        o.pull_k = 4;
        o.push_div = 8;
        o.sparse_pull = 0;
        cands.push_back(o);
    }
    // Every candidate's run is created after the one before it was freed, and a
    // release of gigabytes with hipFree slows the next seconds of GPU work by a
    // few percent; one untimed run, created and freed first, puts the first
    // candidate in the same state as the others.
    {
        pp_run r = nullptr;
        if (pp_seeds_init(g, seeds, s, &cands[0], nullptr, &r) == PP_OK) {
            const int err = pp_propagate_until_converged(r, 0, nullptr, 0, nullptr);
            pp_run_free(r);
            if (err != PP_OK) return err;
        }
    }
    float best_ms = INFINITY;
    int tried = 0;
    for (const pp_options &o : cands) {
        pp_run r = nullptr;
        if (pp_seeds_init(g, seeds, s, &o, nullptr, &r) != PP_OK) continue;   // e.g. too many graphs to co-schedule
        float ms = INFINITY;
        int err = pp_propagate_until_converged(r, 0, nullptr, 0, nullptr);   // warm-up (graph capture)
        for (int k = 0; k < reps && err == PP_OK; ++k) {
            const auto t0 = std::chrono::steady_clock::now();
            err = pp_seeds_reset(r, seeds, 0);
            if (err == PP_OK) err = pp_propagate_until_converged(r, 0, nullptr, 0, nullptr);
            const auto t1 = std::chrono::steady_clock::now();
            ms = std::min(ms, (float)std::chrono::duration<double, std::milli>(t1 - t0).count());
        }
        pp_run_free(r);
        if (err != PP_OK) return err;
        if (tried < cap)
            table[tried] = pp_tune_entry{o.pull_k, o.push_div, o.rounds_per_sync, o.persistent, o.sparse_pull, ms};
        ++tried;
        if (ms < best_ms) {
            best_ms = ms;
            *best = o;
        }
    }
    if (ntried) *ntried = tried;
    if (tried == 0) return fail(PP_EDEVICE, "no candidate configuration could run");
    return PP_OK;
}

extern "C" int pp_exact_counts(pp_graph g, int32_t group, const pp_options *opt, int64_t *counts, int32_t cap_rounds,
                               int32_t *D) {
    if (!g || !counts) return fail(PP_EINVAL, "graph or counts is NULL");
    if (g->G != 1) return fail(PP_EINVAL, "one graph only (got a batch of %d)", g->G);
    if (group < 1 || group > 512) return fail(PP_EINVAL, "group = %d outside [1, 512]", group);
    if (cap_rounds < 1) return fail(PP_EINVAL, "cap_rounds < 1");
    const int64_t n = g->n;
    pp_options o;
    pp_options_default(&o);
    if (opt) o = *opt;
    o.seed_counts = 0;
    std::memset(counts, 0, sizeof(int64_t) * (size_t)cap_rounds);
    int32_t dmax = 0;
    std::vector<int32_t> seeds((size_t)group);
    std::vector<int64_t> c((size_t)cap_rounds);
    pp_run run = nullptr;     // runs of `group` seeds, reset per group
    int32_t run_s = 0;
    int rc = PP_OK;
    for (int64_t first = 0; first < n && rc == PP_OK; first += group) {
        const int32_t s = (int32_t)std::min<int64_t>(group, n - first);
        for (int32_t i = 0; i < s; ++i) seeds[(size_t)i] = (int32_t)(first + i);
        if (run && run_s != s) {
            pp_run_free(run);
            run = nullptr;
        }
        if (!run) {
            rc = pp_seeds_init(g, seeds.data(), s, &o, nullptr, &run);
            run_s = s;
        } else {
            rc = pp_seeds_reset(run, seeds.data(), 0);
        }
        int32_t d = 0;
        if (rc == PP_OK) rc = pp_propagate_until_converged(run, 0, c.data(), cap_rounds, &d);
        if (rc == PP_OK) {
            for (int32_t k = 0; k < cap_rounds; ++k) counts[k] += c[(size_t)k];
            dmax = std::max(dmax, d);
        }
    }
    if (run) pp_run_free(run);
    if (rc) return rc;
    if (D) *D = dmax;
    return dmax >= cap_rounds ? fail(PP_ERANGE, "D = %d does not fit cap_rounds = %d", dmax, cap_rounds) : PP_OK;
}

// Progressive sampling: groups of seeds from the pool until the average
// distance's Hoeffding half-width (sample D and alpha) meets the target.
extern "C" int pp_progressive_sample(pp_graph g, const int32_t *pool, int32_t pool_len, int32_t group, double target,
                                     double delta, const pp_options *opt, int64_t *counts, int32_t cap_rounds,
                                     pp_progress *out) {
    if (!g || !pool || !counts || !out) return fail(PP_EINVAL, "graph, pool, counts or out is NULL");
    if (g->G != 1) return fail(PP_EINVAL, "one graph only (got a batch of %d)", g->G);
    if (pool_len < 1) return fail(PP_EINVAL, "pool_len < 1");
    if (group < 1 || group > 512) return fail(PP_EINVAL, "group = %d outside [1, 512]", group);
    if (!(delta > 0.0 && delta < 1.0)) return fail(PP_EINVAL, "delta outside (0, 1)");
    if (!(target >= 0.0)) return fail(PP_EINVAL, "target < 0");
    if (cap_rounds < 1) return fail(PP_EINVAL, "cap_rounds < 1");
    int rc = check_host_seeds(g, pool, pool_len);
    if (rc) return rc;
    pp_options o;
    pp_options_default(&o);
    if (opt) o = *opt;
    o.seed_counts = 0;
    std::memset(counts, 0, sizeof(int64_t) * (size_t)cap_rounds);
    std::memset(out, 0, sizeof(*out));
    std::vector<int64_t> c((size_t)cap_rounds);
    pp_run run = nullptr;
    int32_t run_s = 0, used = 0, dmax = 0;
    while (used < pool_len) {
        const int32_t s = std::min(group, pool_len - used);
        if (run && run_s != s) {
            pp_run_free(run);
            run = nullptr;
        }
        if (!run) {
            rc = pp_seeds_init(g, pool + used, s, &o, nullptr, &run);
            run_s = s;
        } else {
            rc = pp_seeds_reset(run, pool + used, 0);
        }
        int32_t d = 0;
        if (rc == PP_OK) rc = pp_propagate_until_converged(run, 0, c.data(), cap_rounds, &d);
        if (rc) break;
        for (int32_t k = 0; k < cap_rounds; ++k) counts[k] += c[(size_t)k];
        dmax = std::max(dmax, d);
        used += s;
        out->groups += 1;
        if (dmax >= cap_rounds) break;
        pp_metrics m;
        if ((rc = pp_estimate_metrics(counts, dmax + 1, g->n, used, 9, 10, &m))) break;
        const double eps = std::sqrt(std::log(2.0 / delta) / (2.0 * (double)used));
        const double bound = dmax == 0 ? 0.0 : (m.alpha > 0.0 ? eps * (double)dmax / m.alpha : INFINITY);
        out->seeds = used;
        out->D = dmax;
        out->alpha = m.alpha;
        out->eps = eps;
        out->bound = bound;
        if (bound <= target) {
            out->met = 1;
            break;
        }
    }
    if (run) pp_run_free(run);
    if (rc) return rc;
    return dmax >= cap_rounds ? fail(PP_ERANGE, "D = %d does not fit cap_rounds = %d", dmax, cap_rounds) : PP_OK;
}

// PROPAGATE-S: batches of k seeds in flight, each run to its last seed's
// first pass without a find; the host checks every 8 passes.
namespace {

// One device region holds every buffer of a PROPAGATE-S call for k seeds in
// flight over ceil(n/64) words and a pass log of cap entries (each part
// 256-byte aligned): both signatures of every seed, per-seed pass counts,
// the pass log, per-seed arcs examined, states, last passes, the count of
// running seeds, and the device copy of the batch's seed ids.
int64_t seq_region_bytes(int64_t k, int64_t nw, int64_t cap) {
    auto up = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
    return up(16 * k * nw) + up(8 * k) + up(8 * cap) + up(8 * k) + up(4 * k) + up(4 * k) + up(4) + up(4 * k);
}

void seq_carve(void *base, int64_t k, int64_t nw, int64_t cap, pp::SeqDev &S, int32_t **dseeds) {
    auto up = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
    char *p = (char *)base;
    S.bits = (uint64_t *)p;
    p += up(16 * k * nw);
    S.pass_cnt = (int64_t *)p;
    p += up(8 * k);
    S.sum_cnt = (int64_t *)p;
    p += up(8 * cap);
    S.examined = (int64_t *)p;
    p += up(8 * k);
    S.done = (int32_t *)p;
    p += up(4 * k);
    S.dpass = (int32_t *)p;
    p += up(4 * k);
    S.active = (int32_t *)p;
    p += up(4);
    *dseeds = (int32_t *)p;
    S.k = (int32_t)k;
    S.nw = nw;
    S.cap = (int32_t)cap;
}

int check_seq_args(pp_graph g, const int32_t *seeds, int32_t s, int32_t concurrent, int64_t *counts, int32_t cap_rounds,
                   int32_t *D) {
    if (!g || !seeds || !counts || !D) return fail(PP_EINVAL, "graph, seeds, counts or D is NULL");
    if (g->G != 1) return fail(PP_EINVAL, "one graph only (got a batch of %d)", g->G);
    if (s < 1) return fail(PP_EINVAL, "s < 1");
    if (concurrent < 0) return fail(PP_EINVAL, "concurrent < 0");
    if (cap_rounds < 1) return fail(PP_EINVAL, "cap_rounds < 1");
    return check_host_seeds(g, seeds, s);
}

// The propagation over buffers laid out by seq_carve (S.k seeds in flight).
// Clears what must start at zero; leaves the stream synchronised.
int propagate_s_run(pp_graph g, const int32_t *seeds, int32_t s, const pp::SeqDev &S, int32_t *dseeds, hipStream_t st,
                    int64_t *counts, int32_t cap_rounds, int32_t *D, int64_t *examined) {
    const int k = S.k;
    const int64_t nw = S.nw, cap = cap_rounds;
    const int32_t *heavy = g->seq_heavy;
    const int64_t nheavy = g->nseq_heavy;
    std::memset(counts, 0, sizeof(int64_t) * (size_t)cap);
    counts[0] = s;
    int32_t dmax = 0;
    int64_t ex_total = 0;
    bool overflow = false;
    const GraphDev gv = graph_view(g, nullptr, 0);
    // about 256 Ki waves in all, at least one block per seed, at most one wave
    // per word (R-MAT 20, 256 seeds: 31.2 ms at 16 Ki waves, 28.7 at 64 Ki,
    // 27.3 at 256 Ki, 29.1 at 1 Mi)
    const int64_t want = (262144 / 4 + k - 1) / k, most = (nw + 3) / 4;
    const int bps = (int)std::max<int64_t>(1, std::min(want, most));
    const int bph = (int)std::max<int64_t>(1, std::min(want, (nheavy + 3) / 4));
    std::vector<int32_t> hs((size_t)k), hd((size_t)k), hdone((size_t)k);
    std::vector<int64_t> hc, hx((size_t)k);
    hipError_t e = hipSuccess;
    for (int first = 0; first < s && e == hipSuccess; first += k) {
        const int kk = std::min(k, s - first);
        for (int i = 0; i < kk; ++i) {
            const int32_t x = seeds[first + i];
            hs[(size_t)i] = g->perm.empty() ? x : g->perm[(size_t)x];
        }
        e = hipMemcpyAsync(dseeds, hs.data(), sizeof(int32_t) * (size_t)kk, hipMemcpyHostToDevice, st);
        int last = 0;   // passes launched
        // buffer 0 of every slot (as 4-byte words) and the pass log; pass 1 writes
        // every word of buffer 1 before anything reads it
        const pp::FillSeg segs[] = {{(uint32_t *)S.bits, 2 * k * nw, 0u}, {(uint32_t *)S.sum_cnt, 2 * cap, 0u}};
        if (e == hipSuccess) e = pp::launch_fills(segs, 2, st);
        if (e == hipSuccess) e = pp::launch_seq_seeds(S, dseeds, kk, st);
        for (int r = 1; r < cap_rounds && e == hipSuccess; ++r) {
            last = r;
            e = pp::launch_seq_pass(gv, S, heavy, nheavy, r, bps, bph, st);
            if (e == hipSuccess && (r % 8 == 0 || r == cap_rounds - 1)) {
                int32_t act = 0;
                e = hipMemcpyAsync(&act, S.active, sizeof(int32_t), hipMemcpyDeviceToHost, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (act == 0) break;
            }
        }
        hc.assign((size_t)last + 1, 0);
        if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), S.sum_cnt, sizeof(int64_t) * hc.size(), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(hx.data(), S.examined, sizeof(int64_t) * (size_t)kk, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(hd.data(), S.dpass, sizeof(int32_t) * (size_t)kk, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(hdone.data(), S.done, sizeof(int32_t) * (size_t)kk, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) break;
        for (int r = 1; r <= last; ++r) counts[r] += hc[(size_t)r];
        for (int j = 0; j < kk; ++j) {
            dmax = std::max(dmax, hd[(size_t)j]);
            ex_total += hx[(size_t)j];
            overflow |= hdone[(size_t)j] == 2;
        }
    }
    (void)hipStreamSynchronize(st);   // also after a failed launch: nothing queued still uses the buffers
    if (e != hipSuccess) return fail(PP_EDEVICE, "PROPAGATE-S: %s", hipGetErrorString(e));
    *D = dmax;
    if (examined) *examined = ex_total;
    if (overflow) return fail(PP_ENOTCONV, "a seed still found nodes at pass %d", cap_rounds - 1);
    return PP_OK;
}

}  // namespace

extern "C" int pp_propagate_s(pp_graph g, const int32_t *seeds, int32_t s, int32_t concurrent, void *stream,
                              int64_t *counts, int32_t cap_rounds, int32_t *D, int64_t *examined) {
    int rc = check_seq_args(g, seeds, s, concurrent, counts, cap_rounds, D);
    if (rc) return rc;
    // seeds in flight: one grid row each (at most 65535)
    const int64_t k = std::min({concurrent > 0 ? concurrent : 256, s, 65535});
    const int64_t nw = (g->n + 63) / 64;
    hipStream_t st = stream ? (hipStream_t)stream : g->stream;
    pp::AllocStream as(st);
    void *region = nullptr;
    const int64_t bytes = seq_region_bytes(k, nw, cap_rounds);
    if ((region = pp::dev_malloc((size_t)bytes)) == nullptr)
        return fail(PP_ENOMEM, "PROPAGATE-S: device buffers of %lld bytes", (long long)bytes);
    pp::SeqDev S{};
    int32_t *dseeds = nullptr;
    seq_carve(region, k, nw, cap_rounds, S, &dseeds);
    rc = propagate_s_run(g, seeds, s, S, dseeds, st, counts, cap_rounds, D, examined);
    pp::dev_release(region);   // propagate_s_run has synchronised the stream
    return rc;
}

extern "C" int pp_propagate_s_noalloc(pp_graph g, const int32_t *seeds, int32_t s, int32_t concurrent, void *stream,
                                      int64_t *counts, int32_t cap_rounds, int32_t *D, int64_t *examined) {
    int rc = check_seq_args(g, seeds, s, concurrent, counts, cap_rounds, D);
    if (rc) return rc;
    const int64_t nw = (g->n + 63) / 64;
    const int64_t most = PP_NOALLOC_BYTES;
    if (seq_region_bytes(1, nw, cap_rounds) > most)
        return fail(PP_EINVAL, "PROPAGATE-S without allocation: one seed over %lld nodes with a log of %d passes "
                               "needs %lld bytes, more than the fixed region's %lld",
                    (long long)g->n, cap_rounds, (long long)seq_region_bytes(1, nw, cap_rounds), (long long)most);
    int64_t k;
    if (concurrent > 0) {
        k = std::min<int64_t>({concurrent, s, 65535});
        if (seq_region_bytes(k, nw, cap_rounds) > most)
            return fail(PP_EINVAL, "PROPAGATE-S without allocation: %lld seeds in flight need %lld bytes, more than "
                                   "the fixed region's %lld",
                        (long long)k, (long long)seq_region_bytes(k, nw, cap_rounds), (long long)most);
    } else {
        // the most seeds in flight, up to min(s, 256), that the region holds
        int64_t lo = 1, hi = std::min<int64_t>(256, s);
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (seq_region_bytes(mid, nw, cap_rounds) <= most) lo = mid; else hi = mid - 1;
        }
        k = lo;
    }
    void *region = nullptr;
    if ((rc = pp::noalloc_region(&region)) != PP_OK) return rc;
    hipStream_t st = stream ? (hipStream_t)stream : g->stream;
    pp::SeqDev S{};
    int32_t *dseeds = nullptr;
    seq_carve(region, k, nw, cap_rounds, S, &dseeds);
    return propagate_s_run(g, seeds, s, S, dseeds, st, counts, cap_rounds, D, examined);
}
