// Internal declarations of the propagation library (not part of the C interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pp.h"

namespace pp {

// Round directions.  INIT marks the seed initialisation (round 0).  A sparse
// round runs either as a push (atomic ORs of the changed nodes' new bits into
// their predecessors) or as a sparse pull (the predecessors that can gain a
// bit gather their whole successor lists); both give the same bits.
// MODE_PUSH_FLAT is a push that walks its frontier as flattened arc ranges
// (the mode logs record it; the control block keeps MODE_PUSH and sets
// bit 0 of `flat`).
enum Mode : int32_t { MODE_PULL = 0, MODE_PUSH = 1, MODE_INIT = 2, MODE_SPULL = 3, MODE_PUSH_FLAT = 4 };

// A pull work unit: a run of consecutive nodes [u0, u1) whose successor
// lists occupy arcs [e0, e1) (at most the tile's arc budget), or one chunk of
// a high-degree node's list (hub >= 0: index into the hub table).
struct Tile {
    int32_t u0, u1;
    int64_t e0, e1;
    int32_t hub;      // -1 for a node run
    int32_t graph;    // graph of the batch the nodes belong to
};

// Push work unit for a frontier entry with many predecessors: arcs
// [off, off + chunk) of entry `entry`'s predecessor list, the chunk being
// four passes of a wave (256 / W arcs for W-word rows).
struct Chunk {
    int32_t entry;
    int32_t off;
};

constexpr int BLOCK = 256;       // threads per block of every bulk kernel
constexpr int TILE_NODES = 64;   // node budget of a pull tile (one wave)
constexpr int PUSH_SLOTS = 4;    // predecessor slots per entry in a small push
constexpr int PUSH_LIGHT = 16;   // entries with more predecessors go through chunks
// frontier entries from which a push walks flattened arc ranges and reads
// predecessor words before its atomics (below: latency-bound, direct slots)
constexpr int PUSH_FILTER_MIN = 16384;
constexpr int PUSH_CHUNK_MIN = 32;   // smallest chunk (W = 8)
// sparse pull: a candidate with at most this many successors gathers them
// itself; a longer list takes the new bits by atomic OR instead
constexpr int SPULL_LIGHT = 16;
#ifndef PP_PULL_GRID_MAX
#define PP_PULL_GRID_MAX 2048
#endif
constexpr int PULL_GRID_MAX = PP_PULL_GRID_MAX;

#ifndef PP_PULL_K
#define PP_PULL_K 4
#endif
#ifndef PP_PULL_K8
#define PP_PULL_K8 4
#endif
#ifndef PP_PULL_WAVES
#define PP_PULL_WAVES 4   // occupancy the pull kernel is compiled for (W <= 4)
#endif
#ifndef PP_PULL_SHORT_WAVES
#define PP_PULL_SHORT_WAVES 5   // the same for its short-list form (W <= 2)
#endif

// A pull tile is the work of one wave, per signature width W (words) and
// arcs per lane K (KK, or the default when KK = 0): the tile's arc budget
// (K per lane) and node budget (one row word per lane and pass).  In the gather, L lanes share each source row, each loading P
// words (16 bytes when W >= 2), and every group of L lanes takes KG = K L
// consecutive arcs.
template <int W, int KK = 0> struct PullShape {
    static constexpr int K = KK > 0 ? KK : (W >= 8 ? PP_PULL_K8 : PP_PULL_K);
    static constexpr int EDGES = K * 64;
    static constexpr int NODES = 64;
    static constexpr int L = W >= 2 ? W / 2 : 1;
    static constexpr int P = W / L;
    static constexpr int KG = K * L;
};

// Sizes of a frontier list, in one 8-byte word so that a block reserves both
// with one atomic (entries in the low half).
struct alignas(8) ListCounts {
    int32_t nodes;    // entries
    int32_t chunks;   // push chunks of its long predecessor lists
};

// Device control block: the round counter and everything the per-round
// kernels hand to each other.  Frontier list p holds the nodes that changed
// in a round of parity p.
struct Ctrl {
    int32_t round;        // round to run next (>= 1 after initialisation)
    int32_t converged;    // every graph has converged (or the log is full)
    int32_t mode;         // direction of the round about to run
    int32_t prev_mode;    // direction of the round before it
    int32_t cur;          // signature buffer holding Sig_{round-1}
    int32_t active;       // graphs not yet converged
    int32_t overflow;     // the round log is full
    int32_t bad_seed;     // a seed id outside its graph was seen (nothing written for it)
    ListCounts lst[2];    // entries and push chunks of frontier list p
    int64_t f_arcs[2];    // predecessor arcs of frontier list p (push work)
    int64_t hub_cnt;      // new bits found by the hub kernel this round
    int64_t hub_nodes;    // hubs that changed this round
    int64_t hub_arcs;     // their predecessor arcs
    int64_t reached;      // new bits of every round so far (R[r] - s)
    int64_t last_count;   // new bits of the last round
    float feat[8];        // scheduler features of the round about to run
    int32_t acc_pending;  // a round (or the initialisation) ran since the last per-node accumulation
    int32_t flat;         // bit 0: the sparse round about to run walks its frontier as flattened
                          // arc ranges (read before atomics) rather than direct slots per entry;
                          // bit 1: the fixed threshold's choice (frontier >= PUSH_FILTER_MIN)
};

static_assert(sizeof(Ctrl) % 4 == 0, "the control block is staged to the host as 32-bit words");

// Counters of the closing launch's two-level ticket: TICKET_GROUP group
// counters, each on its own 128-byte line, then the top counter (launches of
// at most TICKET_GROUP^2 blocks).
constexpr int TICKET_GROUP = 32;
constexpr int TICKET_STRIDE = 32;   // int32 per cache line
constexpr int TICKET_INTS = (TICKET_GROUP + 1) * TICKET_STRIDE;
constexpr int POST_MAX = 1024;      // blocks of the closing launch at most

// Learned cost model: an MLP 8 -> 32 -> 32 -> 4 (ReLU) predicting the log of a
// round's effective cost under each action: 0 dense pull, 1 push over direct
// slots per frontier entry, 2 push over flattened arc ranges, 3 sparse pull.
// Parameter layout (floats): W1[32][8], b1[32], W2[32][32], b2[32], W3[4][32],
// b3[4].
constexpr int MLP_IN = 8, MLP_HID = 32, MLP_OUT = 4;
constexpr int MLP_W1 = 0;
constexpr int MLP_B1 = MLP_W1 + MLP_HID * MLP_IN;
constexpr int MLP_W2 = MLP_B1 + MLP_HID;
constexpr int MLP_B2 = MLP_W2 + MLP_HID * MLP_HID;
constexpr int MLP_W3 = MLP_B2 + MLP_HID;
constexpr int MLP_B3 = MLP_W3 + MLP_OUT * MLP_HID;
constexpr int MLP_PARAMS = MLP_B3 + MLP_OUT;   // 1476
static_assert(MLP_PARAMS == PP_MLP_PARAMS, "cost-model layout");

// State of the grid barrier of the persistent round loop (zero at start).
struct GridBar {
    uint32_t grp[8];      // arrivals per block group
    uint32_t top;         // groups complete
    uint32_t gen;         // barrier generation
    int32_t abort;        // a wait timed out: every block leaves
    uint32_t pad[5];
};

// One graph of a batch as run by the clustered persistent engine: the
// graph's node range, tiles, hubs and push-chunk region, and the range of
// co-resident blocks [b0, b0 + nb) that runs it.
struct Cluster {
    int32_t g;            // graph index
    int32_t b0, nb;       // first block, blocks
    int32_t t0, t1;       // pull tiles
    int32_t h0, h1;       // high-degree nodes
    int32_t pad;
    int64_t n0, n1;       // nodes
    int64_t m;            // stored arcs (scheduler)
    int64_t ch0;          // first push-chunk slot
};

struct GraphDev {
    int64_t n0;               // first node of the view (0 for a whole graph)
    int64_t n, m;             // end of the node range, stored arcs
    const int64_t *rp;        // successor offsets [n+1] (pull)
    const int32_t *col;       // successors [m]
    const int64_t *trp;       // predecessor offsets [n+1] (push)
    const int32_t *tcol;      // predecessors [m]
    const Tile *tiles;
    int32_t ntiles;
    int32_t nhubs;
    const int32_t *hub_node;     // [nhubs]
    const int32_t *node_graph;   // [n], NULL for a single graph
    const int64_t *node_off;     // [G+1] node range of each graph
    int32_t G;
    int32_t pull_grid;           // blocks of the pull launch (= per-block partial slots)
    int32_t short_lists;         // no high-degree chunks and every node at most PULL_NPL
                                 // successors: the pull launches its short-list form
    int32_t skip_dead;           // the pull leaves the rows of nodes without successors
                                 // alone (many such nodes, rows beyond the caches)
};

// A pull tile whose nodes have at most PULL_NPL successors each gathers with
// one lane per node (rows of one or two words).
constexpr int PULL_NPL = 6;

// A run's device state.  Its seeds may be split into seed groups, each with
// its own signature rows (W words), frontier, counters and control block:
// every per-group array holds the groups one after another, and the kernels
// of a launch take group blockIdx.y (group_view).  The fields below describe
// group 0 until a kernel takes its group's view.
struct RunDev {
    int32_t s, W, cap, G; // seeds of the group, words per row, round-log capacity, graphs
    int32_t cstride;      // distance between rounds in counts (groups * graphs)
    int32_t sstride;      // distance between rounds in seed_counts (groups * graphs * sg)
    int32_t ngroups;      // seed groups
    int32_t sg;           // seeds per group (the last one may hold fewer: s_last)
    int32_t s_last;       // seeds of the last group
    int32_t s_all;        // seeds per graph (distance between graphs in a seed list)
    int64_t nn;           // nodes of the graph (size of the per-node arrays of one group)
    int64_t cc;           // push-chunk slots per frontier list of one group
    int32_t pgrid;        // per-block partial slots of one group
    int32_t pad_run;
    uint64_t *sig[2];     // [n][W] each: Sig_{r-1} in sig[cur], the pull writes the other
    uint64_t *acc;        // [n][W] push / hub accumulator, zero between rounds
    int32_t *stamp;       // [n] last round the node was queued
    int32_t *f_ids[2];    // frontier node ids
    uint64_t *f_delta[2]; // frontier delta words [entries][W]
    Chunk *chunks[2];
    int64_t *blk_cnt;     // [pull_grid] per-block new bits of a pull round
    int64_t *blk_nodes;   // [pull_grid] changed nodes
    int64_t *blk_arcs;    // [pull_grid] predecessor arcs of changed nodes
    int64_t *blk_pulled;  // [pull_grid] arcs gathered
    int64_t *counts;      // [cap][groups][G]
    uint32_t *seed_counts;// [cap][groups][G][sg] or NULL
    int32_t *D;           // [G]
    int32_t *gconv;       // [G]
    int32_t *mode_log;    // [G][cap] (row 0 when the graphs run as one union)
    int64_t *arcs_log;    // [G][cap]
    int64_t *phase_log;   // [G][cap][3] device-clock stamps of each round: start, after the main
                          // phase (persistent loop), end
    float *feat_log;      // [G][cap][8] scheduler features of each round (row 0 unused)
    int32_t *tickets;     // [TICKET_INTS] the closing launch's ticket counters (zero between launches)
    int64_t *post_part;   // [3][POST_MAX] the closing launch's per-block partials
    GridBar *bar;         // [G] barrier state per cluster
    Ctrl *ctrl;           // [G]: ctrl[0] for the per-round engine, one per graph when clustered
    // scheduler
    int32_t sched;
    int32_t push_div;
    int32_t pull_k;       // arcs per lane of the pull (the tile set was built for it)
    int32_t sparse_pull;  // sparse rounds: 0 push, 1 sparse pull, 2 either (pseudo-random per round)
    uint64_t fuzz_seed;
    float *mlp;           // [MLP_PARAMS] cost-model weights (NaN: not set, heuristic decides)
    int32_t *plan;        // [cap] action of each round for PP_SCHED_PLAN (-1: the heuristic's)
    int64_t *node_acc;    // [n] per-node sums of popcount(Sig_r(u)) over the states so far, or NULL
};

// Records the message returned by pp_last_error and returns `code`.
int set_error(int code, const char *fmt, ...);

// Device memory for everything the library allocates: through the caller's
// allocator when one is set (pp_set_allocator), else hipMalloc / hipFree.
// dev_malloc returns nullptr on failure; dev_release returns a block to the
// allocator that gave it, after the device has finished with it.
void *dev_malloc(size_t bytes);
void dev_release(void *p);
// The stream handed to the caller's allocator for this thread's allocations
// while the guard lives (the stream of the graph or run being built).
struct AllocStream {
    void *prev;
    explicit AllocStream(void *stream);
    ~AllocStream();
};

// Launchers (pp_kernels.hip).  All enqueue on `st` and return the launch status.
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t st);
// Re-takes the pending direction of nctrl control blocks, `stride` apart,
// with the run's current cost-model weights (PP_SCHED_MLP runs only).
hipError_t launch_redecide(const RunDev &r, int nctrl, int stride, hipStream_t st);
// A fill of n 4-byte words at p (16-byte aligned) with the value v.
struct FillSeg {
    uint32_t *p;
    int64_t n;
    uint32_t v;
};
// Every segment in as few launches as possible (one for up to 16 segments).
hipError_t launch_fills(const FillSeg *segs, int nseg, hipStream_t st);
// One seed group's rows and stamps back to the initial state when only its
// seeds' rows can hold bits: ids [count] stored ids, sig the group's two
// buffers (n rows of W words each, one after the other), stamp its n stamps.
hipError_t launch_clear_seed_rows(const int32_t *ids, int count, int64_t n, int W, uint64_t *sig, int32_t *stamp,
                                  hipStream_t st);
// out[j] = perm[in[j]] (ids outside [0, n) become -1).
hipError_t launch_map_ids(int32_t *out, const int32_t *in, const int32_t *perm, int64_t count, int64_t n,
                          hipStream_t st);
// dst row x = src row perm[x], rows of W words.
// PROPAGATE-S state for k seeds side by side (see pp_seq.hip).
struct SeqDev {
    uint64_t *bits;       // [2][k][nw] signatures, one bit per node
    int64_t *pass_cnt;    // [k] nodes found by the current pass (cleared by its end)
    int64_t *sum_cnt;     // [cap] nodes found at each pass, summed over the seeds
    int64_t *examined;    // [k] arcs examined
    int32_t *done;        // [k] 0 running, 1 done, 2 stopped at the end of the log
    int32_t *dpass;       // [k] last pass that found a node
    int32_t *active;      // [1] seeds still running
    int32_t k, cap;
    int64_t nw;           // 64-bit words per signature
};
hipError_t launch_seq_seeds(const SeqDev &S, const int32_t *seeds, int kk, hipStream_t st);
// The current device's address of the fixed PP_NOALLOC_BYTES region that
// pp_propagate_s_noalloc carves its buffers from (looked up once per device).
int noalloc_region(void **out);
// Nodes with more successors than this go to the wave-per-node launch.
constexpr int SEQ_LIGHT = 32;
// Pass r (short lists, then heavy[0..nheavy)) and its per-seed end.
hipError_t launch_seq_pass(const GraphDev &g, const SeqDev &S, const int32_t *heavy, int64_t nheavy, int r,
                           int blocks_per_seed, int heavy_blocks_per_seed, hipStream_t st);

// Per-node statistics: reached[u] = popcount of u's row of sig, dist_sum[u]
// = K reached[u] - acc[u] (K states accumulated).
hipError_t launch_node_stats(const uint64_t *sig, const int64_t *acc, int64_t n, int W, int64_t K, int32_t *reached,
                             int64_t *dist_sum, hipStream_t st);

hipError_t launch_stage(const void *ctrl, int64_t ctrl_bytes, const int32_t *D, int64_t nD, const int64_t *rows,
                        int64_t nrows, void *h_ctrl, int32_t *h_D, int64_t *h_rows, hipStream_t st);
hipError_t launch_gather_rows(uint64_t *dst, const uint64_t *src, const int32_t *perm, int64_t n, int W,
                              hipStream_t st);
// The internal seed list of a run with seed groups or a seed order (one block
// per graph): out = the stored ids in internal order, pos[i] = the internal
// position of the caller's seed i (see k_seed_order).
hipError_t launch_seed_order(const GraphDev &g, const int32_t *seeds, const int32_t *map, int G, int s_all,
                             int by_reach, int32_t *out, int32_t *pos, hipStream_t st);
// Rows of a grouped run's signatures in the caller's bit order (stored node order).
hipError_t launch_sig_regroup(const uint64_t *sig, int64_t n, int Wg, int Wout, int s_all, int sg, const int32_t *cur,
                              const int32_t *pos, const int32_t *node_graph, uint64_t *out, hipStream_t st);
// seeds: device-readable ids; map (may be NULL): input id -> stored id.
hipError_t launch_seed_init(const GraphDev &g, const RunDev &r, const int32_t *seeds, const int32_t *map,
                            hipStream_t st);
// Sparse-round kernels a round launches: the push's, the sparse pull's, or
// both (SPARSE_BY_RUN: as the run's sparse_pull option asks).
enum SparseKinds : int { SPARSE_BY_RUN = 0, SPARSE_PUSH = 1, SPARSE_PULL = 2, SPARSE_BOTH = 3 };
// One round; when e0/e1 are given they are recorded around the pull launch.
hipError_t launch_round(const GraphDev &g, const RunDev &r, hipStream_t st, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr, int kinds = SPARSE_BY_RUN);
// Rounds up to max_round of every graph in one cooperative launch of `grid`
// blocks split into clusters (device array), initialising graphs at round 0.
hipError_t launch_batch_persistent(const GraphDev &g, const RunDev &r, const Cluster *clusters, int nclusters,
                                   int grid, int max_round, hipStream_t st);
// Seed bits of the clustered engine (per-graph list regions and control blocks).
hipError_t launch_seed_scatter_batch(const GraphDev &g, const RunDev &r, const int32_t *seeds, hipStream_t st);
// Largest co-resident grid for the persistent loop at width W.
int persistent_grid(int W);
int pull_grid_for(int32_t ntiles, int W);

}  // namespace pp
