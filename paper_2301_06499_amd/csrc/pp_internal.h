// Internal declarations of the propagation library (not part of the C interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "pp.h"

namespace pp {

// Round directions.  INIT is the seed-initialisation commit (round 0).
enum Mode : int32_t { MODE_PULL = 0, MODE_PUSH = 1, MODE_INIT = 2 };

// A pull work unit: a run of consecutive nodes [u0, u1) whose successor
// lists occupy arcs [e0, e1) (at most the tile's arc budget), or one chunk of
// a high-degree node's list (hub >= 0: index into the hub tables).
struct Tile {
    int32_t u0, u1;
    int64_t e0, e1;
    int32_t hub;      // -1 for a node run
    int32_t graph;    // graph of the batch the nodes belong to
};

// Push work unit: arcs [off, off + PUSH_CHUNK) of frontier entry `entry`'s
// predecessor list.
struct Chunk {
    int32_t entry;
    int32_t off;
};

constexpr int PUSH_CHUNK = 16;   // predecessor arcs per push chunk
constexpr int BLOCK = 256;       // threads per block of every bulk kernel
constexpr int TILE_NODES = 256;  // node budget of a pull tile

// Edges per thread in the pull gather, per signature width W (words).
template <int W> struct PullShape {
    static constexpr int K = W >= 8 ? 4 : 8;
    static constexpr int EDGES = K * BLOCK;   // arc budget of a pull tile
};

// Device control block: the round counter and everything the per-round
// kernels hand to each other.  List p = round parity.
struct Ctrl {
    int32_t round;        // round to run next (>= 1 after initialisation)
    int32_t converged;    // every graph has converged (or the log is full)
    int32_t mode;         // direction of the round about to run
    int32_t active;       // graphs not yet converged
    int32_t overflow;     // the round log is full
    int32_t pad0;
    int32_t f_count[2];   // entries in frontier list p
    int32_t ch_count[2];  // push chunks built from frontier list p
    int64_t f_arcs[2];    // predecessor arcs of frontier list p (push work)
    int64_t pull_arcs;    // arcs gathered by the last pull round
    int64_t pad1;
};

struct GraphDev {
    int64_t n, m;
    const int64_t *rp;        // successor offsets [n+1] (pull)
    const int32_t *col;       // successors [m]
    const int64_t *trp;       // predecessor offsets [n+1] (push)
    const int32_t *tcol;      // predecessors [m]
    const Tile *tiles;
    int32_t ntiles;
    int32_t nhubs;
    const int32_t *hub_nchunks;
    const int32_t *node_graph;   // [n], NULL for a single graph
    int32_t G;
    int32_t pad;
};

struct RunDev {
    int32_t s, W, cap, G;
    uint64_t *sig;        // [n][W]
    uint64_t *acc;        // [n][W] push accumulator, zero between rounds
    int32_t *stamp;       // [n] last round the node was queued
    int32_t *f_ids[2];    // frontier node ids
    uint64_t *f_delta[2]; // frontier delta words [entries][W]
    Chunk *chunks[2];
    uint64_t *hub_acc;    // [nhubs][W]
    uint32_t *hub_done;   // [nhubs]
    int64_t *counts;      // [cap][G]
    uint32_t *seed_counts;// [cap][G][s] or NULL
    int32_t *D;           // [G]
    int32_t *gconv;       // [G]
    int32_t *mode_log;    // [cap]
    int64_t *arcs_log;    // [cap]
    Ctrl *ctrl;
    // scheduler
    int32_t sched;
    int32_t push_div;
    uint64_t fuzz_seed;
    const float *mlp;     // cost-model weights or NULL
};

// Launchers (pp_kernels.hip).  All enqueue on `st` and return the launch status.
hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t count, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t st);
hipError_t launch_seed_init(const GraphDev &g, const RunDev &r, const int32_t *seeds_dev, hipStream_t st);
hipError_t launch_round(const GraphDev &g, const RunDev &r, hipStream_t st);
int pull_grid(const GraphDev &g);

}  // namespace pp
