/*
 * pp.h -- C interface of the MI355X (gfx950) seed-bitset propagation library.
 *
 * The library computes PROPAGATE-P (Amati et al., "PROPAGATE: a seed
 * propagation framework to compute distance-based metrics on very large
 * graphs", Section 4, Algorithm 1): every node u keeps an s-bit signature
 * Sig(u), bit i set when u can reach seed x_i within the rounds run so far.
 * One synchronous round computes, for every u,
 *     Sig_r(u) = Sig_{r-1}(u)  OR  OR_{u -> v} Sig_{r-1}(v)
 * (the ball recurrence of Section 4, with u's own ball kept as Algorithm 1
 * does), and counts the newly set bits c[r] = sum_u popcount(Sig_r(u) XOR
 * Sig_{r-1}(u)) -- the number of (node, seed) pairs at distance exactly r.
 * The loop stops at the first round that sets no bit.  The metrics of the
 * paper's Section 3 are then estimated from c[0..D].  The library also runs
 * PROPAGATE-S (Algorithm 2: the seeds one at a time, one bit per node),
 * the exact neighbourhood function (every node a seed) and progressive
 * sampling with a Hoeffding stopping rule (Section 4, error bounds).
 *
 * Conventions shared by every entry point
 *   - Every function returns a pp_status (0 = success, < 0 = error); none
 *     throws or aborts.  pp_last_error() gives a message for the calling
 *     thread's last failure.
 *   - Node ids are int32 in [0, n).  Signature bit i (seed i) is word i >> 6,
 *     bit i & 63 of the node's row; rows are W uint64 words, W the smallest
 *     power of two >= ceil(s / 64) (pp_run_words), stored node-major
 *     ([n][W]).  Bits >= s stay zero.
 *   - Round numbering: c[0] = s counts the seeds' own pairs; round r >= 1
 *     adds the pairs at distance exactly r.  D is the last round with
 *     c[D] > 0 (the diameter lower bound); D + 1 rounds run, the last one
 *     finding no new bit.
 *   - Device work is ordered on the HIP stream given at handle creation
 *     (NULL = the library makes its own non-blocking stream).  Calls that
 *     write host memory synchronise that stream before returning.
 *   - Arguments are validated before any device work; a failed validation
 *     leaves the handles unchanged.
 *   - Handles are not thread-safe: use one thread per handle at a time.
 *   - Device memory is owned by the handles and released by the *_free calls;
 *     it comes from hipMalloc, or from the caller's allocator when one is set
 *     (pp_set_allocator).
 */
#ifndef PP_H
#define PP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PP_OK = 0,
    PP_EINVAL = -1,     /* malformed argument (sizes, flags, s out of range, NULL) */
    PP_ERANGE = -2,     /* a node id outside [0, n) or outside its graph */
    PP_ENOMEM = -3,     /* device or host allocation failed */
    PP_EDEVICE = -4,    /* a HIP runtime call failed */
    PP_ENOTCONV = -5,   /* the round cap was reached before convergence */
    PP_ESTATE = -6      /* call not valid in the handle's current state */
} pp_status;

typedef struct pp_graph_s *pp_graph;   /* device CSR + predecessor lists + tiling */
typedef struct pp_run_s *pp_run;       /* signatures, frontier, per-round logs */

/* pp_csr_build flags */
enum {
    PP_UNDIRECTED = 1,       /* each input pair (a, b) stands for arcs a->b and b->a */
    PP_INPUT_ON_DEVICE = 2,  /* src/dst point to device memory */
    PP_TRANSPOSE = 4,        /* propagate along reversed arcs: bit i reaches u when
                                x_i can reach u (instead of u reaching x_i) */
    PP_KEEP_ORDER = 8,       /* store the nodes in input order (by default, per
                                graph, the nodes with the most predecessors are
                                stored first, or, in a graph without such nodes,
                                the nodes are numbered in breadth-first order;
                                either only changes the layout: every result is
                                reported by input node id) */
    PP_BUILD_ON_HOST = 16,   /* sort the arcs on host threads (the default below
                                PP_DEVICE_BUILD_MIN input pairs) */
    PP_BUILD_ON_DEVICE = 32, /* sort the arcs on the device (the default from
                                PP_DEVICE_BUILD_MIN input pairs on); both builds
                                give the same arrays */
    PP_HUBS_ONLY = 64        /* store the high-degree nodes first but leave the
                                others in input order, without the breadth-first
                                numbering: a faster build of a large graph (one
                                host search over every arc) for one that is
                                propagated a few times only */
};
#define PP_DEVICE_BUILD_MIN (1 << 20)

/* per-round direction policy */
enum {
    PP_SCHED_HEURISTIC = 0,  /* fixed-threshold push/pull switch on frontier arcs */
    PP_SCHED_PULL = 1,       /* every round a dense pull over all arcs */
    PP_SCHED_PUSH = 2,       /* every round a push from the changed nodes */
    PP_SCHED_FUZZ = 3,       /* pseudo-random choice per round (testing: outputs must not change) */
    PP_SCHED_MLP = 4,        /* learned cost model, heuristic fallback */
    PP_SCHED_PLAN = 5        /* a given action per round (pp_run_set_plan), heuristic elsewhere */
};

/* Options of a run.  Zero-initialise and set what you need; pp_options_default
 * fills the defaults. */
typedef struct {
    int32_t scheduler;          /* PP_SCHED_* */
    int32_t seed_counts;        /* 1: also record per-seed counts c_i[r] */
    int32_t max_rounds;         /* capacity of the per-round logs (0: n + 1, at most 1<<20) */
    int32_t rounds_per_sync;    /* rounds launched between host convergence checks (0: adaptive:
                                   8, then the rounds run so far, at most 64) */
    int32_t use_graph;          /* 1: replay the round batch as a captured hipGraph */
    int32_t push_div;           /* heuristic: push while frontier arcs * push_div < arcs (0: 8) */
    uint64_t fuzz_seed;         /* PP_SCHED_FUZZ stream */
    int32_t time_kernels;       /* 1: HIP events around every pull launch (pp_get_kernel_times) */
    int32_t persistent;         /* 1: all rounds in one cooperative launch (grid barriers
                                   between phases) instead of launches per round */
    int32_t pull_k;             /* arcs per lane of the pull, 2 or 4 (0: 4); sets the pull
                                   tile (64 K arcs) and so the high-degree threshold
                                   (longer lists are split into tile-sized chunks).
                                   The persistent engine uses 4. */
    int32_t node_stats;         /* 1: per-node reach and distance sums (pp_get_node_stats);
                                   the per-round engine only */
    int32_t sparse_pull;        /* how a round the scheduler makes sparse runs: 0 a push
                                   (atomic OR of the changed nodes' new bits into their
                                   predecessors); 1 a sparse pull (each predecessor that
                                   can gain a bit ORs its whole successor list, as in
                                   Algorithm 1's inner loop, restricted to those nodes);
                                   2 either, by a pseudo-random bit per round from
                                   fuzz_seed (testing).  Same bits every way.  The
                                   per-round engine only */
    int32_t seed_groups;        /* seed groups of the run (the per-round engine): the seeds
                                   of each graph are split, in order, into groups of
                                   sg = ceil(s / seed_groups) (the last may hold fewer);
                                   each group is propagated with rows of its own width
                                   (the smallest power of two >= ceil(sg / 64) words, at
                                   most 8), its own direction per round, counts and
                                   convergence, all groups in the same launches.  Outputs
                                   are the same as one group's, in the caller's bit order.
                                   0: ceil(s / 512) groups (one when s <= 512);
                                   PP_GROUPS_BY_REACH: seed_order 1 and groups sized so
                                   that the initialisation's seeds with a predecessor fill
                                   whole groups first (a group of seeds with none
                                   converges after one round) */
    int32_t seed_order;         /* order of the seeds across the groups: 0 as given;
                                   1 (PP_ORDER_BY_REACH) the seeds whose node has a
                                   predecessor first -- a seed without one reaches no
                                   other node -- each part in the caller's order.
                                   Applied at every initialisation and reset */
} pp_options;

#define PP_GROUPS_BY_REACH (-1)
#define PP_ORDER_BY_REACH 1

/* Metrics estimated from c[0..D] (paper Section 3 and Algorithm 1's closing
 * steps).  T = c[0] + ... + c[D] counts (node, seed) pairs within reach,
 * seeds' own pairs included; every value is computed from exact integers
 * with one final rounding per operand, in the order documented at
 * pp_estimate_metrics. */
typedef struct {
    int32_t diameter;           /* D, the diameter lower bound */
    int32_t rounds_executed;    /* D + 1 */
    int64_t R_final;            /* T */
    double eff_diam;            /* least k with tau_den * R[k] >= tau_num * T */
    double eff_diam_interp;     /* linear interpolation of the crossing between k-1 and k */
    double avg_dist;            /* sum_r r c[r] / (T - s): pairs u != v */
    double avg_dist_paper;      /* sum_r r c[r] / T: self-pairs in the denominator */
    double reachable_pairs;     /* n * T / s, self-pairs included */
    double alpha;               /* (T - s) / (s (n - 1)); 0 when n = 1 */
} pp_metrics;

/* Fills *opt with the defaults (heuristic scheduler, no per-seed counts,
 * adaptive sync, graph replay on). */
void pp_options_default(pp_options *opt);

/*
 * pp_set_allocator -- device memory from the caller (for instance a caching
 * allocator that owns the process's GPU memory) for every block the library
 * allocates from now on: graphs, runs, snapshots and the temporaries of
 * single calls.
 *   alloc(bytes, stream, ctx)   returns device memory of at least `bytes`
 *               bytes, 256-byte aligned, or NULL (the calling entry point
 *               then returns PP_ENOMEM; so does a block off that alignment,
 *               which is handed back first).  stream is the hipStream_t the
 *               library's work on the block is ordered on: the run's stream
 *               for a run's blocks (the one the run creates when the caller
 *               gave none), the call's stream for the temporaries of a call,
 *               the build's stream for a graph (NULL: the legacy default).
 *   release(ptr, stream, ctx)   takes a block back, with the stream it was
 *               allocated for.  Stream-ordered: the library hands a block
 *               back only after waiting for its own streams that used it
 *               (it never waits for the whole device), so the allocator may
 *               give the block out again at once.
 *   ctx         passed to both unchanged.
 * A block always goes back to the allocator that gave it, also after a later
 * call changes or clears the allocator, so both functions must stay callable
 * until every graph and run made under them is freed.  alloc = release = NULL
 * restores hipMalloc / hipFree.  The setting is process-wide: change it while
 * no other thread is inside the library.  Pinned host staging still comes from
 * hipHostMalloc.  PP_EINVAL if exactly one of alloc and release is NULL.
 */
int pp_set_allocator(void *(*alloc)(size_t bytes, void *stream, void *ctx),
                     void (*release)(void *ptr, void *stream, void *ctx), void *ctx);

/*
 * pp_csr_build -- the graph G = (V, E) of Algorithm 1's input.
 *   n, m        nodes and input pairs (m >= 0, 1 <= n < 2^31).
 *   src, dst    m node ids each: pair k is the arc src[k] -> dst[k] (both
 *               directions with PP_UNDIRECTED).  Host memory unless
 *               PP_INPUT_ON_DEVICE; the caller keeps ownership.
 *   flags       PP_UNDIRECTED | PP_INPUT_ON_DEVICE | PP_TRANSPOSE | PP_KEEP_ORDER,
 *               and at most one of PP_BUILD_ON_HOST, PP_BUILD_ON_DEVICE.
 *   node_offsets, num_graphs
 *               a batch of num_graphs disjoint graphs: graph g owns node ids
 *               [node_offsets[g], node_offsets[g+1]) (host array of
 *               num_graphs + 1 entries, node_offsets[0] = 0,
 *               node_offsets[num_graphs] = n, non-decreasing).  NULL with
 *               num_graphs <= 1 means one graph.  An arc joining two graphs
 *               is PP_ERANGE.
 *   stream      hipStream_t the build is ordered on (NULL: legacy default).
 * Self-loops and repeated arcs are removed (they cannot change a bit); the
 * stored arc count is pp_graph_arcs().  The device build radix-sorts packed
 * (row, column) keys on `stream` and needs about 24 bytes per input pair
 * (48 with PP_UNDIRECTED) of device memory while it runs; device-resident
 * input then never goes through the host.  Errors: PP_EINVAL, PP_ERANGE,
 * PP_ENOMEM, PP_EDEVICE; *out is written only on success.
 */
int pp_csr_build(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, uint32_t flags,
                 const int64_t *node_offsets, int32_t num_graphs, void *stream, pp_graph *out);

/* Stored arcs (after dedup, both directions for undirected input) and nodes. */
int64_t pp_graph_arcs(pp_graph g);
/*
 * pp_graph_get_csr -- the stored adjacency, for inspection: rp [n+1] (int64
 * offsets) and col [m] of the successor rows, trp [n+1] and tcol [m] of the
 * predecessor rows, all in storage order, and perm [n] (the stored id of
 * each input node; the identity when the order was kept).  Host arrays, each
 * may be NULL; m = pp_graph_arcs(g).  Synchronous.
 */
int pp_graph_get_csr(pp_graph g, int64_t *rp, int32_t *col, int64_t *trp, int32_t *tcol, int32_t *perm);
int64_t pp_graph_nodes(pp_graph g);
int32_t pp_graph_count(pp_graph g);

/*
 * pp_seeds_init -- Algorithm 1's initialisation: Sig(u) = 0 for all u, then
 * bit i of Sig(x_i) set for every seed, c[0] = s.
 *   seeds       host array of num_graphs * s node ids: seeds[g*s + i] is
 *               seed i of graph g and must lie in graph g's node range.
 *               Repeated seeds are allowed (each owns its own bit).
 *   s           1 <= s <= 4096 seeds per graph; more than 512 need at least
 *               ceil(s / 512) seed groups (opt.seed_groups), which is the default.
 *   opt         NULL for defaults.
 *   stream      hipStream_t for all of the run's device work (NULL: the run
 *               creates its own non-blocking stream).
 * Errors: PP_EINVAL, PP_ERANGE, PP_ENOMEM, PP_EDEVICE.
 */
int pp_seeds_init(pp_graph g, const int32_t *seeds, int32_t s, const pp_options *opt,
                  void *stream, pp_run *out);

/*
 * pp_seeds_reset -- the same initialisation on an existing run, reusing its
 * device memory (no allocation): num_graphs * s seed ids, host memory or,
 * with seeds_on_device, device memory the caller owns.  The call does not
 * wait for the device (with the per-round engine): the initialisation is
 * ordered on the run's stream, and a device seed list must stay valid until
 * the next call that waits.  Host seeds are checked here (PP_ERANGE); device
 * seeds are checked by the device, and an id outside its graph makes the
 * next call that waits (a propagation) fail with PP_ERANGE and leaves the
 * run unusable until a successful reset.  Round logs restart; kernel times
 * keep accumulating.
 */
int pp_seeds_reset(pp_run r, const int32_t *seeds, int32_t seeds_on_device);

/*
 * pp_propagate_round -- one synchronous round (one pass of Algorithm 1's
 * do-while body) for every graph of the batch not yet converged.
 *   new_bits        host [num_graphs]: c_g[r] of the round just run (0 for a
 *                   graph already converged).  May be NULL.
 *   all_converged   host int: 1 once every graph has had a round with no new bit.
 * Synchronises the stream.  After convergence further calls are no-ops that
 * return PP_OK with zeros.  PP_ENOTCONV when the round log is full.
 */
int pp_propagate_round(pp_run r, int64_t *new_bits, int32_t *all_converged);

/*
 * pp_propagate_until_converged -- rounds until every graph converged or
 * max_rounds rounds in total have run (max_rounds <= 0: the log capacity).
 *   counts   host [num_graphs][cap_rounds]: counts[g*cap_rounds + r] = c_g[r]
 *            for r <= D_g, zeros after.  May be NULL.
 *   D        host [num_graphs]: D_g.  May be NULL.
 * Returns PP_ENOTCONV (with the counts so far) if the cap stopped it.
 */
int pp_propagate_until_converged(pp_run r, int32_t max_rounds, int64_t *counts,
                                 int32_t cap_rounds, int32_t *D);

/*
 * pp_estimate_metrics -- host only, pure: the distance metrics from
 * c[0..len-1] of one graph with n nodes and s seeds, tau = tau_num/tau_den
 * (the paper uses 0.9 = 9/10).  Trailing zero rounds are ignored.
 * Errors: PP_EINVAL for len < 1, s < 1, n < 1, tau_den = 0 or
 * tau_num > tau_den.
 */
int pp_estimate_metrics(const int64_t *counts, int32_t len, int64_t n, int32_t s,
                        uint32_t tau_num, uint32_t tau_den, pp_metrics *out);

/* Signatures of the current round into dst ([n][W] uint64 words; device
 * memory when dst_on_device, else host; the caller owns dst). */
int pp_get_signatures(pp_run r, uint64_t *dst, int32_t dst_on_device);

/* Per-seed counts (needs opt.seed_counts): dst host [num_graphs][cap_rounds][s],
 * dst[(g*cap_rounds + r)*s + i] = c_{g,i}[r]. */
int pp_get_seed_counts(pp_run r, uint32_t *dst, int32_t cap_rounds);

/* Rounds run so far (the next round's index) and the number of words W of
 * the signature rows the run reports (pp_get_signatures; W = the smallest
 * power of two >= ceil(s / 64)). */
int32_t pp_run_round(pp_run r);
int32_t pp_run_words(pp_run r);
/* Seed groups of the run and the row width of one group in words. */
int32_t pp_run_groups(pp_run r);
int32_t pp_run_group_words(pp_run r);

/* Per-round record of the last pp_propagate_* call: for each round r <= the
 * current round, mode[r] (PP_MODE_PULL, PP_MODE_PUSH, PP_MODE_PUSH_FLAT or
 * PP_MODE_SPARSE_PULL; 2 for round 0, the initialisation) and arcs[r] (arcs the round touched: all
 * arcs for a pull, the changed nodes' predecessor arcs for a sparse round).
 * Host arrays of cap entries; either may be NULL. */
int pp_get_round_log(pp_run r, int32_t *mode, int64_t *arcs, int32_t cap);
/* The same record for one seed group of a run (pp_get_round_log: group 0's
 * modes, arcs summed over the groups).  PP_EINVAL for a group outside
 * [0, pp_run_groups). */
int pp_get_group_log(pp_run r, int32_t group, int32_t *mode, int64_t *arcs, int32_t cap);

/* With opt.time_kernels: pull_ms[r] = total duration in ms of round r's
 * pull launches (HIP events on the run's stream), summed over every
 * propagation since the run was created (pp_seeds_reset keeps the sums, so
 * a caller differences two reads around repeated runs).  A launch in a push
 * round returns at once (or, after a pull round, lists the push's frontier)
 * and is still timed.  With opt.persistent the value
 * is the main phase of round r (pull, or push for a push round) measured by
 * the device clock between the grid barriers around it.  Host array of cap
 * entries. */
int pp_get_kernel_times(pp_run r, float *pull_ms, int32_t cap);

/*
 * pp_get_node_stats -- per-node outputs for centrality estimates (needs
 * opt.node_stats): for every node u (host arrays [n], by input node id)
 *   reached[u]  = the seeds u reaches within the rounds run so far (seed bits
 *                 set in Sig(u); a repeated seed counts once per bit),
 *   dist_sum[u] = the sum of d(u, x_i) over those seeds.
 * The paper leaves per-node centralities to future work and defines none:
 * these are the plain per-node quantities the propagation determines, from
 * which a caller forms sampled closeness or similar estimates.  The run
 * keeps, per node, the sum of popcount(Sig(u)) over its states (after the
 * initialisation and after every round run), one extra pass per round.
 * Synchronises.  PP_ESTATE if the run was created without node_stats.
 */
int pp_get_node_stats(pp_run r, int32_t *reached, int64_t *dist_sum);

/* Copy of a run's whole state (signatures, frontier, logs) / restore from a
 * copy of the same graph and s.  A restored run continues bit-identically. */
int pp_run_snapshot(pp_run r, pp_run *copy);
int pp_run_restore(pp_run r, pp_run from);

/*
 * Learned scheduler.  Every round of PROPAGATE-P (Algorithm 1) computes the
 * same Sig_r whether it pulls (each node ORs its successors' signatures) or
 * pushes (each changed node ORs its delta into its predecessors), and however
 * a push spreads the frontier's arcs over the lanes; these choices only
 * change the cost.  PP_SCHED_MLP picks, before each round, the action with
 * the smallest predicted cost of a cost model evaluated on the device from
 * eight features of the last round (all normalised to about [0, 1]):
 *   f0 nodes changed / n            f1 their predecessor arcs / stored arcs
 *   f2 pairs reached past the seeds / (n s)
 *   f3 new pairs of the round / (n s)
 *   f4 min(c[r] / max(c[r-1], 1), 4) / 4   (c[-1] = 0)
 *   f5 log2(index of the next round + 1) / 16
 *   f6 log2(f1's arcs / max(f0's nodes, 1) + 1) / 16
 *   f7 1 if the last round pulled, else 0
 * The model is a fully connected network 8 -> 32 -> 32 -> 4, ReLU on both
 * hidden layers, outputs in log-milliseconds of the round's effective cost
 * under each action:
 *   y0 dense pull (every node gathers its successors' rows)
 *   y1 push over direct slots: a few lanes per frontier entry walk its
 *      predecessor list (lean for small frontiers)
 *   y2 push over flattened arc ranges: the frontier's arcs laid out as one
 *      range per wave, each predecessor word read before its atomic (for
 *      large frontiers)
 *   y3 sparse pull (the predecessors that can gain a bit gather their lists)
 * and takes the allowed action with the least output (the first on a tie):
 * the pushes unless the run's sparse_pull is 1, the sparse pull when it is 1
 * or 2 (the persistent engine's pushes always use direct slots).  Weights are
 * PP_MLP_PARAMS floats in the order W1[32][8], b1[32], W2[32][32], b2[32],
 * W3[4][32], b3[4] (row = output unit).  A non-finite output of an allowed
 * action, or weights never set, falls back to the heuristic (direction by
 * frontier arcs, tiling by frontier size: flattened from 16384 entries).
 * The scheduler never changes a result bit, only the work.
 */
#define PP_MLP_PARAMS 1476

/* Sets the run's cost-model weights (host array of PP_MLP_PARAMS floats,
 * copied) or clears them (NULL: the heuristic decides).  Used only when the
 * run was created with scheduler = PP_SCHED_MLP.  The direction of the
 * round about to run (taken at the end of the last round, for a new run at
 * pp_seeds_init) is taken again with the new weights.  The weights persist
 * across pp_seeds_reset.  Synchronises. */
int pp_run_set_mlp(pp_run r, const float *params);

/* The actions of PP_SCHED_PLAN: plan[r] (host, len entries) for round r, an
 * action index of the cost model (0 dense pull, 1 push over direct slots, 2
 * push over flattened ranges, 3 sparse pull; an action the run does not
 * allow, or -1, leaves the round to the heuristic, as do rounds >= len).
 * Kept across resets.  Used to measure fixed schedules.  Synchronises. */
int pp_run_set_plan(pp_run r, const int32_t *plan, int32_t len);

/* Device-clock duration of each round of the run's last propagation (the
 * per-round engine; seed group 0): ms[r] (host, cap entries) from the start
 * of round r's first launch to the end of its closing launch, 0 for rounds
 * not run.  Synchronises. */
int pp_get_round_times(pp_run r, float *ms, int32_t cap);

/* Scheduler features of every round: feat[r][8] (host, cap rows) holds the
 * features computed at the end of round r-1 for round r; row 0 is zero. */
int pp_get_round_features(pp_run r, float *feat, int32_t cap);

/* Training samples for the cost model.  Runs the next round of a run on the
 * per-round engine with the given action (PP_MODE_PULL, PP_MODE_PUSH (direct
 * slots), PP_MODE_PUSH_FLAT (flattened arc ranges) or PP_MODE_SPARSE_PULL;
 * PP_MODE_PUSH stands for the run's sparse direction, i.e. a sparse pull
 * when the run was created with sparse_pull = 1)
 * instead of the scheduler's, and stores its duration in milliseconds in
 * *ms (HIP events around the whole round, every launch of the round
 * included).  features (host [8] or NULL) receives the round's features.
 * With pp_run_snapshot / pp_run_restore a caller times a round both ways,
 * and after either kind of previous round.  PP_ESTATE if the run has
 * converged or is persistent; PP_ENOTCONV if its round log is full. */
enum { PP_MODE_PULL = 0, PP_MODE_PUSH = 1, PP_MODE_SPARSE_PULL = 3, PP_MODE_PUSH_FLAT = 4 };
int pp_time_round(pp_run r, int32_t mode, float *features, float *ms);

/* The cost model on the device, for training and its tests.  All arrays
 * are host memory owned by the caller; n samples, 1 <= n <= 2^26; rows are
 * samples (x[n][8], t and y [n][2]); fp32 arithmetic, sums over samples in
 * double in a fixed order (bit-reproducible).  Synchronous. */
/* y = model(x). */
int pp_mlp_forward(const float *params, const float *x, int64_t n, float *y);
/* loss = 1/(2n) sum_n sum_k (y_nk - t_nk)^2 and its gradient with respect to
 * every parameter (grad [PP_MLP_PARAMS]); either output may be NULL. */
int pp_mlp_loss_grad(const float *params, const float *x, const float *t, int64_t n, float *grad, float *loss);
/* `steps` full-batch Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning
 * rate lr, moments starting at zero) on that loss; params is updated in
 * place; loss_log (host [steps] or NULL) receives the loss before each step. */
int pp_mlp_train(float *params, const float *x, const float *t, int64_t n, int32_t steps, float lr, float *loss_log);

/*
 * pp_exact_counts -- the exact neighbourhood function: PROPAGATE-P with
 * every node as a seed (s = n, the paper's ground-truth use of the method),
 * run as ceil(n / group) seed groups of up to `group` (1..512) nodes each,
 * in node order, their per-round counts summed: counts[r] = the number of
 * ordered pairs (u, v) with d(u, v) = r (counts[0] = n), for r < cap_rounds
 * (host array, zeroed first); *D (may be NULL) = the largest distance, the
 * exact diameter of the reachable pairs.  One graph only.  opt (NULL:
 * defaults) sets the engine and scheduler of the runs; per-seed counts are
 * off.  PP_ERANGE if D >= cap_rounds (counts then hold the rounds that fit).
 */
int pp_exact_counts(pp_graph g, int32_t group, const pp_options *opt, int64_t *counts, int32_t cap_rounds,
                    int32_t *D);

/*
 * pp_progressive_sample -- progressive sampling with a Hoeffding stopping
 * rule (Section 4, error bounds).  Seeds are taken from pool (host [pool_len]
 * input ids, checked), in order, `group` (1..512) at a time; after each
 * group the per-round counts of all seeds so far are summed, and with
 * eps = sqrt(ln(2 / delta) / (2 s)) the run stops at the first group after
 * which eps x D / alpha <= target, where D and alpha = (T - s) / (s (n - 1))
 * are the sample's (the average distance's half-width at confidence
 * 1 - delta, with the sample's values for the unknown Delta and alpha; 0
 * when D = 0), or when the pool runs out.  0 < delta < 1, target >= 0.
 * counts (host [cap_rounds], zeroed first) receives the summed counts
 * c[0..D] of the seeds used; out the figures below.  opt (NULL: defaults)
 * sets the engine and scheduler of the runs.  One graph only.  PP_ERANGE if
 * D >= cap_rounds.
 */
typedef struct {
    int32_t seeds;          /* seeds used */
    int32_t groups;         /* groups run */
    int32_t met;            /* 1: the bound met the target; 0: the pool ran out first */
    int32_t D;              /* D of the sample */
    double alpha;           /* the sample's connectivity rate */
    double eps;             /* sqrt(ln(2 / delta) / (2 seeds)) */
    double bound;           /* eps x D / alpha (0 when D = 0) */
} pp_progress;
int pp_progressive_sample(pp_graph g, const int32_t *pool, int32_t pool_len, int32_t group, double target,
                          double delta, const pp_options *opt, int64_t *counts, int32_t cap_rounds,
                          pp_progress *out);

/*
 * pp_propagate_s -- PROPAGATE-S (Algorithm 2): the seeds one at a time with
 * one bit per node, each pass a synchronous bottom-up step in which a node
 * not reached yet stops at its first reached successor (the early break).
 * Same counts as PROPAGATE-P for the same seeds, in O(n) bits per seed
 * instead of O(n s) for all of them.
 *   seeds      host [s] input node ids, checked (PP_ERANGE if outside [0, n));
 *              duplicates count once each, as seed bits do in PROPAGATE-P.
 *   concurrent seeds in flight at once (0: min(s, 256), at most 65535);
 *              device memory is 2 x concurrent x ceil(n/64) x 8 bytes of
 *              signatures plus cap_rounds x 8 bytes of counts, allocated
 *              here and freed before return (the graph keeps a list of its
 *              nodes with long successor lists from the first call on).
 *   stream     hipStream_t or NULL (the graph's stream); synchronous.
 *   counts     host [cap_rounds], zeroed first: counts[r] = pairs (u, x_i)
 *              with d(u, x_i) = r, counts[0] = s.
 *   D          host, the largest r with counts[r] > 0.
 *   examined   host or NULL: arcs examined over all passes and seeds, each
 *              node's walk counted up to and including its first hit (the
 *              work the early break leaves).
 * One graph only (PP_EINVAL for a batch).  PP_ENOTCONV if a seed still finds
 * nodes at pass cap_rounds - 1 (counts then hold the passes that fit).
 */
int pp_propagate_s(pp_graph g, const int32_t *seeds, int32_t s, int32_t concurrent, void *stream, int64_t *counts,
                   int32_t cap_rounds, int32_t *D, int64_t *examined);

/*
 * pp_propagate_s_noalloc -- pp_propagate_s for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, same results bit for bit; it calls
 * no allocator (neither hipMalloc nor the caller's allocator of
 * pp_set_allocator).  Its device buffers (every seed's signature pair, the
 * pass log, per-seed counters, the seed ids) come from one fixed region of
 * PP_NOALLOC_BYTES bytes that every device the library runs on holds from its
 * first such call until the process ends.
 *   concurrent  0: the most seeds in flight, up to min(s, 256), whose buffers
 *               fit the region; > 0: that many (at most s), PP_EINVAL if they
 *               do not fit.
 * The buffers of k seeds over n nodes with a log of cap_rounds passes take
 * about 16 k ceil(n/64) + 8 cap_rounds bytes; PP_EINVAL (with the sizes in
 * the message) when even one seed does not fit.  Calls on one device share
 * that device's region, which keeps the last call's contents (each call
 * clears what must start at zero): two calls that overlap on one device race
 * and give wrong results; run them one after the other (one stream, or the
 * caller's own ordering).  Synchronous, like pp_propagate_s.
 */
#define PP_NOALLOC_BYTES (64u << 20)
int pp_propagate_s_noalloc(pp_graph g, const int32_t *seeds, int32_t s, int32_t concurrent, void *stream,
                           int64_t *counts, int32_t cap_rounds, int32_t *D, int64_t *examined);

/* One configuration tried by pp_autotune and its best time. */
typedef struct {
    int32_t pull_k, push_div, rounds_per_sync, persistent, sparse_pull;
    float ms;                   /* least wall time of a reset plus a propagation to convergence */
} pp_tune_entry;

/*
 * pp_autotune -- picks run options for a graph by measurement.  Candidates:
 * the pull tile (2 or 4 arcs per lane, which also sets the length above
 * which a list is split into tile-sized chunks) times the push threshold
 * (push_div 4, 8, 16, 32) on the per-round engine, the same thresholds with
 * sparse pulls for the sparse rounds (4 arcs per lane), and the persistent
 * engine.  Each is run once to warm up (graph capture), then `reps` times
 * (>= 1) from pp_seeds_reset to convergence; the least wall time counts.
 *   seeds, s    a representative seed list (host, as for pp_seeds_init).
 *   base        options to start from (NULL: defaults); the scheduler,
 *               per-seed counts, round cap and replay settings are kept
 *               (the learned scheduler runs without weights, i.e. as the
 *               heuristic, during tuning).
 *   best        receives the fastest candidate's options.
 *   table, cap  host array for every candidate tried (may be NULL if cap is
 *               0); *ntried (may be NULL) receives how many were tried.
 * A candidate whose run cannot be created (the persistent engine with more
 * graphs than co-resident blocks) is skipped.  Outputs never depend on the
 * options, only the time does.  Allocates and frees a run per candidate,
 * and one untimed run first: releasing gigabytes of device memory slows
 * the next seconds of GPU work by a few percent, so every candidate is
 * timed after a release, the first one included.
 */
int pp_autotune(pp_graph g, const int32_t *seeds, int32_t s, const pp_options *base, int32_t reps,
                pp_options *best, pp_tune_entry *table, int32_t cap, int32_t *ntried);

/* Free a run (waits for its stream first) / a graph.  Free every run made on
 * a graph, and let every call that uses the graph return, before freeing the
 * graph: its blocks go back to the allocator without a device-wide wait. */
void pp_run_free(pp_run r);
void pp_graph_free(pp_graph g);
const char *pp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PP_H */
