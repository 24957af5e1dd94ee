// HIP kernels for PROPAGATE-P rounds on gfx950 (wave64).
//
// A round r (one pass of Algorithm 1's do-while body) is a fixed sequence of
// three launches that hand work to each other through the device control
// block, so no host decision is needed between rounds and a batch of rounds
// can be replayed as a captured graph.  Kernels of the direction not chosen
// for the round return at once.
//
// Dense pull (the ball recurrence of Section 4, Sig_r(u) = Sig_{r-1}(u) OR
// the rows of u's successors):
//   k_pull<W>        tiles of consecutive nodes: successor ids staged in LDS;
//                    groups of lanes share each source row (one 16-byte load
//                    per lane), OR K consecutive arcs in registers and flush
//                    them into the node's LDS row; the new row is written to
//                    the other signature buffer (the update is synchronous
//                    because Sig_{r-1} is only read).  New bits are counted
//                    per block (Algorithm 1's XOR count).  Chunks of
//                    high-degree nodes OR into the accumulator.
// Sparse push (equal to the pull: only the bits a node gained in round r-1
// can give new bits in round r, every older bit having reached its
// predecessors already):
//   k_pull<W>        in a push round after a pull round: lists the nodes
//                    that changed in the pull (same launch slot).
//   k_push<W>        ORs those new bits into the predecessors' rows with
//                    atomics; a bit is new when the atomic that sets it saw
//                    it clear; nodes that gained bits are queued once.
// Closing launch:
//   k_post<W>        a push round's commit (collects the gained bits, counts
//                    and lists them) or a pull round's high-degree nodes;
//                    then its last block runs the round's end: counts,
//                    convergence (a graph converges at its first round
//                    without a new bit), diameter bookkeeping, the per-round
//                    log, the features and direction of the next round.
#include "pp_internal.h"

namespace pp {

#define PP_DEV __device__ __forceinline__

// Reads of the control block: atomic loads, so they are never served from
// the scalar cache, which a persistent launch would leave stale.
#define CTL(x) __hip_atomic_load(&(x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
// Device-scope store of a value another block of the same launch reads.
#define PUT(x, v) __hip_atomic_store(&(x), (v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)

PP_DEV int lane_id() { return __lane_id(); }

template <int W> struct WordMask {
    static constexpr uint64_t rep = ~0ull / ((1ull << W) - 1);   // lanes with (lane % W) == 0
    static constexpr uint64_t row = (1ull << W) - 1;              // the W lanes of one row
};

// arcs of a push chunk: four passes of a whole wave (64 / W slots)
template <int W> struct PushShape {
    static constexpr int SLOTS = 64 / W;
    static constexpr int CHUNK = 4 * SLOTS;
};

PP_DEV uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Group grp's view of a run: its signature pair, accumulator, stamps,
// frontier lists, partial slots, counters, logs and control block (each
// per-group array holds the groups one after another; counts and per-seed
// counts interleave the groups within each round's row).
PP_DEV RunDev group_view(const RunDev &R0, int grp) {
    RunDev R = R0;
    const int64_t n = R0.nn, W = R0.W, G = R0.G, cap = R0.cap;
    R.s = grp == R0.ngroups - 1 ? R0.s_last : R0.sg;
    R.sig[0] = R0.sig[0] + grp * 2 * n * W;
    R.sig[1] = R.sig[0] + n * W;
    R.acc = R0.acc + grp * n * W;
    R.stamp = R0.stamp + grp * n;
    R.f_ids[0] = R0.f_ids[0] + grp * 2 * n;
    R.f_ids[1] = R.f_ids[0] + n;
    R.f_delta[0] = R0.f_delta[0] + grp * 2 * n * W;
    R.f_delta[1] = R.f_delta[0] + n * W;
    R.chunks[0] = R0.chunks[0] + grp * 2 * R0.cc;
    R.chunks[1] = R.chunks[0] + R0.cc;
    R.blk_cnt = R0.blk_cnt + (int64_t)grp * R0.pgrid;
    R.blk_nodes = R0.blk_nodes + (int64_t)grp * R0.pgrid;
    R.blk_arcs = R0.blk_arcs + (int64_t)grp * R0.pgrid;
    R.blk_pulled = R0.blk_pulled + (int64_t)grp * R0.pgrid;
    R.counts = R0.counts + grp * G;
    R.seed_counts = R0.seed_counts ? R0.seed_counts + grp * G * R0.sg : nullptr;
    R.D = R0.D + grp * G;
    R.gconv = R0.gconv + grp * G;
    R.mode_log = R0.mode_log + grp * G * cap;
    R.arcs_log = R0.arcs_log + grp * G * cap;
    R.phase_log = R0.phase_log + grp * G * cap * 3;
    R.feat_log = R0.feat_log + grp * G * cap * MLP_IN;
    R.tickets = R0.tickets + (int64_t)grp * TICKET_INTS;
    R.post_part = R0.post_part + (int64_t)grp * 3 * POST_MAX;
    R.bar = R0.bar + grp * G;
    R.ctrl = R0.ctrl + grp * G;
    return R;
}

// Buffer k & 1 of a pair by arithmetic on both pointers rather than a
// run-time index into the pair (which would keep a struct copy of the run in
// scratch memory).  Both members of every pair live in one allocation.
template <typename T> PP_DEV T *sel(T *const (&a)[2], int k) { return a[0] + (ptrdiff_t)(k & 1) * (a[1] - a[0]); }

template <typename T> PP_DEV T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

PP_DEV int wave_inclusive_scan(int v) {
    const int ln = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o);
        if (ln >= o) v += t;
    }
    return v;
}

// Appends one slot per lane with `want` to a shared counter with one atomic
// per wave; returns the lane's slot (or -1).  Safe in divergent code: the
// leader is a lane that wants a slot, hence active.
PP_DEV int32_t wave_append(int32_t *counter, bool want) {
    const uint64_t m = __ballot(want);
    if (m == 0) return -1;
    const int ln = lane_id();
    const int leader = __ffsll((long long)m) - 1;
    int32_t base = 0;
    if (ln == leader) base = atomicAdd(counter, (int32_t)__popcll(m));
    base = __shfl(base, leader);
    return want ? base + (int32_t)__popcll(m & ((1ull << ln) - 1ull)) : -1;
}

// Block-wide sum of a per-thread value (all threads must call).
template <typename T> PP_DEV T block_sum(T v, T *scratch) {
    v = wave_sum(v);
    const int wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 0) scratch[wv] = v;
    __syncthreads();
    T t = 0;
#pragma unroll
    for (int k = 0; k < BLOCK / 64; ++k) t += scratch[k];
    return t;
}

template <int W> PP_DEV void load_row(const uint64_t *__restrict__ p, uint64_t (&out)[W]) {
    if constexpr (W == 1) {
        out[0] = p[0];
    } else {
#pragma unroll
        for (int k = 0; k < W; k += 2) {
            const ulonglong2 v = *reinterpret_cast<const ulonglong2 *>(p + k);
            out[k] = v.x;
            out[k + 1] = v.y;
        }
    }
}

template <int W> PP_DEV void store_row(uint64_t *__restrict__ p, const uint64_t (&v)[W]) {
    if constexpr (W == 1) {
        p[0] = v[0];
    } else {
#pragma unroll
        for (int k = 0; k < W; k += 2) {
            ulonglong2 q;
            q.x = v[k];
            q.y = v[k + 1];
            *reinterpret_cast<ulonglong2 *>(p + k) = q;
        }
    }
}
template <int W> PP_DEV void flush_lds(unsigned long long *dst, uint64_t (&acc)[W]) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
        if (acc[w]) atomicOr(dst + w, (unsigned long long)acc[w]);
        acc[w] = 0;
    }
}

// Per-seed counts, wave-wide: lane b accumulates how many lanes holding word
// k have bit b set in d (lanes hold word lane % W).  Call with the whole
// wave active.
template <int W> PP_DEV void seed_ballot(uint64_t d, uint32_t (&sc)[W]) {
    if (__ballot(d != 0) == 0) return;
    const int ln = lane_id();
    for (int bit = 0; bit < 64; ++bit) {
        const uint64_t m = __ballot((int)((d >> bit) & 1ull));
        if (m) {
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const uint32_t c = (uint32_t)__popcll(m & (WordMask<W>::rep << k));
                if (ln == bit) sc[k] += c;
            }
        }
    }
}

template <int W> PP_DEV void seed_flush(const RunDev &R, int r, const uint32_t (&sc)[W]) {
    const int ln = lane_id();
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const int bitidx = k * 64 + ln;
        if (sc[k] && bitidx < R.s) atomicAdd(&R.seed_counts[(int64_t)r * R.sstride + bitidx], sc[k]);
    }
}

// Counts of a batch of graphs, combined over the wave before the atomics: the
// lanes of a wave mostly hold nodes of one graph (a list's entries and a
// tile's nodes are in node order, and each graph is a node range), and every
// lane adding into its graph's counter on its own would queue thousands of
// same-address atomics per round on a few cache lines.  Every lane of the
// wave calls; key: the lane's graph (any value where v = 0).
PP_DEV void wave_add_keyed(unsigned long long *base, int key, unsigned long long v) {
    const int ln = lane_id();
    uint64_t todo = __ballot(v != 0);
    while (todo) {   // wave-uniform: one pass per graph present
        const int lead = __builtin_ctzll(todo);
        const int k = __shfl(key, lead);
        const bool mine = ((todo >> ln) & 1ull) && key == k;
        const unsigned long long t = wave_sum(mine ? v : 0ull);
        if (ln == lead) atomicAdd(base + k, t);
        todo &= ~__ballot(mine);
    }
}

// Per-seed counts of a batch: lane ln holds word ln % W of a row of graph
// gi, d its new bits; the lanes of one graph are counted per seed bit by
// ballot and each seed with new bits takes one atomic.  Every lane of the
// wave calls.
template <int W> PP_DEV void seed_bits_keyed(const RunDev &R, int r, int gi, uint64_t d, bool valid) {
    const int ln = lane_id();
    uint64_t todo = __ballot(valid && d != 0);
    while (todo) {   // wave-uniform
        const int k = __shfl(gi, __builtin_ctzll(todo));
        const bool mine = valid && gi == k;
        const uint64_t dm = mine ? d : 0ull;
        uint64_t any = dm;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) any |= __shfl_xor(any, o);
        uint32_t c[W];
#pragma unroll
        for (int w = 0; w < W; ++w) c[w] = 0;
        while (any) {   // the seed bits set in any lane of the graph
            const int b = __builtin_ctzll(any);
            any &= any - 1;
            const uint64_t m = __ballot((int)((dm >> b) & 1ull));
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint32_t cw = (uint32_t)__popcll(m & (WordMask<W>::rep << w));
                if (ln == b) c[w] = cw;
            }
        }
        const int64_t base = (int64_t)r * R.sstride + (int64_t)k * R.sg;
#pragma unroll
        for (int w = 0; w < W; ++w)
            if (c[w]) atomicAdd(&R.seed_counts[base + w * 64 + ln], c[w]);
        todo &= ~__ballot(mine && d != 0);
    }
}

// Block-wide exclusive prefix sum of v in thread order, with the block total;
// every thread of the block must call (scratch: BLOCK/64 ints of LDS).
PP_DEV int block_scan(int v, int *scratch, int &total) {
    const int incl = wave_inclusive_scan(v);
    const int wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 63) scratch[wv] = incl;
    __syncthreads();
    int before = 0;
    total = 0;
#pragma unroll
    for (int k = 0; k < BLOCK / 64; ++k) {
        const int c = scratch[k];
        if (k < wv) before += c;
        total += c;
    }
    return before + incl - v;
}

// Push chunks needed by a frontier entry with `deg` predecessors (0 when the
// light path walks its list).
template <int W> PP_DEV int chunks_for(int64_t deg) {
    constexpr int CH = PushShape<W>::CHUNK;
    return deg > PUSH_LIGHT ? (int)((deg + CH - 1) / CH) : 0;
}

// Push chunk records of one block iteration, written by the whole block:
// thread t owns nchk[k] chunks of entry entry[k] (k < U), at slots from
// `before` on, in (thread, k) order (before: the block's exclusive scan of
// the threads' sums; total: the block's sum).  Each thread writes every
// BLOCK-th slot, finding the owner by binary search over the block's scan, so
// one long list costs no thread more than total/BLOCK stores.  All threads of
// the block call; s_pre and s_ent hold BLOCK * U ints; ends with a barrier.
template <int U>
PP_DEV void write_chunks(Chunk *out, int before, const int (&nchk)[U], const int32_t (&entry)[U], int total,
                         int chunk, int *s_pre, int32_t *s_ent) {
    int run = before;
#pragma unroll
    for (int k = 0; k < U; ++k) {
        s_pre[threadIdx.x * U + k] = run;
        s_ent[threadIdx.x * U + k] = entry[k];
        run += nchk[k];
    }
    __syncthreads();
    for (int c = threadIdx.x; c < total; c += BLOCK) {
        int lo = 0, hi = BLOCK * U - 1;   // the last (thread, k) whose first slot is <= c owns slot c
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_pre[mid] <= c) lo = mid; else hi = mid - 1;
        }
        out[c] = Chunk{s_ent[lo], (c - s_pre[lo]) * chunk};
    }
    __syncthreads();
}
PP_DEV void write_chunks(Chunk *out, int before, int nchk, int32_t entry, int total, int chunk, int *s_pre,
                         int32_t *s_ent) {
    const int n1[1] = {nchk};
    const int32_t e1[1] = {entry};
    write_chunks<1>(out, before, n1, e1, total, chunk, s_pre, s_ent);
}

// Lists nodes in a block-private LDS queue and moves the queue to the global
// list with one atomic per block (fewer same-address atomics than a per-wave
// append).  An entry that does not fit falls back to a global atomic.
struct BlockQueue {
    static constexpr int CAP = 2048;
    int32_t *q;      // LDS [CAP]
    int *n;          // LDS counter
    PP_DEV void push(bool want, int32_t u, int32_t *gcount, int32_t *glist) {
        const uint64_t m = __ballot(want);
        if (m == 0) return;
        const int ln = lane_id();
        const int leader = __ffsll((long long)m) - 1;
        int base = 0;
        if (ln == leader) base = atomicAdd(n, (int)__popcll(m));
        base = __shfl(base, leader);
        if (want) {
            const int pos = base + (int)__popcll(m & ((1ull << ln) - 1ull));
            if (pos < CAP) {
                q[pos] = u;
            } else {
                glist[atomicAdd(gcount, 1)] = u;
            }
        }
    }
    // all threads of the block; ends with the queue moved out
    PP_DEV void flush(int32_t *gcount, int32_t *glist, int *s_base) {
        __syncthreads();
        const int cnt = *n < CAP ? *n : CAP;
        if (threadIdx.x == 0) *s_base = cnt ? atomicAdd(gcount, cnt) : 0;
        __syncthreads();
        for (int i = threadIdx.x; i < cnt; i += BLOCK) glist[*s_base + i] = q[i];
    }
};

// ---------------------------------------------------------------- fills


__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static int fill_grid(int64_t count) {
    int64_t b = (count + BLOCK - 1) / BLOCK;
    return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}


hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(count)), dim3(BLOCK), 0, st, p, v, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------- fused fills

// Several fills in one launch: block b fills chunk b - first_block[k] of
// segment k (FILL_CHUNK 4-byte words; 16-byte stores for whole quadruples).
constexpr int FILL_SEGS = 16;
constexpr int64_t FILL_CHUNK = (int64_t)BLOCK * 16;
struct FillPlan {
    FillSeg seg[FILL_SEGS];
    int64_t first_block[FILL_SEGS + 1];
    int32_t nseg;
};

__global__ void __launch_bounds__(BLOCK) k_fill_plan(FillPlan P) {
    const int64_t b = blockIdx.x;
    int k = 0;
    while (k + 1 < P.nseg && P.first_block[k + 1] <= b) ++k;
    const FillSeg S = P.seg[k];
    const int64_t w0 = (b - P.first_block[k]) * FILL_CHUNK;
    const int64_t w1 = w0 + FILL_CHUNK < S.n ? w0 + FILL_CHUNK : S.n;
    const int64_t body = w0 + ((w1 - w0) & ~(int64_t)3);
    const uint4 q = make_uint4(S.v, S.v, S.v, S.v);
    for (int64_t i = w0 + threadIdx.x * 4; i < body; i += BLOCK * 4) *reinterpret_cast<uint4 *>(S.p + i) = q;
    for (int64_t i = body + threadIdx.x; i < w1; i += BLOCK) S.p[i] = S.v;
}

hipError_t launch_fills(const FillSeg *segs, int nseg, hipStream_t st) {
    FillPlan P{};
    int k = 0;
    int64_t blocks = 0;
    auto flush = [&]() -> hipError_t {
        if (k == 0) return hipSuccess;
        P.nseg = k;
        P.first_block[k] = blocks;
        hipLaunchKernelGGL(k_fill_plan, dim3((unsigned)blocks), dim3(BLOCK), 0, st, P);
        P = FillPlan{};
        k = 0;
        blocks = 0;
        return hipGetLastError();
    };
    for (int i = 0; i < nseg; ++i) {
        if (segs[i].n <= 0) continue;
        if (k == FILL_SEGS) {
            const hipError_t e = flush();
            if (e != hipSuccess) return e;
        }
        P.seg[k] = segs[i];
        P.first_block[k] = blocks;
        blocks += (segs[i].n + FILL_CHUNK - 1) / FILL_CHUNK;
        ++k;
    }
    return flush();
}

// A seed group's rows back to their initial state where only its seeds can
// have set bits: the rows of the given stored ids (both buffers) and their
// stamps.  Ids outside [0, n) are skipped.
__global__ void __launch_bounds__(BLOCK) k_clear_seed_rows(const int32_t *ids, int count, int64_t n, int W,
                                                           uint64_t *sig, int32_t *stamp) {
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < count; i += gridDim.x * BLOCK) {
        const int32_t x = ids[i];
        if (x < 0 || x >= n) continue;
        for (int w = 0; w < W; ++w) {
            sig[(int64_t)x * W + w] = 0;
            sig[n * W + (int64_t)x * W + w] = 0;
        }
        stamp[x] = -1;
    }
}

hipError_t launch_clear_seed_rows(const int32_t *ids, int count, int64_t n, int W, uint64_t *sig, int32_t *stamp,
                                  hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_seed_rows, dim3((count + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, ids, count, n, W,
                       sig, stamp);
    return hipGetLastError();
}

// ---------------------------------------------------------------- node ids

// out[j] = perm[in[j]] for ids in [0, n), -1 otherwise.
__global__ void __launch_bounds__(BLOCK) k_map_ids(int32_t *out, const int32_t *in, const int32_t *perm, int64_t count,
                                                   int64_t n) {
    for (int64_t j = blockIdx.x * (int64_t)BLOCK + threadIdx.x; j < count; j += (int64_t)gridDim.x * BLOCK) {
        const int32_t x = in[j];
        out[j] = (x >= 0 && x < n) ? perm[x] : -1;
    }
}

hipError_t launch_map_ids(int32_t *out, const int32_t *in, const int32_t *perm, int64_t count, int64_t n,
                          hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_map_ids, dim3(fill_grid(count)), dim3(BLOCK), 0, st, out, in, perm, count, n);
    return hipGetLastError();
}

// dst row x = src row perm[x] (W words per row).
__global__ void __launch_bounds__(BLOCK) k_gather_rows(uint64_t *dst, const uint64_t *src, const int32_t *perm,
                                                       int64_t n, int W) {
    const int64_t total = n * W;
    for (int64_t j = blockIdx.x * (int64_t)BLOCK + threadIdx.x; j < total; j += (int64_t)gridDim.x * BLOCK) {
        const int64_t x = j / W;
        dst[j] = src[(int64_t)perm[x] * W + (j - x * W)];
    }
}

// The host's view of a run in one launch: control blocks and D (as 32-bit
// words) and a range of count rows, stored straight into pinned host memory
// (coherent, mapped), which the host reads after waiting on the stream.
__global__ void k_stage(const int32_t *ctrl, int64_t nctrl, const int32_t *D, int64_t nD, const int64_t *rows,
                        int64_t nrows, int32_t *h_ctrl, int32_t *h_D, int64_t *h_rows) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nctrl + nD + nrows; i += stride) {
        if (i < nctrl) h_ctrl[i] = ctrl[i];
        else if (i < nctrl + nD) h_D[i - nctrl] = D[i - nctrl];
        else h_rows[i - nctrl - nD] = rows[i - nctrl - nD];
    }
}

hipError_t launch_stage(const void *ctrl, int64_t ctrl_bytes, const int32_t *D, int64_t nD, const int64_t *rows,
                        int64_t nrows, void *h_ctrl, int32_t *h_D, int64_t *h_rows, hipStream_t st) {
    const int64_t nctrl = ctrl_bytes / 4;
    hipLaunchKernelGGL(k_stage, dim3(fill_grid(nctrl + nD + nrows)), dim3(BLOCK), 0, st, (const int32_t *)ctrl, nctrl,
                       D, nD, rows, nrows, (int32_t *)h_ctrl, h_D, h_rows);
    return hipGetLastError();
}

hipError_t launch_gather_rows(uint64_t *dst, const uint64_t *src, const int32_t *perm, int64_t n, int W,
                              hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_rows, dim3(fill_grid(n * W)), dim3(BLOCK), 0, st, dst, src, perm, n, W);
    return hipGetLastError();
}

// ---------------------------------------------------------------- seeds

// The internal seed list of a run with seed groups or a seed order, one block
// per graph: the caller's ids (mapped to stored ids by `map` when given; ids
// outside [0, n) become -1, which the seed placement reports) in internal
// order, out[gi * s_all + q], and pos[gi * s_all + i] = q, the internal
// position of the caller's seed i.  With by_reach, the seeds whose node has a
// predecessor come first and the rest after them, each part in the caller's
// order (a seed without a predecessor can set no bit but its own); otherwise
// q = i.  Group j holds internal positions [j sg, (j + 1) sg).
__global__ void __launch_bounds__(BLOCK) k_seed_order(GraphDev g, const int32_t *seeds, const int32_t *map,
                                                      int s_all, int by_reach, int32_t *out, int32_t *pos) {
    __shared__ int s_scan[BLOCK / 64];
    const int64_t base = (int64_t)blockIdx.x * s_all;
    auto stored = [&](int i) -> int32_t {
        int32_t x = seeds[base + i];
        if (map) x = (x >= 0 && x < g.n) ? map[x] : -1;
        return x;
    };
    // a seed the placement will reject keeps its place among the first part
    auto live = [&](int32_t x) -> bool { return !by_reach || x < 0 || x >= g.n || g.trp[x + 1] > g.trp[x]; };
    int nlive = 0;
    for (int i0 = 0; i0 < s_all; i0 += BLOCK) {   // block-uniform
        const int i = i0 + threadIdx.x;
        int t = 0;
        (void)block_scan(i < s_all && live(stored(i)) ? 1 : 0, s_scan, t);
        nlive += t;
    }
    int done_live = 0, done_dead = 0;
    for (int i0 = 0; i0 < s_all; i0 += BLOCK) {   // block-uniform
        const int i = i0 + threadIdx.x;
        const bool valid = i < s_all;
        const int32_t x = valid ? stored(i) : 0;
        const bool lv = valid && live(x);
        int tl = 0, td = 0;
        const int rl = block_scan(lv ? 1 : 0, s_scan, tl);
        const int rd = block_scan(valid && !lv ? 1 : 0, s_scan, td);
        if (valid) {
            const int q = lv ? done_live + rl : nlive + done_dead + rd;
            out[base + q] = x;
            pos[base + i] = q;
        }
        done_live += tl;
        done_dead += td;
    }
}

// Signature rows in the caller's bit order from the rows of a run's seed
// groups: word j of row u holds the caller's seeds 64 j .. 64 j + 63 of u's
// graph; seed i sits at internal position q = pos[gi * s_all + i], bit q % sg
// of group q / sg's row (group grp's current buffer is cur[grp]; each group
// holds a pair of [n][Wg] buffers, the groups one after another).  Rows in
// stored order.
__global__ void __launch_bounds__(BLOCK) k_sig_regroup(const uint64_t *sig, int64_t n, int Wg, int Wout, int s_all,
                                                       int sg, const int32_t *cur, const int32_t *pos,
                                                       const int32_t *node_graph, uint64_t *out) {
    const int64_t total = n * Wout;
    for (int64_t t = blockIdx.x * (int64_t)BLOCK + threadIdx.x; t < total; t += (int64_t)gridDim.x * BLOCK) {
        const int64_t u = t / Wout;
        const int j = (int)(t - u * Wout);
        const int64_t gb = (node_graph ? (int64_t)node_graph[u] : 0) * s_all;
        uint64_t word = 0;
        for (int b = 0; b < 64; ++b) {
            const int i = j * 64 + b;
            if (i >= s_all) break;
            const int q = pos[gb + i];
            const int grp = q / sg, p = q - grp * sg;
            const uint64_t *row = sig + ((int64_t)grp * 2 + cur[grp]) * n * Wg + u * Wg;
            word |= ((row[p >> 6] >> (p & 63)) & 1ull) << b;
        }
        out[t] = word;
    }
}

hipError_t launch_seed_order(const GraphDev &g, const int32_t *seeds, const int32_t *map, int G, int s_all,
                             int by_reach, int32_t *out, int32_t *pos, hipStream_t st) {
    hipLaunchKernelGGL(k_seed_order, dim3(G), dim3(BLOCK), 0, st, g, seeds, map, s_all, by_reach, out, pos);
    return hipGetLastError();
}

hipError_t launch_sig_regroup(const uint64_t *sig, int64_t n, int Wg, int Wout, int s_all, int sg, const int32_t *cur,
                              const int32_t *pos, const int32_t *node_graph, uint64_t *out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sig_regroup, dim3(fill_grid(n * Wout)), dim3(BLOCK), 0, st, sig, n, Wg, Wout, s_all, sg, cur,
                       pos, node_graph, out);
    return hipGetLastError();
}

// Seed bit i of graph g goes to node seeds[g*s + i] (Algorithm 1's
// initialisation).  Bits are gathered in the accumulator first so that a node
// holding several seeds is listed once; the round-0 commit writes them.  A
// seed outside its graph's node range is skipped and flagged.
// map (may be NULL): input id -> stored id for ids in [0, n), -1 otherwise.
// seeds: the group's first seed of graph 0 (graph gi's at gi * s_all).
template <int W>
PP_DEV void phase_seed_scatter(const GraphDev &g, const RunDev &R, const int32_t *seeds, const int32_t *map,
                               int bid, int nb) {
    const int64_t total = (int64_t)R.G * R.s;
    for (int64_t j = bid * (int64_t)BLOCK + threadIdx.x; j < total; j += (int64_t)nb * BLOCK) {
        const int i = (int)(j % R.s);
        const int gi = (int)(j / R.s);
        int32_t x = seeds[(int64_t)gi * R.s_all + i];
        if (map) x = (x >= 0 && x < g.n) ? map[x] : -1;
        const bool ok = x >= g.node_off[gi] && x < g.node_off[gi + 1];
        if (!ok) atomicOr(&R.ctrl->bad_seed, 1);
        if (ok) atomicOr((unsigned long long *)&R.acc[(int64_t)x * W + (i >> 6)], 1ull << (i & 63));
        const bool want = ok && atomicMax(&R.stamp[x], 0) < 0;
        const int pos = wave_append(&R.ctrl->lst[0].nodes, want);
        if (want) R.f_ids[0][pos] = x;
    }
}
template <int W>
__global__ void __launch_bounds__(BLOCK) k_seed_scatter(GraphDev g, RunDev R0, const int32_t *seeds,
                                                        const int32_t *map) {
    const RunDev R = group_view(R0, blockIdx.y);
    phase_seed_scatter<W>(g, R, seeds + (int64_t)blockIdx.y * R0.sg, map, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------- list commit

// The commit's items (entry, word) of list p: U per thread and pass, their
// loads in flight together, taken U grid-widths apart so that a short list
// still spreads over every block.
template <int W, int U>
PP_DEV void commit_items(const GraphDev &g, const RunDev &R, int init, bool apply, int r, int p, int64_t items, int bid,
                         int nb, uint64_t &pop, int64_t &arcs, uint32_t (&sc)[W]) {
    Ctrl *C = R.ctrl;
    uint64_t *sg = sel(R.sig, CTL(C->cur));
    const int32_t *ids = sel(R.f_ids, p);
    uint64_t *dl = sel(R.f_delta, p);
    Chunk *chunks = sel(R.chunks, p);
    const int w = lane_id() & (W - 1);
    const bool per_seed = R.seed_counts != nullptr;
    __shared__ int s_scan[BLOCK / 64];
    __shared__ int s_cbase;
    __shared__ int s_pre[BLOCK * U];
    __shared__ int32_t s_ent[BLOCK * U];
    const int64_t width = (int64_t)nb * BLOCK;
    for (int64_t bb = bid * (int64_t)BLOCK; bb < items; bb += width * U) {   // block-uniform
        int64_t idx[U];
        bool valid[U];
        int32_t u[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            idx[k] = bb + (int64_t)k * width + threadIdx.x;   // word idx % W == w
            valid[k] = idx[k] < items;
            u[k] = valid[k] ? ids[idx[k] / W] : 0;
        }
        uint64_t d[U];
        int64_t lo[U], hi[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            d[k] = valid[k] ? R.acc[(int64_t)u[k] * W + w] : 0;
            const bool head = valid[k] && w == 0;
            lo[k] = head ? g.trp[u[k]] : 0;
            hi[k] = head ? g.trp[u[k] + 1] : 0;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (!valid[k]) continue;
            R.acc[(int64_t)u[k] * W + w] = 0;
            dl[idx[k]] = d[k];
            if (init) {
                R.sig[0][(int64_t)u[k] * W + w] |= d[k];
                R.sig[1][(int64_t)u[k] * W + w] |= d[k];
            } else if (apply) {   // a sparse pull left the row as it was
                sg[(int64_t)u[k] * W + w] |= d[k];
            }
        }
        int nchk[U];
        int32_t ent[U];
        int tc = 0;
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t deg = hi[k] - lo[k];
            arcs += deg;
            nchk[k] = chunks_for<W>(deg);
            ent[k] = (int32_t)(idx[k] / W);
            tc += nchk[k];
        }
        // push chunks of long predecessor lists: one reservation per block and pass
        if (__syncthreads_or(tc > 0)) {
            int total = 0;
            const int before = block_scan(tc, s_scan, total);
            if (threadIdx.x == 0) s_cbase = atomicAdd(&C->lst[p].chunks, total);
            __syncthreads();
            write_chunks<U>(chunks + s_cbase, before, nchk, ent, total, PushShape<W>::CHUNK, s_pre, s_ent);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int pc = __popcll(d[k]);
            if (R.G == 1) {
                pop += (uint64_t)pc;
                if (per_seed) seed_ballot<W>(d[k], sc);
            } else {
                const int gi = valid[k] ? g.node_graph[u[k]] : 0;
                wave_add_keyed((unsigned long long *)&R.counts[(int64_t)r * R.cstride], gi, (unsigned long long)pc);
                if (per_seed) seed_bits_keyed<W>(R, r, gi, d[k], valid[k]);
            }
        }
    }
}

// Collects the bits gathered in the accumulator for the entries of frontier
// list r&1, writes them into the list, counts them, and reserves push chunks
// for the next round.  Round 0 (init) also writes them into both signature
// buffers; a push round has set them in Sig already; after a sparse pull
// (apply) they are set in Sig here.
// parts (the closing launch): the block's new-bit count and predecessor arcs
// go to its slots of the per-block partials instead of the round's
// counters, which the round's end then sums.
// UMAX: at most this many items per thread and pass (1 keeps the LDS and
// registers small, for the persistent kernel).  pstride: distance between
// the three partials' arrays (a one-block cluster keeps its three in LDS).
template <int W, int UMAX = 4>
PP_DEV void phase_push_commit(const GraphDev &g, const RunDev &R, int init, int bid, int nb, int64_t *parts = nullptr,
                              bool apply = false, int pstride = POST_MAX) {
    Ctrl *C = R.ctrl;
    const int r = init ? 0 : CTL(C->round);
    const int p = r & 1;
    const int32_t cnt = CTL(C->lst[p].nodes);
    const int64_t items = (int64_t)cnt * W;
    const bool per_seed = R.seed_counts != nullptr;
    uint64_t pop = 0;
    int64_t arcs = 0;
    uint32_t sc[W];
#pragma unroll
    for (int k = 0; k < W; ++k) sc[k] = 0;
    // long lists: four items per thread and pass
    if (UMAX >= 4 && items > 2 * (int64_t)nb * BLOCK)
        commit_items<W, 4>(g, R, init, apply, r, p, items, bid, nb, pop, arcs, sc);
    else
        commit_items<W, 1>(g, R, init, apply, r, p, items, bid, nb, pop, arcs, sc);
    __shared__ unsigned long long s_red[BLOCK / 64];
    const unsigned long long tp = block_sum<unsigned long long>(pop, s_red);
    const unsigned long long ta = block_sum<unsigned long long>((unsigned long long)arcs, s_red);
    if (threadIdx.x == 0) {
        if (parts) {
            PUT(parts[0 * pstride + bid], (int64_t)tp);
            PUT(parts[1 * pstride + bid], (int64_t)0);
            PUT(parts[2 * pstride + bid], (int64_t)ta);
        } else {
            if (R.G == 1 && tp) atomicAdd((unsigned long long *)&R.counts[(int64_t)r * R.cstride], tp);
            if (ta) atomicAdd((unsigned long long *)&C->f_arcs[p], ta);
        }
    }
    if (per_seed && R.G == 1) seed_flush<W>(R, r, sc);
}

// ---------------------------------------------------------------- pull

// Issues the loads that stage a pull tile: K column ids per lane and the
// tile's row offsets (relative to its first arc; a hub chunk is one row).
template <int K, int NODES>
PP_DEV void stage_tile(const GraphDev &g, const Tile &T, int ln, int32_t (&cv)[K], int32_t &rv0, int32_t &rv1) {
    const int nn = T.u1 - T.u0;
    const int ne = (int)(T.e1 - T.e0);
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int i = ln + j * 64;
        cv[j] = i < ne ? g.col[T.e0 + i] : 0;
    }
    rv0 = 0;
    rv1 = 0;
    if (T.hub >= 0) {
        rv0 = ln == 0 ? 0 : ne;
    } else {
        if (ln <= nn) rv0 = (int)(g.rp[T.u0 + ln] - T.e0);
        if (ln == 0 && nn == NODES) rv1 = (int)(g.rp[T.u0 + NODES] - T.e0);
    }
}

// SHORT: every tile of the graph takes the one-lane-per-node gather (rows of
// one or two words, no high-degree chunks): the general gather is not
// compiled in, which leaves the kernel fewer registers and more waves.
// DEAD: the rows of nodes without successors are left alone (see below).
template <int W, int KK = 0, bool SHORT = false, bool DEAD = false>
PP_DEV void phase_pull(const GraphDev &g, const RunDev &R, int bid, int nb) {
    Ctrl *C = R.ctrl;
    using PS = PullShape<W, KK>;
    constexpr int K = PS::K;
    constexpr int EDGES = PS::EDGES;
    constexpr int NODES = PS::NODES;
    constexpr int WAVES = BLOCK / 64;
    // each wave stages its own tile: no block barrier inside the tile loop
    __shared__ int32_t s_col[WAVES][EDGES];
    __shared__ int32_t s_rp[WAVES][NODES + 1];
    __shared__ unsigned long long s_acc[WAVES][NODES * W];
    __shared__ unsigned long long s_red[BLOCK / 64];
    const int r = CTL(C->round);
    const int cur = CTL(C->cur);
    const uint64_t *__restrict__ sig = sel(R.sig, cur);
    uint64_t *__restrict__ nxt = sel(R.sig, cur ^ 1);
    const int ln = lane_id();
    const int wv = threadIdx.x >> 6;
    int32_t *col_l = s_col[wv];
    int32_t *rp_l = s_rp[wv];
    unsigned long long *acc_l = s_acc[wv];
    const bool per_seed = R.seed_counts != nullptr;
    uint64_t pop = 0;
    int64_t nodes = 0, parcs = 0, pulled = 0;
    uint32_t sc[W];
#pragma unroll
    for (int k = 0; k < W; ++k) sc[k] = 0;

    const int64_t nw = (int64_t)nb * WAVES;
    // Software pipeline over the wave's tiles: the column and offset loads of
    // the next tile are issued before this tile's row gathers, so one memory
    // latency per tile is exposed instead of two.
    int64_t t = (int64_t)bid * WAVES + wv;
    Tile T = t < g.ntiles ? g.tiles[t] : Tile{0, 0, 0, 0, -1, 0};
    int32_t cv[K];
    int32_t rv0 = 0, rv1 = 0;
    stage_tile<K, NODES>(g, T, ln, cv, rv0, rv1);
    for (; t < g.ntiles; t += nw) {   // wave-uniform
        const int64_t tn = t + nw;
        const Tile Tn = tn < g.ntiles ? g.tiles[tn] : T;
        const int nn = T.u1 - T.u0;
        const int ne = (int)(T.e1 - T.e0);
        const bool hub = T.hub >= 0;
        const bool skip = R.G > 1 && R.gconv[T.graph];
        if (!skip) {
#pragma unroll
            for (int j = 0; j < K; ++j) col_l[ln + j * 64] = cv[j];
            if (ln <= nn) rp_l[ln] = rv0;
            if (ln == 0 && nn == NODES) rp_l[NODES] = rv1;
#pragma unroll
            for (int j = 0; j < W; ++j) acc_l[ln + j * 64] = 0ull;
        }
        if (tn < g.ntiles) stage_tile<K, NODES>(g, Tn, ln, cv, rv0, rv1);
        if (skip) {
            // a graph of the batch that has converged gathers nothing, but its
            // rows still go to the other buffer: its last round may have been a
            // push, which set bits in this buffer only, and the pull is about
            // to make the other one current
            if (!hub) {
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    const int idx = ln + j * 64;
                    if (idx < nn * W) nxt[(int64_t)T.u0 * W + idx] = sig[(int64_t)T.u0 * W + idx];
                }
            }
            T = Tn;
            continue;
        }
        // A node without successors keeps its row for good, and the row is the
        // same in both buffers (the initialisation writes the seed bits into
        // both): with DEAD it is neither read nor written here (rowmask bit i:
        // the tile's node i has successors).  On a large R-MAT graph most
        // nodes have none.
        uint64_t rowmask = 0;
        if constexpr (DEAD) rowmask = hub ? 0ull : __ballot(ln < nn && rp_l[ln + 1] > rp_l[ln]);
        uint64_t own[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const int idx = ln + j * 64;   // word idx % W of node idx / W (< 64)
            const bool rw = DEAD ? ((rowmask >> (idx / W)) & 1ull) != 0 : (!hub && idx < nn * W);
            own[j] = rw ? sig[(int64_t)T.u0 * W + idx] : 0;
        }

        // a tile whose lists are all short (one- and two-word rows, at most
        // NPL successors): one lane per node walks its own list, so load j
        // of the wave takes the j-th successor of 64 consecutive nodes
        // (neighbouring rows on a lattice: few cache lines per load)
        constexpr int NPL = PULL_NPL;
        int dmax = 0;
        if constexpr (W <= 2 && !SHORT) {
            if (!hub) {
                int d = ln < nn ? rp_l[ln + 1] - rp_l[ln] : 0;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) d = max(d, __shfl_xor(d, o));
                dmax = d;
            }
        }
        if (SHORT || (W <= 2 && !hub && dmax <= NPL)) {
            const int b0 = ln < nn ? rp_l[ln] : 0;
            const int d = ln < nn ? rp_l[ln + 1] - b0 : 0;
            uint64_t rows[NPL][W];
#pragma unroll
            for (int j = 0; j < NPL; ++j) {
#pragma unroll
                for (int w = 0; w < W; ++w) rows[j][w] = 0;
                if (j < d) load_row<W>(sig + (int64_t)col_l[b0 + j] * W, rows[j]);
            }
            if (ln < nn) {
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    uint64_t a = 0;
#pragma unroll
                    for (int j = 0; j < NPL; ++j) a |= rows[j][w];
                    acc_l[ln * W + w] = a;
                }
            }
        } else if constexpr (!SHORT) {
        // gather: a group of L lanes shares arcs [a, a + KG); each lane loads
        // and ORs its P-word slice of every source row (one 16-byte load per
        // lane, so the group's loads of one row fall in one cache line and
        // cost one L2 request), keeps a running accumulator, and flushes it
        // into the LDS row of each node it leaves
        constexpr int L = PS::L, P = PS::P, KG = PS::KG;
        const int sub = ln % L;
        const int a = (ln / L) * KG;
        if (a < ne) {
            const int b = min(a + KG, ne);
            int lo = 0, hi = nn - 1;          // node i with rp[i] <= a < rp[i+1]
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (rp_l[mid] <= a) lo = mid; else hi = mid - 1;
            }
            int i = lo;
            uint64_t rows[KG][P];
#pragma unroll
            for (int j = 0; j < KG; ++j) {
                if (a + j < b) {
                    load_row<P>(sig + (int64_t)col_l[a + j] * W + sub * P, rows[j]);
                } else {
#pragma unroll
                    for (int w = 0; w < P; ++w) rows[j][w] = 0;
                }
            }
            uint64_t acc[P];
#pragma unroll
            for (int w = 0; w < P; ++w) acc[w] = 0;
            int nx = rp_l[i + 1];
#pragma unroll
            for (int j = 0; j < KG; ++j) {
                const int e = a + j;
                if (e < b) {
                    while (e >= nx) {
                        flush_lds<P>(acc_l + i * W + sub * P, acc);
                        ++i;
                        nx = rp_l[i + 1];
                    }
#pragma unroll
                    for (int w = 0; w < P; ++w) acc[w] |= rows[j][w];
                }
            }
            flush_lds<P>(acc_l + i * W + sub * P, acc);
        }
        }
        if (ln == 0) pulled += ne;

        if (hub) {
            // a chunk of a high-degree node: combined by the hub phase
            if (ln < W && acc_l[ln]) atomicOr((unsigned long long *)&R.acc[(int64_t)T.u0 * W + ln], acc_l[ln]);
        } else {
            uint64_t tpop = 0;
#pragma unroll
            for (int j = 0; j < W; ++j) {   // same trip count for every lane
                const int idx = ln + j * 64;
                const bool valid = idx < nn * W;
                uint64_t nw2 = 0;
                const int32_t u = T.u0 + idx / W;
                if (DEAD ? ((rowmask >> (idx / W)) & 1ull) != 0 : valid) {
                    const uint64_t av = acc_l[idx];
                    nw2 = av & ~own[j];
                    nxt[(int64_t)T.u0 * W + idx] = own[j] | av;
                }
                tpop += (uint64_t)__popcll(nw2);
                const uint64_t bal = __ballot(nw2 != 0);
                const int gb = ln & ~(W - 1);
                const bool lead = valid && (ln & (W - 1)) == 0 && ((bal >> gb) & WordMask<W>::row) != 0;
                if (lead) {
                    nodes += 1;
                    parcs += g.trp[u + 1] - g.trp[u];
                    R.stamp[u] = r;   // changed in this round: listed by a push that follows
                }
                if (per_seed) {
                    if (R.G == 1) seed_ballot<W>(nw2, sc);
                    else seed_bits_keyed<W>(R, r, T.graph, nw2, valid);
                }
            }
            if (R.G == 1) {
                pop += tpop;
            } else {
                const uint64_t tt = wave_sum(tpop);
                if (ln == 0 && tt) atomicAdd((unsigned long long *)&R.counts[(int64_t)r * R.cstride + T.graph], (unsigned long long)tt);
            }
        }
        T = Tn;
    }
    const unsigned long long tp = block_sum<unsigned long long>(pop, s_red);
    const unsigned long long tn = block_sum<unsigned long long>((unsigned long long)nodes, s_red);
    const unsigned long long ta = block_sum<unsigned long long>((unsigned long long)parcs, s_red);
    const unsigned long long tq = block_sum<unsigned long long>((unsigned long long)pulled, s_red);
    if (threadIdx.x == 0) {
        R.blk_cnt[bid] = (int64_t)tp;
        R.blk_nodes[bid] = (int64_t)tn;
        R.blk_arcs[bid] = (int64_t)ta;
        R.blk_pulled[bid] = (int64_t)tq;
    }
    if (per_seed && R.G == 1) seed_flush<W>(R, r, sc);
}

// High-degree nodes of a pull round: the chunks left their ORed rows in the
// accumulator.
template <int W>
PP_DEV void phase_pull_hubs(const GraphDev &g, const RunDev &R, int bid, int nb, int64_t *parts = nullptr) {
    Ctrl *C = R.ctrl;
    if (g.nhubs == 0) {
        if (parts && threadIdx.x == 0) {
            PUT(parts[0 * POST_MAX + bid], (int64_t)0);
            PUT(parts[1 * POST_MAX + bid], (int64_t)0);
            PUT(parts[2 * POST_MAX + bid], (int64_t)0);
        }
        return;
    }
    const int r = CTL(C->round);
    const int cur = CTL(C->cur);
    const uint64_t *sig = sel(R.sig, cur);
    uint64_t *nxt = sel(R.sig, cur ^ 1);
    const int ln = lane_id();
    const int w = ln & (W - 1);
    const bool per_seed = R.seed_counts != nullptr;
    uint64_t pop = 0;
    int64_t nodes = 0, parcs = 0;
    uint32_t sc[W];
#pragma unroll
    for (int k = 0; k < W; ++k) sc[k] = 0;
    const int64_t items = (int64_t)g.nhubs * W;
    const int64_t stride = (int64_t)nb * BLOCK;
    for (int64_t base = bid * (int64_t)BLOCK + (threadIdx.x & ~63); base < items; base += stride) {
        const int64_t idx = base + ln;
        const bool valid = idx < items;
        uint64_t nw = 0;
        int32_t u = 0;
        if (valid) {
            u = g.hub_node[idx / W];
            const int64_t o = (int64_t)u * W + w;
            const uint64_t av = R.acc[o];
            R.acc[o] = 0;
            const uint64_t ow = sig[o];
            nw = av & ~ow;
            nxt[o] = ow | av;
        }
        const uint64_t bal = __ballot(nw != 0);
        const int gb = ln & ~(W - 1);
        const bool lead = valid && w == 0 && ((bal >> gb) & WordMask<W>::row) != 0;
        if (lead) {
            nodes += 1;
            parcs += g.trp[u + 1] - g.trp[u];
            R.stamp[u] = r;
        }
        const int pc = __popcll(nw);
        if (R.G == 1) {
            pop += (uint64_t)pc;
            if (per_seed) seed_ballot<W>(nw, sc);
        } else {
            const int gi = valid ? g.node_graph[u] : 0;
            wave_add_keyed((unsigned long long *)&R.counts[(int64_t)r * R.cstride], gi, (unsigned long long)pc);
            if (per_seed) seed_bits_keyed<W>(R, r, gi, nw, valid);
        }
    }
    __shared__ unsigned long long s_red[BLOCK / 64];
    const unsigned long long tp = block_sum<unsigned long long>(pop, s_red);
    const unsigned long long tn = block_sum<unsigned long long>((unsigned long long)nodes, s_red);
    const unsigned long long ta = block_sum<unsigned long long>((unsigned long long)parcs, s_red);
    if (threadIdx.x == 0) {
        if (parts) {
            PUT(parts[0 * POST_MAX + bid], (int64_t)tp);
            PUT(parts[1 * POST_MAX + bid], (int64_t)tn);
            PUT(parts[2 * POST_MAX + bid], (int64_t)ta);
        } else {
            if (tp) atomicAdd((unsigned long long *)&C->hub_cnt, tp);
            if (tn) atomicAdd((unsigned long long *)&C->hub_nodes, tn);
            if (ta) atomicAdd((unsigned long long *)&C->hub_arcs, ta);
        }
    }
    if (per_seed && R.G == 1) seed_flush<W>(R, r, sc);
}

// ---------------------------------------------------------------- push

// After a pull round the frontier is not listed; this lists the nodes that
// changed in round r-1 (the pull stamped them with r-1) with their new bits
// (Sig_{r-1} and Sig_{r-2} are the two buffers), into list (r-1)&1.  Each
// block owns a contiguous node range, one thread per node.  A first pass
// reads the stamps, counts the block's entries, arcs and push chunks, and
// collects the changed nodes in LDS; one atomic per block reserves their
// slots; a second pass writes the entries (rows read for the changed nodes
// only).  A block whose changed nodes overflow the LDS list rescans its
// range instead.
template <int W, int CAP = 2048>   // CAP: LDS list capacity per block
PP_DEV void phase_frontier(const GraphDev &g, const RunDev &R, int bid, int nb) {
    Ctrl *C = R.ctrl;
    const int r = CTL(C->round);
    const int p = (r - 1) & 1;
    const int cur = CTL(C->cur);
    const uint64_t *now = sel(R.sig, cur);
    const uint64_t *old = sel(R.sig, cur ^ 1);
    const int64_t span = g.n - g.n0;   // the view's node range [n0, n)
    const int64_t per = ((span + nb - 1) / nb + BLOCK - 1) / BLOCK * BLOCK;
    const int64_t u_begin = g.n0 + (int64_t)bid * per;
    const int64_t u_end = u_begin + per < g.n ? u_begin + per : g.n;
    __shared__ int s_scan[BLOCK / 64];
    __shared__ unsigned long long s_red[BLOCK / 64];
    __shared__ int s_nbase, s_cbase, s_len;
    __shared__ int s_pre[BLOCK];
    __shared__ int32_t s_ent[BLOCK];
    __shared__ int32_t s_list[CAP];
    __shared__ int32_t s_deg[CAP];
    if (threadIdx.x == 0) s_len = 0;
    __syncthreads();

    int nodes = 0, nchunks = 0;
    int64_t arcs = 0;
    const int ln = lane_id();
    constexpr int U = 4;   // nodes per thread whose loads are in flight together
    for (int64_t u0 = u_begin + threadIdx.x; u0 < u_end; u0 += (int64_t)U * BLOCK) {
        bool ch[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t u = u0 + (int64_t)k * BLOCK;
            ch[k] = u < u_end && R.stamp[u] == r - 1;
        }
        int64_t lo[U], hi[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t u = u0 + (int64_t)k * BLOCK;
            lo[k] = ch[k] ? g.trp[u] : 0;
            hi[k] = ch[k] ? g.trp[u + 1] : 0;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t deg = hi[k] - lo[k];
            nodes += ch[k] ? 1 : 0;
            arcs += deg;
            nchunks += chunks_for<W>(deg);
            // append to the block's LDS list: one LDS atomic per wave
            const uint64_t m = __ballot(ch[k]);
            if (m) {
                const int leader = __ffsll((long long)m) - 1;
                int base = 0;
                if (ln == leader) base = atomicAdd(&s_len, (int)__popcll(m));
                base = __shfl(base, leader);
                const int pos = base + (int)__popcll(m & ((1ull << ln) - 1ull));
                if (ch[k] && pos < CAP) {
                    s_list[pos] = (int32_t)(u0 + (int64_t)k * BLOCK);
                    s_deg[pos] = (int32_t)deg;
                }
            }
        }
    }
    const int tn = block_sum<int>(nodes, s_scan);
    const int tc = block_sum<int>(nchunks, s_scan);
    const unsigned long long ta = block_sum<unsigned long long>((unsigned long long)arcs, s_red);
    // the list's arcs are the pull's changed nodes' arcs, which the round's
    // end of that pull has recorded already
    (void)ta;
    if (threadIdx.x == 0 && (tn | tc)) {
        const unsigned long long old = atomicAdd(reinterpret_cast<unsigned long long *>(&C->lst[p]),
                                                 (unsigned long long)tn | ((unsigned long long)tc << 32));
        s_nbase = (int)(uint32_t)old;
        s_cbase = (int)(old >> 32);
    }
    __syncthreads();
    if (tn == 0) return;   // same for the whole block
    int32_t *ids = sel(R.f_ids, p);
    uint64_t *dl = sel(R.f_delta, p);
    Chunk *chunks = sel(R.chunks, p);
    int crun = s_cbase;
    if (tn <= CAP) {
        // the listed nodes only (in the order the waves appended them)
        for (int i0 = 0; i0 < tn; i0 += BLOCK) {   // block-uniform
            const int i = i0 + threadIdx.x;
            const bool valid = i < tn;
            const int64_t u = valid ? s_list[i] : 0;
            const int nchk = valid ? chunks_for<W>(s_deg[i]) : 0;
            const int pos = s_nbase + i;
            int it_chunks = 0;
            const int cfirst = crun + block_scan(nchk, s_scan, it_chunks);
            if (valid) {
                uint64_t a[W], b[W];
                load_row<W>(now + u * W, a);
                load_row<W>(old + u * W, b);
#pragma unroll
                for (int w = 0; w < W; ++w) a[w] &= ~b[w];
                ids[pos] = (int32_t)u;
                store_row<W>(dl + (int64_t)pos * W, a);
            }
            if (it_chunks) write_chunks(chunks + crun, cfirst - crun, nchk, pos, it_chunks, PushShape<W>::CHUNK, s_pre, s_ent);
            crun += it_chunks;
        }
        return;
    }
    int done = 0;
    for (int64_t ub = u_begin; ub < u_end && done < tn; ub += BLOCK) {   // block-uniform
        const int64_t u = ub + threadIdx.x;
        const bool changed = u < u_end && R.stamp[u] == r - 1;
        const int64_t deg = changed ? g.trp[u + 1] - g.trp[u] : 0;
        const int nchk = changed ? chunks_for<W>(deg) : 0;
        int it_nodes = 0, it_chunks = 0;
        const int pos = s_nbase + done + block_scan(changed ? 1 : 0, s_scan, it_nodes);
        const int cfirst = crun + block_scan(nchk, s_scan, it_chunks);
        if (changed) {
            uint64_t a[W], b[W];
            load_row<W>(now + u * W, a);
            load_row<W>(old + u * W, b);
#pragma unroll
            for (int w = 0; w < W; ++w) a[w] &= ~b[w];
            ids[pos] = (int32_t)u;
            store_row<W>(dl + (int64_t)pos * W, a);
        }
        if (it_chunks) write_chunks(chunks + crun, cfirst - crun, nchk, pos, it_chunks, PushShape<W>::CHUNK, s_pre, s_ent);
        done += it_nodes;
        crun += it_chunks;
    }
}

// Pushes new bits d[it] of frontier entries to up to IT predecessors per
// lane (the W lanes of a slot share the predecessor and hold its words).  All
// predecessor ids are loaded, then all rows read, then the atomic ORs of the
// bits not seen set issued, before any result is used; a bit is new when the
// atomic that set it saw it clear.  Predecessors
// that gained a bit are queued once per round (stamp).
template <int W, int IT>
PP_DEV void push_slots(const RunDev &R, uint64_t *sig, int r, const int64_t (&k)[IT], const bool (&kv)[IT],
                       const int32_t *tcol, int w, const uint64_t (&d)[IT], BlockQueue &bq, Ctrl *C, int pn,
                       bool filter) {
    int32_t u[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) u[it] = kv[it] ? tcol[k[it]] : 0;
    // filter: a plain read first -- bits only ever get set, so a bit seen set
    // (even in a stale copy) needs no atomic, and most pushes of a late round
    // bring nothing new; a small push, bound by latency, skips the read
    uint64_t seen[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it)
        seen[it] = (filter && kv[it] && d[it]) ? __hip_atomic_load(&sig[(int64_t)u[it] * W + w], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP)
                                     : 0ull;
    uint64_t nb[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        nb[it] = 0;
        const uint64_t need = d[it] & ~seen[it];
        if (kv[it] && need) {
            const uint64_t oldv =
                atomicOr((unsigned long long *)&sig[(int64_t)u[it] * W + w], (unsigned long long)need);
            nb[it] = need & ~oldv;
        }
    }
    const int ln = lane_id();
    const int gb = ln & ~(W - 1);
    bool want[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        if (nb[it]) atomicOr((unsigned long long *)&R.acc[(int64_t)u[it] * W + w], (unsigned long long)nb[it]);
        const uint64_t bal = __ballot(nb[it] != 0);
        const bool any = kv[it] && ((bal >> gb) & WordMask<W>::row) != 0;
        want[it] = any && w == 0 && atomicMax(&R.stamp[u[it]], r) < r;
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) bq.push(want[it], u[it], &C->lst[pn].nodes, sel(R.f_ids, pn));
}

// Sparse pull over up to IT (frontier entry, predecessor u) pairs per slot of
// W lanes (lane w holds word w of the entry's new bits d).  No signature is
// written in this phase, so u gains a bit in this round exactly when some
// entry's new bits are not all in u's row; such a u is claimed once per round
// (stamp).  A u with at most SPULL_LIGHT successors is then gathered whole by
// the claiming slot (every successor's row, as in a pull) and the bits its
// row lacks go to the accumulator; a u with a longer list instead takes each
// entry's missing bits by atomic OR into the accumulator.  Either way u is
// queued once, and the commit sets the accumulated bits in its row.
template <int W, int IT>
PP_DEV void spull_slots(const GraphDev &g, const RunDev &R, const uint64_t *sig, int r, const int64_t (&k)[IT],
                        const bool (&kv)[IT], int w, const uint64_t (&d)[IT], BlockQueue &bq, Ctrl *C, int pn) {
    int32_t u[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) u[it] = kv[it] ? g.tcol[k[it]] : 0;
    // the row and the list bounds of every slot's predecessor, in one batch
    uint64_t own[IT];
    int64_t b[IT], e[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        own[it] = kv[it] ? sig[(int64_t)u[it] * W + w] : 0ull;
        b[it] = kv[it] ? g.rp[u[it]] : 0;
        e[it] = kv[it] ? g.rp[u[it] + 1] : 0;
    }
    const int ln = lane_id();
    const int gb = ln & ~(W - 1);
    bool claim[IT], light[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const uint64_t need = kv[it] ? d[it] & ~own[it] : 0ull;
        const bool any = ((__ballot(need != 0) >> gb) & WordMask<W>::row) != 0;
        light[it] = e[it] - b[it] <= SPULL_LIGHT;
        if (!light[it] && need) atomicOr((unsigned long long *)&R.acc[(int64_t)u[it] * W + w], (unsigned long long)need);
        const bool c = any && w == 0 && atomicMax(&R.stamp[u[it]], r) < r;
        claim[it] = ((__ballot(c) >> gb) & 1ull) != 0;   // the slot's first lane holds the claim
    }
    // claimed short lists: the first four successors of every slot in one
    // batch of loads, then the rest of the longer ones
    uint64_t a[IT];
    int32_t v4[IT][4];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const bool go = claim[it] && light[it];
#pragma unroll
        for (int q = 0; q < 4; ++q) v4[it][q] = go && b[it] + q < e[it] ? g.col[b[it] + q] : -1;
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        a[it] = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (v4[it][q] >= 0) a[it] |= sig[(int64_t)v4[it][q] * W + w];
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        if (claim[it] && light[it]) {
            for (int64_t j = b[it] + 4; j < e[it]; j += 4) {
                int32_t vv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) vv[q] = j + q < e[it] ? g.col[j + q] : -1;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (vv[q] >= 0) a[it] |= sig[(int64_t)vv[q] * W + w];
            }
            R.acc[(int64_t)u[it] * W + w] = a[it] & ~own[it];
        }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) bq.push(claim[it] && w == 0, u[it], &C->lst[pn].nodes, sel(R.f_ids, pn));
}

// FLAT: large frontiers take the flattened, read-first path (false keeps
// only the direct path, with fewer registers, for the persistent kernel).
// SPARSE: the same walk over the frontier's predecessor arcs as a sparse
// pull (spull_slots) instead of a push.
template <int W, bool FLAT = true, bool SPARSE = false>
PP_DEV void phase_push(const GraphDev &g, const RunDev &R, int bid, int nb) {
    Ctrl *C = R.ctrl;
    const int r = CTL(C->round);
    const int pp = (r - 1) & 1, pn = r & 1;
    uint64_t *sig = sel(R.sig, CTL(C->cur));
    const int32_t cnt = CTL(C->lst[pp].nodes);
    const int32_t nch = CTL(C->lst[pp].chunks);
    const bool filter = FLAT && (CTL(C->flat) & 1);   // the round's tiling of the frontier's arcs
    const int32_t *ids = sel(R.f_ids, pp);
    const uint64_t *dl = sel(R.f_delta, pp);
    const int ln = lane_id();
    const int w = ln & (W - 1);
    const int64_t wave = (bid * (int64_t)BLOCK + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)nb * BLOCK) >> 6;
    __shared__ int32_t s_q[BlockQueue::CAP];
    __shared__ int s_qn, s_qbase;
    BlockQueue bq{s_q, &s_qn};
    if (threadIdx.x == 0) s_qn = 0;
    __syncthreads();

    // light entries (at most PUSH_LIGHT predecessors)
    if (FLAT && filter) {
        // light entries (at most PUSH_LIGHT predecessors): a wave takes G = 64/W
        // entries at a time, one per group of W lanes, and walks their arcs as
        // one flat range (an exclusive scan of the entries' degrees), one arc per
        // group per step, so short lists leave no lane idle; a group finds the
        // entry of its arc by binary search over the scan held in the lanes
        {
            constexpr int G = 64 / W;
            constexpr int IT = 4;
            const int grp = ln / W;
            for (int64_t e0 = wave * G; e0 < cnt; e0 += nwaves * G) {   // wave-uniform
                const int64_t e = e0 + grp;
                int64_t b = 0;
                int deg = 0;
                uint64_t d = 0;
                if (e < cnt) {
                    const int32_t v = ids[e];
                    b = g.trp[v];
                    const int64_t len = g.trp[v + 1] - b;
                    deg = len <= PUSH_LIGHT ? (int)len : 0;   // long lists go through chunks
                    d = dl[e * W + w];
                }
                const int contrib = w == 0 ? deg : 0;
                const int incl = wave_inclusive_scan(contrib);
                const int start = __shfl(incl - contrib, grp * W);   // the group's first flat arc
                const int total = __shfl(incl, 63);
                for (int a0 = 0; a0 < total; a0 += G * IT) {   // wave-uniform
                    int64_t k[IT];
                    bool kv[IT];
                    uint64_t dd[IT];
    #pragma unroll
                    for (int it = 0; it < IT; ++it) {
                        const int a = a0 + it * G + grp;
                        int lo = 0;   // the last group whose first flat arc is <= a
    #pragma unroll
                        for (int step = G >> 1; step > 0; step >>= 1)   // lo + step stays below G
                            if (__shfl(start, (lo + step) * W) <= a) lo += step;
                        const int so = __shfl(start, lo * W);
                        const int64_t bo = __shfl(b, lo * W);
                        dd[it] = __shfl(d, lo * W + w);
                        kv[it] = a < total;
                        k[it] = bo + (a - so);
                    }
                    if constexpr (SPARSE) spull_slots<W, IT>(g, R, sig, r, k, kv, w, dd, bq, C, pn);
                    else push_slots<W, IT>(R, sig, r, k, kv, g.tcol, w, dd, bq, C, pn, filter);
                }
            }
        }
    } else {
        // a small frontier, bound by latency: PUSH_SLOTS slots of W lanes per
        // entry walk its list directly (no scan, no search)
        constexpr int L = W * PUSH_SLOTS;
        constexpr int GPW = 64 / L;
        constexpr int IT = PUSH_LIGHT / PUSH_SLOTS;
        const int grp = ln / L, slot = (ln % L) / W;
        for (int64_t e0 = wave * GPW; e0 < cnt; e0 += nwaves * GPW) {   // wave-uniform
            const int64_t e = e0 + grp;
            bool ev = e < cnt;
            int64_t b = 0, end = 0;
            uint64_t d = 0;
            if (ev) {
                const int32_t v = ids[e];
                b = g.trp[v];
                end = g.trp[v + 1];
                ev = end - b <= PUSH_LIGHT;
                d = dl[e * W + w];
            }
            int64_t k[IT];
            bool kv[IT];
            uint64_t dd[IT];
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                k[it] = b + slot + it * PUSH_SLOTS;
                kv[it] = ev && k[it] < end;
                dd[it] = d;
            }
            if constexpr (SPARSE) spull_slots<W, IT>(g, R, sig, r, k, kv, w, dd, bq, C, pn);
            else push_slots<W, IT>(R, sig, r, k, kv, g.tcol, w, dd, bq, C, pn, false);
        }
    }
    // long lists: chunks of CHUNK arcs, one wave each
    {
        constexpr int SL = PushShape<W>::SLOTS;
        constexpr int CH = PushShape<W>::CHUNK;
        constexpr int IT = CH / SL;
        const int slot = ln / W;
        for (int64_t c = wave; c < nch; c += nwaves) {   // wave-uniform
            const Chunk cd = sel(R.chunks, pp)[c];
            const int32_t v = ids[cd.entry];
            const uint64_t d = dl[(int64_t)cd.entry * W + w];
            const int64_t b = g.trp[v] + cd.off;
            const int64_t lim = g.trp[v + 1];
            const int64_t end = (b + CH < lim) ? b + CH : lim;
            int64_t k[IT];
            bool kv[IT];
            uint64_t dd[IT];
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                k[it] = b + slot + it * SL;
                kv[it] = k[it] < end;
                dd[it] = d;
            }
            if constexpr (SPARSE) spull_slots<W, IT>(g, R, sig, r, k, kv, w, dd, bq, C, pn);
            else push_slots<W, IT>(R, sig, r, k, kv, g.tcol, w, dd, bq, C, pn, filter);
        }
    }
    bq.flush(&C->lst[pn].nodes, sel(R.f_ids, pn), &s_qbase);
}

// ---------------------------------------------------------------- round end

PP_DEV int32_t schedule(const GraphDev &g, const RunDev &R, int32_t r, int64_t fnodes, int64_t farcs) {
    switch (R.sched) {
        case PP_SCHED_PULL: return MODE_PULL;
        case PP_SCHED_PUSH: return MODE_PUSH;
        case PP_SCHED_FUZZ:
            return (mix64(R.fuzz_seed + (uint64_t)r * 0x9E3779B97F4A7C15ull) >> 63) ? MODE_PUSH : MODE_PULL;
        default:
            (void)fnodes;
            return (farcs * (int64_t)R.push_div < g.m) ? MODE_PUSH : MODE_PULL;
    }
}

// The sparse direction of round r: a push, or a sparse pull when the run asks
// for it (sparse_pull 1), or either by a pseudo-random bit per round
// (sparse_pull 2, for testing: the bits do not depend on it).
PP_DEV int32_t sparse_dir(const RunDev &R, int32_t r, int32_t d) {
    if (d != MODE_PUSH || R.sparse_pull == 0) return d;
    if (R.sparse_pull == 1) return MODE_SPULL;
    return (mix64(~R.fuzz_seed + (uint64_t)r * 0xD1B54A32D192ED03ull) >> 63) ? MODE_SPULL : MODE_PUSH;
}

// log2(x) for x >= 1, to about 1e-15 relative: x = m 2^e with m in
// [sqrt(1/2), sqrt(2)) (frexp, then one halving of the range), and
// ln m = 2 artanh(t) = 2 (t + t^3/3 + t^5/5 + ...) with t = (m - 1)/(m + 1),
// |t| <= 0.1716, summed to t^17/17 (the next term is below 1e-16 of the sum).
// It stands in for the library's double log2, whose long dependent chain sat
// on every round's path through the round's end (about 0.5 us per round of a
// one-block cluster), for features that are then rounded to float.
PP_DEV double log2_series(double x) {
    int e = 0;
    double m = frexp(x, &e);   // m in [0.5, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double t = (m - 1.0) / (m + 1.0), t2 = t * t;
    double p = 1.0 / 17.0;
#pragma unroll
    for (int k = 15; k >= 1; k -= 2) p = p * t2 + 1.0 / (double)k;
    return (double)e + 2.0 * t * p * 1.44269504088896340736;   // 1 / ln 2
}

// The eight frontier features of the round after `r` (each roughly in [0, 1]):
// changed nodes / n, their predecessor arcs / m, reached (node, seed) pairs /
// (n s), new bits of round r / (n s), growth of the new-bit count (ratio to
// the round before, clipped at 4, / 4), log2(r + 1) / 16, log2 of the mean
// predecessor degree of the changed nodes / 16, and whether round r pulled.
PP_DEV void sched_features(const GraphDev &g, const RunDev &R, int r, int mode, int64_t fnodes, int64_t farcs,
                           int64_t cnt, int64_t reached, int64_t last, float (&f)[MLP_IN]) {
    const double nv = (double)(g.n - g.n0 > 0 ? g.n - g.n0 : 1);
    const double mv = (double)(g.m > 0 ? g.m : 1);
    const double pairs = nv * (double)R.s;
    f[0] = (float)((double)fnodes / nv);
    f[1] = (float)((double)farcs / mv);
    f[2] = (float)((double)reached / pairs);
    f[3] = (float)((double)cnt / pairs);
    const double grow = (double)cnt / (double)(last > 0 ? last : 1);
    f[4] = (float)((grow < 4.0 ? grow : 4.0) / 4.0);
    f[5] = (float)(log2_series((double)r + 1.0) / 16.0);
    f[6] = (float)(log2_series((double)farcs / (double)(fnodes > 0 ? fnodes : 1) + 1.0) / 16.0);
    f[7] = mode == MODE_PULL ? 1.0f : 0.0f;
}

// The cost model's actions a run may take: dense pull always; the pushes
// unless sparse rounds must be sparse pulls; the sparse pull when the run
// launches its kernel (the per-round engine with sparse_pull 1 or 2).
PP_DEV uint32_t allowed_actions(const RunDev &R, bool direct_only) {
    uint32_t a = 1u;
    if (R.sparse_pull != 1) a |= direct_only ? 2u : 6u;
    if (R.sparse_pull != 0 && !direct_only) a |= 8u;
    return a;
}

// MLP inference for the closing launch of a round, where it lies on the path
// from one round to the next: every weight is loaded ahead into the threads
// that use it (the loads overlap the round's sums), layer 1 takes the whole
// block of BLOCK = 256 threads (thread t: hidden unit t / 8, input t % 8, a
// reduction over 8 lanes) and hands over through LDS with one barrier, and
// one wave takes layers 2 and 3 without further barriers: lane j sums half of
// hidden unit j % 32's inputs (j < 32 the first 16, else the last 16, read as
// LDS broadcasts) and the halves meet by one shuffle; then lane j takes
// output j / 16 over hidden units 2 (j % 16) and 2 (j % 16) + 1 (shuffled in)
// and 16 lanes reduce each output.
static_assert(BLOCK == 256 && MLP_IN == 8 && MLP_HID == 32 && MLP_OUT == 4, "block inference layout");
struct MlpThread {
    float w1, b1;       // layer 1: unit t / 8, input t % 8
    float w2[16], b2;   // wave 0, lane j: unit j % 32, inputs 16 (j / 32) .. + 15
    float w3[2], b3;    // wave 0, lane j: output j / 16, hidden units 2 (j % 16), + 1
};

PP_DEV void mlp_load_block(const float *w, MlpThread &m) {
    const int t = threadIdx.x;
    m.w1 = w[MLP_W1 + (t >> 3) * MLP_IN + (t & 7)];
    m.b1 = w[MLP_B1 + (t >> 3)];
    if (t < 64) {
        const int jj = t & 31, h0 = 16 * (t >> 5);
#pragma unroll
        for (int u = 0; u < 16; ++u) m.w2[u] = w[MLP_W2 + jj * MLP_HID + h0 + u];
        m.b2 = w[MLP_B2 + jj];
        const int k = t >> 4, i0 = 2 * (t & 15);
        m.w3[0] = w[MLP_W3 + k * MLP_HID + i0];
        m.w3[1] = w[MLP_W3 + k * MLP_HID + i0 + 1];
        m.b3 = w[MLP_B3 + k];
    }
}

// Every thread of the block calls; returns the action (as mlp_decide) in every thread.
PP_DEV int32_t mlp_eval_block(const MlpThread &m, const float (&f)[MLP_IN], uint32_t allow) {
    __shared__ float s_h1[MLP_HID];
    __shared__ int32_t s_act;
    const int t = threadIdx.x, q = t & 7;
    float fq = f[0];
#pragma unroll
    for (int i = 1; i < MLP_IN; ++i) fq = q == i ? f[i] : fq;   // input q, without indexing a register array
    float p = m.w1 * fq;
    p += __shfl_xor(p, 1);
    p += __shfl_xor(p, 2);
    p += __shfl_xor(p, 4);
    if (q == 0) s_h1[t >> 3] = fmaxf(p + m.b1, 0.0f);
    __syncthreads();
    if (t < 64) {
        const int h0 = 16 * (t >> 5);
        float h = 0.0f;
#pragma unroll
        for (int u = 0; u < 16; ++u) h += m.w2[u] * s_h1[h0 + u];
        h += __shfl_xor(h, 32);
        const float h2 = fmaxf(h + m.b2, 0.0f);   // lanes j and j + 32 hold hidden unit j % 32
        const int i0 = 2 * (t & 15);
        float o = m.w3[0] * __shfl(h2, i0) + m.w3[1] * __shfl(h2, i0 + 1);
#pragma unroll
        for (int d = 1; d < 16; d <<= 1) o += __shfl_xor(o, d);
        o += m.b3;   // lanes 16 k .. 16 k + 15 hold output k
        int32_t best = -1;
        float bo = 0.0f;
#pragma unroll
        for (int a = 0; a < MLP_OUT; ++a) {
            const float oa = __shfl(o, 16 * a);
            if (!((allow >> a) & 1u) || best == -2) continue;
            if (!__builtin_isfinite(oa)) {
                best = -2;
                continue;
            }
            if (best < 0 || oa < bo) {
                best = a;
                bo = oa;
            }
        }
        if (t == 0) s_act = best < 0 ? -1 : best;
    }
    __syncthreads();
    return s_act;
}

// The same inference with the weights read where they are used (few
// registers: for the kernels that keep their footprint small).
PP_DEV int32_t mlp_decide(const float *w, const float (&f)[MLP_IN], uint32_t allow) {
    const int j = lane_id();
    const int jj = j & (MLP_HID - 1);
    float h1 = w[MLP_B1 + jj];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) h1 += w[MLP_W1 + jj * MLP_IN + i] * f[i];
    h1 = h1 > 0.0f ? h1 : 0.0f;
    float h2 = w[MLP_B2 + jj];
    for (int i = 0; i < MLP_HID; ++i) h2 += w[MLP_W2 + jj * MLP_HID + i] * __shfl(h1, i);
    h2 = h2 > 0.0f ? h2 : 0.0f;
    const int k = j & (MLP_OUT - 1);
    float o = w[MLP_B3 + k];
    for (int i = 0; i < MLP_HID; ++i) o += w[MLP_W3 + k * MLP_HID + i] * __shfl(h2, i);
    int32_t best = -1;
    float bo = 0.0f;
    for (int a = 0; a < MLP_OUT; ++a) {
        const float oa = __shfl(o, a);
        if (!((allow >> a) & 1u)) continue;
        if (!__builtin_isfinite(oa)) return -1;
        if (best < 0 || oa < bo) {
            best = a;
            bo = oa;
        }
    }
    return best;
}

// The direction and frontier tiling of the next round from a cost-model
// action (>= 0), else from the fixed rule: `fallback` (pull or push, turned
// into a sparse pull as the run's option asks) with the threshold's tiling.
// Returns the mode; *flat receives the control block's tiling bits.
PP_DEV int32_t take_action(const RunDev &R, int32_t round, int32_t action, int32_t fallback, bool heur_flat,
                           bool direct_only, int32_t *flat) {
    const int32_t hf = heur_flat && !direct_only ? 1 : 0;
    int32_t mode;
    int32_t f = hf;
    switch (action) {
        case 0: mode = MODE_PULL; break;
        case 1: mode = MODE_PUSH; f = 0; break;
        case 2: mode = MODE_PUSH; f = direct_only ? 0 : 1; break;
        case 3: mode = MODE_SPULL; break;
        default: mode = sparse_dir(R, round, fallback); break;
    }
    *flat = f | (hf << 1);
    return mode;
}

// nparts: blocks of the pull that left per-block partials.  parts/npost:
// the closing launch's per-block partials (new bits, hub nodes, arcs), or
// NULL when its blocks added into the control block instead.  direct_only:
// the caller's pushes walk direct slots only (the persistent loop).
// INFER: how the cost model (a run under PP_SCHED_MLP) is evaluated:
// INFER_WAVE by one wave, weights read where used (few registers: the
// initialisation, the persistent loop); INFER_BLOCK by the whole block,
// weights loaded before the sums (the per-round engine's closing launch);
// INFER_NONE for callers whose run does not use the model.
enum { INFER_WAVE = 0, INFER_BLOCK = 1, INFER_NONE = 2 };
template <int INFER = INFER_WAVE>
PP_DEV void phase_round_end(const GraphDev &g, const RunDev &R, int init, int nparts, const int64_t *parts = nullptr,
                            int npost = 0, bool direct_only = false, int pstride = POST_MAX) {
    Ctrl *C = R.ctrl;
    const int r = init ? 0 : CTL(C->round);
    const int mode = init ? MODE_INIT : CTL(C->mode);
    __shared__ long long s_red4[4][BLOCK / 64];
    __shared__ int s_active;
    __shared__ int s_next;
    // every control-block value the end needs, loaded up front, and the
    // scheduler's inputs: the cost model's weights (first wave) or the plan's
    // next action
    const bool use_mlp = R.sched == PP_SCHED_MLP;
    MlpThread mw;
    if (INFER == INFER_BLOCK && use_mlp) mlp_load_block(R.mlp, mw);
    const int32_t planned = (R.sched == PP_SCHED_PLAN && r + 1 < R.cap) ? R.plan[r + 1] : -1;
    const long long hub_cnt = CTL(C->hub_cnt), hub_nodes = CTL(C->hub_nodes), hub_arcs = CTL(C->hub_arcs);
    const long long lst_count = CTL(C->lst[r & 1].nodes), lst_arcs = CTL(C->f_arcs[r & 1]);
    const long long prev_arcs = CTL(C->f_arcs[(r - 1) & 1]);
    const int64_t reached0 = CTL(C->reached), last = CTL(C->last_count);
    // one reduction for the four sums: pull partials (pull rounds) and the
    // closing launch's partials
    long long v[4] = {0, 0, 0, 0};
    if (mode == MODE_PULL) {
#pragma unroll 4
        for (int b = threadIdx.x; b < nparts; b += BLOCK) {
            v[0] += R.blk_cnt[b];
            v[1] += R.blk_nodes[b];
            v[2] += R.blk_arcs[b];
            v[3] += R.blk_pulled[b];
        }
    }
#pragma unroll
    for (int j = 0; j < POST_MAX / BLOCK; ++j) {   // all loads issued before the sums
        const int b = threadIdx.x + j * BLOCK;
        if (b < npost) {
            v[0] += CTL(parts[0 * pstride + b]);
            v[1] += CTL(parts[1 * pstride + b]);
            v[2] += CTL(parts[2 * pstride + b]);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = wave_sum(v[k]);
    if (lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s_red4[k][threadIdx.x >> 6] = v[k];
    }
    if (threadIdx.x == 0) s_active = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = 0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) v[k] += s_red4[k][w];
    }
    long long fnodes = 0, farcs = 0, pulled = 0;
    long long own = -1;   // this round's count of a single graph when known here
    if (mode == MODE_PULL) {
        fnodes = v[1] + hub_nodes;
        farcs = v[2] + hub_arcs;
        pulled = v[3];
        if (R.G == 1) own = v[0] + hub_cnt;
    } else {
        fnodes = lst_count;
        farcs = lst_arcs + v[2];
        if (R.G == 1 && parts) own = v[0];
    }
    if (own >= 0 && threadIdx.x == 0) R.counts[(int64_t)r * R.cstride] = own;
    int act = 0;
    long long cnt = 0;
    for (int gi = threadIdx.x; gi < R.G; gi += BLOCK) {
        const long long c = own >= 0 ? own : CTL(R.counts[(int64_t)r * R.cstride + gi]);
        cnt += c;
        // a single graph whose round ends here has not converged (its
        // rounds stop with it), so its flag need not be read
        if (own < 0 && R.gconv[gi]) continue;
        if (c == 0) {
            R.gconv[gi] = 1;
        } else {
            R.D[gi] = r;
            ++act;
        }
    }
    if (act) atomicAdd(&s_active, act);
    if (own >= 0) cnt = own;
    else cnt = block_sum<long long>(cnt, s_red4[0]);
    const int64_t reached = reached0 + (init ? 0 : cnt);
    float f[MLP_IN];
    sched_features(g, R, r + 1, mode, fnodes, farcs, cnt, reached, last, f);
    const int32_t fallback = schedule(g, R, r + 1, fnodes, farcs);
    const uint32_t allow = allowed_actions(R, direct_only);
    if (INFER == INFER_BLOCK && use_mlp) {
        const int32_t a = mlp_eval_block(mw, f, allow);   // the whole block
        if (threadIdx.x == 0) s_next = a;
    } else if (threadIdx.x < 64) {
        int32_t a = (INFER == INFER_WAVE && use_mlp) ? mlp_decide(R.mlp, f, allow) : -1;
        if (R.sched == PP_SCHED_PLAN)   // a given plan (outside its actions: the heuristic)
            a = (planned >= 0 && planned < MLP_OUT && ((allow >> planned) & 1u)) ? planned : -1;
        if (threadIdx.x == 0) s_next = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (r < R.cap) R.phase_log[(int64_t)r * 3 + 2] = (int64_t)wall_clock64();   // the round's end
        C->acc_pending = 1;   // a state for the per-node sums
        R.mode_log[r] = (mode == MODE_PUSH && !direct_only && (CTL(C->flat) & 1)) ? MODE_PUSH_FLAT : mode;
        R.arcs_log[r] = mode == MODE_PULL ? pulled : (mode == MODE_INIT ? 0 : prev_arcs);
        // the arcs of the nodes changed in this round: a following push's work
        if (mode == MODE_PULL || parts) C->f_arcs[r & 1] = farcs;
        if (mode == MODE_PULL) C->cur ^= 1;
        C->prev_mode = mode;
        C->hub_cnt = 0;
        C->hub_nodes = 0;
        C->hub_arcs = 0;
        C->active = s_active;
        C->reached = reached;
        C->last_count = cnt;
#pragma unroll
        for (int i = 0; i < MLP_IN; ++i) C->feat[i] = f[i];
        if (r + 1 < R.cap) {
#pragma unroll
            for (int i = 0; i < MLP_IN; ++i) R.feat_log[(int64_t)(r + 1) * MLP_IN + i] = f[i];
        }
        if (s_active == 0) {
            C->converged = 1;
        } else if (r + 1 >= R.cap) {
            C->converged = 1;
            C->overflow = 1;
        } else {
            const int nr = r + 1, q = nr & 1;
            C->lst[q].nodes = 0;
            C->lst[q].chunks = 0;
            C->f_arcs[q] = 0;
            int32_t fl = 0;
            C->mode = take_action(R, nr, s_next, fallback, fnodes >= PUSH_FILTER_MIN, direct_only, &fl);
            C->flat = fl;
            C->round = nr;
        }
    }
}


// ---------------------------------------------------------------- kernels

// One launch per phase; a phase whose direction is not the round's returns.
template <int W> __global__ void __launch_bounds__(BLOCK) k_push_commit(GraphDev g, RunDev R0, int init) {
    const RunDev R = group_view(R0, blockIdx.y);
    if (R.ctrl->converged || (!init && R.ctrl->mode != MODE_PUSH)) return;
    phase_push_commit<W>(g, R, init, blockIdx.x, gridDim.x);
}
// The pull, or in a push round that follows a pull the frontier listing (the
// push's first phase, in the same launch slot so that a round takes three
// launches).  The listing uses at most FRONTIER_BLOCKS blocks: each takes one
// reservation atomic on a single address, and those serialise.
constexpr int FRONTIER_BLOCKS = 1024;
template <int W, int KK, bool DEAD = false>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(W >= 8 ? 2 : PP_PULL_WAVES)))
k_pull(GraphDev g, RunDev R0) {
    const RunDev R = group_view(R0, blockIdx.y);
    const Ctrl *C = R.ctrl;
    if (C->converged) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {   // the round's start: its first launch's first block
        const int r = C->round;
        if (r < R.cap) R.phase_log[(int64_t)r * 3] = (int64_t)wall_clock64();
    }
    if (C->mode == MODE_PULL) {
        phase_pull<W, KK, false, DEAD>(g, R, blockIdx.x, gridDim.x);
    } else if (C->prev_mode == MODE_PULL && blockIdx.x < FRONTIER_BLOCKS) {
        const int nb = gridDim.x < FRONTIER_BLOCKS ? (int)gridDim.x : FRONTIER_BLOCKS;
        phase_frontier<W, 1024>(g, R, blockIdx.x, nb);
    }
}
// The pull of a graph whose lists are all short (one- and two-word rows):
// the same phases as k_pull with only the one-lane-per-node gather compiled.
template <int W>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(PP_PULL_SHORT_WAVES)))
k_pull_short(GraphDev g, RunDev R0) {
    const RunDev R = group_view(R0, blockIdx.y);
    const Ctrl *C = R.ctrl;
    if (C->converged) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {   // the round's start: its first launch's first block
        const int r = C->round;
        if (r < R.cap) R.phase_log[(int64_t)r * 3] = (int64_t)wall_clock64();
    }
    if (C->mode == MODE_PULL) {
        phase_pull<W, 0, true>(g, R, blockIdx.x, gridDim.x);
    } else if (C->prev_mode == MODE_PULL && blockIdx.x < FRONTIER_BLOCKS) {
        const int nb = gridDim.x < FRONTIER_BLOCKS ? (int)gridDim.x : FRONTIER_BLOCKS;
        phase_frontier<W, 1024>(g, R, blockIdx.x, nb);
    }
}
template <int W> __global__ void __launch_bounds__(BLOCK) k_push(GraphDev g, RunDev R0) {
    const RunDev R = group_view(R0, blockIdx.y);
    if (R.ctrl->converged || R.ctrl->mode != MODE_PUSH) return;
    phase_push<W>(g, R, blockIdx.x, gridDim.x);
}
// The sparse pull's kernel, apart from the push's so that a run that never
// takes it keeps the push kernel's smaller register and LDS footprint.
template <int W> __global__ void __launch_bounds__(BLOCK) k_spull(GraphDev g, RunDev R0) {
    const RunDev R = group_view(R0, blockIdx.y);
    if (R.ctrl->converged || R.ctrl->mode != MODE_SPULL) return;
    phase_push<W, true, true>(g, R, blockIdx.x, gridDim.x);
}
__global__ void __launch_bounds__(BLOCK) k_round_end(GraphDev g, RunDev R0, int init) {
    const RunDev R = group_view(R0, blockIdx.y);
    if (R.ctrl->converged) return;
    phase_round_end(g, R, init, g.pull_grid);
}
// Algorithm 1's initialisation for a short seed list in one block: the seed
// bits, the round-0 commit and the round's end, one after the other (the
// block's barriers order them; its global writes are visible to its own
// threads after a barrier).
template <int W>
__global__ void __launch_bounds__(BLOCK) k_seed_init(GraphDev g, RunDev R0, const int32_t *seeds, const int32_t *map) {
    const RunDev R = group_view(R0, blockIdx.y);
    phase_seed_scatter<W>(g, R, seeds + (int64_t)blockIdx.y * R0.sg, map, 0, 1);
    __syncthreads();
    phase_push_commit<W>(g, R, 1, 0, 1);
    __syncthreads();
    phase_round_end(g, R, 1, g.pull_grid);
}

// Blocks of a closing launch of nb blocks that items (words to commit or
// combine) keep busy: POST_ITEMS per thread, at least one block.  Blocks
// without items would only add ticket latency, and more than one item per
// thread adds serial passes of dependent loads; one item measured best.
constexpr int POST_ITEMS = 1;
PP_DEV int post_blocks(int64_t items, int nb) {
    const int64_t b = (items + (int64_t)BLOCK * POST_ITEMS - 1) / ((int64_t)BLOCK * POST_ITEMS);
    return b < 1 ? 1 : (b < nb ? (int)b : nb);
}

// Waits until every global memory operation this thread issued has been
// performed (s_waitcnt with vmcnt 0; expcnt 7 and lgkmcnt 15 leave the other
// counters alone), with compiler fences so that no memory access moves
// across it.
PP_DEV void wait_global_ops() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Two-level ticket (one thread per block, after every thread of the block
// has waited for its global operations and a block barrier): true for the
// block that finishes last.  Blocks count off in groups of TICKET_GROUP, each
// group on its own cache line, and the last block of each group counts off
// at the top, so no address takes more than TICKET_GROUP atomics.  Whoever
// completes a counter resets it for the next launch.
PP_DEV bool last_block(int32_t *tickets, int bid, int nb) {
    const int ngroups = (nb + TICKET_GROUP - 1) / TICKET_GROUP;
    const int gi = bid / TICKET_GROUP;
    const int gsize = nb - gi * TICKET_GROUP < TICKET_GROUP ? nb - gi * TICKET_GROUP : TICKET_GROUP;
    int32_t *gc = tickets + gi * TICKET_STRIDE;
    if (__hip_atomic_fetch_add(gc, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != gsize - 1) return false;
    __hip_atomic_store(gc, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int32_t *top = tickets + TICKET_GROUP * TICKET_STRIDE;
    if (__hip_atomic_fetch_add(top, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ngroups - 1) return false;
    __hip_atomic_store(top, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// The closing launch of a round: the list commit of a push round or the
// high-degree nodes of a pull round, then the round's end, run by the last
// block to finish.  Everything the round's end reads from the other blocks
// of this launch was written by device-scope atomics (per-block partials,
// counts, hub totals), which are coherent across the XCDs' L2 caches once
// performed, and is read back with device-scope atomic loads.  So each thread
// waits for its own global operations to be performed before the block
// counts off; the block barrier alone would not wait for them (a workgroup
// release emits no such wait on CDNA), and the last block could read a
// partial of the previous round.  An agent-scope release would also write
// back every dirty L2 line, which this launch's plain writes (rows, deltas,
// lists) need only at the launch boundary: up to 12 us per round on large
// commits.
template <int W, bool MLP> __global__ void __launch_bounds__(BLOCK) k_post(GraphDev g, RunDev R0) {
    const RunDev R = group_view(R0, blockIdx.y);
    Ctrl *C = R.ctrl;
    if (CTL(C->converged)) {   // set only by the last block, after every block has finished
        if (blockIdx.x == 0 && threadIdx.x == 0) PUT(C->acc_pending, 0);   // no round ran in this slot
        return;
    }
    const int32_t mode = CTL(C->mode);
    // the blocks this round's items need (every block reads the same count):
    // the rest leave at once and take no ticket, so a small round's end does
    // not wait for the whole grid to count off
    const int64_t items = mode == MODE_PULL ? (int64_t)g.nhubs * W : (int64_t)CTL(C->lst[CTL(C->round) & 1].nodes) * W;
    const int nb = post_blocks(items, (int)gridDim.x);
    if ((int)blockIdx.x >= nb) return;
    if (mode == MODE_PULL) phase_pull_hubs<W>(g, R, blockIdx.x, nb, R.post_part);
    else phase_push_commit<W>(g, R, 0, blockIdx.x, nb, R.post_part, mode == MODE_SPULL);
    __shared__ int s_last;
    wait_global_ops();
    __syncthreads();
    if (threadIdx.x == 0) s_last = last_block(R.tickets, (int)blockIdx.x, nb);
    __syncthreads();
    if (!s_last) return;
    phase_round_end<MLP ? INFER_BLOCK : INFER_NONE>(g, R, 0, g.pull_grid, R.post_part, nb);
}

// Per-node sums for reach and distance statistics: after the initialisation
// and after every round that ran, each node adds the popcount of its current
// signature.  A seed bit that u gains at round d stays, so over the states
// 0..E it is counted E - d + 1 times, and sum_i d(u, x_i) = (E + 1) reached(u)
// - sum (see k_node_stats).
template <int W> __global__ void __launch_bounds__(BLOCK) k_node_acc(GraphDev g, RunDev R0) {
    const RunDev R = group_view(R0, blockIdx.y);
    Ctrl *C = R.ctrl;
    if (!CTL(C->acc_pending)) return;
    const uint64_t *sig = sel(R.sig, CTL(C->cur));
    for (int64_t u = blockIdx.x * (int64_t)BLOCK + threadIdx.x; u < g.n; u += (int64_t)gridDim.x * BLOCK) {
        int c = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) c += __popcll(sig[u * W + w]);
        if (c) R.node_acc[u] += c;
    }
}

__global__ void __launch_bounds__(BLOCK) k_node_stats(const uint64_t *sig, const int64_t *acc, int64_t n, int W,
                                                      int64_t K, int32_t *reached, int64_t *dist_sum) {
    for (int64_t u = blockIdx.x * (int64_t)BLOCK + threadIdx.x; u < n; u += (int64_t)gridDim.x * BLOCK) {
        int c = 0;
        for (int w = 0; w < W; ++w) c += __popcll(sig[u * W + w]);
        reached[u] = c;
        dist_sum[u] = K * (int64_t)c - acc[u];
    }
}

hipError_t launch_node_stats(const uint64_t *sig, const int64_t *acc, int64_t n, int W, int64_t K, int32_t *reached,
                             int64_t *dist_sum, hipStream_t st) {
    hipLaunchKernelGGL(k_node_stats, dim3(fill_grid(n)), dim3(BLOCK), 0, st, sig, acc, n, W, K, reached, dist_sum);
    return hipGetLastError();
}

// New cost-model weights for a run in progress: the direction of the round
// about to run was taken at the end of the last one, so take it again from
// the features saved in each live control block (one wave per block).
__global__ void __launch_bounds__(64) k_redecide(RunDev R, int nctrl, int stride) {
    Ctrl *C = R.ctrl + (int64_t)blockIdx.x * stride;
    if ((int)blockIdx.x >= nctrl || R.sched != PP_SCHED_MLP) return;
    const int32_t mode = CTL(C->mode);
    if (CTL(C->round) < 1 || CTL(C->converged) || mode == MODE_INIT) return;
    float f[MLP_IN];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) f[i] = C->feat[i];
    const int32_t a = mlp_decide(R.mlp, f, allowed_actions(R, false));
    if (threadIdx.x == 0 && a >= 0) {
        int32_t fl = 0;
        C->mode = take_action(R, CTL(C->round), a, MODE_PUSH, (CTL(C->flat) >> 1) & 1, false, &fl);
        C->flat = fl;
    }
}

hipError_t launch_redecide(const RunDev &R, int nctrl, int stride, hipStream_t st) {
    if (nctrl <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_redecide, dim3(nctrl), dim3(64), 0, st, R, nctrl, stride);
    return hipGetLastError();
}

// ---------------------------------------------------------------- persistent rounds

// Barrier among the nb blocks of one cluster (block rank bid).  A cluster of
// one block only needs the block barrier.  Otherwise blocks arrive on one of
// up to eight group counters (rank i in group i % 8, matching the
// round-robin placement of blocks on the XCDs), the last of a group arrives
// on the top counter, and the last group advances the generation everyone
// waits on.  The agent-scope fences publish each block's writes before it
// arrives and make the others' writes visible after it leaves.  A wait longer
// than about ten seconds sets `abort`; every later barrier and the round loop
// then return, so the grid always drains.
PP_DEV bool cluster_barrier(GridBar *b, int bid, int nb) {
    __shared__ int s_abort;
    __syncthreads();
    if (nb == 1) return true;   // one block: nothing to wait for, and no one to time out
    if (threadIdx.x == 0) {
        const uint32_t ng = nb < 8 ? (uint32_t)nb : 8u;
        const uint32_t grp = (uint32_t)bid % ng;
        const uint32_t gsize = (uint32_t)nb / ng + (grp < (uint32_t)nb % ng ? 1u : 0u);
        int ab = CTL(b->abort);
        if (!ab) {
            const uint32_t gen = CTL(b->gen);
            __threadfence();
            if (atomicAdd(&b->grp[grp], 1u) + 1 == gsize) {
                atomicExch(&b->grp[grp], 0u);
                __threadfence();
                if (atomicAdd(&b->top, 1u) + 1 == ng) {
                    atomicExch(&b->top, 0u);
                    __threadfence();
                    atomicAdd(&b->gen, 1u);
                }
            }
            const uint64_t t0 = wall_clock64();
            while (CTL(b->gen) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (wall_clock64() - t0 > 1000000000ull) {   // ~10 s at 100 MHz
                    atomicExch(&b->abort, 1);
                    break;
                }
                if (CTL(b->abort)) break;
            }
            __threadfence();
            ab = CTL(b->abort);
        }
        s_abort = ab;
    }
    __syncthreads();
    return s_abort == 0;
}

// The slice of a batch that one cluster runs: graph cl.g as a graph of its
// own (its node range, tiles, hubs, list regions, log rows, control block).
PP_DEV void cluster_view(const GraphDev &g, const RunDev &R, const Cluster &cl, GraphDev &gv, RunDev &rv) {
    gv = g;
    gv.n0 = cl.n0;
    gv.n = cl.n1;
    gv.m = cl.m;
    gv.tiles = g.tiles + cl.t0;
    gv.ntiles = cl.t1 - cl.t0;
    gv.hub_node = g.hub_node + cl.h0;
    gv.nhubs = cl.h1 - cl.h0;
    gv.G = 1;
    gv.pull_grid = cl.nb;
    rv = R;
    rv.G = 1;
    rv.ctrl = R.ctrl + cl.g;
    rv.bar = R.bar + cl.g;
    rv.counts = R.counts + cl.g;
    rv.seed_counts = R.seed_counts ? R.seed_counts + (int64_t)cl.g * R.sg : nullptr;
    rv.D = R.D + cl.g;
    rv.gconv = R.gconv + cl.g;
    rv.mode_log = R.mode_log + (int64_t)cl.g * R.cap;
    rv.arcs_log = R.arcs_log + (int64_t)cl.g * R.cap;
    rv.phase_log = R.phase_log + (int64_t)cl.g * R.cap * 3;
    rv.feat_log = R.feat_log + (int64_t)cl.g * R.cap * MLP_IN;
    const int W = R.W;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        rv.f_ids[k] = R.f_ids[k] + cl.n0;
        rv.f_delta[k] = R.f_delta[k] + cl.n0 * W;
        rv.chunks[k] = R.chunks[k] + cl.ch0;
    }
    rv.blk_cnt = R.blk_cnt + cl.b0;
    rv.blk_nodes = R.blk_nodes + cl.b0;
    rv.blk_arcs = R.blk_arcs + cl.b0;
    rv.blk_pulled = R.blk_pulled + cl.b0;
}

// Every graph of a batch in one cooperative launch: cluster c (a range of
// co-resident blocks) runs graph clusters[c].g round after round, with
// barriers among its own blocks only, until the graph converges or its round
// passes max_round.  A graph still at round 0 is first initialised (its seed
// bits were scattered by k_seed_scatter_batch).  Every block of a cluster
// runs every phase and every barrier of its cluster; the loop condition is
// read by all of them after a barrier, so they leave together.  Rank 0 logs
// device-clock stamps per round: [start, after the main phase, end].
template <int W>
__global__ void __launch_bounds__(BLOCK) k_batch(GraphDev g, RunDev R, const Cluster *clusters, int nclusters,
                                                 int max_round) {
    int lo = 0, hi = nclusters - 1;   // cluster holding this block
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (clusters[mid].b0 <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
    }
    const Cluster cl = clusters[lo];
    const int bid = (int)blockIdx.x - cl.b0;
    const int nb = cl.nb;
    if (bid >= nb) return;   // spare block outside every cluster: never waited for
    GraphDev gv;
    RunDev rv;
    cluster_view(g, R, cl, gv, rv);
    // A cluster of one block keeps its control block in LDS for the launch:
    // every read of it in a round is then an LDS access instead of a trip to
    // the L2, and no other block reads it before the launch ends.
    __shared__ Ctrl s_ctrl;
    Ctrl *const gctrl = rv.ctrl;
    const bool local = nb == 1;
    constexpr int CTRL_WORDS = (int)(sizeof(Ctrl) / 4);
    if (local) {
        for (int i = threadIdx.x; i < CTRL_WORDS; i += BLOCK)
            reinterpret_cast<int32_t *>(&s_ctrl)[i] = reinterpret_cast<const int32_t *>(gctrl)[i];
        __syncthreads();
        rv.ctrl = &s_ctrl;
    }
    Ctrl *C = rv.ctrl;
    GridBar *bar = rv.bar;
    const bool lead = bid == 0 && threadIdx.x == 0;
    // a one-block cluster's commit hands its new-bit count and arcs to the
    // round's end through LDS, not through the graph's counter in memory
    __shared__ int64_t s_parts[3];
    int64_t *const lparts = local ? s_parts : nullptr;
    bool ok = true;
    if (CTL(C->round) == 0 && !CTL(C->converged)) {
        phase_push_commit<W, 1>(gv, rv, 1, bid, nb);
        ok = cluster_barrier(bar, bid, nb);
        if (ok && bid == 0) phase_round_end(gv, rv, 1, nb, nullptr, 0, true);
        if (ok) ok = cluster_barrier(bar, bid, nb);
    }
    while (ok) {
        const int conv = CTL(C->converged);
        const int r = CTL(C->round);
        const int mode = CTL(C->mode);
        const int prev = CTL(C->prev_mode);
        if (conv || r > max_round || (!local && CTL(bar->abort))) break;
        int64_t *stamp = r < rv.cap ? rv.phase_log + (int64_t)r * 3 : nullptr;
        if (lead && stamp) stamp[0] = (int64_t)wall_clock64();
        if (mode == MODE_PUSH) {
            if (prev == MODE_PULL) {
                phase_frontier<W, 256>(gv, rv, bid, nb);
                if (!cluster_barrier(bar, bid, nb)) break;
            }
            phase_push<W, false>(gv, rv, bid, nb);
            if (!cluster_barrier(bar, bid, nb)) break;
            if (lead && stamp) stamp[1] = (int64_t)wall_clock64();
            phase_push_commit<W, 1>(gv, rv, 0, bid, nb, lparts, false, 1);
            if (!cluster_barrier(bar, bid, nb)) break;
        } else {
            phase_pull<W>(gv, rv, bid, nb);
            if (!cluster_barrier(bar, bid, nb)) break;
            if (lead && stamp) stamp[1] = (int64_t)wall_clock64();
            if (gv.nhubs) {
                phase_pull_hubs<W>(gv, rv, bid, nb);
                if (!cluster_barrier(bar, bid, nb)) break;
            }
        }
        const bool lp = local && mode == MODE_PUSH;
        if (bid == 0) phase_round_end(gv, rv, 0, nb, lp ? lparts : nullptr, lp ? 1 : 0, true, 1);
        if (lead && stamp) stamp[2] = (int64_t)wall_clock64();
        if (!cluster_barrier(bar, bid, nb)) break;
    }
    if (local) {   // the control block back for the host and the next launch
        __syncthreads();
        for (int i = threadIdx.x; i < CTRL_WORDS; i += BLOCK)
            reinterpret_cast<int32_t *>(gctrl)[i] = reinterpret_cast<const int32_t *>(&s_ctrl)[i];
    }
}

// Seed bits for the clustered engine: like k_seed_scatter, but each graph's
// seed nodes go to its own region of list 0 and its own control block.
template <int W>
__global__ void __launch_bounds__(BLOCK) k_seed_scatter_batch(GraphDev g, RunDev R, const int32_t *seeds, int64_t total) {
    for (int64_t j = blockIdx.x * (int64_t)BLOCK + threadIdx.x; j < total; j += (int64_t)gridDim.x * BLOCK) {
        const int i = (int)(j % R.s);
        const int gi = (int)(j / R.s);
        const int32_t x = seeds[j];
        const int64_t n0 = g.node_off[gi];
        const bool ok = x >= n0 && x < g.node_off[gi + 1];
        if (!ok) atomicOr(&R.ctrl[0].bad_seed, 1);
        if (!ok) continue;
        atomicOr((unsigned long long *)&R.acc[(int64_t)x * W + (i >> 6)], 1ull << (i & 63));
        if (atomicMax(&R.stamp[x], 0) < 0) {
            const int pos = atomicAdd(&R.ctrl[gi].lst[0].nodes, 1);
            R.f_ids[0][n0 + pos] = x;
        }
    }
}

// ---------------------------------------------------------------- launchers

// blocks of a pull launch: one wave per tile, four waves per block, up to a
// cap measured per row width.  The dispatcher starts blocks in order, so many
// short-lived blocks keep the blocks in flight on neighbouring tiles and
// balance themselves; each block also costs its start and its partial sums.
// One- and two-word rows: 1024 (4096^2 grid 138.4 ms per propagation, 140.3
// at 2048); four and eight words: 2048 below 2^20 tiles (R-MAT 20, four
// words: 0.709 ms; 0.723 at 1024, 0.734 at 4096), else 32768 (R-MAT 26: with
// s = 512 a dense pull takes 19.2 ms at 2048, 18.0 at 8192, 17.4 at 32768;
// two groups of 256 seeds take 105.1 ms at 2048, 102.2 at 32768).
int pull_grid_for(int32_t ntiles, int W) {
    const int b = (ntiles + BLOCK / 64 - 1) / (BLOCK / 64);
    const int cap = W <= 2 ? PULL_GRID_MAX / 2 : (ntiles >= (1 << 20) ? 16 * PULL_GRID_MAX : PULL_GRID_MAX);
    return b < 1 ? 1 : (b < cap ? b : cap);
}

// blocks of the per-node launches (node sums), and the push launch's least
// width: one per 256 nodes, 64 to 1024
static int list_grid(const GraphDev &g) {
    const int64_t b = (g.n + BLOCK - 1) / BLOCK;
    return (int)(b < 64 ? 64 : (b > 1024 ? 1024 : b));
}

// blocks of the push and sparse-pull launches: as many as the list launches,
// and on graphs of more than 2^27 arcs one per 2^17 arcs up to 8192, since a
// push there can walk a hundred million arcs at once (R-MAT scale 26: 76.3 ->
// 67.6 ms per propagation from 1024 to 8192 blocks).  A launch that finds
// little or nothing to do costs more the more blocks it has, which is why
// smaller graphs keep the list launches' 1024 (R-MAT scale 20 lost 7% at
// 2048, the 4096^2 grid 9%).
static int push_grid(const GraphDev &g) {
    const int lg = list_grid(g);
    const int64_t by_arcs = g.m >> 17;
    return by_arcs > lg ? (int)(by_arcs < 8192 ? by_arcs : 8192) : lg;
}

static_assert(TICKET_GROUP * TICKET_GROUP >= POST_MAX, "the closing launch's ticket covers its blocks");
// blocks of the closing launch: a push round's commit lists up to n nodes,
// but a launch of many blocks that mostly find nothing to do costs time in
// every round; one block per 4096 nodes, 64 to POST_MAX
static int post_grid(const GraphDev &g) {
    const int64_t b = (g.n + 4095) / 4096;
    return (int)(b < 64 ? 64 : (b > POST_MAX ? POST_MAX : b));
}

// seed lists up to this length initialise in one single-block launch
constexpr int64_t SEED_INIT_ONE_BLOCK = 4096;

template <int W>
static hipError_t seed_init_impl(const GraphDev &g, const RunDev &R, const int32_t *seeds, const int32_t *map,
                                 hipStream_t st) {
    const int64_t total = (int64_t)R.G * R.sg;   // seeds of the largest group
    const unsigned ng = (unsigned)R.ngroups;
    if (total <= SEED_INIT_ONE_BLOCK) {
        hipLaunchKernelGGL(k_seed_init<W>, dim3(1, ng), dim3(BLOCK), 0, st, g, R, seeds, map);
        if (R.node_acc) hipLaunchKernelGGL(k_node_acc<W>, dim3(list_grid(g), ng), dim3(BLOCK), 0, st, g, R);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_seed_scatter<W>, dim3(fill_grid(total), ng), dim3(BLOCK), 0, st, g, R, seeds, map);
    hipLaunchKernelGGL(k_push_commit<W>, dim3(fill_grid(total * W), ng), dim3(BLOCK), 0, st, g, R, 1);
    hipLaunchKernelGGL(k_round_end, dim3(1, ng), dim3(BLOCK), 0, st, g, R, 1);
    if (R.node_acc) hipLaunchKernelGGL(k_node_acc<W>, dim3(list_grid(g), ng), dim3(BLOCK), 0, st, g, R);
    return hipGetLastError();
}

template <int W>
static hipError_t round_impl(const GraphDev &g, const RunDev &R, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                             int kinds) {
    if (kinds == SPARSE_BY_RUN) kinds = R.sparse_pull == 0 ? SPARSE_PUSH : (R.sparse_pull == 1 ? SPARSE_PULL : SPARSE_BOTH);
    if (e0) {
        const hipError_t e = hipEventRecord(e0, st);
        if (e != hipSuccess) return e;
    }
    const unsigned ng = (unsigned)R.ngroups;   // every launch covers every seed group (blockIdx.y)
    // the pull's form for this graph: short lists only, rows of nodes without
    // successors left alone, or the general one
    bool short_form = false;
    if constexpr (W <= 2) short_form = g.short_lists && R.pull_k != 2;
    if (short_form) {
        if constexpr (W <= 2) hipLaunchKernelGGL(k_pull_short<W>, dim3(g.pull_grid, ng), dim3(BLOCK), 0, st, g, R);
    } else if (R.pull_k == 2) {
        hipLaunchKernelGGL((k_pull<W, 2>), dim3(g.pull_grid, ng), dim3(BLOCK), 0, st, g, R);
    } else if (g.skip_dead) {
        hipLaunchKernelGGL((k_pull<W, 0, true>), dim3(g.pull_grid, ng), dim3(BLOCK), 0, st, g, R);
    } else {
        hipLaunchKernelGGL((k_pull<W, 0>), dim3(g.pull_grid, ng), dim3(BLOCK), 0, st, g, R);
    }
    if (e1) {
        const hipError_t e = hipEventRecord(e1, st);
        if (e != hipSuccess) return e;
    }
    if (kinds & SPARSE_PUSH) hipLaunchKernelGGL(k_push<W>, dim3(push_grid(g), ng), dim3(BLOCK), 0, st, g, R);
    if (kinds & SPARSE_PULL) hipLaunchKernelGGL(k_spull<W>, dim3(push_grid(g), ng), dim3(BLOCK), 0, st, g, R);
    if (R.sched == PP_SCHED_MLP) hipLaunchKernelGGL((k_post<W, true>), dim3(post_grid(g), ng), dim3(BLOCK), 0, st, g, R);
    else hipLaunchKernelGGL((k_post<W, false>), dim3(post_grid(g), ng), dim3(BLOCK), 0, st, g, R);
    if (R.node_acc) hipLaunchKernelGGL(k_node_acc<W>, dim3(list_grid(g), ng), dim3(BLOCK), 0, st, g, R);
    return hipGetLastError();
}

hipError_t launch_seed_init(const GraphDev &g, const RunDev &R, const int32_t *seeds, const int32_t *map,
                            hipStream_t st) {
    switch (R.W) {
        case 1: return seed_init_impl<1>(g, R, seeds, map, st);
        case 2: return seed_init_impl<2>(g, R, seeds, map, st);
        case 4: return seed_init_impl<4>(g, R, seeds, map, st);
        case 8: return seed_init_impl<8>(g, R, seeds, map, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_round(const GraphDev &g, const RunDev &R, hipStream_t st, hipEvent_t e0, hipEvent_t e1, int kinds) {
    switch (R.W) {
        case 1: return round_impl<1>(g, R, st, e0, e1, kinds);
        case 2: return round_impl<2>(g, R, st, e0, e1, kinds);
        case 4: return round_impl<4>(g, R, st, e0, e1, kinds);
        case 8: return round_impl<8>(g, R, st, e0, e1, kinds);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pp

namespace pp {

template <int W> static const void *batch_fn() { return reinterpret_cast<const void *>(&k_batch<W>); }

static const void *batch_kernel(int W) {
    switch (W) {
        case 1: return batch_fn<1>();
        case 2: return batch_fn<2>();
        case 4: return batch_fn<4>();
        default: return batch_fn<8>();
    }
}

int persistent_grid(int W) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_kernel(W), BLOCK, 0) != hipSuccess) return 0;
    if (per > 4) per = 4;
    return per * cus;
}

hipError_t launch_batch_persistent(const GraphDev &g, const RunDev &R, const Cluster *clusters, int nclusters,
                                   int grid, int max_round, hipStream_t st) {
    GraphDev gg = g;
    RunDev rr = R;
    const Cluster *cc = clusters;
    int nc = nclusters;
    int mr = max_round;
    void *args[] = {&gg, &rr, &cc, &nc, &mr};
    return hipLaunchCooperativeKernel(batch_kernel(R.W), dim3(grid), dim3(BLOCK), args, 0, st);
}

template <int W> static hipError_t scatter_batch_impl(const GraphDev &g, const RunDev &R, const int32_t *seeds, hipStream_t st) {
    const int64_t total = (int64_t)R.G * R.s;
    hipLaunchKernelGGL(k_seed_scatter_batch<W>, dim3(fill_grid(total)), dim3(BLOCK), 0, st, g, R, seeds, total);
    return hipGetLastError();
}

hipError_t launch_seed_scatter_batch(const GraphDev &g, const RunDev &R, const int32_t *seeds, hipStream_t st) {
    switch (R.W) {
        case 1: return scatter_batch_impl<1>(g, R, seeds, st);
        case 2: return scatter_batch_impl<2>(g, R, seeds, st);
        case 4: return scatter_batch_impl<4>(g, R, seeds, st);
        case 8: return scatter_batch_impl<8>(g, R, seeds, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pp
