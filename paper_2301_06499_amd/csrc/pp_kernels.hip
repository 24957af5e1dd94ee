// HIP kernels for PROPAGATE-P rounds on gfx950 (wave64).
//
// One round r (Algorithm 1's do-while body) is four launches that hand work
// to each other through the device control block, so a round needs no host
// decision and a batch of rounds can be replayed as a captured graph:
//
//   k_pull<W>       dense pull: for every node u, OR the rows of u's
//                   successors (the ball recurrence of Section 4) into an LDS
//                   accumulator; nodes whose accumulated bits are not all in
//                   Sig(u) are appended to frontier list r&1 with their new
//                   bits.  Sig is only read, so the update is synchronous.
//   k_push<W>       sparse push: for every predecessor u of a node v that
//                   changed in round r-1, atomically OR v's new bits of round
//                   r-1 into Sig(u); bits u did not have are collected in the
//                   accumulator and u is queued once.  Only new bits of round
//                   r-1 can produce new bits in round r (every older bit of v
//                   already reached u), so this equals the pull.
//   k_commit<W>     applies (pull) or collects (push) the new bits of the
//                   frontier entries, counts them (c[r] = popcount of the new
//                   bits, Algorithm 1's XOR count), optionally per seed with
//                   wave ballots, and prepares the push chunks for round r+1.
//   k_round_end     convergence (a graph converges at its first round with no
//                   new bit), diameter bookkeeping, the per-round log, and the
//                   direction of round r+1.
//
// Whichever of pull/push is not selected returns at once.
#include "pp_internal.h"

namespace pp {

#define PP_DEV __device__ __forceinline__

PP_DEV int lane_id() { return __lane_id(); }

template <int W> struct WordMask {
    // lanes holding word w of a row when W consecutive lanes share a row
    static constexpr uint64_t rep = ~0ull / ((W == 64) ? ~0ull : ((1ull << W) - 1));
    static constexpr uint64_t row = (W == 64) ? ~0ull : ((1ull << W) - 1);
};

PP_DEV uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

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

template <int W> PP_DEV void flush_lds(unsigned long long *dst, uint64_t (&acc)[W]) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
        if (acc[w]) atomicOr(dst + w, (unsigned long long)acc[w]);
        acc[w] = 0;
    }
}

// ---------------------------------------------------------------- fills

__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static int fill_grid(int64_t count) {
    int64_t b = (count + BLOCK - 1) / BLOCK;
    return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t v, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(count)), dim3(BLOCK), 0, st, p, v, count);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(count)), dim3(BLOCK), 0, st, p, v, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------- seeds

// Seed bit i of graph g goes to node seeds[g*s + i] (Algorithm 1's
// initialisation).  Bits are gathered in the accumulator first so that a node
// holding several seeds is queued once; the INIT commit then writes them.
template <int W>
__global__ void __launch_bounds__(BLOCK) k_seed_scatter(RunDev R, const int32_t *seeds, int64_t total) {
    for (int64_t j = blockIdx.x * (int64_t)BLOCK + threadIdx.x; j < total; j += (int64_t)gridDim.x * BLOCK) {
        const int i = (int)(j % R.s);
        const int32_t x = seeds[j];
        atomicOr((unsigned long long *)&R.acc[(int64_t)x * W + (i >> 6)], 1ull << (i & 63));
        const bool want = atomicMax(&R.stamp[x], 0) < 0;
        const int pos = wave_append(&R.ctrl->f_count[0], want);
        if (want) R.f_ids[0][pos] = x;
    }
}

// ---------------------------------------------------------------- pull

template <int W>
__global__ void __launch_bounds__(BLOCK) k_pull(GraphDev g, RunDev R) {
    Ctrl *C = R.ctrl;
    if (C->converged || C->mode != MODE_PULL) return;
    constexpr int K = PullShape<W>::K;
    constexpr int EDGES = PullShape<W>::EDGES;
    __shared__ int32_t s_col[EDGES];
    __shared__ int32_t s_rp[TILE_NODES + 1];
    __shared__ unsigned long long s_acc[TILE_NODES * W];
    __shared__ int s_last;
    const int r = C->round;
    const int p = r & 1;
    const int tid = threadIdx.x;
    const int ln = lane_id();
    int64_t arcs_done = 0;

    for (int t = blockIdx.x; t < g.ntiles; t += gridDim.x) {
        const Tile T = g.tiles[t];
        if (R.G > 1 && R.gconv[T.graph]) continue;  // same for the whole block
        const int nn = T.u1 - T.u0;
        const int ne = (int)(T.e1 - T.e0);
        const bool hub = T.hub >= 0;
        for (int i = tid; i <= nn; i += BLOCK)
            s_rp[i] = hub ? (i == 0 ? 0 : ne) : (int)(g.rp[T.u0 + i] - T.e0);
        for (int i = tid; i < ne; i += BLOCK) s_col[i] = g.col[T.e0 + i];
        for (int i = tid; i < nn * W; i += BLOCK) s_acc[i] = 0ull;
        __syncthreads();

        // gather: thread tid ORs the rows of arcs [a, a+K) into its running
        // accumulator and flushes it to the LDS row of each node it leaves
        const int a = tid * K;
        if (a < ne) {
            const int b = min(a + K, ne);
            int lo = 0, hi = nn - 1;          // node i with s_rp[i] <= a < s_rp[i+1]
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_rp[mid] <= a) lo = mid; else hi = mid - 1;
            }
            int i = lo;
            uint64_t rows[K][W];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                if (a + j < b) {
                    load_row<W>(R.sig + (int64_t)s_col[a + j] * W, rows[j]);
                } else {
#pragma unroll
                    for (int w = 0; w < W; ++w) rows[j][w] = 0;
                }
            }
            uint64_t acc[W];
#pragma unroll
            for (int w = 0; w < W; ++w) acc[w] = 0;
            int nxt = s_rp[i + 1];
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int e = a + j;
                if (e < b) {
                    while (e >= nxt) {
                        flush_lds<W>(s_acc + i * W, acc);
                        ++i;
                        nxt = s_rp[i + 1];
                    }
#pragma unroll
                    for (int w = 0; w < W; ++w) acc[w] |= rows[j][w];
                }
            }
            flush_lds<W>(s_acc + i * W, acc);
        }
        arcs_done += ne;
        __syncthreads();

        bool finalize = true;
        if (hub) {
            // combine the chunks of a high-degree node; the last one finishes it
            if (tid < W && s_acc[tid]) atomicOr((unsigned long long *)&R.hub_acc[(int64_t)T.hub * W + tid], s_acc[tid]);
            __threadfence();
            __syncthreads();
            if (tid == 0) {
                const uint32_t prev = atomicAdd(&R.hub_done[T.hub], 1u);
                s_last = (int)(prev + 1 == (uint32_t)g.hub_nchunks[T.hub]);
            }
            __syncthreads();
            finalize = s_last != 0;
            if (finalize) {
                __threadfence();
                if (tid < W) s_acc[tid] = atomicExch((unsigned long long *)&R.hub_acc[(int64_t)T.hub * W + tid], 0ull);
                if (tid == 0) atomicExch(&R.hub_done[T.hub], 0u);
                __syncthreads();
            }
        }
        if (finalize) {
            for (int idx0 = 0; idx0 < nn * W; idx0 += BLOCK) {   // same trip count for all lanes
                const int idx = idx0 + tid;
                const bool valid = idx < nn * W;
                uint64_t nw = 0;
                int32_t u = 0;
                if (valid) {
                    u = T.u0 + idx / W;
                    const uint64_t av = s_acc[idx];
                    if (av) nw = av & ~R.sig[(int64_t)u * W + (idx & (W - 1))];
                }
                const uint64_t bal = __ballot(nw != 0);
                const int gb = ln & ~(W - 1);
                const bool changed = valid && ((bal >> gb) & WordMask<W>::row) != 0;
                const bool leader = changed && ((ln & (W - 1)) == 0);
                int pos = wave_append(&C->f_count[p], leader);
                pos = __shfl(pos, gb);
                if (changed) {
                    if (leader) R.f_ids[p][pos] = u;
                    R.f_delta[p][(int64_t)pos * W + (ln & (W - 1))] = nw;
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0 && arcs_done) atomicAdd((unsigned long long *)&C->pull_arcs, (unsigned long long)arcs_done);
}

// ---------------------------------------------------------------- push

template <int W>
__global__ void __launch_bounds__(BLOCK) k_push(GraphDev g, RunDev R) {
    Ctrl *C = R.ctrl;
    if (C->converged || C->mode != MODE_PUSH) return;
    constexpr int P = 4;            // slots per chunk
    constexpr int L = W * P;        // lanes per chunk
    constexpr int GPW = 64 / L;     // chunks per wave
    const int r = C->round;
    const int pp = (r - 1) & 1, pn = r & 1;
    const int32_t nch = C->ch_count[pp];
    const Chunk *ch = R.chunks[pp];
    const int32_t *ids = R.f_ids[pp];
    const uint64_t *dl = R.f_delta[pp];
    const int ln = lane_id();
    const int grp = ln / L, sub = ln % L, w = sub % W, slot = sub / W;
    const int64_t wave = (blockIdx.x * (int64_t)BLOCK + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * BLOCK) >> 6;
    for (int64_t c0 = wave * GPW; c0 < nch; c0 += nwaves * GPW) {   // wave-uniform loop
        const int64_t c = c0 + grp;
        const bool cv = c < nch;
        int64_t b = 0, end = 0;
        uint64_t d = 0;
        if (cv) {
            const Chunk cd = ch[c];
            const int32_t v = ids[cd.entry];
            d = dl[(int64_t)cd.entry * W + w];
            b = g.trp[v] + cd.off;
            const int64_t lim = g.trp[v + 1];
            end = (b + PUSH_CHUNK < lim) ? b + PUSH_CHUNK : lim;
        }
#pragma unroll
        for (int it = 0; it < PUSH_CHUNK / P; ++it) {
            const int64_t k = b + slot + it * P;
            const bool kv = cv && k < end;
            int32_t u = 0;
            uint64_t nb = 0;
            if (kv) {
                u = g.tcol[k];
                if (d) {
                    const uint64_t old = atomicOr((unsigned long long *)&R.sig[(int64_t)u * W + w], (unsigned long long)d);
                    nb = d & ~old;
                    if (nb) atomicOr((unsigned long long *)&R.acc[(int64_t)u * W + w], (unsigned long long)nb);
                }
            }
            const uint64_t bal = __ballot(nb != 0);
            const int gb = ln & ~(W - 1);
            const bool any = kv && ((bal >> gb) & WordMask<W>::row) != 0;
            bool want = false;
            if (any && (ln & (W - 1)) == 0) want = atomicMax(&R.stamp[u], r) < r;
            const int pos = wave_append(&C->f_count[pn], want);
            if (want) R.f_ids[pn][pos] = u;
        }
    }
}

// ---------------------------------------------------------------- commit

template <int W>
__global__ void __launch_bounds__(BLOCK) k_commit(GraphDev g, RunDev R, int init) {
    Ctrl *C = R.ctrl;
    if (C->converged) return;
    const int r = init ? 0 : C->round;
    const int p = r & 1;
    const int mode = init ? MODE_INIT : C->mode;
    const int32_t cnt = C->f_count[p];
    const int64_t items = (int64_t)cnt * W;
    int32_t *ids = R.f_ids[p];
    uint64_t *dl = R.f_delta[p];
    Chunk *chunks = R.chunks[p];
    const int ln = lane_id();
    const int w = ln & (W - 1);
    const bool per_seed = R.seed_counts != nullptr;
    uint64_t pop = 0;
    int64_t arcs = 0;
    uint32_t sc[W];
#pragma unroll
    for (int k = 0; k < W; ++k) sc[k] = 0;
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    for (int64_t base = blockIdx.x * (int64_t)BLOCK + (threadIdx.x & ~63); base < items; base += stride) {
        const int64_t idx = base + ln;
        const bool valid = idx < items;
        const int64_t e = idx / W;
        uint64_t d = 0;
        int32_t u = 0;
        if (valid) {
            u = ids[e];
            uint64_t *sp = R.sig + (int64_t)u * W + w;
            if (mode == MODE_PULL) {
                d = dl[idx];
                *sp |= d;
            } else {
                uint64_t *ap = R.acc + (int64_t)u * W + w;
                d = *ap;
                *ap = 0;
                dl[idx] = d;
                if (mode == MODE_INIT) *sp |= d;
            }
        }
        const int pc = __popcll(d);
        int gi = 0;
        if (R.G == 1) {
            pop += (uint64_t)pc;
        } else if (valid) {
            gi = g.node_graph[u];
            if (pc) atomicAdd((unsigned long long *)&R.counts[(int64_t)r * R.G + gi], (unsigned long long)pc);
        }
        // push chunks of this entry for round r+1 (one slot block per wave)
        int nchk = 0;
        if (valid && w == 0) {
            const int64_t deg = g.trp[u + 1] - g.trp[u];
            nchk = (int)((deg + PUSH_CHUNK - 1) / PUSH_CHUNK);
            arcs += deg;
        }
        const int incl = wave_inclusive_scan(nchk);
        const int total = __shfl(incl, 63);
        if (total) {
            int cbase = 0;
            if (ln == 0) cbase = atomicAdd(&C->ch_count[p], total);
            cbase = __shfl(cbase, 0);
            const int first = cbase + incl - nchk;
            for (int j = 0; j < nchk; ++j) chunks[first + j] = Chunk{(int32_t)e, j * PUSH_CHUNK};
        }
        if (per_seed) {
            if (R.G == 1) {
                if (__ballot(d != 0)) {
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
            } else if (valid) {
                uint64_t x = d;
                while (x) {
                    const int bit = __ffsll((long long)x) - 1;
                    x &= x - 1;
                    atomicAdd(&R.seed_counts[((int64_t)r * R.G + gi) * R.s + w * 64 + bit], 1u);
                }
            }
        }
    }
    __shared__ unsigned long long s_red[2][BLOCK / 64];
    pop = wave_sum(pop);
    uint64_t ua = wave_sum((uint64_t)arcs);
    const int wv = threadIdx.x >> 6;
    if (ln == 0) {
        s_red[0][wv] = pop;
        s_red[1][wv] = ua;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tp = 0, ta = 0;
        for (int k = 0; k < BLOCK / 64; ++k) {
            tp += s_red[0][k];
            ta += s_red[1][k];
        }
        if (R.G == 1 && tp) atomicAdd((unsigned long long *)&R.counts[r], tp);
        if (ta) atomicAdd((unsigned long long *)&C->f_arcs[p], ta);
    }
    if (per_seed && R.G == 1) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int bitidx = k * 64 + ln;
            if (sc[k] && bitidx < R.s) atomicAdd(&R.seed_counts[(int64_t)r * R.s + bitidx], sc[k]);
        }
    }
}

// ---------------------------------------------------------------- round end

PP_DEV int32_t schedule(const GraphDev &g, const RunDev &R, int32_t r, int32_t fcount, int64_t farcs) {
    switch (R.sched) {
        case PP_SCHED_PULL: return MODE_PULL;
        case PP_SCHED_PUSH: return MODE_PUSH;
        case PP_SCHED_FUZZ:
            return (mix64(R.fuzz_seed + (uint64_t)r * 0x9E3779B97F4A7C15ull) >> 63) ? MODE_PUSH : MODE_PULL;
        default:
            (void)fcount;
            return (farcs * (int64_t)R.push_div < g.m) ? MODE_PUSH : MODE_PULL;
    }
}

__global__ void k_round_end(GraphDev g, RunDev R, int init) {
    Ctrl *C = R.ctrl;
    if (C->converged) return;
    const int r = init ? 0 : C->round;
    __shared__ int s_active;
    if (threadIdx.x == 0) s_active = 0;
    __syncthreads();
    int act = 0;
    for (int gi = threadIdx.x; gi < R.G; gi += blockDim.x) {
        if (R.gconv[gi]) continue;
        if (R.counts[(int64_t)r * R.G + gi] == 0) {
            R.gconv[gi] = 1;
        } else {
            R.D[gi] = r;
            ++act;
        }
    }
    if (act) atomicAdd(&s_active, act);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int mode = init ? MODE_INIT : C->mode;
        R.mode_log[r] = mode;
        R.arcs_log[r] = init ? 0 : (mode == MODE_PULL ? C->pull_arcs : C->f_arcs[(r - 1) & 1]);
        C->pull_arcs = 0;
        C->active = s_active;
        if (s_active == 0) {
            C->converged = 1;
        } else if (r + 1 >= R.cap) {
            C->converged = 1;
            C->overflow = 1;
        } else {
            const int nr = r + 1, q = nr & 1;
            C->f_count[q] = 0;
            C->ch_count[q] = 0;
            C->f_arcs[q] = 0;
            C->mode = schedule(g, R, nr, C->f_count[r & 1], C->f_arcs[r & 1]);
            C->round = nr;
        }
    }
}

// ---------------------------------------------------------------- launchers

int pull_grid(const GraphDev &g) {
    const int cap = 256 * 8;
    return g.ntiles < 1 ? 1 : (g.ntiles < cap ? g.ntiles : cap);
}

template <int W> static hipError_t seed_init_impl(const GraphDev &g, const RunDev &R, const int32_t *seeds, hipStream_t st) {
    const int64_t total = (int64_t)R.G * R.s;
    hipLaunchKernelGGL(k_seed_scatter<W>, dim3(fill_grid(total)), dim3(BLOCK), 0, st, R, seeds, total);
    hipLaunchKernelGGL(k_commit<W>, dim3(fill_grid(total * W)), dim3(BLOCK), 0, st, g, R, 1);
    hipLaunchKernelGGL(k_round_end, dim3(1), dim3(256), 0, st, g, R, 1);
    return hipGetLastError();
}

template <int W> static hipError_t round_impl(const GraphDev &g, const RunDev &R, hipStream_t st) {
    hipLaunchKernelGGL(k_pull<W>, dim3(pull_grid(g)), dim3(BLOCK), 0, st, g, R);
    hipLaunchKernelGGL(k_push<W>, dim3(1024), dim3(BLOCK), 0, st, g, R);
    hipLaunchKernelGGL(k_commit<W>, dim3(1024), dim3(BLOCK), 0, st, g, R, 0);
    hipLaunchKernelGGL(k_round_end, dim3(1), dim3(256), 0, st, g, R, 0);
    return hipGetLastError();
}

hipError_t launch_seed_init(const GraphDev &g, const RunDev &R, const int32_t *seeds, hipStream_t st) {
    switch (R.W) {
        case 1: return seed_init_impl<1>(g, R, seeds, st);
        case 2: return seed_init_impl<2>(g, R, seeds, st);
        case 4: return seed_init_impl<4>(g, R, seeds, st);
        case 8: return seed_init_impl<8>(g, R, seeds, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_round(const GraphDev &g, const RunDev &R, hipStream_t st) {
    switch (R.W) {
        case 1: return round_impl<1>(g, R, st);
        case 2: return round_impl<2>(g, R, st);
        case 4: return round_impl<4>(g, R, st);
        case 8: return round_impl<8>(g, R, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pp
