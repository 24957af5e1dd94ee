// PROPAGATE-S (Algorithm 2) on gfx950 (wave64): the seeds one at a time with
// one bit per node, k seeds side by side.
//
// Each of the k seeds in flight owns a pair of n-bit signatures (node u is
// bit u & 63 of word u >> 6).  Pass r reads buffer (r-1) & 1 and writes
// buffer r & 1 in full, so the update is synchronous.  A wave takes a word of
// 64 nodes of one seed, one node per lane: a node not reached yet walks its
// successor list and stops at the first successor already reached (the
// algorithm's early break); one ballot gives the word's new bits.  A lane
// walks a short list itself, four arcs per step.  Nodes with more than
// SEQ_LIGHT successors (listed once per graph) are left to a second launch
// in which a group of 32 lanes takes one such node and walks its list 128
// arcs per step up to the first step with a hit, so a hub costs one group,
// not the word that holds it.  Each pass counts, per seed, the nodes it found and
// the arcs it examined (up to and including the first hit of each node); a
// seed is done at its first pass that finds nothing.
#include <mutex>

#include "pp_internal.h"

namespace pp {

#define PS_DEV __device__ __forceinline__

namespace {

PS_DEV int lane() { return __lane_id(); }

PS_DEV bool reached(const uint64_t *sig, int32_t v) { return (sig[v >> 6] >> (v & 63)) & 1ull; }

PS_DEV uint64_t *buffer(const SeqDev &S, int b, int j) {
    return S.bits + ((int64_t)(b & 1) * S.k + j) * S.nw;
}

template <typename T> PS_DEV T block_total(T v, T *scratch) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if (lane() == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    T t = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) t += scratch[w];
    return t;
}

}  // namespace

// Seed j of the batch (kk of them) starts with its own bit; slots kk..k-1
// are idle.  Buffer 0 of every slot was cleared before.
__global__ void __launch_bounds__(BLOCK) k_seq_seeds(SeqDev S, const int32_t *seeds, int kk) {
    for (int j = blockIdx.x * BLOCK + threadIdx.x; j < S.k; j += gridDim.x * BLOCK) {
        S.done[j] = j < kk ? 0 : 1;
        S.dpass[j] = 0;
        S.examined[j] = 0;
        S.pass_cnt[j] = 0;
        if (j < kk) {
            const int32_t x = seeds[j];
            buffer(S, 0, j)[x >> 6] |= 1ull << (x & 63);
        }
        if (j == 0) S.active[0] = kk;
    }
}

// Pass r, nodes with short lists, of every seed still running (grid: blocks
// per seed x k).  Writes every word of the next signature.
__global__ void __launch_bounds__(BLOCK) k_seq_pass(GraphDev g, SeqDev S, int r) {
    const int j = blockIdx.y;
    if (S.done[j]) return;   // the same for the whole block
    const uint64_t *cur = buffer(S, r - 1, j);
    uint64_t *nxt = buffer(S, r, j);
    const int ln = lane();
    const int64_t wave = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (BLOCK / 64);
    int64_t found = 0, exam = 0;
    for (int64_t wd = wave; wd < S.nw; wd += nwaves) {   // wave-uniform
        const uint64_t word = cur[wd];
        const int64_t u = wd * 64 + ln;
        const bool open = u < g.n && !((word >> ln) & 1ull);
        int64_t b = 0, e = 0;
        if (open) {
            b = g.rp[u];
            e = g.rp[u + 1];
        }
        bool hit = false;
        if (open && e - b <= SEQ_LIGHT) {   // longer lists: k_seq_heavy
            // the lane's own list, four arcs in flight per step
            for (int64_t a = b; a < e && !hit; a += 4) {
                int32_t v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = a + q < e ? g.col[a + q] : -1;
                bool t[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) t[q] = v[q] >= 0 && reached(cur, v[q]);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (!hit && v[q] >= 0) {
                        ++exam;
                        hit = t[q];
                    }
                }
            }
        }
        const uint64_t nb = __ballot(hit);
        if (ln == 0) {
            nxt[wd] = word | nb;
            found += __popcll(nb);
        }
    }
    __shared__ long long s_red[BLOCK / 64];
    const long long tf = block_total<long long>(found, s_red);
    const long long te = block_total<long long>(exam, s_red);
    if (threadIdx.x == 0) {
        if (tf) atomicAdd((unsigned long long *)&S.pass_cnt[j], (unsigned long long)tf);
        if (te) atomicAdd((unsigned long long *)&S.examined[j], (unsigned long long)te);
    }
}

// Pass r, nodes with long lists (heavy[0..nheavy), stored ids): a group of
// 32 lanes per node, two nodes per wave, each lane four arcs per step (128
// arcs per node and step, in arc order); a hit sets the node's bit in the
// next signature (written by k_seq_pass before, in stream order).  R-MAT 20,
// 256 seeds: 25.3 ms per propagation with 32 lanes, 27.4 with 16, 34.1 with
// 8, 27.5 with 64.
__global__ void __launch_bounds__(BLOCK) k_seq_heavy(GraphDev g, SeqDev S, const int32_t *heavy, int64_t nheavy,
                                                    int r) {
    constexpr int GL = 32;                 // lanes per node
    constexpr int GW = 64 / GL;            // nodes per wave
    const int j = blockIdx.y;
    if (S.done[j]) return;   // the same for the whole block
    const uint64_t *cur = buffer(S, r - 1, j);
    uint64_t *nxt = buffer(S, r, j);
    const int ln = lane();
    const int grp = ln / GL, sub = ln % GL;
    const uint64_t gmask = GL == 64 ? ~0ull : (((1ull << (GL & 63)) - 1) << (grp * GL));
    const int64_t wave = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (BLOCK / 64);
    int64_t found = 0, exam = 0;
    for (int64_t h0 = wave * GW; h0 < nheavy; h0 += nwaves * GW) {   // wave-uniform
        const int64_t h = h0 + grp;
        int32_t u = 0;
        bool open = false;
        int64_t b = 0, e = 0;
        if (h < nheavy) {
            u = heavy[h];
            open = !reached(cur, u);
            if (open) {
                b = g.rp[u];
                e = g.rp[u + 1];
            }
        }
        bool hit = false;     // the same in every lane of a group
        int64_t ex = 0;
        for (int64_t a0 = b; __ballot(open && !hit && a0 < e); a0 += 4 * GL) {   // wave-uniform condition
            const bool go = open && !hit && a0 < e;
            bool t[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t a = a0 + q * GL + sub;
                t[q] = go && a < e && reached(cur, g.col[a]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint64_t m = (__ballot(t[q]) & gmask) >> (grp * GL);
                if (go && !hit) {
                    if (m) {
                        hit = true;
                        ex += __ffsll((long long)m);   // this chunk's arcs up to the first hit, in arc order
                    } else {
                        const int64_t left = e - (a0 + q * GL);
                        ex += left <= 0 ? 0 : (left < GL ? left : GL);
                    }
                }
            }
        }
        if (sub == 0) {   // one lane per group counts and sets the bit
            exam += ex;
            if (hit) {
                ++found;
                atomicOr((unsigned long long *)&nxt[u >> 6], 1ull << (u & 63));
            }
        }
    }
    __shared__ long long s_red[BLOCK / 64];
    const long long tf = block_total<long long>(found, s_red);
    const long long te = block_total<long long>(exam, s_red);
    if (threadIdx.x == 0) {
        if (tf) atomicAdd((unsigned long long *)&S.pass_cnt[j], (unsigned long long)tf);
        if (te) atomicAdd((unsigned long long *)&S.examined[j], (unsigned long long)te);
    }
}

// After pass r: a seed whose pass found nothing is done; otherwise r is its
// last pass so far with a find.  A seed still running at the last pass the
// log holds is stopped and counted as not converged.
// The pass's finds are summed into sum_cnt[r].
__global__ void __launch_bounds__(BLOCK) k_seq_end(SeqDev S, int r) {
    long long sum = 0;
    for (int j = blockIdx.x * BLOCK + threadIdx.x; j < S.k; j += gridDim.x * BLOCK) {
        if (S.done[j]) continue;
        const int64_t c = S.pass_cnt[j];
        S.pass_cnt[j] = 0;
        sum += c;
        if (c == 0) {
            S.done[j] = 1;
            atomicSub(S.active, 1);
        } else {
            S.dpass[j] = r;
            if (r + 1 >= S.cap) {
                S.done[j] = 2;
                atomicSub(S.active, 1);
            }
        }
    }
    __shared__ long long s_red[BLOCK / 64];
    const long long t = block_total<long long>(sum, s_red);
    if (threadIdx.x == 0 && t) atomicAdd((unsigned long long *)&S.sum_cnt[r], (unsigned long long)t);
}

// The fixed device region of pp_propagate_s_noalloc: PROPAGATE-S's buffers
// for callers that cannot allocate.  Every device the library runs on holds
// its own copy, at its own address, until the process ends.  Host code never
// passes the array's name to a kernel (on the host it only stands for the
// symbol): it takes the device address from hipGetSymbolAddress once per
// device and passes that.
static __device__ __align__(256) unsigned char scratch[PP_NOALLOC_BYTES];

namespace {
constexpr int MAX_DEVICES = 256;
std::mutex &region_mu() {
    static std::mutex *m = new std::mutex();   // lives until the process ends
    return *m;
}
void *g_region[MAX_DEVICES];   // device address of `scratch` per device (NULL: not looked up yet)
}  // namespace

int noalloc_region(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(PP_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return set_error(PP_EDEVICE, "device %d beyond the %d the library tracks", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lk(region_mu());
    if (!g_region[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return set_error(PP_EDEVICE, "address of the fixed region on device %d: %s", dev, hipGetErrorString(e));
        g_region[dev] = ptr;
    }
    *out = g_region[dev];
    return PP_OK;
}

static int small_grid(int64_t items) {
    const int64_t b = (items + BLOCK - 1) / BLOCK;
    return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

hipError_t launch_seq_seeds(const SeqDev &S, const int32_t *seeds, int kk, hipStream_t st) {
    hipLaunchKernelGGL(k_seq_seeds, dim3(small_grid(S.k)), dim3(BLOCK), 0, st, S, seeds, kk);
    return hipGetLastError();
}

hipError_t launch_seq_pass(const GraphDev &g, const SeqDev &S, const int32_t *heavy, int64_t nheavy, int r,
                           int blocks_per_seed, int heavy_blocks_per_seed, hipStream_t st) {
    hipLaunchKernelGGL(k_seq_pass, dim3(blocks_per_seed, S.k), dim3(BLOCK), 0, st, g, S, r);
    if (nheavy > 0)
        hipLaunchKernelGGL(k_seq_heavy, dim3(heavy_blocks_per_seed, S.k), dim3(BLOCK), 0, st, g, S, heavy, nheavy, r);
    hipLaunchKernelGGL(k_seq_end, dim3(small_grid(S.k)), dim3(BLOCK), 0, st, S, r);
    return hipGetLastError();
}

}  // namespace pp
