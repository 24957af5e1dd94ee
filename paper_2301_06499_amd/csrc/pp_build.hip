// Adjacency build on the device (Section 3's graph, as Algorithm 1 reads it):
// the successor rows of the arcs -- self-loops and duplicate arcs removed,
// each row sorted -- and their transpose, from arcs already in device memory.
//
// Each arc u -> v becomes one 64-bit key (u << shift | v), with shift the bit
// width of n, so that a radix sort of the keys' low 2 shift bits orders them
// by row, then by column; equal neighbours are then duplicates, and the row
// boundaries give the row offsets.  A self-loop becomes the key of all ones
// in those bits, above every arc's key (the largest id is below 2^shift - 1),
// which sorts last and is dropped.  The storage order (hub-first, chosen on
// the host from the degrees this file counts) is applied by relabelling the
// sorted keys and sorting again; the transpose is the same keys with the
// halves swapped.
// The result is identical, array for array, to the host build.
#include "pp_internal.h"
#include "pp_build.h"

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>

namespace pp {

namespace {

__global__ void __launch_bounds__(BLOCK) k_check_arcs(const int32_t *a, const int32_t *b, int64_t m, int64_t n,
                                                      const int32_t *node_graph, unsigned long long *first_bad) {
    for (int64_t k = blockIdx.x * (int64_t)BLOCK + threadIdx.x; k < m; k += (int64_t)gridDim.x * BLOCK) {
        const int32_t x = a[k], y = b[k];
        bool bad = x < 0 || x >= n || y < 0 || y >= n;
        if (!bad && node_graph) bad = node_graph[x] != node_graph[y];
        if (bad) atomicMin(first_bad, (unsigned long long)k);
    }
}

// Arc k -> key slot k (and m + k for the reverse arc of an undirected edge).
__global__ void __launch_bounds__(BLOCK) k_arc_keys(const int32_t *a, const int32_t *b, int64_t m, int shift,
                                                    bool undirected, uint64_t no_arc, uint64_t *keys) {
    for (int64_t k = blockIdx.x * (int64_t)BLOCK + threadIdx.x; k < m; k += (int64_t)gridDim.x * BLOCK) {
        const uint64_t x = (uint32_t)a[k], y = (uint32_t)b[k];
        const bool loop = x == y;
        keys[k] = loop ? no_arc : (x << shift | y);
        if (undirected) keys[m + k] = loop ? no_arc : (y << shift | x);
    }
}

// Row lengths from the run boundaries of sorted keys: the run of row r adds
// its end index and subtracts its start index, one atomic each per row.
__global__ void __launch_bounds__(BLOCK) k_row_lengths(const uint64_t *keys, int64_t count, int shift,
                                                       unsigned long long *len) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < count; i += (int64_t)gridDim.x * BLOCK) {
        const uint64_t r = keys[i] >> shift;
        if (i == 0 || (keys[i - 1] >> shift) != r) atomicAdd(&len[r], (unsigned long long)(0 - (uint64_t)i));
        if (i == count - 1 || (keys[i + 1] >> shift) != r) atomicAdd(&len[r], (unsigned long long)(i + 1));
    }
}

__global__ void __launch_bounds__(BLOCK) k_key_cols(const uint64_t *keys, int64_t count, uint64_t mask, int32_t *col) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < count; i += (int64_t)gridDim.x * BLOCK)
        col[i] = (int32_t)(keys[i] & mask);
}

// Column counts (in-degrees) of sorted keys.
__global__ void __launch_bounds__(BLOCK) k_col_counts(const uint64_t *keys, int64_t count, uint64_t mask,
                                                      int32_t *cnt) {
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < count; i += (int64_t)gridDim.x * BLOCK)
        atomicAdd(&cnt[keys[i] & mask], 1);
}

// Relabel (perm: stored id of input node) and / or swap the halves.
__global__ void __launch_bounds__(BLOCK) k_rekey(const uint64_t *in, int64_t count, int shift, const int32_t *perm,
                                                 bool swap, uint64_t *out) {
    const uint64_t mask = (1ull << shift) - 1ull;
    for (int64_t i = blockIdx.x * (int64_t)BLOCK + threadIdx.x; i < count; i += (int64_t)gridDim.x * BLOCK) {
        uint64_t r = in[i] >> shift, c = in[i] & mask;
        if (perm) {
            r = (uint32_t)perm[r];
            c = (uint32_t)perm[c];
        }
        out[i] = swap ? (c << shift | r) : (r << shift | c);
    }
}

__global__ void k_fill_u64(unsigned long long *p, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_fill_i32z(int32_t *p, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

int grid_for(int64_t count) {
    const int64_t b = (count + BLOCK - 1) / BLOCK;
    return (int)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

int bits_for(int64_t n) {
    int s = 1;
    while (s < 31 && (int64_t(1) << s) <= n) ++s;
    return s;
}

// A device block that goes back to the allocator when it leaves scope.
template <typename T> struct DevBuf {
    T *p = nullptr;
    bool get(int64_t count) {
        p = (T *)dev_malloc(sizeof(T) * (size_t)(count > 0 ? count : 1));
        return p != nullptr;
    }
    T *release() {
        T *q = p;
        p = nullptr;
        return q;
    }
    ~DevBuf() {
        if (p) dev_release(p);
    }
};

#define BUILD_TRY(expr)                                                                       \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return set_error(PP_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// keys[0, count) sorted into out (begin..end bits), with temporary storage.
int sort_keys(uint64_t *in, uint64_t *out, int64_t count, int bits, hipStream_t st) {
    size_t bytes = 0;
    BUILD_TRY(rocprim::radix_sort_keys(nullptr, bytes, in, out, (size_t)count, 0u, (unsigned)bits, st));
    DevBuf<unsigned char> tmp;
    if (!tmp.get((int64_t)bytes)) return set_error(PP_ENOMEM, "radix sort storage of %zu bytes", bytes);
    BUILD_TRY(rocprim::radix_sort_keys(tmp.p, bytes, in, out, (size_t)count, 0u, (unsigned)bits, st));
    BUILD_TRY(hipStreamSynchronize(st));   // the storage goes back after the sort
    return PP_OK;
}

// Rows of n nodes from count sorted keys (no duplicates): offsets and columns.
int keys_to_rows(const uint64_t *keys, int64_t count, int64_t n, int shift, DevRows &out, hipStream_t st) {
    DevBuf<unsigned long long> len;
    DevBuf<int64_t> rp;
    DevBuf<int32_t> col;
    if (!len.get(n + 1) || !rp.get(n + 1) || !col.get(count))
        return set_error(PP_ENOMEM, "device rows of %lld nodes and %lld arcs", (long long)n, (long long)count);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n + 1)), dim3(BLOCK), 0, st, len.p, n + 1);
    if (count > 0) {
        hipLaunchKernelGGL(k_row_lengths, dim3(grid_for(count)), dim3(BLOCK), 0, st, keys, count, shift, len.p);
        hipLaunchKernelGGL(k_key_cols, dim3(grid_for(count)), dim3(BLOCK), 0, st, keys, count, (1ull << shift) - 1ull,
                           col.p);
    }
    BUILD_TRY(hipGetLastError());
    size_t bytes = 0;
    const int64_t *lin = reinterpret_cast<const int64_t *>(len.p);
    BUILD_TRY(rocprim::exclusive_scan(nullptr, bytes, lin, rp.p, (int64_t)0, (size_t)(n + 1), rocprim::plus<int64_t>(), st));
    DevBuf<unsigned char> tmp;
    if (!tmp.get((int64_t)bytes)) return set_error(PP_ENOMEM, "scan storage of %zu bytes", bytes);
    BUILD_TRY(rocprim::exclusive_scan(tmp.p, bytes, lin, rp.p, (int64_t)0, (size_t)(n + 1), rocprim::plus<int64_t>(), st));
    BUILD_TRY(hipStreamSynchronize(st));
    out.rp = rp.release();
    out.col = col.release();
    out.m = count;
    return PP_OK;
}

}  // namespace

int device_check_arcs(const int32_t *a, const int32_t *b, int64_t m, int64_t n, const int32_t *node_graph,
                      int64_t *first_bad, hipStream_t st) {
    *first_bad = -1;
    if (m <= 0) return PP_OK;
    DevBuf<unsigned long long> flag;
    if (!flag.get(1)) return set_error(PP_ENOMEM, "a flag");
    const unsigned long long none = ~0ull;
    BUILD_TRY(hipMemcpyAsync(flag.p, &none, sizeof(none), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_check_arcs, dim3(grid_for(m)), dim3(BLOCK), 0, st, a, b, m, n, node_graph, flag.p);
    BUILD_TRY(hipGetLastError());
    unsigned long long got = 0;
    BUILD_TRY(hipMemcpyAsync(&got, flag.p, sizeof(got), hipMemcpyDeviceToHost, st));
    BUILD_TRY(hipStreamSynchronize(st));
    *first_bad = got == none ? -1 : (int64_t)got;
    return PP_OK;
}

int device_build(int64_t n, int64_t m, const int32_t *a, const int32_t *b, bool undirected, const OrderFn &order,
                 DevRows &rows, DevRows &trows, std::vector<int32_t> &perm, hipStream_t st) {
    const int shift = bits_for(n);
    const int bits = 2 * shift;
    const uint64_t mask = (1ull << shift) - 1ull;
    const uint64_t no_arc = (1ull << bits) - 1ull;
    const int64_t slots = undirected ? 2 * m : m;
    if (slots >= (int64_t(1) << 32))
        return set_error(PP_EINVAL, "%lld arc keys: the device build takes fewer than 2^32 (PP_BUILD_ON_HOST)",
                         (long long)slots);
    // sorted keys without self-loops and duplicates
    DevBuf<uint64_t> k0, k1;
    if (!k0.get(slots) || !k1.get(slots)) return set_error(PP_ENOMEM, "%lld arc keys", (long long)slots);
    int64_t count = 0;
    if (m > 0) {
        hipLaunchKernelGGL(k_arc_keys, dim3(grid_for(m)), dim3(BLOCK), 0, st, a, b, m, shift, undirected, no_arc,
                           k0.p);
        BUILD_TRY(hipGetLastError());
        int rc = sort_keys(k0.p, k1.p, slots, bits, st);
        if (rc) return rc;
        DevBuf<unsigned int> ucount;
        if (!ucount.get(1)) return set_error(PP_ENOMEM, "a count");
        size_t bytes = 0;
        BUILD_TRY(rocprim::unique(nullptr, bytes, k1.p, k0.p, ucount.p, (size_t)slots, rocprim::equal_to<uint64_t>(), st));
        DevBuf<unsigned char> tmp;
        if (!tmp.get((int64_t)bytes)) return set_error(PP_ENOMEM, "unique storage of %zu bytes", bytes);
        BUILD_TRY(rocprim::unique(tmp.p, bytes, k1.p, k0.p, ucount.p, (size_t)slots, rocprim::equal_to<uint64_t>(), st));
        unsigned int u = 0;
        BUILD_TRY(hipMemcpyAsync(&u, ucount.p, sizeof(u), hipMemcpyDeviceToHost, st));
        BUILD_TRY(hipStreamSynchronize(st));
        count = (int64_t)u;
        if (count > 0) {
            uint64_t last = 0;
            BUILD_TRY(hipMemcpyAsync(&last, k0.p + (count - 1), sizeof(last), hipMemcpyDeviceToHost, st));
            BUILD_TRY(hipStreamSynchronize(st));
            if (last == no_arc) --count;
        }
    }
    // k0[0, count): the stored arcs by input id, sorted by row then column.
    // Degrees for the storage order: out-degrees from the rows, in-degrees by column.
    {
        DevRows r0;
        int rc = keys_to_rows(k0.p, count, n, shift, r0, st);
        if (rc) return rc;
        DevBuf<int64_t> rp0;
        DevBuf<int32_t> col0;
        rp0.p = r0.rp;
        col0.p = r0.col;
        DevBuf<int32_t> indeg;
        if (!indeg.get(n)) return set_error(PP_ENOMEM, "in-degrees of %lld nodes", (long long)n);
        hipLaunchKernelGGL(k_fill_i32z, dim3(grid_for(n)), dim3(BLOCK), 0, st, indeg.p, n);
        if (count > 0) hipLaunchKernelGGL(k_col_counts, dim3(grid_for(count)), dim3(BLOCK), 0, st, k0.p, count, mask, indeg.p);
        BUILD_TRY(hipGetLastError());
        std::vector<int64_t> rp_h((size_t)n + 1), trp_h((size_t)n + 1, 0);
        std::vector<int32_t> deg_h((size_t)n);
        BUILD_TRY(hipMemcpyAsync(rp_h.data(), rp0.p, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyDeviceToHost, st));
        BUILD_TRY(hipMemcpyAsync(deg_h.data(), indeg.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, st));
        BUILD_TRY(hipStreamSynchronize(st));
        for (int64_t v = 0; v < n; ++v) trp_h[(size_t)v + 1] = trp_h[(size_t)v] + deg_h[(size_t)v];
        std::vector<int32_t> col_h;
        hipError_t col_err = hipSuccess;
        const std::function<const int32_t *()> col = [&]() -> const int32_t * {
            if (col_h.empty() && count > 0) {
                col_h.resize((size_t)count);
                col_err = hipMemcpyAsync(col_h.data(), col0.p, sizeof(int32_t) * (size_t)count, hipMemcpyDeviceToHost, st);
                if (col_err == hipSuccess) col_err = hipStreamSynchronize(st);
            }
            return col_h.data();
        };
        const bool moved = order(rp_h, trp_h, col, perm);
        BUILD_TRY(col_err);
        if (!moved) {
            perm.clear();
            rows.rp = rp0.release();
            rows.col = col0.release();
            rows.m = count;
        }
    }
    DevBuf<int32_t> perm_d;
    if (!perm.empty()) {
        if (!perm_d.get(n)) return set_error(PP_ENOMEM, "the storage order");
        BUILD_TRY(hipMemcpyAsync(perm_d.p, perm.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, st));
        // rows in storage order: relabel, sort
        if (count > 0) {
            hipLaunchKernelGGL(k_rekey, dim3(grid_for(count)), dim3(BLOCK), 0, st, k0.p, count, shift, perm_d.p, false,
                               k1.p);
            BUILD_TRY(hipGetLastError());
            int rc = sort_keys(k1.p, k0.p, count, bits, st);
            if (rc) return rc;
        }
        int rc = keys_to_rows(k0.p, count, n, shift, rows, st);
        if (rc) return rc;
    }
    // the transpose: the (relabelled) keys with the halves swapped, sorted
    if (count > 0) {
        hipLaunchKernelGGL(k_rekey, dim3(grid_for(count)), dim3(BLOCK), 0, st, k0.p, count, shift, nullptr, true, k1.p);
        BUILD_TRY(hipGetLastError());
        int rc = sort_keys(k1.p, k0.p, count, bits, st);
        if (rc) return rc;
    }
    return keys_to_rows(k0.p, count, n, shift, trows, st);
}

}  // namespace pp
