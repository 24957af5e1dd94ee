// Adjacency build on the device (pp_build.hip), used by pp_csr_build.
#pragma once

#include <functional>
#include <vector>

#include "pp_internal.h"

namespace pp {

// Device adjacency build (pp_build.hip).  Rows: offsets [n+1] and columns
// [m], device blocks from dev_malloc (the caller frees them).
struct DevRows {
    int64_t *rp = nullptr;
    int32_t *col = nullptr;
    int64_t m = 0;
};
// First arc k (of m, device arrays) with an id outside [0, n) or whose ends
// lie in different graphs (node_graph, device, may be NULL), or -1.
int device_check_arcs(const int32_t *a, const int32_t *b, int64_t m, int64_t n, const int32_t *node_graph,
                      int64_t *first_bad, hipStream_t st);
// The rows of arcs a[k] -> b[k] (device; and b -> a when undirected), without
// self-loops and duplicates, each sorted, and their transpose.  order(rp, trp,
// col, perm) gets the host offsets of both by input id, and col() the host
// successor ids (by input id, fetched from the device on its first call), and
// may fill perm (the stored id of each input node) and return true; the rows
// are then stored in that order (perm is cleared when it returns false).
using OrderFn = std::function<bool(const std::vector<int64_t> &, const std::vector<int64_t> &,
                                   const std::function<const int32_t *()> &, std::vector<int32_t> &)>;
int device_build(int64_t n, int64_t m, const int32_t *a, const int32_t *b, bool undirected, const OrderFn &order,
                 DevRows &rows, DevRows &trows, std::vector<int32_t> &perm, hipStream_t st);

}  // namespace pp
