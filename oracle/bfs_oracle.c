/*
 * CPU oracle for seed-bitset propagation.  TEST INFRASTRUCTURE ONLY: it is
 * called by the tests, by the package's smoke check and by the benchmark's
 * CPU-baseline leg, never by the product path.  It shares no code with the
 * HIP library.
 *
 * What it computes (paper, Section 3 definitions and Section 4 /
 * Algorithm 1, PROPAGATE-P):
 *   d(u, v) is the number of arcs on a shortest directed path from u to v.
 *   The propagation step ORs into node u the signatures of the heads v of its
 *   arcs u -> v, so bit i (seed x_i) reaches u after r rounds exactly when
 *   d(u, x_i) <= r.  The per-round collision count is therefore
 *       c[0] = s,   c[r] = sum_i #{u : d(u, x_i) = r}   (r >= 1),
 *   i.e. the number of (node, seed) pairs at distance exactly r, and
 *   D = max{r : c[r] > 0} is the last round that set a bit.
 *
 * This follows the plain definition with one breadth-first search per seed
 * over the reversed arcs (from x_i to every u that can reach it), which is
 * the sequential seed-by-seed form the paper states gives the same counts as
 * the parallel one.  Duplicate arcs and self-loops cannot change a BFS, so
 * they are left in.  ``transpose`` runs the BFS over forward arcs instead
 * (bit i reaches u when x_i can reach u).
 *
 * Seeds are split statically over nthreads POSIX threads.  Per-seed counts
 * and signature bits belong to one seed each; signature words shared by
 * several seeds are updated with an atomic OR.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n;
    const int64_t *off;   /* adjacency offsets for the BFS direction, [n+1] */
    const int32_t *adj;   /* adjacency targets */
    const int32_t *seeds;
    int32_t s, W;
    int32_t cap;          /* rows available in the count arrays */
    int32_t t, nthreads;
    int64_t *counts;      /* per-thread [cap] */
    int32_t maxd;
    uint32_t *seed_counts;      /* [cap][s] or NULL */
    const int32_t *sig_rounds;  /* rounds whose signatures are wanted */
    int32_t n_sig;
    uint64_t *sigs;             /* [n_sig][n][W] or NULL */
    uint64_t *final_sig;        /* [n][W] or NULL */
    int32_t *dist_out;          /* [s][n] or NULL: d(u, x_i), -1 if unreachable */
    int overflow;
} job_t;

static void *worker(void *arg) {
    job_t *j = (job_t *)arg;
    int64_t n = j->n;
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!dist || !queue) { j->overflow = 2; free(dist); free(queue); return NULL; }
    for (int32_t i = j->t; i < j->s; i += j->nthreads) {
        for (int64_t u = 0; u < n; ++u) dist[u] = -1;
        int32_t x = j->seeds[i];
        int64_t head = 0, tail = 0;
        dist[x] = 0;
        queue[tail++] = x;
        while (head < tail) {
            int32_t v = queue[head++];
            for (int64_t e = j->off[v]; e < j->off[v + 1]; ++e) {
                int32_t u = j->adj[e];
                if (dist[u] < 0) {
                    dist[u] = dist[v] + 1;
                    queue[tail++] = u;
                }
            }
        }
        /* queue[0..tail) holds every node reached from x_i, in BFS order */
        uint64_t bit = 1ull << (i & 63);
        int32_t w = i >> 6;
        for (int64_t q = 0; q < tail; ++q) {
            int32_t u = queue[q];
            int32_t d = dist[u];
            if (d >= j->cap) { j->overflow = 1; continue; }
            j->counts[d] += 1;
            if (d > j->maxd) j->maxd = d;
            if (j->seed_counts) j->seed_counts[(int64_t)d * j->s + i] += 1;
            if (j->final_sig)
                __atomic_fetch_or(&j->final_sig[(int64_t)u * j->W + w], bit, __ATOMIC_RELAXED);
            for (int32_t k = 0; k < j->n_sig; ++k)
                if (d <= j->sig_rounds[k])
                    __atomic_fetch_or(&j->sigs[((int64_t)k * n + u) * j->W + w], bit, __ATOMIC_RELAXED);
        }
        if (j->dist_out) memcpy(j->dist_out + (int64_t)i * n, dist, sizeof(int32_t) * (size_t)n);
    }
    free(dist);
    free(queue);
    return NULL;
}

/*
 * Returns 0 on success, 1 if some distance did not fit in ``cap`` rows,
 * 2 on allocation failure, 3 on an invalid argument.
 *
 * src/dst: m arcs u -> v (ids in [0, n)); ``undirected`` adds v -> u.
 * counts[cap] receives c[r]; *D_out receives max r with c[r] > 0 (0 if s=0).
 */
int oracle_propagate(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                     int32_t undirected, int32_t transpose,
                     const int32_t *seeds, int32_t s, int32_t nthreads,
                     int64_t *counts, int32_t cap, int32_t *D_out,
                     uint32_t *seed_counts,
                     const int32_t *sig_rounds, int32_t n_sig, uint64_t *sigs,
                     uint64_t *final_sig, int32_t *dist_out) {
    if (n < 0 || m < 0 || s < 0 || cap < 1 || nthreads < 1) return 3;
    for (int64_t e = 0; e < m; ++e)
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return 3;
    for (int32_t i = 0; i < s; ++i)
        if (seeds[i] < 0 || seeds[i] >= n) return 3;
    int32_t W = (s + 63) / 64;

    /* BFS adjacency: for the paper's direction the search runs from x_i
     * backwards along arcs, so node v lists every u with an arc u -> v. */
    int64_t narcs = undirected ? 2 * m : m;
    int64_t *off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(narcs > 0 ? narcs : 1));
    int64_t *fill = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!off || !adj || !fill) { free(off); free(adj); free(fill); return 2; }
    for (int64_t e = 0; e < m; ++e) {
        int32_t from = transpose ? src[e] : dst[e];   /* BFS moves from -> to */
        int32_t to = transpose ? dst[e] : src[e];
        off[from + 1] += 1;
        if (undirected) off[to + 1] += 1;
    }
    for (int64_t v = 0; v < n; ++v) off[v + 1] += off[v];
    memcpy(fill, off, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < m; ++e) {
        int32_t from = transpose ? src[e] : dst[e];
        int32_t to = transpose ? dst[e] : src[e];
        adj[fill[from]++] = to;
        if (undirected) adj[fill[to]++] = from;
    }
    free(fill);

    if (nthreads > s && s > 0) nthreads = s;
    if (s == 0) nthreads = 1;
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    int64_t *tcounts = (int64_t *)calloc((size_t)nthreads * (size_t)cap, sizeof(int64_t));
    if (!jobs || !th || !tcounts) { free(off); free(adj); free(jobs); free(th); free(tcounts); return 2; }
    if (seed_counts) memset(seed_counts, 0, sizeof(uint32_t) * (size_t)cap * (size_t)s);
    if (sigs) memset(sigs, 0, sizeof(uint64_t) * (size_t)n_sig * (size_t)n * (size_t)W);
    if (final_sig) memset(final_sig, 0, sizeof(uint64_t) * (size_t)n * (size_t)W);
    for (int32_t t = 0; t < nthreads; ++t) {
        job_t *j = &jobs[t];
        j->n = n; j->off = off; j->adj = adj; j->seeds = seeds; j->s = s; j->W = W;
        j->cap = cap; j->t = t; j->nthreads = nthreads; j->counts = tcounts + (int64_t)t * cap;
        j->maxd = 0; j->seed_counts = seed_counts; j->sig_rounds = sig_rounds; j->n_sig = n_sig;
        j->sigs = sigs; j->final_sig = final_sig; j->dist_out = dist_out; j->overflow = 0;
        pthread_create(&th[t], NULL, worker, j);
    }
    int rc = 0;
    int32_t D = 0;
    for (int32_t r = 0; r < cap; ++r) counts[r] = 0;
    for (int32_t t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        if (jobs[t].overflow > rc) rc = jobs[t].overflow;
        if (jobs[t].maxd > D) D = jobs[t].maxd;
        for (int32_t r = 0; r < cap; ++r) counts[r] += jobs[t].counts[r];
    }
    *D_out = D;
    free(off); free(adj); free(jobs); free(th); free(tcounts);
    return rc;
}
