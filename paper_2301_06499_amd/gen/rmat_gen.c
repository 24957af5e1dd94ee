/*
 * Native R-MAT edge generator: the same counter-based definition as
 * inputs.rmat (SplitMix64 draw k*ceil(scale/2) + l/2 of the stream, high
 * 32 bits for even levels l, low 32 bits for odd ones, compared with the
 * integer thresholds of the cumulative quadrant probabilities), so both
 * produce identical edge lists; this one runs on every host core for the
 * large scales.  Input generation only: no propagation arithmetic.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

static inline uint64_t draw(uint64_t seed, uint64_t idx) {
    uint64_t z = seed + (idx + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct {
    int scale;
    int64_t lo, hi;
    uint64_t seed, t1, t2, t3;
    int32_t *src, *dst;
} job_t;

static void *work(void *arg) {
    const job_t *j = (const job_t *)arg;
    const uint64_t per = (uint64_t)(j->scale + 1) / 2;
    for (int64_t k = j->lo; k < j->hi; ++k) {
        const uint64_t base = (uint64_t)k * per;
        uint64_t s = 0, d = 0, x = 0, u;
        for (int lvl = 0; lvl < j->scale; ++lvl) {
            if ((lvl & 1) == 0) {
                x = draw(j->seed, base + (uint64_t)(lvl / 2));
                u = x >> 32;
            } else {
                u = x & 0xFFFFFFFFull;
            }
            const int bit = j->scale - 1 - lvl;
            const uint64_t sb = u >= j->t2;
            const uint64_t db = (u >= j->t1 && u < j->t2) || u >= j->t3;
            s |= sb << bit;
            d |= db << bit;
        }
        j->src[k] = (int32_t)s;
        j->dst[k] = (int32_t)d;
    }
    return NULL;
}

/* Edges [0, m) of R-MAT(scale) for stream `seed` into src/dst; 0 on success. */
int rmat_edges(int scale, int64_t m, uint64_t seed, uint64_t t1, uint64_t t2, uint64_t t3, int32_t *src,
               int32_t *dst, int nthreads) {
    if (scale < 1 || scale > 31 || m < 0 || nthreads < 1) return -1;
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) {
        free(jobs);
        free(th);
        return -2;
    }
    int started = 0;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (job_t){scale, m * t / nthreads, m * (t + 1) / nthreads, seed, t1, t2, t3, src, dst};
        if (pthread_create(&th[t], NULL, work, &jobs[t]) == 0) {
            ++started;
        } else {
            work(&jobs[t]);
            th[t] = 0;
        }
    }
    for (int t = 0; t < nthreads; ++t)
        if (th[t]) pthread_join(th[t], NULL);
    (void)started;
    free(jobs);
    free(th);
    return 0;
}
