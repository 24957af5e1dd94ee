// Distance metrics from the per-round counts (host only, no device work).
//
// Paper: Section 3 (diameter, effective diameter, average distance, number
// of reachable pairs, connectivity rate) and Algorithm 1's closing steps.
// Readings: c[0] = s counts the seeds' own pairs and rounds are numbered
// from 1, so R[k] = c[0] + ... + c[k] is the number of (node, seed) pairs
// within distance k and T = R[D] includes the s self-pairs.  Sums are exact
// 128-bit integers; each reported double is formed by converting the exact
// operands and dividing once, in the order written below.
#include <stdint.h>

#include "pp.h"

namespace pp {
// Records the message pp_last_error returns (defined with the rest of the
// interface) and returns `code`.
int set_error(int code, const char *fmt, ...);
}  // namespace pp

extern "C" int pp_estimate_metrics(const int64_t *counts, int32_t len, int64_t n, int32_t s, uint32_t tau_num,
                                   uint32_t tau_den, pp_metrics *out) {
    if (!counts || !out) return pp::set_error(PP_EINVAL, "counts or out is NULL");
    if (len < 1) return pp::set_error(PP_EINVAL, "len = %d < 1", len);
    if (s < 1 || n < 1) return pp::set_error(PP_EINVAL, "s = %d and n = %lld must be >= 1", s, (long long)n);
    if (tau_den == 0 || tau_num > tau_den)
        return pp::set_error(PP_EINVAL, "tau = %u/%u outside [0, 1]", tau_num, tau_den);
    for (int32_t r = 0; r < len; ++r)
        if (counts[r] < 0) return pp::set_error(PP_EINVAL, "counts[%d] = %lld < 0", r, (long long)counts[r]);
    // D: last round with new collisions
    int32_t D = 0;
    for (int32_t r = 0; r < len; ++r)
        if (counts[r] > 0) D = r;
    __int128 T = 0, Sd = 0;
    for (int32_t r = 0; r <= D; ++r) {
        T += counts[r];
        Sd += (__int128)r * counts[r];
    }
    const __int128 P1 = T - s;
    // effective diameter: least k with tau_den * R[k] >= tau_num * T, exactly
    int32_t k = D;
    __int128 R = 0, Rprev = 0;
    for (int32_t j = 0; j <= D; ++j) {
        Rprev = R;
        R += counts[j];
        if ((__int128)tau_den * R >= (__int128)tau_num * T) {
            k = j;
            break;
        }
    }
    double interp = 0.0;
    if (k > 0) {
        const __int128 num = (__int128)tau_num * T - (__int128)tau_den * Rprev;
        const __int128 den = (__int128)tau_den * (R - Rprev);
        interp = (double)(k - 1) + (double)num / (double)den;
    }
    out->diameter = D;
    out->rounds_executed = D + 1;
    out->R_final = (int64_t)T;
    out->eff_diam = (double)k;
    out->eff_diam_interp = interp;
    out->avg_dist = P1 > 0 ? (double)Sd / (double)P1 : 0.0;
    out->avg_dist_paper = T > 0 ? (double)Sd / (double)T : 0.0;
    out->reachable_pairs = (double)((__int128)n * T) / (double)s;
    out->alpha = n > 1 ? (double)P1 / (double)((__int128)s * (n - 1)) : 0.0;
    return PP_OK;
}
