/*
 * Input-generator helpers for the seeded synthetic tensors.
 *
 * This file is part of the input generator only: it draws nothing itself
 * (all random numbers come from numpy's PCG64 in synthetic.py) and holds
 * none of the MTTKRP / CP arithmetic.  It provides two bulk operations that
 * are too slow in numpy at 10^8 scale:
 *
 *   synth_inverse_cdf  - map uniform doubles u to ranks via a sorted CDF
 *                        (upper_bound: the rank k with cdf[k-1] <= u < cdf[k])
 *   synth_dedupe_first - keep the first occurrence of every distinct
 *                        N-tuple of coordinates, in input order
 *
 * Built with gcc -O2 -fopenmp into libsynth.so; loaded with ctypes.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* out[i] = number of cdf entries <= u[i]  (0-based rank of the draw). */
void synth_inverse_cdf(const double *cdf, int64_t ncdf, const double *u,
                       int64_t n, int32_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double x = u[i];
        int64_t lo = 0, hi = ncdf; /* first index with cdf[idx] > x */
        while (lo < hi) {
            int64_t mid = lo + ((hi - lo) >> 1);
            if (cdf[mid] <= x) lo = mid + 1; else hi = mid;
        }
        if (lo >= ncdf) lo = ncdf - 1; /* u == 1.0 cannot happen, guard anyway */
        out[i] = (int32_t)lo;
    }
}

static inline uint64_t mix64(uint64_t z)
{
    z ^= z >> 33; z *= 0xff51afd7ed558ccdULL;
    z ^= z >> 33; z *= 0xc4ceb9fe1a85ec53ULL;
    z ^= z >> 33;
    return z;
}

/*
 * coords: nmodes pointers, each to n int32 coordinates.
 * keep:   output, at most n entries: indices of first occurrences, ascending.
 * Returns the number of kept entries, or -1 on allocation failure.
 */
int64_t synth_dedupe_first(int nmodes, const int32_t *const *coords, int64_t n,
                           int64_t *keep)
{
    uint64_t cap = 1;
    while (cap < (uint64_t)n * 2u + 16u) cap <<= 1;
    int64_t *table = (int64_t *)malloc(cap * sizeof(int64_t));
    if (!table) return -1;
    memset(table, 0xff, cap * sizeof(int64_t)); /* -1 = empty */
    uint64_t mask = cap - 1;
    int64_t nk = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t h = 0x9e3779b97f4a7c15ULL;
        for (int m = 0; m < nmodes; ++m)
            h = mix64(h ^ (uint64_t)(uint32_t)coords[m][i] ^ ((uint64_t)m << 40));
        uint64_t slot = h & mask;
        for (;;) {
            int64_t j = table[slot];
            if (j < 0) { table[slot] = i; keep[nk++] = i; break; }
            int same = 1;
            for (int m = 0; m < nmodes; ++m)
                if (coords[m][j] != coords[m][i]) { same = 0; break; }
            if (same) break;
            slot = (slot + 1) & mask;
        }
    }
    free(table);
    return nk;
}
