/*
 * Seeded synthetic instances for expander l0-decoding.
 *
 * This module only draws inputs: the expander's column-index store, the
 * support and nonzero values of the k-sparse signal x, and the measurement
 * y = A x.  It holds none of the decoder's arithmetic (no scoring, no
 * selection, no residual update) and is shared, as an input source only, by
 * the CPU oracle and the GPU decoder's tests and benchmark.
 *
 * Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used as a counter-based
 * generator: word c of stream (seed, tag, j) is mix64(K + (c+1)*GAMMA) with
 * K = mix64(mix64(seed + (tag+1)*GAMMA) + (j+1)*GAMMA).  Every column, every
 * support slot and every value has its own stream, so results do not depend
 * on the number of threads used to draw them.
 *
 * Matrix model (Section 2.2, Definition 2.2 and the footnote on generating
 * expanders in Section 1.1): each column has exactly d ones, their rows drawn
 * uniformly from all C(m, d) subsets, independently over columns.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

enum { TAG_COLUMNS = 1, TAG_SUPPORT = 2, TAG_VALUES = 3, TAG_WEIGHTS = 4 };

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t tag, uint64_t j) {
    return mix64(mix64(seed + (tag + 1) * GAMMA) + (j + 1) * GAMMA);
}

static inline uint64_t word(uint64_t key, uint64_t c) { return mix64(key + (c + 1) * GAMMA); }

/* Unbiased integer in [0, range): reject the 2^64 mod range lowest words. */
static uint64_t bounded(uint64_t key, uint64_t* ctr, uint64_t range) {
    uint64_t thresh = (0 - range) % range;
    for (;;) {
        uint64_t u = word(key, (*ctr)++);
        if (u >= thresh) return u % range;
    }
}

/* Uniform double in [0, 1) with 53 random bits. */
static double unit53(uint64_t key, uint64_t* ctr) {
    return (double)(word(key, (*ctr)++) >> 11) * (1.0 / 9007199254740992.0);
}

/*
 * col_idx[j*d + t], t = 0..d-1: the d distinct rows of column j, ascending.
 * Returns 0, or -1 on bad arguments.
 */
int l0gen_columns(uint64_t seed, int64_t n, int32_t m, int32_t d, int32_t* col_idx) {
    if (n < 0 || m < 1 || d < 1 || d > m || (n > 0 && !col_idx)) return -1;
#pragma omp parallel for schedule(static, 4096)
    for (int64_t j = 0; j < n; ++j) {
        uint64_t key = stream_key(seed, TAG_COLUMNS, (uint64_t)j);
        uint64_t ctr = 0;
        int32_t* rows = col_idx + j * (int64_t)d;
        int32_t have = 0;
        while (have < d) {
            int32_t r = (int32_t)bounded(key, &ctr, (uint64_t)m);
            int dup = 0;
            for (int32_t u = 0; u < have; ++u) dup |= (rows[u] == r);
            if (dup) continue;
            /* insertion keeps the list ascending */
            int32_t p = have++;
            while (p > 0 && rows[p - 1] > r) { rows[p] = rows[p - 1]; --p; }
            rows[p] = r;
        }
    }
    return 0;
}

/*
 * k distinct indices in [0, n), uniform (Floyd's sampling without
 * replacement), written ascending to supp[0..k).  Returns 0 or -1.
 */
int l0gen_support(uint64_t seed, int64_t n, int64_t k, int64_t* supp) {
    if (n < 0 || k < 0 || k > n || (k > 0 && !supp)) return -1;
    if (k == 0) return 0;
    unsigned char* in = (unsigned char*)calloc((size_t)n, 1);
    if (!in) return -1;
    uint64_t key = stream_key(seed, TAG_SUPPORT, 0);
    uint64_t ctr = 0;
    for (int64_t i = n - k; i < n; ++i) {
        int64_t t = (int64_t)bounded(key, &ctr, (uint64_t)(i + 1));
        if (in[t]) in[i] = 1; else in[t] = 1;
    }
    int64_t p = 0;
    for (int64_t i = 0; i < n; ++i)
        if (in[i]) supp[p++] = i;
    free(in);
    return p == k ? 0 : -1;
}

/*
 * Nonzero values for the support slots: kind 0 draws N(0,1) by Marsaglia's
 * polar method, kind 1 draws uniformly from {-1, +1}.  The value of index j
 * comes from its own stream, so it does not depend on k.  Returns 0 or -1.
 */
int l0gen_values(uint64_t seed, int64_t k, const int64_t* supp, int32_t kind, double* vals) {
    if (k < 0 || (k > 0 && (!supp || !vals)) || kind < 0 || kind > 1) return -1;
    for (int64_t s = 0; s < k; ++s) {
        uint64_t key = stream_key(seed, TAG_VALUES, (uint64_t)supp[s]);
        uint64_t ctr = 0;
        if (kind == 1) {
            vals[s] = (word(key, ctr) >> 63) ? 1.0 : -1.0;
            continue;
        }
        for (;;) {
            double v1 = 2.0 * unit53(key, &ctr) - 1.0;
            double v2 = 2.0 * unit53(key, &ctr) - 1.0;
            double q = v1 * v1 + v2 * v2;
            if (q > 0.0 && q < 1.0) { vals[s] = v1 * sqrt(-2.0 * log(q) / q); break; }
        }
    }
    return 0;
}

/*
 * Column weights for a column-scaled matrix (Section 4.3.3: every column of A
 * multiplied by an i.i.d. draw from a continuous distribution): w_j uniform
 * on [lo, hi] (a 53-bit draw scaled to the interval), from column j's own
 * stream.  Returns 0 or -1.
 */
int l0gen_weights(uint64_t seed, int64_t n, double lo, double hi, double* w) {
    if (n < 0 || (n > 0 && !w) || !(lo < hi) || !isfinite(lo) || !isfinite(hi)) return -1;
    for (int64_t j = 0; j < n; ++j) {
        uint64_t key = stream_key(seed, TAG_WEIGHTS, (uint64_t)j);
        uint64_t ctr = 0;
        w[j] = lo + (hi - lo) * unit53(key, &ctr);
    }
    return 0;
}

/*
 * Measurement y = A x for x given by (supp, vals), supp ascending:
 * y_i is the sum, starting from +0.0 and taken over ascending column index,
 * of the entries A_ij x_j over the support columns j whose neighbourhood
 * contains row i.  A_ij is 1, or w[j] when w is given (each product rounded
 * once before it is added).  Returns 0 or -1.
 */
int l0gen_measure(int64_t n, int32_t m, int32_t d, const int32_t* col_idx,
                  int64_t k, const int64_t* supp, const double* vals, const double* w, double* y) {
    if (n < 0 || m < 1 || d < 1 || !y || (k > 0 && (!col_idx || !supp || !vals))) return -1;
    for (int32_t i = 0; i < m; ++i) y[i] = 0.0;
    for (int64_t s = 0; s < k; ++s) {
        int64_t j = supp[s];
        if (j < 0 || j >= n || (s > 0 && supp[s - 1] >= j)) return -1;
        const double term = w ? w[j] * vals[s] : vals[s];
        for (int32_t t = 0; t < d; ++t) {
            int32_t i = col_idx[j * (int64_t)d + t];
            if (i < 0 || i >= m) return -1;
            y[i] += term;
        }
    }
    return 0;
}
