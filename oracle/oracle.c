/*
 * FP64 CPU oracle for PERMANOVA's within-group statistic s_W, its F statistic,
 * its permutation p-value and its permutation generator.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package's smoke check and
 * the benchmark's CPU-baseline leg may load or call this library.  It shares no
 * code, header, table or helper with the HIP library; the two are compared,
 * never combined.
 *
 * Every function is the plain definition written out, slowly and in the
 * paper's order, with FP64 arithmetic:
 *   - s_W follows Algorithm 1 (section 2): over the strict upper triangle,
 *     row < col, a pair whose two objects carry the same label adds
 *     d^2 * inv_group_sizes[label]; the outer loop runs over permutations.
 *   - s_W in the tiled traversal of Algorithm 2 (section 2) is kept as a second
 *     formulation for cross-checking: per row segment of a TILE x TILE block
 *     the matching d^2 are summed, then multiplied once by the weight.
 *   - s_T, F and the p-value are the standard PERMANOVA quantities the paper
 *     leaves to the "steps before and after" (section 2): s_T = (1/n) sum_{i<j}
 *     d^2, F = ((s_T - s_W)/(k-1)) / (s_W/(n-k)), p = (1 + #{F_p >= F_obs})/(1 + P).
 *   - permutations are Durstenfeld's Fisher-Yates shuffle of the base labels
 *     (the permutation test of section 1), driven by one SplitMix64 stream per
 *     permutation (Steele, Lea & Flood 2014) with Lemire's multiply-shift
 *     bounded draw (Lemire 2019).
 *
 * Parity pins (see tests/test_oracle_pins.py): closed forms (single group,
 * all singletons, constant matrix, Euclidean Huygens identity), invariants
 * (label bijection, object reordering), enumeration of all n! relabelings at
 * tiny n, Algorithm 1 vs Algorithm 2 traversal, a dense FP64 matrix-product
 * formulation, the SplitMix64 published known-answer values.  No function here
 * is "parity unpinned".
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static void set_threads(int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
}

int oracle_max_threads(void) { return omp_get_max_threads(); }

/* ---------------------------------------------------------------------------
 * s_W, Algorithm 1.  rows points at rows [row0, row0 + nrows) of the n x n
 * row-major float matrix (row r of the block is matrix row row0 + r).  acc[p]
 * is a running FP64 sum that this call continues, so splitting the rows over
 * several calls in increasing order reproduces one call over all rows exactly.
 * ------------------------------------------------------------------------- */
void oracle_sW_rows(const float *rows, int64_t row0, int64_t nrows, int64_t n,
                    const int32_t *groupings, int64_t n_perms, const double *inv,
                    double *acc, int nthreads) {
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n_perms; p++) {
        const int32_t *g = groupings + p * n;
        double s = acc[p];
        for (int64_t row = row0; row < row0 + nrows && row < n - 1; row++) {
            const float *mat_row = rows + (uint64_t)(row - row0) * (uint64_t)n;
            int32_t group_idx = g[row];
            for (int64_t col = row + 1; col < n; col++) {
                if (g[col] == group_idx) {
                    double val = (double)mat_row[col];
                    s += val * val * inv[group_idx];
                }
            }
        }
        acc[p] = s;
    }
}

void oracle_sW(const float *mat, int64_t n, const int32_t *groupings, int64_t n_perms,
               const double *inv, double *out, int nthreads) {
    for (int64_t p = 0; p < n_perms; p++) out[p] = 0.0;
    oracle_sW_rows(mat, 0, n, n, groupings, n_perms, inv, out, nthreads);
}

/* s_W, Algorithm 2's tiled traversal (TILE = tile), FP64. */
void oracle_sW_tiled(const float *mat, int64_t n, const int32_t *groupings, int64_t n_perms,
                     const double *inv, int64_t tile, double *out, int nthreads) {
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n_perms; p++) {
        const int32_t *g = groupings + p * n;
        double s = 0.0;
        for (int64_t trow = 0; trow < n - 1; trow += tile) {
            for (int64_t tcol = trow + 1; tcol < n; tcol += tile) {
                int64_t row_end = trow + tile < n - 1 ? trow + tile : n - 1;
                for (int64_t row = trow; row < row_end; row++) {
                    int64_t min_col = tcol > row + 1 ? tcol : row + 1;
                    int64_t max_col = tcol + tile < n ? tcol + tile : n;
                    const float *mat_row = mat + (uint64_t)row * (uint64_t)n;
                    int32_t group_idx = g[row];
                    double local = 0.0;
                    for (int64_t col = min_col; col < max_col; col++) {
                        if (g[col] == group_idx) {
                            double val = (double)mat_row[col];
                            local += val * val;
                        }
                    }
                    s += local * inv[group_idx];
                }
            }
        }
        out[p] = s;
    }
}

/* s_T = (1/n) * sum_{i<j} d_ij^2, sequential FP64.  Continues acc like
 * oracle_sW_rows (call with acc = 0, then divide by n: see oracle_sT). */
void oracle_sq_rows(const float *rows, int64_t row0, int64_t nrows, int64_t n, double *acc) {
    double s = *acc;
    for (int64_t row = row0; row < row0 + nrows && row < n - 1; row++) {
        const float *mat_row = rows + (uint64_t)(row - row0) * (uint64_t)n;
        for (int64_t col = row + 1; col < n; col++) {
            double val = (double)mat_row[col];
            s += val * val;
        }
    }
    *acc = s;
}

double oracle_sT(const float *mat, int64_t n) {
    double s = 0.0;
    oracle_sq_rows(mat, 0, n, n, &s);
    return s / (double)n;
}

/* Sum over pairs in DIFFERENT groups of d^2 (no weights); used for the
 * within + between = total pin. */
double oracle_between_unweighted(const float *mat, int64_t n, const int32_t *grouping) {
    double s = 0.0;
    for (int64_t row = 0; row < n - 1; row++) {
        const float *mat_row = mat + (uint64_t)row * (uint64_t)n;
        for (int64_t col = row + 1; col < n; col++) {
            if (grouping[col] != grouping[row]) {
                double val = (double)mat_row[col];
                s += val * val;
            }
        }
    }
    return s;
}

/* pseudo-F for each s_W: ((s_T - s_W)/(k-1)) / (s_W/(n-k)); NaN when k < 2 or
 * n <= k (the statistic is undefined there). */
void oracle_F(const double *sW, int64_t count, double sT, int64_t n, int32_t k, double *F) {
    for (int64_t i = 0; i < count; i++) {
        if (k < 2 || n <= k) {
            F[i] = NAN;
        } else {
            double s_A = sT - sW[i];
            F[i] = (s_A / (double)(k - 1)) / (sW[i] / (double)(n - k));
        }
    }
}

/* p = (1 + #{p : F_p >= F_obs}) / (1 + P); NaN when P = 0. */
double oracle_pvalue(double F_obs, const double *F_perm, int64_t n_perms) {
    if (n_perms <= 0) return NAN;
    int64_t c = 0;
    for (int64_t p = 0; p < n_perms; p++)
        if (F_perm[p] >= F_obs) c++;
    return (double)(1 + c) / (double)(1 + n_perms);
}

/* The same count through s_W: F_p >= F_obs  <=>  s_W[p] <= s_W_obs when
 * k >= 2, n > k and s_W > 0 (F is strictly decreasing in s_W). */
double oracle_pvalue_sW(double sW_obs, const double *sW_perm, int64_t n_perms) {
    if (n_perms <= 0) return NAN;
    int64_t c = 0;
    for (int64_t p = 0; p < n_perms; p++)
        if (sW_perm[p] <= sW_obs) c++;
    return (double)(1 + c) / (double)(1 + n_perms);
}

/* ---------------------------------------------------------------------------
 * Permutation generator.
 * ------------------------------------------------------------------------- */

/* SplitMix64: advance the state by the golden gamma, return the mixed state. */
uint64_t oracle_splitmix64_next(uint64_t *state) {
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static uint64_t mix_only(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Start state of permutation p's stream: mix(seed XOR mix(p + 1)). */
uint64_t oracle_stream_start(uint64_t seed, uint64_t p) {
    return mix_only(seed ^ mix_only(p + 1));
}

/* Uniform integer in [0, s), s >= 1: Lemire's multiply-shift with rejection
 * on the upper 32 bits of each SplitMix64 output. */
uint32_t oracle_bounded(uint64_t *state, uint32_t s) {
    uint32_t x = (uint32_t)(oracle_splitmix64_next(state) >> 32);
    uint64_t m = (uint64_t)x * (uint64_t)s;
    uint32_t l = (uint32_t)m;
    if (l < s) {
        uint32_t t = (uint32_t)(-s) % s;
        while (l < t) {
            x = (uint32_t)(oracle_splitmix64_next(state) >> 32);
            m = (uint64_t)x * (uint64_t)s;
            l = (uint32_t)m;
        }
    }
    return (uint32_t)(m >> 32);
}

/* Test helper: number of draws the bounded draws of oracle_permute discard
 * (Lemire rejections) over n_perms shuffles of n labels -- which inputs
 * exercise a generator's rejection path. */
int64_t oracle_count_rejections(int64_t n, int64_t n_perms, uint64_t seed) {
    int64_t total = 0;
    for (int64_t p = 0; p < n_perms; p++) {
        uint64_t st = oracle_stream_start(seed, (uint64_t)p);
        for (int64_t i = n - 1; i >= 1; i--) {
            const uint32_t s = (uint32_t)(i + 1);
            for (;;) {
                const uint32_t x = (uint32_t)(oracle_splitmix64_next(&st) >> 32);
                const uint32_t l = (uint32_t)((uint64_t)x * (uint64_t)s);
                if (l >= s || l >= (uint32_t)(-s) % s) break;
                total++;
            }
        }
    }
    return total;
}

/* groupings[p*n + i]: Fisher-Yates (Durstenfeld, i from n-1 down to 1, swap
 * with a uniform j in [0, i]) applied to a copy of base, stream of perm p. */
void oracle_permute(const int32_t *base, int64_t n, int64_t n_perms, uint64_t seed,
                    int32_t *groupings, int nthreads) {
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n_perms; p++) {
        int32_t *a = groupings + p * n;
        memcpy(a, base, (size_t)n * sizeof(int32_t));
        uint64_t st = oracle_stream_start(seed, (uint64_t)p);
        for (int64_t i = n - 1; i >= 1; i--) {
            int64_t j = (int64_t)oracle_bounded(&st, (uint32_t)(i + 1));
            int32_t t = a[i];
            a[i] = a[j];
            a[j] = t;
        }
    }
}
