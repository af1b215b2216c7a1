/*
 * FP64 CPU oracle for PERMANOVA's within-group statistic s_W, its F statistic,
 * its permutation p-value and its permutation generator.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package's smoke check and
 * the benchmark's CPU-baseline leg may load or call this library.  It shares no
 * code, header, table or helper with the HIP library; the two are compared,
 * never combined.
 *
 * What is computed, each from its definition, slowly and in FP64:
 *
 *   s_W (section 2: the quantity Algorithm 1 returns).  For a grouping g of
 *   the n objects and per-group weights w,
 *       s_W = sum over groups c of  w_c * S_c,
 *       S_c = sum over the unordered pairs {a, b}, a < b, whose objects both
 *             belong to group c, of d_ab^2,
 *   where d_ab is read above the diagonal only (row a, column b > a): the
 *   paper never reads the diagonal or the lower triangle.  Each S_c walks the
 *   members of group c (listed in increasing object order) and is a Neumaier
 *   compensated FP64 sum, so its error is a few units in the last place for
 *   any n.  The weighted terms w_c * S_c are then added in increasing order of
 *   value (compensated as well).  The result therefore depends only on the
 *   partition and on which weight each block carries: relabelling the groups
 *   by a bijection (weights moved with them) gives the same bits, and two
 *   groupings that induce the same partition give the same bits.
 *
 *   s_T, F and the p-value: the standard PERMANOVA quantities the paper leaves
 *   to the steps "before and after" (section 2): s_T = (1/n) sum_{a<b} d_ab^2,
 *   F = ((s_T - s_W)/(k-1)) / (s_W/(n-k)), p = (1 + #{q : F_q >= F_obs})/(1 + P).
 *   The count is also offered through s_W (F falls strictly as s_W grows),
 *   with a relative tie tolerance: permutation q counts when
 *   s_W[q] <= s_W_obs + rtol * |s_W_obs|.
 *
 *   The random relabelings of the permutation test (section 1): Durstenfeld's
 *   Fisher-Yates shuffle of the base labels, one SplitMix64 stream per
 *   permutation (Steele, Lea & Flood 2014), Lemire's bounded draw with
 *   rejection (Lemire 2019).
 *
 * Pins (tests/test_oracle_pins.py) compare every function here with something
 * other than itself: closed forms, invariants, enumeration of all relabelings
 * of tiny inputs, exact rationals, brute force, a dense matrix-product
 * formulation, published known-answer values of SplitMix64 and closed-form
 * draw sequences of Lemire's method.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#define _GNU_SOURCE
#include <math.h>
#include <sched.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static void set_threads(int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
}

int oracle_max_threads(void) { return omp_get_max_threads(); }

/* Measurement helper of the CPU baseline, no part of any statistic: sets the
 * CPU affinity of the threads of a team of `nthreads` (the same threads later
 * parallel regions of that size reuse).  With one_each (and ncpus >= nthreads)
 * thread t runs on cpus[t] alone; otherwise every thread may run on all ncpus
 * CPUs (to undo a pinning).  Returns 0, or -1 if a call failed. */
int oracle_pin_threads(const int *cpus, int ncpus, int nthreads, int one_each) {
    int bad = 0;
    if (one_each && ncpus < nthreads) return -1;
    omp_set_num_threads(nthreads);
#pragma omp parallel num_threads(nthreads) reduction(| : bad)
    {
        cpu_set_t set;
        CPU_ZERO(&set);
        if (one_each) {
            CPU_SET(cpus[omp_get_thread_num()], &set);
        } else {
            for (int c = 0; c < ncpus; c++) CPU_SET(cpus[c], &set);
        }
        if (sched_setaffinity(0, sizeof(set), &set) != 0) bad = 1;
    }
    return bad ? -1 : 0;
}

/* ---------------------------------------------------------------------------
 * Compensated summation (Neumaier 1974): *hi + *lo carries the running sum.
 * ------------------------------------------------------------------------- */
static inline void kadd(double *hi, double *lo, double x) {
    const double t = *hi + x;
    if (fabs(*hi) >= fabs(x))
        *lo += (*hi - t) + x;
    else
        *lo += (x - t) + *hi;
    *hi = t;
}

/* Members of every group of one grouping in increasing object order:
 * first[c] .. first[c + 1] - 1 index `member`; slot[a] is object a's index
 * there.  Returns -1 if a label lies outside [0, k). */
static int list_members(const int32_t *g, int64_t n, int32_t k, int64_t *first,
                        int64_t *member, int64_t *slot) {
    for (int32_t c = 0; c <= k; c++) first[c] = 0;
    for (int64_t a = 0; a < n; a++) {
        if (g[a] < 0 || g[a] >= k) return -1;
        first[g[a] + 1]++;
    }
    for (int32_t c = 0; c < k; c++) first[c + 1] += first[c];
    int64_t *fill = (int64_t *)malloc((size_t)k * sizeof(int64_t));
    if (!fill) return -1;
    for (int32_t c = 0; c < k; c++) fill[c] = first[c];
    for (int64_t a = 0; a < n; a++) {
        const int64_t at = fill[g[a]]++;
        member[at] = a;
        slot[a] = at;
    }
    free(fill);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Within-group sums of squared distances.
 *
 * rows points at matrix rows [row0, row0 + nrows) of an n x n row-major float
 * matrix (block row r is matrix row row0 + r; only its columns > row0 + r are
 * read).  For every grouping p (row p of groupings, labels in [0, k)) and group
 * c, sums[(p * k + c) * 2 + {0, 1}] is a compensated pair that this call
 * continues with the pairs {a, b}, a in the block, b > a, both in group c --
 * so calls over consecutive row blocks make up the whole triangle.
 * Returns 0, or -1 on a label outside [0, k) (sums then undefined).
 * ------------------------------------------------------------------------- */
int oracle_group_sums(const float *rows, int64_t row0, int64_t nrows, int64_t n,
                      const int32_t *groupings, int64_t n_perms, int32_t k, double *sums,
                      int nthreads) {
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel reduction(| : bad)
    {
        int64_t *first = (int64_t *)malloc((size_t)(k + 1) * sizeof(int64_t));
        int64_t *member = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        int64_t *slot = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        if (!first || !member || !slot) bad = 1;
#pragma omp for schedule(dynamic, 1)
        for (int64_t p = 0; p < n_perms; p++) {
            if (!first || !member || !slot) continue;
            const int32_t *g = groupings + p * n;
            if (list_members(g, n, k, first, member, slot)) {
                bad = 1;
                continue;
            }
            double *acc = sums + (size_t)p * (size_t)k * 2;
            for (int64_t a = row0; a < row0 + nrows && a < n; a++) {
                const int32_t c = g[a];
                const float *row = rows + (uint64_t)(a - row0) * (uint64_t)n;
                double hi = acc[2 * c], lo = acc[2 * c + 1];
                for (int64_t m = slot[a] + 1; m < first[c + 1]; m++) {
                    const double x = (double)row[member[m]];
                    kadd(&hi, &lo, x * x);
                }
                acc[2 * c] = hi;
                acc[2 * c + 1] = lo;
            }
        }
        free(first);
        free(member);
        free(slot);
    }
    return bad ? -1 : 0;
}

static int cmp_double(const void *x, const void *y) {
    const double a = *(const double *)x, b = *(const double *)y;
    return (a > b) - (a < b);
}

/* out[p] = sum_c w[c] * S_c from the compensated group sums, the k weighted
 * terms added in increasing order of value. */
void oracle_sW_from_sums(const double *sums, int64_t n_perms, int32_t k, const double *w,
                         double *out) {
    double *t = (double *)malloc((size_t)(k > 0 ? k : 1) * sizeof(double));
    for (int64_t p = 0; p < n_perms; p++) {
        const double *acc = sums + (size_t)p * (size_t)k * 2;
        for (int32_t c = 0; c < k; c++) t[c] = w[c] * (acc[2 * c] + acc[2 * c + 1]);
        qsort(t, (size_t)k, sizeof(double), cmp_double);
        double hi = 0.0, lo = 0.0;
        for (int32_t c = 0; c < k; c++) kadd(&hi, &lo, t[c]);
        out[p] = hi + lo;
    }
    free(t);
}

/* s_W of every grouping row over the whole n x n matrix.  Returns 0, or -1 on
 * a label outside [0, k) or an allocation failure. */
int oracle_sW(const float *mat, int64_t n, const int32_t *groupings, int64_t n_perms, int32_t k,
              const double *w, double *out, int nthreads) {
    double *sums = (double *)calloc((size_t)(n_perms > 0 ? n_perms : 1) * (size_t)k * 2,
                                    sizeof(double));
    if (!sums) return -1;
    int rc = oracle_group_sums(mat, 0, n, n, groupings, n_perms, k, sums, nthreads);
    if (rc == 0) oracle_sW_from_sums(sums, n_perms, k, w, out);
    free(sums);
    return rc;
}

/* ---------------------------------------------------------------------------
 * s_T and the between-group sum.
 * ------------------------------------------------------------------------- */

/* Continues the compensated pair acc[0] + acc[1] with d_ab^2 over the block's
 * rows, columns b > a (see oracle_group_sums for the block convention). */
void oracle_sq_sum(const float *rows, int64_t row0, int64_t nrows, int64_t n, double *acc) {
    double hi = acc[0], lo = acc[1];
    for (int64_t a = row0; a < row0 + nrows && a < n; a++) {
        const float *row = rows + (uint64_t)(a - row0) * (uint64_t)n;
        for (int64_t b = a + 1; b < n; b++) {
            const double x = (double)row[b];
            kadd(&hi, &lo, x * x);
        }
    }
    acc[0] = hi;
    acc[1] = lo;
}

double oracle_sT(const float *mat, int64_t n) {
    double acc[2] = {0.0, 0.0};
    oracle_sq_sum(mat, 0, n, n, acc);
    return (acc[0] + acc[1]) / (double)n;
}

/* Sum of d_ab^2 over the pairs a < b in DIFFERENT groups (no weights): the
 * "between" part, for the within + between = total pin. */
double oracle_between_unweighted(const float *mat, int64_t n, const int32_t *grouping) {
    double hi = 0.0, lo = 0.0;
    for (int64_t a = 0; a < n; a++) {
        const float *row = mat + (uint64_t)a * (uint64_t)n;
        for (int64_t b = a + 1; b < n; b++) {
            if (grouping[a] == grouping[b]) continue;
            const double x = (double)row[b];
            kadd(&hi, &lo, x * x);
        }
    }
    return hi + lo;
}

/* ---------------------------------------------------------------------------
 * F and the p-value.
 * ------------------------------------------------------------------------- */

/* pseudo-F for each s_W: ((s_T - s_W)/(k-1)) / (s_W/(n-k)); NaN when k < 2 or
 * n <= k (the statistic is undefined there). */
void oracle_F(const double *sW, int64_t count, double sT, int64_t n, int32_t k, double *F) {
    for (int64_t i = 0; i < count; i++) {
        if (k < 2 || n <= k) {
            F[i] = NAN;
        } else {
            const double between = (sT - sW[i]) / (double)(k - 1);
            const double within = sW[i] / (double)(n - k);
            F[i] = between / within;
        }
    }
}

/* Textbook count: p = (1 + #{q : F_q >= F_obs}) / (1 + P); NaN when P = 0. */
double oracle_pvalue_F(double F_obs, const double *F_perm, int64_t n_perms) {
    if (n_perms <= 0) return NAN;
    int64_t hits = 0;
    for (int64_t q = 0; q < n_perms; q++) hits += F_perm[q] >= F_obs;
    return (double)(1 + hits) / (double)(1 + n_perms);
}

/* The same count through s_W with a relative tie tolerance:
 * p = (1 + #{q : s_W[q] <= s_W_obs + rtol |s_W_obs|}) / (1 + P).  With
 * rtol = 0 it equals oracle_pvalue_F whenever k >= 2, n > k and s_W > 0. */
double oracle_pvalue(double sW_obs, const double *sW_perm, int64_t n_perms, double rtol) {
    if (n_perms <= 0) return NAN;
    const double edge = sW_obs + rtol * fabs(sW_obs);
    int64_t hits = 0;
    for (int64_t q = 0; q < n_perms; q++) hits += sW_perm[q] <= edge;
    return (double)(1 + hits) / (double)(1 + n_perms);
}

/* ---------------------------------------------------------------------------
 * Permutation generator.
 * ------------------------------------------------------------------------- */

static uint64_t splitmix_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* SplitMix64: advance the state by the golden gamma, return the mixed state. */
uint64_t oracle_splitmix64_next(uint64_t *state) {
    *state += 0x9E3779B97F4A7C15ULL;
    return splitmix_mix(*state);
}

/* Start state of permutation p's stream: mix(seed XOR mix(p + 1)). */
uint64_t oracle_stream_start(uint64_t seed, uint64_t p) {
    return splitmix_mix(seed ^ splitmix_mix(p + 1));
}

/* Uniform integer in [0, s), s >= 1 (Lemire 2019): x = the upper 32 bits of the
 * next output, m = x * s; the low word of m below 2^32 mod s means x falls in
 * the over-represented part and is redrawn; the high word of m is the value. */
uint32_t oracle_bounded(uint64_t *state, uint32_t s) {
    const uint32_t reject_below = (uint32_t)(0u - s) % s;   /* 2^32 mod s */
    for (;;) {
        const uint32_t x = (uint32_t)(oracle_splitmix64_next(state) >> 32);
        const uint64_t m = (uint64_t)x * (uint64_t)s;
        if ((uint32_t)m >= reject_below) return (uint32_t)(m >> 32);
    }
}

/* Test helper: the number of draws oracle_permute's bounded draws discard
 * over n_perms shuffles of n labels (which inputs exercise the rejection). */
int64_t oracle_count_rejections(int64_t n, int64_t n_perms, uint64_t seed) {
    int64_t total = 0;
    for (int64_t p = 0; p < n_perms; p++) {
        uint64_t st = oracle_stream_start(seed, (uint64_t)p);
        for (int64_t top = n - 1; top >= 1; top--) {
            const uint32_t s = (uint32_t)(top + 1);
            const uint32_t reject_below = (uint32_t)(0u - s) % s;
            for (;;) {
                const uint32_t x = (uint32_t)(oracle_splitmix64_next(&st) >> 32);
                if ((uint32_t)((uint64_t)x * (uint64_t)s) >= reject_below) break;
                total++;
            }
        }
    }
    return total;
}

/* groupings[p*n + a]: Durstenfeld's Fisher-Yates on a copy of base with the
 * stream of permutation p -- for top = n-1 down to 1, swap the entry at top
 * with the one at a uniform position in [0, top]. */
void oracle_permute(const int32_t *base, int64_t n, int64_t n_perms, uint64_t seed,
                    int32_t *groupings, int nthreads) {
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n_perms; p++) {
        int32_t *lab = groupings + p * n;
        memcpy(lab, base, (size_t)n * sizeof(int32_t));
        uint64_t st = oracle_stream_start(seed, (uint64_t)p);
        for (int64_t top = n - 1; top >= 1; top--) {
            const int64_t pick = (int64_t)oracle_bounded(&st, (uint32_t)(top + 1));
            const int32_t held = lab[top];
            lab[top] = lab[pick];
            lab[pick] = held;
        }
    }
}
