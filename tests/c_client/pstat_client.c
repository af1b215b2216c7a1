/* A consumer of the pstat C ABI written in plain C: no Python, no torch.
 * Device memory comes from the HIP runtime's C API; the program runs the
 * shuffle, the group weights, s_W on four forms and the whole permutation
 * test on a matrix whose every off-diagonal distance is 0.5, where the
 * statistic has a closed form (section 2's sum): every pair in a group adds
 * 0.25 / n_g, so s_W = 0.25 * sum_g (n_g - 1) / 2 = (n - k) / 8 for any
 * grouping with those sizes, s_T = (n - 1) / 8, F = 1 and, all statistics
 * being equal, p = 1.  Exit status 0 when every check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "pstat.h"

#define CHECK(x)                                                                     \
    do {                                                                             \
        int rc_ = (x);                                                               \
        if (rc_ != PSTAT_OK) {                                                       \
            fprintf(stderr, "%s:%d: %s -> %d (%s)\n", __FILE__, __LINE__, #x, rc_,   \
                    pstat_last_error());                                             \
            return 1;                                                                \
        }                                                                            \
    } while (0)
#define HCHECK(x)                                                                    \
    do {                                                                             \
        hipError_t e_ = (x);                                                         \
        if (e_ != hipSuccess) {                                                      \
            fprintf(stderr, "%s:%d: %s -> %s\n", __FILE__, __LINE__, #x,             \
                    hipGetErrorString(e_));                                          \
            return 1;                                                                \
        }                                                                            \
    } while (0)

static int close_to(double got, double want, double rtol) {
    return fabs(got - want) <= rtol * fabs(want);
}

int main(void) {
    enum { N = 1000, K = 4, P = 63 };
    static const int sizes[K] = {100, 200, 300, 400};
    const double sW_want = (double)(N - K) / 8.0, sT_want = (double)(N - 1) / 8.0;

    float *hm = (float *)malloc(sizeof(float) * N * N);
    int32_t *hb = (int32_t *)malloc(sizeof(int32_t) * N);
    double *hout = (double *)malloc(sizeof(double) * P);
    if (!hm || !hb || !hout) return 1;
    for (int i = 0; i < N; i++)
        for (int j = 0; j < N; j++) hm[(size_t)i * N + j] = i == j ? 0.0f : 0.5f;
    for (int g = 0, i = 0; g < K; g++)
        for (int c = 0; c < sizes[g]; c++) hb[i++] = g;

    CHECK(pstat_init(0));
    float *mat;
    int32_t *base, *groupings;
    double *inv, *out, *result;
    HCHECK(hipMalloc((void **)&mat, sizeof(float) * N * N));
    HCHECK(hipMalloc((void **)&base, sizeof(int32_t) * N));
    HCHECK(hipMalloc((void **)&groupings, sizeof(int32_t) * N * P));
    HCHECK(hipMalloc((void **)&inv, sizeof(double) * K));
    HCHECK(hipMalloc((void **)&out, sizeof(double) * P));
    HCHECK(hipMalloc((void **)&result, sizeof(double) * 4));
    HCHECK(hipMemcpy(mat, hm, sizeof(float) * N * N, hipMemcpyHostToDevice));
    HCHECK(hipMemcpy(base, hb, sizeof(int32_t) * N, hipMemcpyHostToDevice));

    CHECK(pstat_permute(base, N, P, 3000, groupings));
    CHECK(pstat_group_weights(base, N, K, inv));

    static const int paths[4] = {PSTAT_PATH_PLAIN_F32, PSTAT_PATH_PLAIN_F64,
                                 PSTAT_PATH_MFMA_SPLIT_BF16, PSTAT_PATH_MFMA_BF16};
    for (int q = 0; q < 4; q++) {
        CHECK(pstat_set_path(paths[q]));
        CHECK(pstat_sW(mat, N, groupings, P, inv, out));
        HCHECK(hipMemcpy(hout, out, sizeof(double) * P, hipMemcpyDeviceToHost));
        for (int p = 0; p < P; p++)
            if (!close_to(hout[p], sW_want, 1e-12)) {
                fprintf(stderr, "path %d: s_W[%d] = %.17g, want %.17g\n", paths[q], p, hout[p],
                        sW_want);
                return 1;
            }
    }

    int64_t rechecked = -1;
    double hr[4];
    CHECK(pstat_set_path(PSTAT_PATH_MFMA_SPLIT_BF16));
    CHECK(pstat_permanova(mat, N, base, K, P, 3000, result, NULL, &rechecked));
    HCHECK(hipMemcpy(hr, result, sizeof hr, hipMemcpyDeviceToHost));
    if (!close_to(hr[0], 1.0, 1e-9) || hr[1] != 1.0 || !close_to(hr[2], sW_want, 1e-12) ||
        !close_to(hr[3], sT_want, 1e-12)) {
        fprintf(stderr, "permanova: F %.17g p %.17g s_W %.17g s_T %.17g\n", hr[0], hr[1], hr[2],
                hr[3]);
        return 1;
    }
    /* a bad size is refused before any launch */
    if (pstat_sW(mat, 1, groupings, P, inv, out) != PSTAT_EINVAL) {
        fprintf(stderr, "n = 1 was not refused\n");
        return 1;
    }

    HCHECK(hipFree(mat));
    HCHECK(hipFree(base));
    HCHECK(hipFree(groupings));
    HCHECK(hipFree(inv));
    HCHECK(hipFree(out));
    HCHECK(hipFree(result));
    free(hm);
    free(hb);
    free(hout);
    printf("ok: s_W %.6f on 4 forms, F %.6f, p %.6f, %lld rechecked\n", sW_want, hr[0], hr[1],
           (long long)rechecked);
    return 0;
}
