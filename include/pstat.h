/*
 * pstat -- PERMANOVA's permuted within-group statistic s_W on AMD MI355X (gfx950).
 *
 * C ABI of libpstat.so.  Every entry point is extern "C", returns an int status
 * (PSTAT_OK or a negative PSTAT_E* code), never throws, and leaves its outputs
 * unwritten when it returns an error.  pstat_last_error() gives a readable
 * reason (thread-local; includes the HIP error string where one exists).
 *
 * Memory.  Unless stated otherwise every array argument is a DEVICE pointer
 * (hipMalloc'd or a torch CUDA tensor's storage) owned by the caller; the library
 * never frees or keeps a caller pointer after a call returns, except a matrix
 * registered with pstat_matrix_register, which must stay alive until
 * pstat_matrix_release.  A host pointer passed where a device pointer is
 * required gives PSTAT_EPTR.
 *
 * Streams.  Work is enqueued on the calling thread's stream (pstat_set_stream;
 * default: the null stream).  Results are valid once the caller synchronises
 * that stream.  Calls that must look at a value on the device before they can
 * decide what to do (label validation in pstat_sW, the tie recheck in
 * pstat_permanova) synchronise the stream themselves and say so below.
 *
 * Scratch.  The library needs device scratch (staged labels, per-block
 * partials, pre-squared matrix tiles).  If the thread has set a workspace with
 * pstat_set_workspace it is used (PSTAT_ENOMEM if too small, see
 * pstat_workspace_bytes); otherwise the library allocates and caches its own.
 *
 * Layouts.  mat is n x n float32, row-major, 64-bit element offsets
 * (row * n + col); only the strict upper triangle (col > row) is ever read,
 * so it may also be given alone, packed (pstat_set_matrix_layout).
 * groupings is int32, permutation-major: row p (n labels) starts at p * n.
 * Labels are group indices 0 <= g < k (k <= 65535) and index inv_group_sizes.
 */
#ifndef PSTAT_H
#define PSTAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PSTAT_OK 0
#define PSTAT_EINVAL (-1)  /* bad size or argument                         */
#define PSTAT_ELABEL (-2)  /* a label < 0 or >= 65535                      */
#define PSTAT_EDOMAIN (-3) /* F undefined: k < 2 or n <= k                 */
#define PSTAT_ENOMEM (-4)  /* workspace too small / device allocation fail */
#define PSTAT_EHIP (-5)    /* a HIP runtime call failed                    */
#define PSTAT_EPTR (-6)    /* pointer is not device-accessible memory      */
#define PSTAT_ESTATE (-7)  /* pstat_init not called on this thread/device  */

/* ---- computation forms of s_W ------------------------------------------ */
#define PSTAT_PATH_AUTO (-1)           /* the tuned default                */
#define PSTAT_PATH_PLAIN_F32 0         /* VALU kernel, FP32 row segments   */
#define PSTAT_PATH_MFMA_BF16 1         /* MFMA, D^2 in BF16                */
#define PSTAT_PATH_MFMA_F16 2          /* MFMA, D^2 in FP16                */
#define PSTAT_PATH_MFMA_SPLIT_BF16 3   /* MFMA, D^2 as BF16 hi + BF16 lo   */
#define PSTAT_PATH_PLAIN_F64 4         /* VALU kernel, FP64 throughout     */
#define PSTAT_PATH_MFMA_SPLIT3_BF16 5  /* MFMA, D^2 as BF16 hi + mid + lo:
                                          every FP32 square represented
                                          exactly (1.5x the split cost)  */
#define PSTAT_N_PATHS 6

/* ---- context ------------------------------------------------------------ */

/* Library version, major * 10000 + minor * 100 + patch. */
int pstat_version(void);

/* Text of the last error on this thread ("" if none).  Never NULL. */
const char *pstat_last_error(void);

/* Make `device` current for this thread, read its properties and prepare the
 * library's per-device state.  Must precede every other call on the thread. */
int pstat_init(int device);

/* Stream (a hipStream_t, NULL = null stream) for this thread's later calls. */
int pstat_set_stream(void *hip_stream);

/* ---- matrix layouts --------------------------------------------------------
 * Every call reads D only above the diagonal (section 2, Algorithm 1), so it
 * can be given either as the full row-major n x n square or as that strict
 * upper triangle alone, packed row after row: row i holds d_i,i+1 .. d_i,n-1
 * and starts at float i (2n - i - 1) / 2, n (n - 1) / 2 floats in all (half
 * the memory, which is what lets larger n fit on one device).  The layout
 * applies to the `mat` of this thread's later calls (pstat_sW, pstat_sW_k,
 * pstat_sT, pstat_permanova, pstat_matrix_register, pstat_job_create);
 * results are bit-identical in both.  PSTAT_EINVAL for an unknown layout. */
#define PSTAT_LAYOUT_SQUARE 0
#define PSTAT_LAYOUT_UPPER_PACKED 1
int pstat_set_matrix_layout(int layout);

/* Form used by pstat_sW / pstat_sW_k / pstat_permanova on this thread.
 * PSTAT_PATH_AUTO (default) = the tuned choice for the problem shape.  The
 * MFMA forms need at least two groups: with a single group the plain FP32
 * form runs instead. */
int pstat_set_path(int path);

/* The form PSTAT_PATH_AUTO stands for at n objects and n_groups groups (other
 * paths are returned unchanged; PSTAT_EINVAL for an unknown path -- a resolved
 * path is never negative).  Host only; needs no device. */
int pstat_resolve_path(int path, int64_t n, int32_t n_groups);

/* Tuning of one path for this thread: `tile` and `batch` override the tuned
 * values (0 = keep the tuned value).  Plain paths: tile = square tile edge
 * (32 or 64), batch = permutation lanes per work-group (64, 128 or 256).  MFMA
 * paths: tile = K-chunk length in columns (multiple of 64, rounded up to a
 * multiple of 128; 0 = the library's choice: 2,048 columns for 16,256 < n <=
 * 130,944, 1,536 for 8,064 < n <= 16,256, else 1,024), batch = N columns per
 * work-group (256 or 512).
 * Invalid values give PSTAT_EINVAL. */
int pstat_set_tuning(int path, int tile, int batch);

/* Caller-owned device workspace for this thread (NULL, 0 = library-managed). */
int pstat_set_workspace(void *dev_ptr, size_t bytes);

/* Free the library-managed workspace of this thread (after the device's
 * queued work has finished); the next call that needs one allocates it
 * again.  For callers that alternate very large problems with other device
 * work.  PSTAT_OK when there is none. */
int pstat_free_workspace(void);

/* Workspace pstat_sW_k needs for this shape and path (bytes), 0 on bad input. */
size_t pstat_workspace_bytes(int64_t n, int64_t n_perms, int32_t n_groups, int path);

/* ---- the statistic (section 2, Algorithm 1) ------------------------------ */

/* out[p] = s_W of grouping row p, p = 0 .. n_perms-1:
 *   s_W = sum over 0 <= i < j < n with g[i] == g[j] of mat[i*n+j]^2 * inv_group_sizes[g[i]],
 * the paper's permanova_f_stat_sW_T with the paper's argument order.  k is
 * found as 1 + the largest label, so inv_group_sizes must hold at least that
 * many FP64 weights (normally 1/n_g).  Validates every label first and
 * SYNCHRONISES the stream once to read the result: PSTAT_ELABEL on a label
 * outside [0, 65535).  n >= 2, n_perms >= 0 (0: nothing to do). */
int pstat_sW(const float *mat, int64_t n, const int32_t *groupings, int64_t n_perms,
             const double *inv_group_sizes, double *out);

/* pstat_sW with the number of groups given (labels must lie in [0, n_groups)):
 * no synchronisation.  A label out of range is reported asynchronously: the
 * affected out[p] are set to NaN and the next pstat_check_labels on this
 * thread returns PSTAT_ELABEL. */
int pstat_sW_k(const float *mat, int64_t n, const int32_t *groupings, int64_t n_perms,
               int32_t n_groups, const double *inv_group_sizes, double *out);

/* pstat_sW_k for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * calls no hipMalloc, hipFree or other allocating routine; its scratch is a
 * static device array of pstat_noalloc_scratch_bytes() bytes (64 MiB), one
 * per device, reserved when the library's code is loaded on that device and
 * held until the process ends; the thread's workspace (pstat_set_workspace)
 * is not used.  Same arguments, results and asynchronous label check as
 * pstat_sW_k, on the thread's form, layout and stream (pstat_profile does not
 * time it).  *scratch_bytes (host, may be NULL) receives the scratch the
 * shape needs; a shape needing more than the array gives PSTAT_ENOMEM before
 * any launch, with out untouched.  Every call on one device shares that
 * device's array: calls that overlap on one device (two threads, or two
 * streams without ordering between them) race and give wrong results; calls
 * ordered on one stream are safe (each call writes before it reads every
 * byte of scratch it uses, so nothing left by an earlier call is read). */
int pstat_sW_k_noalloc(const float *mat, int64_t n, const int32_t *groupings, int64_t n_perms,
                       int32_t n_groups, const double *inv_group_sizes, double *out,
                       size_t *scratch_bytes);

/* Size of pstat_sW_k_noalloc's static scratch array, bytes. */
size_t pstat_noalloc_scratch_bytes(void);

/* PSTAT_OK if no out-of-range label was seen by this thread's pstat_sW_k calls
 * since the previous check, else PSTAT_ELABEL.  Synchronises the stream. */
int pstat_check_labels(void);

/* ---- the steps around it (section 2: "before and after") ---------------- */

/* *s_T = (1/n) * sum_{i<j} mat[i*n+j]^2, FP64 (device scalar). */
int pstat_sT(const float *mat, int64_t n, double *s_T);

/* F[i] = ((s_T - s_W[i]) / (k-1)) / (s_W[i] / (n-k)), FP64; s_T is a device
 * scalar.  PSTAT_EDOMAIN if k < 2 or n <= k. */
int pstat_F(const double *s_W, int64_t count, const double *s_T, int64_t n, int32_t k,
            double *F);

/* Relative tie tolerance of the p-value (a reading of the permutation test of
 * section 1): a permutation's statistic counts as at least as extreme as the
 * observed one when s_W_perm <= s_W_obs + PSTAT_TIE_RTOL * |s_W_obs|.
 * Groupings whose s_W are equal in exact arithmetic -- the observed partition
 * reached again under other labels, any grouping of a constant matrix -- then
 * tie whatever order their FP64 sums were taken in (FP64 rounding of s_W is
 * ~1e-13 relative at n = 10^5), while statistics that differ by more than
 * 1e-10 are told apart (FP32 storage of d already blurs s_W at ~1e-8). */
#define PSTAT_TIE_RTOL 1e-10

/* *p = (1 + #{q : s_W_perm[q] <= *s_W_obs + PSTAT_TIE_RTOL |*s_W_obs|}) /
 * (1 + n_perms), FP64, device scalars: the count of F_q >= F_obs (F falls as
 * s_W grows, for k >= 2, n > k, s_W > 0) with ties taken at that tolerance.
 * NaN values never count.  n_perms = 0 gives NaN. */
int pstat_pvalue(const double *s_W_obs, const double *s_W_perm, int64_t n_perms, double *p);

/* inv[g] = 1 / #{i : grouping[i] == g} for g < n_groups (0 for an empty group),
 * FP64 (the weights PERMANOVA passes as inv_group_sizes). */
int pstat_group_weights(const int32_t *grouping, int64_t n, int32_t n_groups, double *inv);

/* groupings[p*n + i], p < n_perms: Durstenfeld's Fisher-Yates shuffle of base
 * (n labels, device) for permutation p, driven by SplitMix64 started at
 * mix(seed XOR mix(p + 1)) with Lemire's bounded draw -- the random relabeling
 * of the permutation test (section 1).  Labels must lie in [0, 65535). */
int pstat_permute(const int32_t *base, int64_t n, int64_t n_perms, uint64_t seed,
                  int32_t *groupings);

/* The whole permutation test on one matrix, all on the device:
 * weights 1/n_g from `grouping` (n_groups groups), n_perms shuffles
 * (pstat_permute with `seed`), s_W of the observed grouping and of every
 * shuffle, s_T, F and p (as pstat_pvalue, ties at PSTAT_TIE_RTOL).  The
 * observed grouping and the first 7 shuffles are recomputed in FP64; the
 * largest relative error of the form over those 8, times 16, is the band
 * (at least 1e-13): every shuffle whose s_W lies within the band of the
 * p-value's edge (from the observed value to PSTAT_TIE_RTOL above it) is
 * recomputed in FP64 too before counting.  The band is measured, not a
 * proven bound: a shuffle outside it whose error exceeded it could land on
 * the wrong side.  The call SYNCHRONISES the
 * stream twice (label check, count of near ties).  F counts the non-empty
 * groups among the n_groups labels.  result (device, 4 doubles) =
 * {F_obs, p, s_W_obs, s_T}; sW_all (device, n_perms + 1 doubles, may be NULL)
 * receives s_W of the observed grouping then of each shuffle; n_rechecked
 * (host, may be NULL) receives how many permutations were recomputed.  On
 * the MFMA forms every grouping here has the observed group sizes, so the
 * largest group's within-group sum is taken as the complement of the others
 * (k - 1 one-hot columns instead of k); its values agree with pstat_sW's to
 * the form's tolerance, not bit for bit. */
int pstat_permanova(const float *mat, int64_t n, const int32_t *grouping, int32_t n_groups,
                    int64_t n_perms, uint64_t seed, double *result, double *sW_all,
                    int64_t *n_rechecked);

/* ---- resident matrices -------------------------------------------------- */

/* Register a resident matrix for repeated tests: the library keeps the MFMA
 * forms' pre-squared tiles (when `path` is an MFMA path) so later calls skip
 * that staging.  `mat` must stay valid until release.  *handle > 0. */
int pstat_matrix_register(const float *mat, int64_t n, int path, int64_t *handle);
int pstat_matrix_release(int64_t handle);

/* pstat_sW_k on a registered matrix with that registration's path. */
int pstat_sW_registered(int64_t handle, const int32_t *groupings, int64_t n_perms,
                        int32_t n_groups, const double *inv_group_sizes, double *out);

/* ---- many tests at once (serving) ----------------------------------------- */
/* Not part of the paper's statement of the problem: the device side of a
 * serving loop that keeps several permutation tests resident and runs their
 * work in shared launches.  A job is one whole test (as pstat_permanova) on
 * the plain FP32 kernel (tile 32, 256 permutation lanes) or the split-BF16
 * MFMA kernel (512 columns per work-group); its work is n_units units (one
 * work-group each).  A round runs any list of units of any live jobs in one
 * launch per form of the work-list kernels, replayed from a captured hipGraph
 * (two graphs alternate, so a round's unit list can be filled while the
 * previous round runs).  A job's result depends only on its own units and a
 * fixed reduction order: it is bit-identical alone and in any mix. */

/* Server with room for max_jobs live jobs and max_units units per round. */
int pstat_serve_create(int64_t max_jobs, int64_t max_units, int64_t *server);
/* Waits for its rounds, frees the server (job scratch stays the caller's). */
int pstat_serve_destroy(int64_t server);

/* Device scratch bytes one job needs (caller-owned, kept until release);
 * path: PSTAT_PATH_PLAIN_F32, PSTAT_PATH_MFMA_SPLIT_BF16 or PSTAT_PATH_AUTO. */
size_t pstat_job_bytes(int64_t n, int64_t n_perms, int32_t n_groups, int path);

/* Stage a test into `scratch` for form `path` (as pstat_job_bytes): validates
 * `grouping` (SYNCHRONISES the stream), weights, the n_perms shuffles of
 * pstat_permute(seed), staged labels (and for MFMA the pre-squared tiles).  mat
 * must stay valid until release.  *job: the job's id; *n_units: its units,
 * numbered 0 .. n_units-1. */
int pstat_job_create(int64_t server, const float *mat, int64_t n, const int32_t *grouping,
                     int32_t n_groups, int64_t n_perms, uint64_t seed, int path, void *scratch,
                     size_t scratch_bytes, int64_t *job, int64_t *n_units);

/* Run `count` units (host array of (job, unit) pairs, 2*count int64) in one
 * launch on the thread's stream (which must not be the null stream).  Returns
 * once the launch is queued; waits only for the round that used the same
 * unit buffer two rounds ago.  Each unit of a job must run exactly once before
 * pstat_job_finish. */
int pstat_serve_round(int64_t server, const int64_t *units, int64_t count);

/* After all of a job's units have run: FP64 reduction, s_T, FP64 recheck of
 * the observed grouping and near ties, F and p.  SYNCHRONISES the stream.
 * result (HOST, 4 doubles) = {F_obs, p, s_W_obs, s_T}; sW_all (device, may be
 * NULL) receives s_W of the observed grouping then of each shuffle. */
int pstat_job_finish(int64_t server, int64_t job, double *result, double *sW_all,
                     int64_t *n_rechecked);

/* Free the job's slot (waits for rounds still in flight). */
int pstat_job_release(int64_t server, int64_t job);

/* ---- measurement -------------------------------------------------------- */

/* While enabled (on != 0), every s_W evaluation on this thread records a pair
 * of HIP events on its stream around its main kernel (the plain kernel or the
 * MFMA kernel; not staging, pre-pass or reduction).  Enabling clears earlier
 * records. */
int pstat_profile(int on);

/* Synchronises the recorded events and returns the summed duration of the
 * main-kernel launches recorded since pstat_profile(1) (*ms, milliseconds)
 * and their count (*launches); both host pointers, either may be NULL. */
int pstat_profile_read(double *ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* PSTAT_H */
