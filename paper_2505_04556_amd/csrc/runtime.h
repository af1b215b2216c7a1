// Runtime internals shared by the C-ABI translation units (pstat_runtime.hip,
// pstat_serve.hip).  Not installed.
#pragma once

#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/pstat.h"
#include "internal.h"

namespace pstat {
namespace rt {

constexpr int kVersion = 10000;  // 1.0.0

struct Tuning {
    int tile = 0;
    int batch = 0;
};

struct DeviceInfo {
    bool ready = false;
    int n_cu = 256;
    size_t lds_limit = 65536;
    // this device's copy of the static scratch array of pstat_sW_k_noalloc
    // (its device address, from hipGetSymbolAddress at pstat_init)
    char *static_scratch = nullptr;
};

struct Thread {
    int device = -1;
    hipStream_t stream = nullptr;
    int path = PSTAT_PATH_AUTO;
    int packed = 0;   // layout of the matrices passed on this thread (PSTAT_LAYOUT_*)
    Tuning tuning[PSTAT_N_PATHS];
    void *ws_user = nullptr;
    size_t ws_user_bytes = 0;
    // library-managed workspace (per thread, per device in use)
    void *ws_own = nullptr;
    size_t ws_own_bytes = 0;
    int ws_own_device = -1;
    // small device scalars: [0] label error flag (sticky for pstat_sW_k),
    // [1] max label, [2] tie count
    int32_t *flags = nullptr;
    int flags_device = -1;
    int32_t *host_flags = nullptr;  // pinned
    // main-kernel timing (pstat_profile)
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    char err[512] = {0};
};

extern thread_local Thread tls;

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
#define HIP_TRY(expr)                                      \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);  \
    } while (0)
int check_launch(const char *what);
int need_init();
const DeviceInfo &dev_info();
int check_dev_ptr(const void *p, const char *name);

// ---- workspace carving --------------------------------------------------------
struct Carver {
    char *base;
    size_t cap;
    size_t used = 0;
    bool dry;  // size-only pass
    void *take(size_t bytes) {
        used = (used + 255) & ~(size_t)255;
        void *p = dry ? nullptr : base + used;
        used += bytes;
        return p;
    }
};

int acquire_workspace(size_t bytes, char **out);

bool is_mfma(int path);
int mfma_dtype(int path);
int resolve_path(int path, int64_t n, int32_t k);
void plain_params(int path, int64_t P, int *tile, int *lanes);
void mfma_params(int path, int *kchunk_cols, int *ncols);

// ---- s_W on a staged problem ------------------------------------------------
// Scratch of one s_W evaluation of P permutations on the given path.
struct SwLayout {
    int path = 0;
    uint8_t *bad = nullptr;      // per-permutation "had a bad label" flags
    uint16_t *lab = nullptr;     // staged labels
    uint32_t *lab4 = nullptr;    // MFMA, k <= 15: the same packed four bits each
    double *partial = nullptr;   // plain: [chunks][P_pad]
    void *tiles = nullptr;       // MFMA: pre-squared tiles (unless registered)
    int32_t *tab = nullptr;      // MFMA: work-item table
    float *z = nullptr;          // MFMA: [items][P][k] (complement: [items][P][k-1][2])
    double *tmp = nullptr;       // MFMA: [P][k] (complement: [P][k-1][2])
    Complement cx{};             // MFMA complement form (mp.cx)
    PlainPlan pp{};
    MfmaPlan mp{};
};

// cx: the MFMA forms may use the complement form (every grouping must have
// the group sizes of the first; the pre-pass must run, not registered tiles).
void layout_sW(Carver &c, int64_t n, int64_t P, int32_t k, int path, bool own_tiles,
               SwLayout &L, bool cx = false);
size_t sW_bytes(int64_t n, int64_t P, int32_t k, int path, bool own_tiles, bool cx = false);

// Event pair around the main kernel when this thread is profiling.
struct KernelTimer {
    hipEvent_t a = nullptr, b = nullptr;
    KernelTimer(hipStream_t s, bool timed) {
        if (!tls.profiling || !timed) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            (void)hipGetLastError();
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, s);
    }
    void stop(hipStream_t s) {
        if (!a) return;
        (void)hipEventRecord(b, s);
        tls.events.emplace_back(a, b);
        a = b = nullptr;
    }
};

int exec_sW(const SwLayout &L, const float *mat, int64_t n, const int32_t *g,
            const int32_t *rows, int64_t P, int32_t k, int32_t limit, const double *w,
            double *out, const void *tiles, int32_t *err_flag, bool timed = true,
            double *sT_part = nullptr, double *sT = nullptr, bool staged = false,
            const PrepassRecheck *samples = nullptr, int packed = 0);
int scan_labels_sync(const int32_t *g, int64_t count, int32_t limit, int32_t *max_label);

// ---- the whole permutation test in phases ------------------------------------
// Device buffers of one test with R = n_perms + 1 groupings (the observed one
// first); they live through the test.
struct TestHead {
    int32_t *allg;     // int32 [R][n]
    double *w;         // [k] weights 1/n_g
    uint32_t *counts;  // [k]
    double *sw;        // [R] s_W
    double *sTp;       // [nsT + 1] s_T partials, then s_T
    double *sT;
    double *pv;        // p-value
    int32_t *list;     // [R] row lists of the recheck
    double *vals;      // [R] recheck values
    double *band;      // tie band
    double *result;    // [4] F_obs, p, s_W_obs, s_T
    double *rcp;       // [prepass_blocks(n)][kRecheckRows] partials of the
                       // pre-pass's FP64 recheck of the first rows
};
void carve_head(Carver &c, int64_t n, int64_t R, int32_t k, TestHead &h);
// Observed grouping into row 0, n_perms shuffles after it, weights.
int prepare_test(const TestHead &h, int64_t n, const int32_t *grouping, int32_t k,
                 int64_t n_perms, uint64_t seed, int32_t max_label);
// After h.sw holds the fast path's s_W of all R rows: s_T, FP64 recheck of the
// observed grouping, band samples and near ties, p-value, result.  `region` is
// scratch of at least few_partial_bytes(n, R) bytes.
// sT_ready: s_T was already left in h.sT (by the pre-pass of the MFMA forms).
// lab16: the groupings as staged u16 rows of stride16 entries (else h.allg);
// region must not overlap them.  samples_ready: the FP64 s_W of the observed
// grouping and the first kBandSamples permutations is already in h.vals (the
// MFMA pre-pass computed it).
int finish_test(const TestHead &h, const float *mat, int64_t n, int32_t k, int64_t n_perms,
                int path, char *region, size_t region_bytes, int64_t *rechecked,
                bool sT_ready = false, const uint16_t *lab16 = nullptr, int64_t stride16 = 0,
                bool samples_ready = false, int packed = 0);

// Tie band of the p-value recheck: kBandMargin times the largest relative
// error of the fast path over the observed grouping and the first
// kBandSamples permutations (all recomputed in FP64).
constexpr int64_t kBandSamples = 7;
constexpr double kBandMargin = 16.0;

} // namespace rt
} // namespace pstat
