// C ABI of libpstat.so (include/pstat.h): argument checks, per-thread context,
// workspace carving, path dispatch and the whole-test driver.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <vector>

#include "../../include/pstat.h"
#include "runtime.h"

namespace pstat {
namespace rt {

thread_local Thread tls;  // declared in runtime.h

// Scratch of pstat_sW_k_noalloc: a file-scope device array, one copy per
// device, held until the process ends.  Host code never uses this name as an
// address (on the host it is only a stand-in for the symbol): pstat_init
// takes each device's address with hipGetSymbolAddress and keeps it in
// DeviceInfo::static_scratch.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

std::mutex g_mu;
std::map<int, DeviceInfo> g_devices;

struct Registered {
    const float *mat;
    int64_t n;
    int path;
    int device;
    void *tiles;
    int packed;   // layout of mat
};
std::map<int64_t, Registered> g_registered;
int64_t g_next_handle = 1;

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(tls.err, sizeof(tls.err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    (void)hipGetLastError();
    return fail(PSTAT_EHIP, "%s: %s", what, hipGetErrorString(e));
}


int check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PSTAT_EHIP, "%s launch: %s", what, hipGetErrorString(e));
    return PSTAT_OK;
}

int need_init() {
    if (tls.device < 0) return fail(PSTAT_ESTATE, "pstat_init has not been called on this thread");
    return PSTAT_OK;
}

const DeviceInfo &dev_info() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_devices[tls.device];
}

// A device pointer: hipMalloc'd or managed memory.
int check_dev_ptr(const void *p, const char *name) {
    if (!p) return fail(PSTAT_EINVAL, "%s is NULL", name);
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PSTAT_EPTR, "%s is not device memory", name);
    }
    if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
        return fail(PSTAT_EPTR, "%s is not device memory (memory type %d)", name, (int)a.type);
    return PSTAT_OK;
}


int acquire_workspace(size_t bytes, char **out) {
    if (tls.ws_user) {
        if (tls.ws_user_bytes < bytes)
            return fail(PSTAT_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed",
                        tls.ws_user_bytes, bytes);
        *out = (char *)tls.ws_user;
        return PSTAT_OK;
    }
    if (tls.ws_own && tls.ws_own_device == tls.device && tls.ws_own_bytes >= bytes) {
        *out = (char *)tls.ws_own;
        return PSTAT_OK;
    }
    if (tls.ws_own) {
        // The previous owner may still be in use by queued work on this stream.
        HIP_TRY(hipStreamSynchronize(tls.stream));
        (void)hipFree(tls.ws_own);
        tls.ws_own = nullptr;
        tls.ws_own_bytes = 0;
    }
    size_t grow = bytes + bytes / 4 + (1 << 20);
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, grow);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        e = hipMalloc(&p, bytes);
        grow = bytes;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PSTAT_ENOMEM, "could not allocate %zu bytes of device workspace", bytes);
    }
    tls.ws_own = p;
    tls.ws_own_bytes = grow;
    tls.ws_own_device = tls.device;
    *out = (char *)p;
    return PSTAT_OK;
}

bool is_mfma(int path) {
    return path == PSTAT_PATH_MFMA_BF16 || path == PSTAT_PATH_MFMA_F16 ||
           path == PSTAT_PATH_MFMA_SPLIT_BF16 || path == PSTAT_PATH_MFMA_SPLIT3_BF16;
}
int mfma_dtype(int path) {
    return path == PSTAT_PATH_MFMA_BF16 ? 0 : path == PSTAT_PATH_MFMA_F16 ? 1
         : path == PSTAT_PATH_MFMA_SPLIT3_BF16 ? 3 : 2;
}

// Default form for a shape when the thread asked for PSTAT_PATH_AUTO (the
// autotuner's per-shape choices are applied through pstat_set_path): the MFMA
// contraction costs 4k flops per pair-permutation in split BF16 against two
// VALU operations for the plain kernel at 1/64 of the matrix-core rate,
// so it wins while k stays small; tiny matrices stay on the plain kernel.
int resolve_path(int path, int64_t n, int32_t k) {
    if (path == PSTAT_PATH_AUTO)
        return (n >= 512 && k >= 2 && k <= 16) ? PSTAT_PATH_MFMA_SPLIT_BF16 : PSTAT_PATH_PLAIN_F32;
    // The MFMA kernels stage the labels of at most half a work-group's
    // columns' worth of permutations (k >= 2); a single group runs plain.
    if (is_mfma(path) && k < 2) return PSTAT_PATH_PLAIN_F32;
    return path;
}

void plain_params(int path, int64_t P, int *tile, int *lanes) {
    const Tuning &t = tls.tuning[path];
    *tile = t.tile ? t.tile : 32;
    // Few permutations (the FP64 recheck): narrower work-groups keep more of
    // the lanes busy.
    *lanes = t.batch ? t.batch : (P <= 64 ? 64 : P <= 128 ? 128 : 256);
    if (path == PSTAT_PATH_PLAIN_F64 && *tile > 32) *tile = 32;
}

void mfma_params(int path, int *kchunk_cols, int *ncols) {
    const Tuning &t = tls.tuning[path];
    *kchunk_cols = t.tile;   // 0 = planner's choice
    *ncols = t.batch ? t.batch : 512;
}

void layout_sW(Carver &c, int64_t n, int64_t P, int32_t k, int path, bool own_tiles,
               SwLayout &L, bool cx) {
    L.path = path;
    L.bad = (uint8_t *)c.take((size_t)(P > 0 ? P : 1));
    if (!is_mfma(path)) {
        int tile, lanes;
        plain_params(path, P, &tile, &lanes);
        L.pp = plain_plan(n, P, tile, lanes, dev_info().n_cu);
        L.lab = (uint16_t *)c.take((size_t)L.pp.n_pad * L.pp.P_pad * sizeof(uint16_t));
        L.partial = (double *)c.take((size_t)L.pp.chunks * L.pp.P_pad * sizeof(double));
        return;
    }
    int kchunk_cols, ncols;
    mfma_params(path, &kchunk_cols, &ncols);
    L.mp = mfma_plan(n, P, k, mfma_dtype(path), kchunk_cols, ncols, dev_info().n_cu,
                     cx && own_tiles);
    L.lab = (uint16_t *)c.take((size_t)L.mp.n_pad * L.mp.P_pad * sizeof(uint16_t));
    // fewer than 16 groups: the MFMA kernel copies labels packed four bits
    // each
    if (mfma_use_nibbles(L.mp, k))
        L.lab4 = (uint32_t *)c.take((size_t)L.mp.n_pad * L.mp.P_pad / 2);
    if (own_tiles) L.tiles = c.take(mfma_tile_bytes(n, mfma_dtype(path)));
    L.tab = (int32_t *)c.take(mfma_table_bytes(L.mp));
    const int32_t zc = L.mp.cx ? 2 * L.mp.kcol : k;   // z entries per grouping
    L.z = (float *)c.take((size_t)L.mp.items * (P > 0 ? P : 1) * zc * sizeof(float));
    L.tmp = (double *)c.take(reduce_tmp_doubles(L.mp.items, P, zc) * sizeof(double));
    if (L.mp.cx) {
        L.cx.L = (int32_t *)c.take(sizeof(int32_t));
        L.cx.rcs = (double *)c.take((size_t)complement_part_doubles(n) * sizeof(double));
        L.cx.slices = (double *)c.take((size_t)complement_slice_doubles(n) * sizeof(double));
        L.cx.v = (double *)c.take((size_t)L.mp.n_pad * sizeof(double));
        L.cx.r = (double *)c.take((size_t)L.mp.n_pad * sizeof(double));
        L.cx.S = (double *)c.take(sizeof(double));
        L.cx.vnot = (double *)c.take((size_t)(P > 0 ? P : 1) * sizeof(double));
    }
}

size_t sW_bytes(int64_t n, int64_t P, int32_t k, int path, bool own_tiles, bool cx) {
    Carver c{nullptr, 0, 0, true};
    SwLayout L;
    layout_sW(c, n, P, k, path, own_tiles, L, cx);
    return c.used + 256;
}

// Runs one evaluation: stage labels (row q of the staged problem is row
// rows[q] of g, or row q when rows is NULL; rows is only used by plain paths),
// run the kernel, reduce into out[0..P).  tiles: pre-squared tiles of a
// registered matrix, or NULL to run the pre-pass into L.tiles (which also
// leaves s_T in *sT when sT_part is set).  staged: L.lab and L.bad already
// hold the MFMA forms' labels (g is then not read).

int exec_sW(const SwLayout &L, const float *mat, int64_t n, const int32_t *g,
            const int32_t *rows, int64_t P, int32_t k, int32_t limit, const double *w,
            double *out, const void *tiles, int32_t *err_flag, bool timed, double *sT_part,
            double *sT, bool staged, const PrepassRecheck *samples, int packed) {
    hipStream_t s = tls.stream;
    int rc;
    if (!staged) launch_fill_u8(L.bad, P, 0, s);
    if (!is_mfma(L.path)) {
        launch_stage_labels_om(g, rows, n, P, L.pp.n_pad, L.pp.P_pad, limit, L.lab, L.bad,
                               err_flag, s);
        if ((rc = check_launch("label staging"))) return rc;
        KernelTimer timer(s, timed);
        if (launch_plain(L.pp, L.path == PSTAT_PATH_PLAIN_F64, mat, n, L.lab, w, k, L.partial, s,
                         packed))
            return fail(PSTAT_EINVAL, "no plain kernel for tile %d, lanes %d", L.pp.tile,
                        L.pp.lanes);
        timer.stop(s);
        if ((rc = check_launch("plain s_W"))) return rc;
        launch_reduce_plain(L.partial, L.pp.chunks, L.pp.P_pad, P, L.bad, out, s);
        return check_launch("plain reduce");
    }
    if (rows) return fail(PSTAT_EINVAL, "row lists are only supported on the plain paths");
    if (!staged) {
        launch_stage_labels_pm(g, n, P, L.mp.n_pad, L.mp.P_pad, limit, L.lab, L.bad, err_flag, s);
        if ((rc = check_launch("label staging"))) return rc;
    }
    if (L.mp.cx && tiles) return fail(PSTAT_EINVAL, "complement form needs the pre-pass");
    if (!tiles) {
        launch_mfma_prepass(mat, n, L.mp.dtype, L.tiles, s, sT_part, sT, samples,
                            L.mp.cx ? L.cx.rcs : nullptr, packed);
        if ((rc = check_launch("mfma prepass"))) return rc;
        tiles = L.tiles;
    }
    if (L.mp.cx) {
        // *L.cx.L (the largest group) was set by the caller
        launch_complement_sums(L.cx, n, s);
        launch_vnot(L.cx, L.lab, L.mp.n_pad, n, P, s);
        if ((rc = check_launch("complement sums"))) return rc;
    }
    if (L.lab4) {
        launch_pack_nibbles(L.lab, L.mp.n_pad * L.mp.P_pad, L.lab4, s);
        if ((rc = check_launch("label packing"))) return rc;
    }
    KernelTimer timer(s, timed);
    if (launch_mfma(L.mp, tiles, n, L.lab, k, P, L.tab, L.z, s, L.mp.cx ? L.cx.L : nullptr,
                    L.lab4))
        return fail(PSTAT_EINVAL, "no MFMA kernel for %d columns", L.mp.ncols);
    timer.stop(s);
    if ((rc = check_launch("mfma s_W"))) return rc;
    launch_reduce_mfma(L.z, L.mp.items, P, k, w, L.bad, L.tmp, out, s,
                       L.mp.dtype == 1 ? f16_max_cell(tiles, n) : nullptr,
                       L.mp.cx ? &L.cx : nullptr);
    return check_launch("mfma reduce");
}

// Scan `count` labels against `limit`; synchronises; *max_label on success.
int scan_labels_sync(const int32_t *g, int64_t count, int32_t limit, int32_t *max_label) {
    hipStream_t s = tls.stream;
    launch_fill_i32(tls.flags + 3, 1, 0, s);
    launch_fill_i32(tls.flags + 1, 1, -1, s);
    launch_scan_labels(g, count, limit, tls.flags + 3, tls.flags + 1, s);
    int rc = check_launch("label scan");
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(tls.host_flags, tls.flags, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (tls.host_flags[3]) return fail(PSTAT_ELABEL, "a label is negative or >= %d", limit);
    *max_label = tls.host_flags[1];
    return PSTAT_OK;
}

int sW_common(const float *mat, int64_t n, const int32_t *groupings, int64_t n_perms,
              int32_t n_groups, const double *w, double *out, bool validate_sync,
              const void *tiles, int path, int packed) {
    int rc = need_init();
    if (rc) return rc;
    if (n < 2) return fail(PSTAT_EINVAL, "n must be >= 2 (got %lld)", (long long)n);
    if (n_perms < 0) return fail(PSTAT_EINVAL, "n_perms must be >= 0");
    if (!validate_sync && (n_groups < 1 || n_groups > kMaxGroups))
        return fail(PSTAT_EINVAL, "n_groups must be in [1, %d]", kMaxGroups);
    if (n_perms == 0) return PSTAT_OK;
    if ((rc = check_dev_ptr(mat, "mat"))) return rc;
    if ((rc = check_dev_ptr(groupings, "groupings"))) return rc;
    if ((rc = check_dev_ptr(w, "inv_group_sizes"))) return rc;
    if ((rc = check_dev_ptr(out, "out"))) return rc;
    int32_t k = n_groups;
    if (validate_sync) {
        int32_t mx = -1;
        if ((rc = scan_labels_sync(groupings, n_perms * n, kMaxGroups, &mx))) return rc;
        k = mx + 1;
    }
    path = resolve_path(path, n, k);
    const size_t need = sW_bytes(n, n_perms, k, path, tiles == nullptr);
    char *ws;
    if ((rc = acquire_workspace(need, &ws))) return rc;
    Carver c{ws, need, 0, false};
    SwLayout L;
    layout_sW(c, n, n_perms, k, path, tiles == nullptr, L);
    return exec_sW(L, mat, n, groupings, nullptr, n_perms, k, k, w, out, tiles, tls.flags, true,
                   nullptr, nullptr, false, nullptr, packed);
}

int init_flags() {
    if (tls.flags && tls.flags_device == tls.device) return PSTAT_OK;
    if (!tls.host_flags) HIP_TRY(hipHostMalloc((void **)&tls.host_flags, 256, hipHostMallocDefault));
    if (tls.flags) (void)hipFree(tls.flags);
    HIP_TRY(hipMalloc((void **)&tls.flags, 64));
    HIP_TRY(hipMemset(tls.flags, 0, 64));
    tls.flags_device = tls.device;
    return PSTAT_OK;
}


// ---- the whole permutation test in phases ------------------------------------
void carve_head(Carver &c, int64_t n, int64_t R, int32_t k, TestHead &h) {
    const int64_t nsT = sT_partials_count(n);
    h.allg = (int32_t *)c.take((size_t)R * n * sizeof(int32_t));
    h.w = (double *)c.take((size_t)k * sizeof(double));
    h.counts = (uint32_t *)c.take((size_t)k * sizeof(uint32_t));
    h.sw = (double *)c.take((size_t)R * sizeof(double));
    h.sTp = (double *)c.take((size_t)(nsT + 1) * sizeof(double));
    h.sT = h.sTp ? h.sTp + nsT : nullptr;
    h.pv = (double *)c.take(sizeof(double));
    h.list = (int32_t *)c.take((size_t)R * sizeof(int32_t));
    h.vals = (double *)c.take((size_t)R * sizeof(double));
    h.band = (double *)c.take(sizeof(double));
    h.result = (double *)c.take(4 * sizeof(double));
    h.rcp = (double *)c.take((size_t)prepass_blocks(n) * kRecheckRows * sizeof(double));
}

int prepare_test(const TestHead &h, int64_t n, const int32_t *grouping, int32_t k,
                 int64_t n_perms, uint64_t seed, int32_t max_label) {
    hipStream_t s = tls.stream;
    HIP_TRY(hipMemcpyAsync(h.allg, grouping, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    launch_permute(grouping, n, n_perms, seed, max_label, h.allg + n, dev_info().lds_limit,
                   dev_info().n_cu, s);
    int rc = check_launch("permute");
    if (rc) return rc;
    launch_group_weights(grouping, n, k, h.counts, h.w, s);
    return check_launch("group weights");
}

int finish_test(const TestHead &h, const float *mat, int64_t n, int32_t k, int64_t n_perms,
                int path, char *region, size_t region_bytes, int64_t *rechecked_out,
                bool sT_ready, const uint16_t *lab16, int64_t stride16, bool samples_ready,
                int packed) {
    hipStream_t s = tls.stream;
    int rc;
    const int64_t R = n_perms + 1;
    if (!sT_ready) {
        launch_sT(mat, n, h.sTp, h.sT, s, packed);
        if ((rc = check_launch("s_T"))) return rc;
    }
    // FP64 recheck.  First the observed grouping and the first few
    // permutations: the observed value gives F_obs, and the largest relative
    // error of the fast path over these samples sets the tie band.  Then every
    // permutation whose fast s_W lies within the band of the observed value is
    // recomputed, so that the p-value count is decided at FP64 accuracy.
    int64_t rechecked = 0;
    if (path != PSTAT_PATH_PLAIN_F64) {
        const int64_t S = (n_perms < kBandSamples ? n_perms : kBandSamples) + 1;
        if (region_bytes < few_partial_bytes(n, R)) return fail(PSTAT_ENOMEM, "recheck region too small");
        double *partial = (double *)region;
        // FP64 s_W of the groupings listed in h.list[0..m)
        auto recheck = [&](int64_t m) {
            if (lab16)
                launch_sw_few_u16(mat, n, lab16, stride16, h.list, m, k, h.w, partial, h.vals, s,
                                  packed);
            else
                launch_sw_few(mat, n, h.allg, h.list, m, k, h.w, partial, h.vals, s, packed);
        };
        launch_iota(h.list, S, s);
        if (!samples_ready) recheck(S);
        if ((rc = check_launch("FP64 recheck"))) return rc;
        launch_tie_band(h.sw, h.vals, S, kBandMargin, h.band, s);
        launch_scatter(h.vals, h.list, S, h.sw, s);
        if ((rc = check_launch("tie band"))) return rc;
        int64_t m = 0;
        if (n_perms >= S) {
            launch_fill_i32(tls.flags + 2, 1, 0, s);
            launch_flag_ties(h.sw, S, R, h.band, h.list, tls.flags + 2, s);
            if ((rc = check_launch("tie flags"))) return rc;
            HIP_TRY(hipMemcpyAsync(tls.host_flags, tls.flags, 3 * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            m = tls.host_flags[2];
        }
        if (m > 0) {
            recheck(m);
            launch_scatter(h.vals, h.list, m, h.sw, s);
            if ((rc = check_launch("recheck"))) return rc;
        }
        rechecked = S - 1 + m;
    }
    launch_pvalue(h.sw, h.sw + 1, n_perms, h.pv, s);
    launch_pack_result(h.sw, h.sT, n, k, h.counts, h.pv, h.result, s);
    if ((rc = check_launch("result"))) return rc;
    if (rechecked_out) *rechecked_out = rechecked;
    return PSTAT_OK;
}

} // namespace rt
} // namespace pstat

using namespace pstat;
using namespace pstat::rt;

extern "C" {

int pstat_version(void) { return kVersion; }

const char *pstat_last_error(void) { return tls.err; }

int pstat_init(int device) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) {
        (void)hipGetLastError();
        return fail(PSTAT_EHIP, "no HIP device available");
    }
    if (device < 0 || device >= count) return fail(PSTAT_EINVAL, "device %d out of range", device);
    HIP_TRY(hipSetDevice(device));
    {
        std::lock_guard<std::mutex> lk(g_mu);
        DeviceInfo &d = g_devices[device];
        if (!d.ready) {
            int v = 0;
            if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) ==
                    hipSuccess && v > 0)
                d.n_cu = v;
            v = 0;
            if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
                    hipSuccess && v > 0)
                d.lds_limit = (size_t)v;
            // this device is current: its own copy of the static scratch
            void *addr = nullptr;
            const hipError_t se = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
            if (se != hipSuccess || !addr) return hip_fail(se, "hipGetSymbolAddress(scratch)");
            d.static_scratch = (char *)addr;
            d.ready = true;
        }
    }
    tls.device = device;
    tls.err[0] = 0;
    return init_flags();
}

int pstat_set_matrix_layout(int layout) {
    if (layout != PSTAT_LAYOUT_SQUARE && layout != PSTAT_LAYOUT_UPPER_PACKED)
        return fail(PSTAT_EINVAL, "unknown matrix layout %d", layout);
    tls.packed = layout == PSTAT_LAYOUT_UPPER_PACKED;
    return PSTAT_OK;
}

int pstat_set_stream(void *hip_stream) {
    tls.stream = (hipStream_t)hip_stream;
    return PSTAT_OK;
}

int pstat_resolve_path(int path, int64_t n, int32_t n_groups) {
    if (path < PSTAT_PATH_AUTO || path >= PSTAT_N_PATHS)
        return fail(PSTAT_EINVAL, "unknown path %d", path);
    return resolve_path(path, n, n_groups);
}

int pstat_set_path(int path) {
    if (path != PSTAT_PATH_AUTO && (path < 0 || path >= PSTAT_N_PATHS))
        return fail(PSTAT_EINVAL, "unknown path %d", path);
    tls.path = path;
    return PSTAT_OK;
}

int pstat_set_tuning(int path, int tile, int batch) {
    if (path < 0 || path >= PSTAT_N_PATHS) return fail(PSTAT_EINVAL, "unknown path %d", path);
    if (is_mfma(path)) {
        if (tile < 0 || tile % 64) return fail(PSTAT_EINVAL, "K chunk must be a multiple of 64");
        if (batch != 0 && batch != 256 && batch != 512)
            return fail(PSTAT_EINVAL, "MFMA N columns must be 256 or 512");
    } else {
        if (tile != 0 && tile != 32 && tile != 64) return fail(PSTAT_EINVAL, "tile must be 32 or 64");
        if (path == PSTAT_PATH_PLAIN_F64 && tile == 64)
            return fail(PSTAT_EINVAL, "the FP64 plain kernel uses tile 32");
        if (batch != 0 && batch != 64 && batch != 128 && batch != 256)
            return fail(PSTAT_EINVAL, "lanes must be 64, 128 or 256");
    }
    tls.tuning[path].tile = tile;
    tls.tuning[path].batch = batch;
    return PSTAT_OK;
}

int pstat_free_workspace(void) {
    if (!tls.ws_own) return PSTAT_OK;
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    HIP_TRY(hipSetDevice(tls.ws_own_device));
    // work queued on any stream of that device may still read it
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipFree(tls.ws_own);
    (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "freeing the library workspace");
    tls.ws_own = nullptr;
    tls.ws_own_bytes = 0;
    tls.ws_own_device = -1;
    return PSTAT_OK;
}

int pstat_set_workspace(void *dev_ptr, size_t bytes) {
    if (dev_ptr) {
        int rc = need_init();
        if (rc) return rc;
        if ((rc = check_dev_ptr(dev_ptr, "workspace"))) return rc;
    }
    tls.ws_user = dev_ptr;
    tls.ws_user_bytes = dev_ptr ? bytes : 0;
    return PSTAT_OK;
}

size_t pstat_workspace_bytes(int64_t n, int64_t n_perms, int32_t n_groups, int path) {
    if (n < 2 || n_perms < 0 || n_groups < 1 || n_groups > kMaxGroups) return 0;
    if (path != PSTAT_PATH_AUTO && (path < 0 || path >= PSTAT_N_PATHS)) return 0;
    if (tls.device < 0) return 0;
    return sW_bytes(n, n_perms, n_groups, resolve_path(path, n, n_groups), true);
}

int pstat_sW(const float *mat, int64_t n, const int32_t *groupings, int64_t n_perms,
             const double *inv_group_sizes, double *out) {
    return sW_common(mat, n, groupings, n_perms, 0, inv_group_sizes, out, true, nullptr, tls.path,
                     tls.packed);
}

int pstat_sW_k(const float *mat, int64_t n, const int32_t *groupings, int64_t n_perms,
               int32_t n_groups, const double *inv_group_sizes, double *out) {
    return sW_common(mat, n, groupings, n_perms, n_groups, inv_group_sizes, out, false, nullptr,
                     tls.path, tls.packed);
}

int pstat_sW_k_noalloc(const float *mat, int64_t n, const int32_t *groupings, int64_t n_perms,
                       int32_t n_groups, const double *inv_group_sizes, double *out,
                       size_t *scratch_bytes) {
    int rc = need_init();
    if (rc) return rc;
    if (n < 2) return fail(PSTAT_EINVAL, "n must be >= 2 (got %lld)", (long long)n);
    if (n_perms < 0) return fail(PSTAT_EINVAL, "n_perms must be >= 0");
    if (n_groups < 1 || n_groups > kMaxGroups)
        return fail(PSTAT_EINVAL, "n_groups must be in [1, %d]", kMaxGroups);
    const int path = resolve_path(tls.path, n, n_groups);
    const size_t need = sW_bytes(n, n_perms, n_groups, path, true);
    if (scratch_bytes) *scratch_bytes = need;
    if (n_perms == 0) return PSTAT_OK;
    if (need > kStaticScratchBytes)
        return fail(PSTAT_ENOMEM,
                    "this shape needs %zu bytes of scratch, beyond the %zu-byte static scratch "
                    "of pstat_sW_k_noalloc (use pstat_sW_k)",
                    need, kStaticScratchBytes);
    if ((rc = check_dev_ptr(mat, "mat"))) return rc;
    if ((rc = check_dev_ptr(groupings, "groupings"))) return rc;
    if ((rc = check_dev_ptr(inv_group_sizes, "inv_group_sizes"))) return rc;
    if ((rc = check_dev_ptr(out, "out"))) return rc;
    char *base = dev_info().static_scratch;
    if (!base) return fail(PSTAT_ESTATE, "no static scratch on device %d", tls.device);
    Carver c{base, kStaticScratchBytes, 0, false};
    SwLayout L;
    layout_sW(c, n, n_perms, n_groups, path, true, L);
    // untimed: the event pairs of pstat_profile would be created here
    return exec_sW(L, mat, n, groupings, nullptr, n_perms, n_groups, n_groups, inv_group_sizes,
                   out, nullptr, tls.flags, false, nullptr, nullptr, false, nullptr, tls.packed);
}

size_t pstat_noalloc_scratch_bytes(void) { return kStaticScratchBytes; }

int pstat_check_labels(void) {
    int rc = need_init();
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(tls.host_flags, tls.flags, sizeof(int32_t), hipMemcpyDeviceToHost,
                           tls.stream));
    HIP_TRY(hipStreamSynchronize(tls.stream));
    if (tls.host_flags[0]) {
        launch_fill_i32(tls.flags, 1, 0, tls.stream);
        HIP_TRY(hipStreamSynchronize(tls.stream));
        return fail(PSTAT_ELABEL, "an out-of-range label was seen");
    }
    return PSTAT_OK;
}

int pstat_sT(const float *mat, int64_t n, double *s_T) {
    int rc = need_init();
    if (rc) return rc;
    if (n < 2) return fail(PSTAT_EINVAL, "n must be >= 2");
    if ((rc = check_dev_ptr(mat, "mat")) || (rc = check_dev_ptr(s_T, "s_T"))) return rc;
    char *ws;
    const size_t need = (size_t)sT_partials_count(n) * sizeof(double) + 256;
    if ((rc = acquire_workspace(need, &ws))) return rc;
    launch_sT(mat, n, (double *)ws, s_T, tls.stream, tls.packed);
    return check_launch("s_T");
}

int pstat_F(const double *s_W, int64_t count, const double *s_T, int64_t n, int32_t k,
            double *F) {
    int rc = need_init();
    if (rc) return rc;
    if (k < 2 || n <= k) return fail(PSTAT_EDOMAIN, "F needs k >= 2 and n > k (k=%d, n=%lld)", k,
                                     (long long)n);
    if (count < 0) return fail(PSTAT_EINVAL, "count must be >= 0");
    if (count == 0) return PSTAT_OK;
    if ((rc = check_dev_ptr(s_W, "s_W")) || (rc = check_dev_ptr(s_T, "s_T")) ||
        (rc = check_dev_ptr(F, "F")))
        return rc;
    launch_F(s_W, count, s_T, n, k, F, tls.stream);
    return check_launch("F");
}

int pstat_pvalue(const double *s_W_obs, const double *s_W_perm, int64_t n_perms, double *p) {
    int rc = need_init();
    if (rc) return rc;
    if (n_perms < 0) return fail(PSTAT_EINVAL, "n_perms must be >= 0");
    if ((rc = check_dev_ptr(s_W_obs, "s_W_obs")) || (rc = check_dev_ptr(p, "p"))) return rc;
    if (n_perms > 0 && (rc = check_dev_ptr(s_W_perm, "s_W_perm"))) return rc;
    launch_pvalue(s_W_obs, s_W_perm, n_perms, p, tls.stream);
    return check_launch("p-value");
}

int pstat_group_weights(const int32_t *grouping, int64_t n, int32_t n_groups, double *inv) {
    int rc = need_init();
    if (rc) return rc;
    if (n < 1 || n_groups < 1 || n_groups > kMaxGroups)
        return fail(PSTAT_EINVAL, "need n >= 1 and 1 <= n_groups <= %d", kMaxGroups);
    if ((rc = check_dev_ptr(grouping, "grouping")) || (rc = check_dev_ptr(inv, "inv"))) return rc;
    char *ws;
    if ((rc = acquire_workspace((size_t)n_groups * 4 + 256, &ws))) return rc;
    launch_group_weights(grouping, n, n_groups, (uint32_t *)ws, inv, tls.stream);
    return check_launch("group weights");
}

int pstat_permute(const int32_t *base, int64_t n, int64_t n_perms, uint64_t seed,
                  int32_t *groupings) {
    int rc = need_init();
    if (rc) return rc;
    if (n < 1 || n_perms < 0) return fail(PSTAT_EINVAL, "need n >= 1 and n_perms >= 0");
    if (n > 0xFFFFFFFFll) return fail(PSTAT_EINVAL, "n must be < 2^32");
    if (n_perms == 0) return PSTAT_OK;
    if ((rc = check_dev_ptr(base, "base")) || (rc = check_dev_ptr(groupings, "groupings")))
        return rc;
    int32_t max_label = -1;
    if ((rc = scan_labels_sync(base, n, kMaxGroups, &max_label))) return rc;
    launch_permute(base, n, n_perms, seed, max_label, groupings, dev_info().lds_limit,
                   dev_info().n_cu, tls.stream);
    return check_launch("permute");
}

int pstat_permanova(const float *mat, int64_t n, const int32_t *grouping, int32_t n_groups,
                    int64_t n_perms, uint64_t seed, double *result, double *sW_all,
                    int64_t *n_rechecked) {
    int rc = need_init();
    if (rc) return rc;
    if (n < 2 || n_perms < 0) return fail(PSTAT_EINVAL, "need n >= 2 and n_perms >= 0");
    if (n > 0xFFFFFFFFll) return fail(PSTAT_EINVAL, "n must be < 2^32");
    if (n_groups < 2 || n <= n_groups || n_groups > kMaxGroups)
        return fail(PSTAT_EDOMAIN, "F needs 2 <= n_groups < n (n_groups=%d)", n_groups);
    if ((rc = check_dev_ptr(mat, "mat")) || (rc = check_dev_ptr(grouping, "grouping")) ||
        (rc = check_dev_ptr(result, "result")))
        return rc;
    if (sW_all && (rc = check_dev_ptr(sW_all, "sW_all"))) return rc;
    const int32_t k = n_groups;
    const int path = resolve_path(tls.path, n, k);
    hipStream_t s = tls.stream;
    int32_t max_label = -1;
    if ((rc = scan_labels_sync(grouping, n, k, &max_label))) return rc;

    const int64_t R = n_perms + 1;  // the observed grouping is row 0
    TestHead h;
    Carver dry{nullptr, 0, 0, true};
    carve_head(dry, n, R, k, h);
    const size_t head = (size_t)round_up((int64_t)dry.used, 256) + 256;
    // s_W workspace, then the FP64 recheck's partials (the recheck may read
    // the staged labels, so the two must not overlap)
    const size_t swb = sW_bytes(n, R, k, path, true, true);
    const size_t fpb = few_partial_bytes(n, R);
    char *ws;
    if ((rc = acquire_workspace(head + swb + fpb, &ws))) return rc;
    Carver hc{ws, head, 0, false};
    carve_head(hc, n, R, k, h);
    if (sW_all) h.sw = sW_all;
    if (result) h.result = result;

    Carver c{ws + head, swb, 0, false};
    SwLayout L;
    layout_sW(c, n, R, k, path, true, L, true);
    // MFMA forms: the shuffle writes the permutations straight into the
    // staged u16 layout (row 0 the observed grouping, rows past R padding)
    bool staged = false;
    if (is_mfma(path)) {
        const int64_t np = L.mp.n_pad;
        launch_fill_u8(L.bad, R, 0, s);
        staged = launch_permute_u16(grouping, n, n_perms, seed, max_label, L.lab + np, np,
                                    dev_info().lds_limit, dev_info().n_cu, s) == 0;
        if (staged) {
            if ((rc = check_launch("permute"))) return rc;
            launch_stage_labels_pm(grouping, n, 1, np, 1, k, L.lab, L.bad, tls.flags, s);
            if (L.mp.P_pad > R)
                launch_stage_labels_pm(grouping, n, 0, np, L.mp.P_pad - R, k, L.lab + R * np,
                                       L.bad, tls.flags, s);
            launch_group_weights(grouping, n, k, h.counts, h.w, s);
            if ((rc = check_launch("label staging"))) return rc;
        }
    }
    if (!staged && (rc = prepare_test(h, n, grouping, k, n_perms, seed, max_label))) return rc;
    // Complement form: every row is a permutation of the observed grouping,
    // so all share its group sizes; the largest group gets no columns.
    if (is_mfma(path) && L.mp.cx) launch_largest_group(h.counts, k, L.cx.L, s);
    // The MFMA forms' pre-pass also leaves s_T and the FP64 s_W of the
    // observed grouping and the first permutations (the recheck's samples).
    const bool mf = is_mfma(path);
    PrepassRecheck prc;
    if (mf) {
        prc.lab = L.lab;
        prc.stride = L.mp.n_pad;
        prc.m = (int32_t)((n_perms < kBandSamples ? n_perms : kBandSamples) + 1);
        prc.w = h.w;
        prc.k = k;
        prc.part = h.rcp;
        prc.out = h.vals;
    }
    if ((rc = exec_sW(L, mat, n, h.allg, nullptr, R, k, k, h.w, h.sw, nullptr, tls.flags, true,
                      h.sTp, h.sT, staged, mf ? &prc : nullptr, tls.packed)))
        return rc;
    int64_t rechecked = 0;
    if ((rc = finish_test(h, mat, n, k, n_perms, path, ws + head + swb, fpb, &rechecked, mf,
                          staged ? L.lab : nullptr, L.mp.n_pad, mf, tls.packed)))
        return rc;
    if (n_rechecked) *n_rechecked = rechecked;
    return PSTAT_OK;
}

int pstat_matrix_register(const float *mat, int64_t n, int path, int64_t *handle) {
    int rc = need_init();
    if (rc) return rc;
    if (!handle) return fail(PSTAT_EINVAL, "handle is NULL");
    if (n < 2) return fail(PSTAT_EINVAL, "n must be >= 2");
    if ((rc = check_dev_ptr(mat, "mat"))) return rc;
    if (path == PSTAT_PATH_AUTO) path = PSTAT_PATH_MFMA_SPLIT_BF16;
    if (path < 0 || path >= PSTAT_N_PATHS) return fail(PSTAT_EINVAL, "unknown path %d", path);
    void *tiles = nullptr;
    if (is_mfma(path)) {
        HIP_TRY(hipMalloc(&tiles, mfma_tile_bytes(n, mfma_dtype(path))));
        launch_mfma_prepass(mat, n, mfma_dtype(path), tiles, tls.stream, nullptr, nullptr,
                            nullptr, nullptr, tls.packed);
        if ((rc = check_launch("mfma prepass"))) {
            (void)hipFree(tiles);
            return rc;
        }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    const int64_t h = g_next_handle++;
    g_registered[h] = Registered{mat, n, path, tls.device, tiles, tls.packed};
    *handle = h;
    return PSTAT_OK;
}

int pstat_matrix_release(int64_t handle) {
    Registered r;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_registered.find(handle);
        if (it == g_registered.end()) return fail(PSTAT_EINVAL, "unknown handle %lld", (long long)handle);
        r = it->second;
        g_registered.erase(it);
    }
    if (r.tiles) {
        // queued work may still read the tiles
        HIP_TRY(hipStreamSynchronize(tls.stream));
        HIP_TRY(hipFree(r.tiles));
    }
    return PSTAT_OK;
}

int pstat_sW_registered(int64_t handle, const int32_t *groupings, int64_t n_perms,
                        int32_t n_groups, const double *inv_group_sizes, double *out) {
    Registered r;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_registered.find(handle);
        if (it == g_registered.end()) return fail(PSTAT_EINVAL, "unknown handle %lld", (long long)handle);
        r = it->second;
    }
    if (r.device != tls.device) return fail(PSTAT_EINVAL, "handle belongs to device %d", r.device);
    return sW_common(r.mat, r.n, groupings, n_perms, n_groups, inv_group_sizes, out, false,
                     r.tiles, r.path, r.packed);
}

int pstat_profile(int on) {
    for (auto &e : tls.events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    tls.events.clear();
    tls.profiling = on != 0;
    return PSTAT_OK;
}

int pstat_profile_read(double *ms, int64_t *launches) {
    double total = 0.0;
    for (auto &e : tls.events) {
        HIP_TRY(hipEventSynchronize(e.second));
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, e.first, e.second));
        total += t;
    }
    if (ms) *ms = total;
    if (launches) *launches = (int64_t)tls.events.size();
    return PSTAT_OK;
}

}  // extern "C"
