// Batched execution of many permutation tests (the serving loop's device
// side).  A server owns a device table of staged jobs; each round executes a
// list of work units -- (job, tile chunk, permutation group) -- of any mix of
// jobs in one launch of the work-list plain kernel, replayed from a captured
// hipGraph: copy the unit list from pinned host memory, then run the kernel.
// Two graphs alternate so the host can fill one unit list while the other
// round runs.  A job's result depends only on its own units and its fixed
// reduction order, so it is the same whether it runs alone or in a mix.
#include <string.h>

#include "runtime.h"

namespace pstat {
namespace rt {
namespace {

constexpr int kKinds = 3;

struct Job {
    bool live = false;
    int kind = 0;                  // 0 plain FP32, 1 MFMA split BF16 (512-column
                                   // work-groups), 2 the same with 256 columns
    const float *mat = nullptr;
    int packed = 0;                // layout of mat
    int64_t n = 0, n_perms = 0;
    int32_t k = 0;
    TestHead head{};
    PlainPlan pl{};
    MfmaPlan mp{};
    uint16_t *lab = nullptr;
    double *partial = nullptr;
    float *z = nullptr;
    double *tmp = nullptr;
    Complement cx{};               // MFMA complement form (mp.cx)
    uint8_t *bad = nullptr;
    int64_t units = 0;
    int64_t split = 1;             // units are (a, b) with b in [0, split)
};

struct Server {
    int device = -1;
    int64_t max_jobs = 0, max_units = 0;
    JobDesc *jobs_dev = nullptr;
    JobDesc *jobs_host = nullptr;           // pinned, one entry per slot
    // per alternating slot b: unit lists of the plain [0] and the two MFMA
    // [1], [2] kinds
    UnitDesc *units_dev[2][kKinds] = {};
    int32_t *count_dev[2] = {nullptr, nullptr};    // [kind] counts of slot b
    UnitDesc *units_host[2][kKinds] = {};          // pinned
    int32_t *count_host[2] = {nullptr, nullptr};   // pinned
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr};
    bool in_flight[2] = {false, false};
    int next = 0;
    std::vector<Job> jobs;
};

std::mutex g_srv_mu;
std::map<int64_t, Server *> g_servers;
int64_t g_next_server = 1;

Server *find_server(int64_t h) {
    std::lock_guard<std::mutex> lk(g_srv_mu);
    auto it = g_servers.find(h);
    return it == g_servers.end() ? nullptr : it->second;
}

// Scratch layout of one job inside the caller's buffer.
struct JobLayout {
    TestHead head;
    uint16_t *lab = nullptr;
    double *partial = nullptr;
    uint8_t *bad = nullptr;
    PlainPlan pl{};
    MfmaPlan mp{};
    void *tiles = nullptr;
    int32_t *tab = nullptr;
    float *z = nullptr;
    double *tmp = nullptr;
    Complement cx{};
};

void layout_job(Carver &c, int64_t n, int64_t n_perms, int32_t k, int kind, JobLayout &L) {
    const int64_t R = n_perms + 1;
    carve_head(c, n, R, k, L.head);
    L.bad = (uint8_t *)c.take((size_t)R);
    if (kind == 0) {
        L.pl = plain_plan(n, R, kServeTile, kServeLanes, dev_info().n_cu);
        L.lab = (uint16_t *)c.take((size_t)L.pl.n_pad * L.pl.P_pad * sizeof(uint16_t));
        L.partial = (double *)c.take((size_t)L.pl.chunks * L.pl.P_pad * sizeof(double));
        return;
    }
    // the same plan as the whole-test entry point's (complement form; 256
    // columns per work-group with two groups), so a job's results equal that
    // call's bit for bit
    L.mp = mfma_plan(n, R, k, 2, 0, 512, dev_info().n_cu, true);
    L.lab = (uint16_t *)c.take((size_t)L.mp.n_pad * L.mp.P_pad * sizeof(uint16_t));
    L.tiles = c.take(mfma_tile_bytes(n, 2));
    L.tab = (int32_t *)c.take(mfma_table_bytes(L.mp));
    const int32_t zc = L.mp.cx ? 2 * L.mp.kcol : k;   // z entries per grouping
    L.z = (float *)c.take((size_t)L.mp.items * R * zc * sizeof(float));
    L.tmp = (double *)c.take(reduce_tmp_doubles(L.mp.items, R, zc) * sizeof(double));
    if (L.mp.cx) {
        L.cx.L = (int32_t *)c.take(sizeof(int32_t));
        L.cx.rcs = (double *)c.take((size_t)complement_part_doubles(n) * sizeof(double));
        L.cx.slices = (double *)c.take((size_t)complement_slice_doubles(n) * sizeof(double));
        L.cx.v = (double *)c.take((size_t)L.mp.n_pad * sizeof(double));
        L.cx.r = (double *)c.take((size_t)L.mp.n_pad * sizeof(double));
        L.cx.S = (double *)c.take(sizeof(double));
        L.cx.vnot = (double *)c.take((size_t)R * sizeof(double));
    }
}

int job_kind(int path, int64_t n, int32_t k) {
    path = resolve_path(path, n, k);
    if (path == PSTAT_PATH_PLAIN_F32) return 0;
    if (path == PSTAT_PATH_MFMA_SPLIT_BF16) return 1;
    return -1;
}

void destroy_server(Server *sv) {
    for (int b = 0; b < 2; b++) {
        if (sv->exec[b]) (void)hipGraphExecDestroy(sv->exec[b]);
        if (sv->graph[b]) (void)hipGraphDestroy(sv->graph[b]);
        if (sv->done[b]) (void)hipEventDestroy(sv->done[b]);
        for (int t = 0; t < kKinds; t++) {
            if (sv->units_dev[b][t]) (void)hipFree(sv->units_dev[b][t]);
            if (sv->units_host[b][t]) (void)hipHostFree(sv->units_host[b][t]);
        }
        if (sv->count_dev[b]) (void)hipFree(sv->count_dev[b]);
        if (sv->count_host[b]) (void)hipHostFree(sv->count_host[b]);
    }
    if (sv->jobs_dev) (void)hipFree(sv->jobs_dev);
    if (sv->jobs_host) (void)hipHostFree(sv->jobs_host);
    delete sv;
}

}  // namespace
}  // namespace rt
}  // namespace pstat

using namespace pstat;
using namespace pstat::rt;

extern "C" {

int pstat_serve_create(int64_t max_jobs, int64_t max_units, int64_t *server) {
    int rc = need_init();
    if (rc) return rc;
    if (!server) return fail(PSTAT_EINVAL, "server is NULL");
    if (max_jobs < 1 || max_jobs > (1 << 20) || max_units < 1 || max_units > (1 << 22))
        return fail(PSTAT_EINVAL, "max_jobs in [1, 2^20] and max_units in [1, 2^22] required");
    Server *sv = new Server();
    sv->device = tls.device;
    sv->max_jobs = max_jobs;
    sv->max_units = max_units;
    sv->jobs.resize((size_t)max_jobs);
    auto bail = [&](hipError_t e, const char *what) {
        destroy_server(sv);
        return hip_fail(e, what);
    };
    hipError_t e;
    if ((e = hipMalloc((void **)&sv->jobs_dev, sizeof(JobDesc) * max_jobs)) != hipSuccess)
        return bail(e, "hipMalloc(job table)");
    if ((e = hipHostMalloc((void **)&sv->jobs_host, sizeof(JobDesc) * max_jobs,
                           hipHostMallocDefault)) != hipSuccess)
        return bail(e, "hipHostMalloc(job table)");
    memset(sv->jobs_host, 0, sizeof(JobDesc) * max_jobs);
    for (int b = 0; b < 2; b++) {
        for (int t = 0; t < kKinds; t++) {
            if ((e = hipMalloc((void **)&sv->units_dev[b][t], sizeof(UnitDesc) * max_units)) !=
                hipSuccess)
                return bail(e, "hipMalloc(units)");
            if ((e = hipHostMalloc((void **)&sv->units_host[b][t], sizeof(UnitDesc) * max_units,
                                   hipHostMallocDefault)) != hipSuccess)
                return bail(e, "hipHostMalloc(units)");
            memset(sv->units_host[b][t], 0, sizeof(UnitDesc) * max_units);
        }
        if ((e = hipMalloc((void **)&sv->count_dev[b], 64)) != hipSuccess)
            return bail(e, "hipMalloc(count)");
        if ((e = hipHostMalloc((void **)&sv->count_host[b], 64, hipHostMallocDefault)) != hipSuccess)
            return bail(e, "hipHostMalloc(count)");
        for (int t = 0; t < kKinds; t++) sv->count_host[b][t] = 0;
        if ((e = hipEventCreateWithFlags(&sv->done[b], hipEventDisableTiming)) != hipSuccess)
            return bail(e, "hipEventCreate");
    }
    std::lock_guard<std::mutex> lk(g_srv_mu);
    const int64_t h = g_next_server++;
    g_servers[h] = sv;
    *server = h;
    return PSTAT_OK;
}

int pstat_serve_destroy(int64_t server) {
    Server *sv = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_srv_mu);
        auto it = g_servers.find(server);
        if (it == g_servers.end()) return fail(PSTAT_EINVAL, "unknown server %lld", (long long)server);
        sv = it->second;
        g_servers.erase(it);
    }
    for (int b = 0; b < 2; b++)
        if (sv->in_flight[b]) (void)hipEventSynchronize(sv->done[b]);
    destroy_server(sv);
    return PSTAT_OK;
}

size_t pstat_job_bytes(int64_t n, int64_t n_perms, int32_t n_groups, int path) {
    if (tls.device < 0 || n < 2 || n_perms < 0 || n_groups < 1 || n_groups > kMaxGroups) return 0;
    const int kind = job_kind(path, n, n_groups);
    if (kind < 0) return 0;
    Carver c{nullptr, 0, 0, true};
    JobLayout L;
    layout_job(c, n, n_perms, n_groups, kind, L);
    return c.used + 256;
}

int pstat_job_create(int64_t server, const float *mat, int64_t n, const int32_t *grouping,
                     int32_t n_groups, int64_t n_perms, uint64_t seed, int path, void *scratch,
                     size_t scratch_bytes, int64_t *job, int64_t *n_units) {
    int rc = need_init();
    if (rc) return rc;
    Server *sv = find_server(server);
    if (!sv) return fail(PSTAT_EINVAL, "unknown server %lld", (long long)server);
    if (sv->device != tls.device) return fail(PSTAT_EINVAL, "server belongs to device %d", sv->device);
    if (!job || !n_units) return fail(PSTAT_EINVAL, "job and n_units must not be NULL");
    if (n < 2 || n_perms < 0 || n > 0xFFFFFFFFll) return fail(PSTAT_EINVAL, "bad n or n_perms");
    if (n_groups < 2 || n <= n_groups || n_groups > kMaxGroups)
        return fail(PSTAT_EDOMAIN, "F needs 2 <= n_groups < n (n_groups=%d)", n_groups);
    if ((rc = check_dev_ptr(mat, "mat")) || (rc = check_dev_ptr(grouping, "grouping")) ||
        (rc = check_dev_ptr(scratch, "scratch")))
        return rc;
    int kind = job_kind(path, n, n_groups);
    if (kind < 0) return fail(PSTAT_EINVAL, "serving jobs run the plain FP32 or split-BF16 MFMA form");
    const size_t need = pstat_job_bytes(n, n_perms, n_groups, path);
    if (scratch_bytes < need)
        return fail(PSTAT_ENOMEM, "job scratch of %zu bytes is smaller than the %zu needed",
                    scratch_bytes, need);
    int64_t slot = -1;
    for (int64_t i = 0; i < sv->max_jobs; i++)
        if (!sv->jobs[i].live) { slot = i; break; }
    if (slot < 0) return fail(PSTAT_ENOMEM, "all %lld job slots are in use", (long long)sv->max_jobs);

    int32_t max_label = -1;
    if ((rc = scan_labels_sync(grouping, n, n_groups, &max_label))) return rc;
    Carver c{(char *)scratch, scratch_bytes, 0, false};
    JobLayout L;
    layout_job(c, n, n_perms, n_groups, kind, L);
    if (kind == 1 && L.mp.ncols == 256) kind = 2;   // one column per permutation: k = 2
    const int64_t R = n_perms + 1;
    if ((rc = prepare_test(L.head, n, grouping, n_groups, n_perms, seed, max_label))) return rc;
    hipStream_t s = tls.stream;
    launch_fill_u8(L.bad, R, 0, s);
    JobDesc &d = sv->jobs_host[slot];
    memset(&d, 0, sizeof(JobDesc));
    d.mat = mat;
    d.packed = tls.packed;
    d.w = L.head.w;
    d.n = n;
    d.k = n_groups;
    d.kind = kind;
    d.R = R;
    if (kind == 0) {
        launch_stage_labels_om(L.head.allg, nullptr, n, R, L.pl.n_pad, L.pl.P_pad, n_groups, L.lab,
                               L.bad, tls.flags, s);
        d.lab = L.lab;
        d.partial = L.partial;
        d.nt = L.pl.n_t;
        d.n_tiles = L.pl.n_tiles;
        d.tiles_per_chunk = L.pl.tiles_per_chunk;
        d.P_pad = L.pl.P_pad;
    } else {
        launch_stage_labels_pm(L.head.allg, n, R, L.mp.n_pad, L.mp.P_pad, n_groups, L.lab, L.bad,
                               tls.flags, s);
        // the pre-pass also leaves s_T and the recheck samples' FP64 s_W, as
        // in the whole-test entry point
        PrepassRecheck prc;
        prc.lab = L.lab;
        prc.stride = L.mp.n_pad;
        prc.m = (int32_t)((n_perms < kBandSamples ? n_perms : kBandSamples) + 1);
        prc.w = L.head.w;
        prc.k = n_groups;
        prc.part = L.head.rcp;
        prc.out = L.head.vals;
        if (L.mp.cx) launch_largest_group(L.head.counts, n_groups, L.cx.L, s);
        launch_mfma_prepass(mat, n, 2, L.tiles, s, L.head.sTp, L.head.sT, &prc,
                            L.mp.cx ? L.cx.rcs : nullptr, tls.packed);
        if (L.mp.cx) {
            launch_complement_sums(L.cx, n, s);
            launch_vnot(L.cx, L.lab, L.mp.n_pad, n, R, s);
        }
        launch_item_table(L.mp, L.tab, s);
        d.tiles = L.tiles;
        d.lab_pm = L.lab;
        d.tab = L.tab;
        d.z = L.z;
        d.comp_units = L.mp.panels * (L.mp.panels + 1);
        d.kb_total = L.mp.kb_total;
        d.n_pad_m = L.mp.n_pad;
        d.cx = L.mp.cx ? 1 : 0;
        d.Lp = L.cx.L;
    }
    if ((rc = check_launch("job staging"))) return rc;
    HIP_TRY(hipMemcpyAsync(sv->jobs_dev + slot, &d, sizeof(JobDesc), hipMemcpyHostToDevice, s));

    Job &J = sv->jobs[slot];
    J.live = true;
    J.kind = kind;
    J.mat = mat;
    J.packed = tls.packed;
    J.n = n;
    J.n_perms = n_perms;
    J.k = n_groups;
    J.head = L.head;
    J.pl = L.pl;
    J.mp = L.mp;
    J.lab = L.lab;
    J.partial = L.partial;
    J.z = L.z;
    J.tmp = L.tmp;
    J.cx = L.cx;
    J.bad = L.bad;
    if (kind == 0) {
        J.units = L.pl.chunks * L.pl.pgroups;
        J.split = L.pl.pgroups;
    } else {
        J.units = L.mp.items * L.mp.nblocks;
        J.split = L.mp.nblocks;
    }
    *job = slot;
    *n_units = J.units;
    return PSTAT_OK;
}

int pstat_serve_round(int64_t server, const int64_t *units, int64_t count) {
    int rc = need_init();
    if (rc) return rc;
    Server *sv = find_server(server);
    if (!sv) return fail(PSTAT_EINVAL, "unknown server %lld", (long long)server);
    if (count < 0 || count > sv->max_units)
        return fail(PSTAT_EINVAL, "count must be in [0, %lld]", (long long)sv->max_units);
    if (count > 0 && !units) return fail(PSTAT_EINVAL, "units is NULL");
    if (!tls.stream) return fail(PSTAT_EINVAL, "serving rounds need a created stream, not the null stream");
    const int b = sv->next;
    if (sv->in_flight[b]) {
        HIP_TRY(hipEventSynchronize(sv->done[b]));
        sv->in_flight[b] = false;
    }
    // Host pairs (job, unit) -> (job, a, b) in the list of the job's kind:
    // plain (tile chunk, permutation group), MFMA (work item, column block);
    // a job's units are numbered a-major so neighbouring units share data.
    int32_t cnt[kKinds] = {0, 0, 0};
    for (int64_t i = 0; i < count; i++) {
        const int64_t j = units[2 * i], u = units[2 * i + 1];
        if (j < 0 || j >= sv->max_jobs || !sv->jobs[j].live)
            return fail(PSTAT_EINVAL, "unit %lld names job %lld, which is not live", (long long)i,
                        (long long)j);
        const Job &J = sv->jobs[j];
        if (u < 0 || u >= J.units)
            return fail(PSTAT_EINVAL, "unit %lld of job %lld out of range", (long long)u, (long long)j);
        sv->units_host[b][J.kind][cnt[J.kind]++] =
            UnitDesc{(int32_t)j, (int32_t)(u / J.split), (int32_t)(u % J.split)};
    }
    for (int t = 0; t < kKinds; t++) sv->count_host[b][t] = cnt[t];
    if (!sv->exec[b]) {
        hipStream_t s = tls.stream;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
        hipError_t e[8];
        for (int t = 0; t < kKinds; t++)
            e[t] = hipMemcpyAsync(sv->units_dev[b][t], sv->units_host[b][t],
                                  sizeof(UnitDesc) * sv->max_units, hipMemcpyHostToDevice, s);
        e[3] = hipMemcpyAsync(sv->count_dev[b], sv->count_host[b], kKinds * sizeof(int32_t),
                              hipMemcpyHostToDevice, s);
        launch_plain_worklist(sv->jobs_dev, sv->units_dev[b][0], sv->count_dev[b], sv->max_units, s);
        e[4] = hipGetLastError();
        launch_mfma_worklist(sv->jobs_dev, sv->units_dev[b][1], sv->count_dev[b] + 1,
                             sv->max_units, s, 512);
        e[5] = hipGetLastError();
        launch_mfma_worklist(sv->jobs_dev, sv->units_dev[b][2], sv->count_dev[b] + 2,
                             sv->max_units, s, 256);
        e[6] = hipGetLastError();
        hipGraph_t g = nullptr;
        e[7] = hipStreamEndCapture(s, &g);
        for (int q = 0; q < 8; q++)
            if (e[q] != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return hip_fail(e[q], "capturing the serving round");
            }
        sv->graph[b] = g;
        HIP_TRY(hipGraphInstantiate(&sv->exec[b], g, nullptr, nullptr, 0));
    }
    HIP_TRY(hipGraphLaunch(sv->exec[b], tls.stream));
    HIP_TRY(hipEventRecord(sv->done[b], tls.stream));
    sv->in_flight[b] = true;
    sv->next = b ^ 1;
    return PSTAT_OK;
}

int pstat_job_finish(int64_t server, int64_t job, double *result, double *sW_all,
                     int64_t *n_rechecked) {
    int rc = need_init();
    if (rc) return rc;
    Server *sv = find_server(server);
    if (!sv) return fail(PSTAT_EINVAL, "unknown server %lld", (long long)server);
    if (job < 0 || job >= sv->max_jobs || !sv->jobs[job].live)
        return fail(PSTAT_EINVAL, "job %lld is not live", (long long)job);
    if (!result) return fail(PSTAT_EINVAL, "result is NULL");
    if (sW_all && (rc = check_dev_ptr(sW_all, "sW_all"))) return rc;
    const Job &J = sv->jobs[job];
    const int64_t R = J.n_perms + 1;
    hipStream_t s = tls.stream;
    if (J.kind == 0)
        launch_reduce_plain(J.partial, J.pl.chunks, J.pl.P_pad, R, J.bad, J.head.sw, s);
    else
        launch_reduce_mfma(J.z, J.mp.items, R, J.k, J.head.w, J.bad, J.tmp, J.head.sw, s, nullptr,
                           J.mp.cx ? &J.cx : nullptr);
    if ((rc = check_launch("job reduce"))) return rc;
    const size_t region = few_partial_bytes(J.n, R);
    char *ws;
    if ((rc = acquire_workspace(region, &ws))) return rc;
    int64_t rechecked = 0;
    if ((rc = finish_test(J.head, J.mat, J.n, J.k, J.n_perms,
                          J.kind == 0 ? PSTAT_PATH_PLAIN_F32 : PSTAT_PATH_MFMA_SPLIT_BF16, ws, region,
                          &rechecked, J.kind != 0, nullptr, 0, J.kind != 0, J.packed)))
        return rc;
    if (sW_all)
        HIP_TRY(hipMemcpyAsync(sW_all, J.head.sw, (size_t)R * sizeof(double),
                               hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(tls.host_flags + 8, J.head.result, 4 * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    memcpy(result, tls.host_flags + 8, 4 * sizeof(double));
    if (n_rechecked) *n_rechecked = rechecked;
    return PSTAT_OK;
}

int pstat_job_release(int64_t server, int64_t job) {
    Server *sv = find_server(server);
    if (!sv) return fail(PSTAT_EINVAL, "unknown server %lld", (long long)server);
    if (job < 0 || job >= sv->max_jobs || !sv->jobs[job].live)
        return fail(PSTAT_EINVAL, "job %lld is not live", (long long)job);
    // Rounds that name this job must be complete before its slot is reused.
    for (int b = 0; b < 2; b++)
        if (sv->in_flight[b]) {
            HIP_TRY(hipEventSynchronize(sv->done[b]));
            sv->in_flight[b] = false;
        }
    sv->jobs[job] = Job();
    return PSTAT_OK;
}

}  // extern "C"
