#!/usr/bin/env python3
"""Benchmark: the whole PERMANOVA permutation test on one MI355X.

One step = one ``pstat_permanova`` call on a matrix already resident in HBM:
Fisher-Yates generation of every permutation, label staging, the s_W kernel
(plain or MFMA form, plus the MFMA pre-pass), the FP64 reductions, s_T, the FP64
recheck of the observed grouping and of near-tie permutations, F and the
p-value.  Headline workload (the largest single instance): n = 100,000
hash-uniform distances in (0, 1) (a 40 GB FP32 matrix resident in HBM), k = 3
groups of 20,000/30,000/50,000, 999 permutations -- a synthetic stand-in with
the top of the paper's size range.  The n = 10,000 and n = 25,000 workloads
are reported beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 3]

Prints one JSON line.  ``value`` is pair-permutations per second of the
fastest form that meets the 1e-5 relative accuracy bar (plain FP32 or split
BF16 MFMA); both forms are timed and reported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak figures of one MI355X used as roofline denominators.
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0
# Plain VALU kernel: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz single (non-packed)
# lane operations per second; the FP32 kernel spends 2 per pair-permutation (a
# compare into a lane mask, and the add that mask enables), plus one scalar
# move of the mask into EXEC per 64 lanes.
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
PLAIN_OPS_PER_PAIRPERM = 2


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def load():
    lib = os.path.join(ROOT, "paper_2505_04556_amd", "libpstat.so")
    if not os.path.exists(lib) or not os.path.exists(os.path.join(ROOT, "synth", "libsynth.so")):
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "pstat_build", os.path.join(ROOT, "paper_2505_04556_amd", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build_all()
    import paper_2505_04556_amd as ps
    return ps


def autotuned(ps, torch, D, cfg, paths):
    """Tile / permutations-per-batch (plain) and K-chunk / columns (MFMA) chosen
    by the autotuner on this workload's own matrix and permutations."""
    import synth
    from paper_2505_04556_amd import autotune
    base = torch.from_numpy(synth.base_labels(cfg["sizes"])).cuda()
    perms = ps.pstat_permute(base, cfg["n_perms"], cfg["perm_seed"])
    w = torch.from_numpy(synth.inv_group_sizes(cfg["sizes"])).cuda()
    # ranked by whole-test time: what the timed steps run
    entry = autotune.tune(D, perms, cfg["k"], w, paths=paths, reps=2, cache={}, save=False,
                          whole=(base, cfg["n_perms"], cfg["perm_seed"]))
    del perms
    return entry


def time_path(ps, torch, path, D, base, cfg, steps, warmup, tuning=None):
    """Warm up, then time exactly `steps` whole tests; returns timings and the
    last step's outputs."""
    ps.pstat_set_path(path)
    if tuning:
        ps.pstat_set_tuning(path, tuning["tile"], tuning["batch"])
    n, k, P, seed = cfg["n"], cfg["k"], cfg["n_perms"], cfg["perm_seed"]
    sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    res = torch.empty(4, dtype=torch.float64, device="cuda")
    rechecked = 0
    for _ in range(warmup):
        _, rechecked = ps.pstat_permanova(D, base, k, P, seed, result=res, sW_all=sw)
    torch.cuda.synchronize()
    ps.pstat_profile(True)
    step_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        # each whole test ends with a synchronisation (it returns the recheck count)
        ts = time.perf_counter()
        _, rechecked = ps.pstat_permanova(D, base, k, P, seed, result=res, sW_all=sw)
        step_ms.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kms, launches = ps.pstat_profile_read()
    ps.pstat_profile(False)
    return dict(path=path, seconds=dt, ms_per_step=dt * 1e3 / steps, kernel_ms_total=kms,
                kernel_launches=launches, rechecked=rechecked, sW=sw.cpu().numpy(),
                result=res.cpu().numpy(), step_ms_median=float(sorted(step_ms)[len(step_ms) // 2]),
                step_ms_best=float(min(step_ms)))


def speedup_leg(ps, torch, sd, synth, steps=3, warmup=1):
    """The precision workload (n=25,000, k=10 uneven groups, 3,999
    permutations): whole tests on the plain FP32 and split-BF16 forms with the
    library defaults; the split form's speedup over the plain one."""
    cfg = synth.config(2)
    D = sd.matrix(cfg)
    base = torch.from_numpy(synth.base_labels(cfg["sizes"])).cuda()
    n, P = cfg["n"], cfg["n_perms"]
    pair_perms = n * (n - 1) // 2 * P
    res = {}
    for path in ("plain_f32", "mfma_split_bf16"):
        r = time_path(ps, torch, path, D, base, cfg, steps, warmup)
        res[path] = dict(ms_per_step=round(r["ms_per_step"], 3),
                         kernel_ms=round(r["kernel_ms_total"] / max(1, r["kernel_launches"]), 3),
                         G_pair_perms_per_s=round(pair_perms / (r["ms_per_step"] / 1e3) / 1e9, 1),
                         F_obs=float(r["result"][0]), p=float(r["result"][1]))
    ps.pstat_set_path(ps.PSTAT_PATH_AUTO)
    del D
    torch.cuda.empty_cache()
    return dict(workload=cfg["name"], steps=steps, forms=res,
                speedup_whole_test=round(res["plain_f32"]["ms_per_step"]
                                         / res["mfma_split_bf16"]["ms_per_step"], 3),
                speedup_kernel=round(res["plain_f32"]["kernel_ms"]
                                     / res["mfma_split_bf16"]["kernel_ms"], 3),
                rel_err_bound=1e-5,
                rel_err_checked_by="tests/test_gpu_fullsize.py::test_n25000_precision_table "
                                   "(every permutation against the FP64 oracle)")


def packed_leg(ps, torch, sd, synth, n, steps=2, warmup=1):
    """The whole test with D given as its packed strict upper triangle (half
    the memory of the square): hash-uniform distances, k = 3 groups of 20/30/50%
    of n, 999 permutations, split BF16 -- the n = 100,000 workload's shape at
    any n, up to sizes whose square layout would not fit beside the tiles."""
    sizes = [n // 5, 3 * n // 10]
    sizes.append(n - sum(sizes))
    cfg = dict(n=n, k=3, n_perms=999, perm_seed=3003, sizes=sizes)
    torch.cuda.empty_cache()
    D = sd.uniform_packed(n, 1001)
    base = torch.from_numpy(synth.base_labels(sizes)).cuda()
    r = time_path(ps, torch, "mfma_split_bf16", D, base, cfg, steps, warmup)
    ps.pstat_set_path(ps.PSTAT_PATH_AUTO)
    del D
    ps.pstat_free_workspace()
    torch.cuda.empty_cache()
    pair_perms = n * (n - 1) // 2 * cfg["n_perms"]
    return dict(workload=f"n{n}_k3_P999_uniform_packed", layout="strict upper triangle, packed",
                matrix_GB=round(2 * n * (n - 1) / 1e9, 1), steps=steps,
                ms_per_step=round(r["ms_per_step"], 3),
                kernel_ms=round(r["kernel_ms_total"] / max(1, r["kernel_launches"]), 3),
                G_pair_perms_per_s=round(pair_perms / (r["ms_per_step"] / 1e3) / 1e9, 1),
                F_obs=float(r["result"][0]), p=float(r["result"][1]), rechecked=r["rechecked"])


def host_description() -> dict:
    """The host the CPU baseline ran on: lscpu's model, sockets, cores, threads
    per core and NUMA nodes, and the CPUs in this process's affinity mask."""
    import subprocess
    keys = ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core",
            "NUMA node(s)", "CPU(s)")
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
    except (OSError, subprocess.SubprocessError):
        out = ""
    for line in out.splitlines():
        if ":" in line:
            key, val = line.split(":", 1)
            if key.strip() in keys and key.strip() not in info:
                info[key.strip()] = val.strip()
    info["affinity_cpus"] = len(os.sched_getaffinity(0))
    return info


def smt_core_sets(max_cores: int):
    """Up to max_cores physical cores of this process's affinity mask that have
    two hardware threads in it: (both threads of each core, one per core), or
    None when the mask has no SMT siblings."""
    mask = sorted(os.sched_getaffinity(0))
    cores = {}
    for c in mask:
        try:
            base = f"/sys/devices/system/cpu/cpu{c}/topology/"
            key = (open(base + "physical_package_id").read().strip(),
                   open(base + "core_id").read().strip())
        except OSError:
            return None
        cores.setdefault(key, []).append(c)
    pairs = [v[:2] for v in cores.values() if len(v) >= 2][:max_cores]
    if not pairs:
        return None
    return [c for pr in pairs for c in pr], [pr[0] for pr in pairs]


def cpu_baseline(D, cfg, target_s=15.0, smt_share=0.15):
    """The FP64 oracle, as it stands, on this host's cores over a bounded
    sample of the same workload: s_W of the first m permutations over the
    whole matrix.  D stays on the device; the oracle is fed row block by row
    block through a pinned host buffer (only the oracle calls are timed), so no
    host copy of the whole matrix is needed.  m is chosen from a timed first
    block so that the sample takes about target_s.  The SMT comparison (the
    paper's finding that SMT matters on the CPU side) runs the oracle on the
    leading share of rows with the team pinned to the same physical cores:
    two threads per core, then one."""
    import numpy as np
    import torch

    import oracle
    import synth
    n, P = cfg["n"], cfg["n_perms"]
    base = synth.base_labels(cfg["sizes"])
    w = synth.inv_group_sizes(cfg["sizes"])
    k = len(cfg["sizes"])
    threads = oracle.max_threads()
    pairs_total = n * (n - 1) // 2
    block = max(1, min(n, (256 << 20) // (4 * n)))
    host = torch.empty((block, n), dtype=torch.float32, pin_memory=True)

    def rows(r0):
        r1 = min(n, r0 + block)
        host[: r1 - r0].copy_(D[r0:r1])
        return host[: r1 - r0].numpy()

    def pairs_in(r0, r1):
        # pairs (a, b), a in [r0, r1), b > a
        return (r1 - r0) * (n - 1) - (r1 * (r1 - 1) // 2 - r0 * (r0 - 1) // 2)

    # calibration: `threads` permutations over the first block
    perms = oracle.permute(base, min(P, max(threads, 1)), cfg["perm_seed"])
    blk = rows(0)
    sums = oracle.new_group_sums(perms.shape[0], k)
    t0 = time.perf_counter()
    oracle.group_sums(blk, 0, n, perms, sums)
    dt = time.perf_counter() - t0
    rate0 = perms.shape[0] * pairs_in(0, blk.shape[0]) / max(dt, 1e-9)
    m = int(target_s * rate0 / pairs_total)
    m = max(threads, (m // threads) * threads)
    m = min(m, P)
    perms = oracle.permute(base, m, cfg["perm_seed"])
    sums = oracle.new_group_sums(m, k)
    seconds = 0.0
    for r0 in range(0, n, block):
        blk = rows(r0)
        t0 = time.perf_counter()
        oracle.group_sums(blk, r0, n, perms, sums)
        seconds += time.perf_counter() - t0
    sW = oracle.sW_from_sums(sums, w)
    out = dict(value=m * pairs_total / seconds / 1e9, seconds=seconds, perms=m, threads=threads,
               sW=sW, host=host_description())
    # SMT: the same cores with two hardware threads each, then one
    sets = smt_core_sets(max(1, threads // 2))
    if sets is None:
        out["smt"] = {"note": "no SMT siblings in this process's affinity mask"}
        return out
    both, one = sets
    mask = sorted(os.sched_getaffinity(0))
    lead = 0
    r_end = 0
    while r_end < n and lead < smt_share * pairs_total:
        r_end = min(n, r_end + block)
        lead = pairs_in(0, r_end)
    smt = {"cores": len(one), "rows": r_end, "pairs": lead}
    try:
        for name, cpus in (("two_threads_per_core", both), ("one_thread_per_core", one)):
            team = len(cpus)
            mp = min(P, team)
            pp = oracle.permute(base, mp, cfg["perm_seed"])
            ss = oracle.new_group_sums(mp, k)
            oracle.pin_threads(cpus, team, True)
            secs = 0.0
            for r0 in range(0, r_end, block):
                b = rows(r0)[: min(block, r_end - r0)]
                t0 = time.perf_counter()
                oracle.group_sums(b, r0, n, pp, ss, nthreads=team)
                secs += time.perf_counter() - t0
            smt[name] = dict(threads=team, cpus=cpus, perms=mp, seconds=round(secs, 3),
                             G_pair_perms_per_s=round(mp * lead / secs / 1e9, 4))
    finally:
        oracle.pin_threads(mask, len(both), False)
        oracle.pin_threads(mask, threads, False)
    smt["smt_speedup"] = round(smt["two_threads_per_core"]["G_pair_perms_per_s"]
                               / smt["one_thread_per_core"]["G_pair_perms_per_s"], 3)
    out["smt"] = smt
    return out


def gemm_ceiling(torch, shapes=((16384, 16384, 16384), (10000, 50000, 10000)), reps=5):
    """The vendor library's dense BF16 rate on this GPU (torch.matmul, which
    runs hipBLASLt): what a plain GEMM reaches here under the chip's power and
    clock limits, beside the nominal 2.5 PFLOP/s peak."""
    res = {}
    g = torch.Generator(device="cuda").manual_seed(0)
    for (m, nn, kk) in shapes:
        a = torch.randn(m, kk, device="cuda", dtype=torch.bfloat16, generator=g)
        b = torch.randn(kk, nn, device="cuda", dtype=torch.bfloat16, generator=g)
        for _ in range(2):
            c = a @ b
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            c = a @ b
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[f"{m}x{nn}x{kk}"] = {"ms": round(ms, 4),
                                 "TFLOP_per_s": round(2.0 * m * nn * kk / (ms * 1e-3) / 1e12, 1)}
        del a, b, c
    torch.cuda.empty_cache()
    return res


def recorded_traffic(kernel_src: str, summary: str):
    """HBM bytes per launch from a committed counter summary, or None when the
    kernel source has changed since the counters were taken."""
    import hashlib
    try:
        fields = dict(line.split(":", 1) for line in open(os.path.join(ROOT, summary))
                      if ":" in line and not line.startswith("#"))
        digest = hashlib.sha256(open(os.path.join(ROOT, kernel_src), "rb").read()).hexdigest()
    except OSError:
        return None
    if fields.get("kernel_source_sha256", "").strip() != digest:
        return None
    return float(fields["traffic_bytes_per_launch"].split()[0])


def serve_trace(budget_bytes: int, count: int, rate: float, arrival_seed: int,
                budget_factor: float = 0.0, burst: bool = False):
    """One serving trace: Poisson arrivals (`rate` requests/s, arrival times from
    `arrival_seed`), n in {1k..20k}, k in 2..12 with Dirichlet sizes, 999 or
    9,999 permutations; continuous batching under an HBM budget (with
    budget_factor > 0: that multiple of the largest request's footprint)."""
    import synth
    import synth.device as sd
    from paper_2505_04556_amd.serve import GpuExecutor, Request, Server
    reqs = []
    for t in synth.serving_requests(count, rate, arrival_seed):
        reqs.append(Request(id=t["id"], n=t["n"], k=t["k"], grouping=synth.base_labels(t["sizes"]),
                            n_perms=t["n_perms"], seed=t["perm_seed"], arrival=t["arrival"],
                            make_matrix=(lambda dev, n=t["n"], s=t["matrix_seed"]:
                                         sd.uniform_matrix(n, s, dev))))
    ex = GpuExecutor(max_jobs=32, max_units=8192, path="auto")
    forms = {}
    for r in reqs:
        f = ex.form(r)
        forms[f] = forms.get(f, 0) + 1
    if budget_factor > 0:
        budget_bytes = int(budget_factor * max(ex.footprint(r) for r in reqs))
    try:
        ex.warmup(reserve_bytes=budget_bytes)   # server start-up, before the first arrival
        srv = Server(ex, hbm_budget=budget_bytes, round_work=1.5e11, max_units=8192)
        res = srv.run(reqs, realtime=not burst)
    finally:
        ex.close()
    res["budget_bytes"] = budget_bytes
    return res, forms


def serve_leg(budget_bytes: int, count: int = 64, rate: float = 4.0, seeds: int = 1,
              budget_factor: float = 0.0, burst: bool = False) -> dict:
    """The serving trace at arrival seed 4000 (latency = result time - arrival
    time, nearest-rank quantiles); with seeds > 1 the same requests are replayed
    under arrival seeds 4001, ... and the latencies of all traces are pooled."""
    from paper_2505_04556_amd.serve import nearest_rank
    res, forms = serve_trace(budget_bytes, count, rate, 4000, budget_factor, burst)
    budget_bytes = res["budget_bytes"]
    st = dict(res["stats"])
    ok = [o for o in res["outcomes"].values() if o.error is None]
    waits = sorted(o.admitted - o.arrival for o in ok)
    waited = sum(1 for w in waits if w > 0.05)
    st.update(rounds=res["rounds"], peak_resident_GB=round(res["peak_bytes"] / 1e9, 3),
              budget_GB=round(budget_bytes / 1e9, 3), requests=count,
              arrivals=("all at t = 0" if burst else f"Poisson, {rate} per s"),
              admissions_delayed_50ms=waited,
              admissions_waited_1ms=sum(1 for w in waits if w > 0.001),
              admission_wait_max_s=round(waits[-1], 4) if waits else None,
              admission_wait_mean_s=round(sum(waits) / len(waits), 4) if waits else None,
              quantiles="nearest rank",
              path="auto: work-list kernels of both forms in each round", jobs_by_form=forms)
    out = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in st.items()}
    if seeds > 1:
        lat = [o.latency for o in res["outcomes"].values() if o.error is None]
        per = [dict(seed=4000, p50_s=out["p50_s"], p99_s=out["p99_s"],
                    G_pair_perms_per_s=out["G_pair_perms_per_s"])]
        failed = out["failed"]
        for sd_ in range(4001, 4000 + seeds):
            r2, _ = serve_trace(budget_bytes, count, rate, sd_)
            lat += [o.latency for o in r2["outcomes"].values() if o.error is None]
            failed += r2["stats"].get("failed", 0)
            per.append(dict(seed=sd_, p50_s=round(r2["stats"]["p50_s"], 5),
                            p99_s=round(r2["stats"]["p99_s"], 5),
                            G_pair_perms_per_s=round(r2["stats"]["G_pair_perms_per_s"], 4)))
        out["pooled"] = dict(arrival_seeds=list(range(4000, 4000 + seeds)), samples=len(lat),
                             failed=failed, p50_s=round(nearest_rank(lat, 0.50), 5),
                             p99_s=round(nearest_rank(lat, 0.99), 5), max_s=round(max(lat), 5),
                             per_seed=per)
    return out


# Counter summaries (profiles/) of each form's main kernel, by workload; a
# recorded figure is used only while the kernel source is the one it was
# taken on.
TRAFFIC_FILES = {
    ("mfma_split_bf16", 1): ("paper_2505_04556_amd/csrc/k_mfma.hip",
                             "profiles/k_mfma_split_n10000_hbm_traffic.txt"),
    ("mfma_split_bf16", 3): ("paper_2505_04556_amd/csrc/k_mfma.hip",
                             "profiles/k_mfma_split_n100000_hbm_traffic.txt"),
    ("plain_f32", 1): ("paper_2505_04556_amd/csrc/k_plain.hip",
                       "profiles/k_plain_f32_n10000_hbm_traffic.txt"),
    ("plain_f32", 3): ("paper_2505_04556_amd/csrc/k_plain.hip",
                       "profiles/k_plain_f32_n100000_hbm_traffic.txt"),
}

DATA = {
    "uniform": "synthetic (seeded hash-uniform distances in (0,1), exact in FP32, symmetric, "
               "zero diagonal)",
    "euclid": "synthetic (seeded Euclidean distances of N(0,1) points, 32 dims, scaled to [0,1])",
}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=3,
                    help="workload: 0 n=1,000; 1 n=10,000; 2 n=25,000; 3 n=100,000 (default)")
    ap.add_argument("--paths", default="plain_f32,mfma_split_bf16")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target duration of the CPU oracle's sample")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving traces")
    ap.add_argument("--no-tune", action="store_true", help="library defaults instead of autotuning")
    ap.add_argument("--no-speedup", action="store_true",
                    help="skip the n=25,000 plain-vs-split-BF16 comparison")
    ap.add_argument("--no-n10000", action="store_true",
                    help="skip the n=10,000 whole tests reported beside the headline")
    ap.add_argument("--no-gemm", action="store_true",
                    help="skip the vendor BF16 GEMM rate measured for context")
    ap.add_argument("--gemm-only", action="store_true",
                    help="measure only the vendor BF16 GEMM rate (for profiling it)")
    ap.add_argument("--serve-budget-gb", type=float, default=8.0)
    ap.add_argument("--plain-tuning", default="",
                    help="TILE,LANES for the plain form instead of the tuned or default ones "
                         "(e.g. 32,64: a lanes sweep)")
    ap.add_argument("--serve-tight-factor", type=float, default=1.0,
                    help="budget of a second serving run, all 64 requests arriving at once, as "
                         "a multiple of the largest request's footprint: admission must queue "
                         "(0 skips it)")
    ap.add_argument("--serve-seeds", type=int, default=1,
                    help="replay the serving trace under this many arrival seeds and pool "
                         "the latencies")
    ap.add_argument("--packed-n", type=int, default=0,
                    help="also time a whole test of this n with D in the packed layout")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the permutation "
              "axis would shard across GPUs, and this benchmark measures one GPU's share.",
              file=sys.stderr)
        return 2
    host = host_description()        # before any device work: lscpu runs as a child

    import numpy as np
    import torch

    import synth
    import synth.device as sd

    ps = load()
    if args.copy_probe_mib:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE calibrate the counters
        src = torch.ones(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.gemm_only:
        print(json.dumps({"gemm_bf16_torch_matmul": gemm_ceiling(torch)}), flush=True)
        return 0
    cfg = synth.config(args.config)
    n, k, P = cfg["n"], cfg["k"], cfg["n_perms"]
    log(f"workload {cfg['name']}: generating the matrix on the device")
    D = sd.matrix(cfg)
    base = torch.from_numpy(synth.base_labels(cfg["sizes"])).cuda()
    torch.cuda.synchronize()
    pairs = n * (n - 1) // 2
    pair_perms = pairs * P
    R = P + 1

    paths = args.paths.split(",")
    tuned = {}
    if not args.no_tune:
        log("autotuning " + ", ".join(paths))
        entry = autotuned(ps, torch, D, cfg, tuple(paths))
        tuned = {p: {kk: v[kk] for kk in ("tile", "batch", "kernel_ms", "whole_ms", "hbm_frac")
                     if kk in v}
                 for p, v in entry["paths"].items()}
        log(f"  tuned: {tuned}")
    if args.plain_tuning:
        t_, l_ = (int(v) for v in args.plain_tuning.split(","))
        tuned["plain_f32"] = {"tile": t_, "batch": l_}
    runs = {}
    for path in paths:
        log(f"timing {path}: {args.warmup} warm-up + {args.steps} steps")
        runs[path] = time_path(ps, torch, path, D, base, cfg, args.steps, args.warmup,
                               tuned.get(path))
        log(f"  {path}: {runs[path]['ms_per_step']:.2f} ms/step, "
            f"kernel {runs[path]['kernel_ms_total'] / max(1, runs[path]['kernel_launches']):.2f} ms")
    ps.pstat_set_path(ps.PSTAT_PATH_AUTO)
    for path in paths:
        ps.pstat_set_tuning(path, 0, 0)

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline (bounded sample, row blocks from the device copy)")
        cpu = cpu_baseline(D, cfg, target_s=args.cpu_seconds)
        cpu["host"] = host
        log(f"  oracle: {cpu['value']:.3f} G pair-perms/s on {cpu['threads']} threads, "
            f"{cpu['perms']} perms in {cpu['seconds']:.1f} s; smt {cpu.get('smt')}")

    # Accuracy of each timed run on the oracle's sample (same generator, same seed).
    acc = {}
    if cpu is not None:
        m = cpu["perms"]
        for path, r in runs.items():
            got = r["sW"][1:1 + m]
            acc[path] = float(np.max(np.abs(got - cpu["sW"]) / np.abs(cpu["sW"])))
    del D
    torch.cuda.empty_cache()
    ps.pstat_free_workspace()

    extra_n10000 = None
    if not args.no_n10000 and args.config != 1:
        log("n=10,000 whole tests (Euclidean, k=5, 9,999 permutations), library defaults")
        c1 = synth.config(1)
        D1 = sd.matrix(c1)
        b1 = torch.from_numpy(synth.base_labels(c1["sizes"])).cuda()
        pp1 = c1["n"] * (c1["n"] - 1) // 2 * c1["n_perms"]
        extra_n10000 = {"workload": c1["name"], "steps": args.steps, "forms": {}}
        for path in paths:
            r1 = time_path(ps, torch, path, D1, b1, c1, args.steps, args.warmup)
            extra_n10000["forms"][path] = dict(
                ms_per_step=round(r1["ms_per_step"], 4),
                kernel_ms=round(r1["kernel_ms_total"] / max(1, r1["kernel_launches"]), 4),
                G_pair_perms_per_s=round(pp1 / (r1["ms_per_step"] / 1e3) / 1e9, 3),
                F_obs=float(r1["result"][0]), p=float(r1["result"][1]),
                rechecked_perms=int(r1["rechecked"]))
        ps.pstat_set_path(ps.PSTAT_PATH_AUTO)
        del D1
        torch.cuda.empty_cache()
        ps.pstat_free_workspace()

    speedup = None
    if not args.no_speedup:
        log("speedup leg: n=25,000, k=10, 3,999 permutations, plain FP32 vs split BF16")
        speedup = speedup_leg(ps, torch, sd, synth)
        ps.pstat_free_workspace()
        log(f"  {speedup}")

    gemm = None
    if not args.no_gemm:
        log("vendor BF16 GEMM rate (torch.matmul) for context")
        gemm = gemm_ceiling(torch)
        log(f"  {gemm}")

    packed = None
    if args.packed_n:
        log(f"packed-layout leg: n={args.packed_n:,}, k=3, 999 permutations, split BF16")
        packed = packed_leg(ps, torch, sd, synth, args.packed_n)
        log(f"  {packed}")

    serve = None
    if not args.no_serve:
        log(f"serving trace: 64 requests, Poisson 4/s, {args.serve_budget_gb:g} GB budget")
        serve = serve_leg(int(args.serve_budget_gb * 1e9), seeds=args.serve_seeds)
        log(f"  serve: p50 {serve.get('p50_s')} s, p99 {serve.get('p99_s')} s, "
            f"{serve.get('G_pair_perms_per_s')} G pair-perms/s")
        if args.serve_tight_factor > 0:
            log(f"serving burst (all 64 at once) under {args.serve_tight_factor:g} x the "
                f"largest footprint")
            tight = serve_leg(0, seeds=1, budget_factor=args.serve_tight_factor, burst=True)
            serve["tight_budget"] = tight
            log(f"  serve (tight): p50 {tight.get('p50_s')} s, p99 {tight.get('p99_s')} s, "
                f"delayed {tight.get('admissions_delayed_50ms')}")

    ok_paths = [p for p in runs if p in ("plain_f32", "mfma_split_bf16", "mfma_split3_bf16")]
    best = min(ok_paths, key=lambda p: runs[p]["ms_per_step"])
    r = runs[best]
    value = pair_perms / (r["ms_per_step"] / 1e3) / 1e9
    kern_ms = r["kernel_ms_total"] / max(1, r["kernel_launches"])
    traffic = None
    if (best, args.config) in TRAFFIC_FILES:
        traffic = recorded_traffic(*TRAFFIC_FILES[(best, args.config)])
    if best.startswith("mfma"):
        s = 3 if "split3" in best else 2 if "split" in best else 1
        # algorithmic work: 2 k s flops per pair-permutation (one-hot columns
        # for all k groups, s BF16 parts); the whole test's kernel executes
        # k - 1 columns (the largest group from the complement)
        work = 2.0 * k * s * pairs * R
        executed = 2.0 * (k - 1) * s * pairs * R
        achieved = work / (kern_ms / 1e3) / 1e12
        roof = dict(bound="mfma", achieved=round(achieved, 2), peak=PEAK_BF16_TFLOPS,
                    unit="TFLOP/s", frac=round(achieved / PEAK_BF16_TFLOPS, 4), traffic=traffic,
                    traffic_unit="HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, each scaled "
                                 "by the same counter's reading for a 1 GiB device copy)",
                    kernel=f"k_mfma ({best}, {k - 1} one-hot columns per grouping)",
                    kernel_ms=round(kern_ms, 4),
                    work_per_launch=f"{2 * k * s} flop x {pairs} pairs x {R} groupings",
                    executed=dict(flop_per_pair_perm=2 * (k - 1) * s,
                                  achieved=round(executed / (kern_ms / 1e3) / 1e12, 2),
                                  frac=round(executed / (kern_ms / 1e3) / 1e12
                                             / PEAK_BF16_TFLOPS, 4)))
    else:
        work = PLAIN_OPS_PER_PAIRPERM * pairs * R
        achieved = work / (kern_ms / 1e3) / 1e12
        roof = dict(bound="alu", achieved=round(achieved, 2), peak=round(PEAK_VALU_TOPS, 2),
                    unit="T lane-op/s", frac=round(achieved / PEAK_VALU_TOPS, 4),
                    traffic=traffic, kernel="k_plain<32,256,float>", kernel_ms=round(kern_ms, 4),
                    work_per_launch=f"{PLAIN_OPS_PER_PAIRPERM} VALU lane-ops x {pairs} pairs x "
                                    f"{R} groupings")

    out = {
        "metric": "G pair-perms/s for s_W (whole permutation test), plain vs MFMA at 1e-5 rel err",
        "value": round(value, 3),
        "unit": "G pair-perms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("bf16 hi+mid+lo -> f32 accumulate -> f64" if best == "mfma_split3_bf16"
                  else "bf16 hi+lo -> f32 accumulate -> f64" if best.startswith("mfma")
                  else "f32 -> f64"),
        "data": DATA[cfg["matrix"]],
        "config": {"workload": cfg["name"], "n": n, "k": k, "group_sizes": cfg["sizes"],
                   "n_perms": P, "path": best},
        "roofline": roof,
        "paths": {p: {"ms_per_step": round(v["ms_per_step"], 4),
                      "ms_per_step_median": round(v["step_ms_median"], 4),
                      "ms_per_step_best": round(v["step_ms_best"], 4),
                      "G_pair_perms_per_s": round(pair_perms / (v["ms_per_step"] / 1e3) / 1e9, 3),
                      "kernel_ms": round(v["kernel_ms_total"] / max(1, v["kernel_launches"]), 4),
                      "F_obs": float(v["result"][0]), "p": float(v["result"][1]),
                      "rechecked_perms": int(v["rechecked"]),
                      "tuning": tuned.get(p),
                      "max_rel_err_vs_oracle_sample": acc.get(p)}
                  for p, v in runs.items()},
    }
    # The plain kernel against HBM: algorithmic bytes (the strict upper
    # triangle once per pass of `lanes` permutations) and, where recorded,
    # counter traffic, over this run's kernel time
    if "plain_f32" in runs:
        v = runs["plain_f32"]
        kms = v["kernel_ms_total"] / max(1, v["kernel_launches"])
        lanes = (tuned.get("plain_f32") or {}).get("batch") or 256
        passes = -(-R // lanes)
        alg = 4.0 * pairs * passes
        hbm = dict(lanes=lanes, passes_over_matrix=passes, algorithmic_bytes=alg,
                   algorithmic_GB_per_s=round(alg / (kms / 1e3) / 1e9, 1),
                   algorithmic_frac_of_8TBps=round(alg / (kms / 1e3) / 8e12, 4))
        t = recorded_traffic(*TRAFFIC_FILES[("plain_f32", args.config)]) \
            if ("plain_f32", args.config) in TRAFFIC_FILES else None
        if t is not None:
            hbm.update(traffic_bytes=t, traffic_GB_per_s=round(t / (kms / 1e3) / 1e9, 1),
                       traffic_frac_of_8TBps=round(t / (kms / 1e3) / 8e12, 4))
        out["paths"]["plain_f32"]["hbm"] = hbm
    if gemm is not None:
        best_gemm = max(v["TFLOP_per_s"] for v in gemm.values())
        out["mfma_context"] = {
            "vendor_bf16_gemm": gemm,
            "note": "torch.matmul (hipBLASLt) dense BF16 on this GPU, same power limits",
            "roofline_executed_over_best_gemm": (round(roof["executed"]["achieved"] / best_gemm, 4)
                                                 if roof["bound"] == "mfma" else None)}
    if extra_n10000 is not None:
        out["n10000"] = extra_n10000
    if speedup is not None:
        out["speedup_n25000"] = speedup
    if packed is not None:
        out["packed_leg"] = packed
    if serve is not None:
        out["serve"] = serve
    if cpu is not None:
        out["cpu_baseline"] = {"value": round(cpu["value"], 4), "unit": "G pair-perms/s",
                               "cores": cpu["threads"], "kind": "oracle",
                               "sample": f"FP64 oracle s_W of the first {cpu['perms']} of the "
                                         f"{P} permutations over the whole matrix (same "
                                         f"generator, row blocks copied from the device), "
                                         f"{cpu['seconds']:.1f} s on {cpu['threads']} threads "
                                         f"(all of the process's OpenMP threads, unpinned)",
                               "host": cpu["host"], "smt": cpu.get("smt")}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
