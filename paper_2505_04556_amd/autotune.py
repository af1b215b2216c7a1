"""Autotuner: picks the computation form and its tile parameters per problem
shape by timing the library's own kernels on the caller's problem.

The search space is the one the C ABI exposes through ``pstat_set_tuning``:

* plain kernels: square tile edge T (32 or 64; the paper's compile-time TILE
  of Algorithm 2, section 2, here chosen by measurement) and permutation lanes
  per work-group (64, 128, 256) -- the number of permutations that reuse one
  staged tile;
* MFMA kernels: K-chunk length in columns (how many K blocks one work item
  accumulates in FP32 before the FP64 reduction) and N columns per work-group
  (256 or 512).

Timings are the main kernel's own duration (HIP events through
``pstat_profile``), median of ``reps`` runs after a warm-up; for the plain
kernels the entry also records the fraction of the 8 TB/s HBM peak that the
algorithmic matrix traffic (the strict upper triangle once per batch of
permutations) reaches at that time.  The form chosen
for ``auto`` is the fastest of those that meet the 1e-5 relative accuracy bar
(plain FP32 and split BF16); BF16 and FP16 are tuned too but never chosen
automatically.

Results are cached in a JSON file (``PSTAT_AUTOTUNE_CACHE`` or
``~/.cache/pstat/autotune.json``) keyed by device name, n bucket (next power of
two), k and permutation-count bucket.
"""
from __future__ import annotations

import json
import math
import os
import statistics
import time

import torch

import paper_2505_04556_amd as ps

PLAIN_SPACE = [(t, b) for t in (32, 64) for b in (64, 128, 256)]
MFMA_SPACE = [(kc, nc) for kc in (512, 1024, 1536, 2048, 4096) for nc in (256, 512)]
ACCURATE = ("plain_f32", "mfma_split_bf16", "mfma_split3_bf16")
PEAK_HBM_BYTES_S = 8e12   # MI355X HBM3E
ALL_PATHS = ("plain_f32", "mfma_split_bf16", "mfma_bf16", "mfma_f16")


def cache_path() -> str:
    return os.environ.get("PSTAT_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "pstat", "autotune.json"))


def bucket(x: int) -> int:
    return 1 << max(0, math.ceil(math.log2(max(1, x))))


def shape_key(n: int, k: int, n_perms: int, device=None) -> str:
    name = torch.cuda.get_device_name(device) if torch.cuda.is_available() else "cpu"
    return f"{name}|n{bucket(n)}|k{k}|P{bucket(n_perms)}"


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_kernel(mat, groupings, k, w, out, reps: int) -> float:
    ps.pstat_sW_k(mat, groupings, k, w, out)          # warm-up (and workspace growth)
    torch.cuda.synchronize()
    samples = []
    for _ in range(reps):
        ps.pstat_profile(True)
        ps.pstat_sW_k(mat, groupings, k, w, out)
        ms, launches = ps.pstat_profile_read()
        samples.append(ms / max(1, launches))
    ps.pstat_profile(False)
    return statistics.median(samples)


def _time_whole(mat, base, k, n_perms, seed, reps: int) -> tuple[float, float]:
    """Median wall time of a whole test (pstat_permanova, which ends with a
    synchronisation) and the median of its main kernel's time."""
    res = torch.empty(4, dtype=torch.float64, device=mat.device)
    ps.pstat_permanova(mat, base, k, n_perms, seed, result=res)    # warm-up
    torch.cuda.synchronize()
    walls, kerns = [], []
    for _ in range(reps):
        ps.pstat_profile(True)
        t0 = time.perf_counter()
        ps.pstat_permanova(mat, base, k, n_perms, seed, result=res)
        torch.cuda.synchronize()
        walls.append((time.perf_counter() - t0) * 1e3)
        ms, launches = ps.pstat_profile_read()
        kerns.append(ms / max(1, launches))
    ps.pstat_profile(False)
    return statistics.median(walls), statistics.median(kerns)


def space_for(path: str) -> list[tuple[int, int]]:
    if path.startswith("plain"):
        return PLAIN_SPACE
    return MFMA_SPACE


def tune(mat: torch.Tensor, groupings: torch.Tensor, n_groups: int, inv: torch.Tensor,
         paths=ALL_PATHS, reps: int = 3, cache: dict | None = None, save: bool = True,
         max_seconds: float = 120.0, whole=None) -> dict:
    """Times every (path, tile, batch) candidate on this problem and records the
    best per path plus the ``auto`` choice.  Returns the cache entry.

    whole = (grouping tensor, n_perms, seed): rank candidates by the time of
    the whole permutation test instead of the s_W kernel alone.  A longer MFMA
    K chunk is faster but accumulates more FP32 rounding, which widens the
    tie band and so the number of permutations the test recomputes in FP64;
    only the whole test sees both."""
    n = mat.shape[0]
    P = groupings.shape[0]
    key = shape_key(n, n_groups, P, mat.device)
    cache = load_cache() if cache is None else cache
    out = torch.empty(P, dtype=torch.float64, device=mat.device)
    entry = {"n": n, "k": n_groups, "n_perms": P, "paths": {}, "tuned_at": time.time()}
    t_start = time.perf_counter()
    for path in paths:
        best = None
        trials = []
        ps.pstat_set_path(path)
        for tile, batch in space_for(path):
            if time.perf_counter() - t_start > max_seconds:
                break
            ps.pstat_set_tuning(path, tile, batch)
            try:
                if whole is not None:
                    wall, ms = _time_whole(mat, whole[0], n_groups, whole[1], whole[2], reps)
                else:
                    ms = _time_kernel(mat, groupings, n_groups, inv, out, reps)
            except ps.PstatError as e:     # e.g. a workspace that does not fit
                trials.append({"tile": tile, "batch": batch, "error": str(e)})
                continue
            t = {"tile": tile, "batch": batch, "kernel_ms": ms}
            if whole is not None:
                t["whole_ms"] = wall
            if path.startswith("plain"):
                # the strict upper triangle streams once per `batch` permutations
                passes = -(-P // batch)
                t["hbm_frac"] = 4.0 * n * (n - 1) / 2 * passes / (ms * 1e-3) / PEAK_HBM_BYTES_S
            trials.append(t)
            rank = "whole_ms" if whole is not None else "kernel_ms"
            if best is None or t[rank] < best[rank]:
                best = dict(t)
        ps.pstat_set_tuning(path, 0, 0)
        if best is not None:
            entry["paths"][path] = dict(best, trials=trials)
    ok = [p for p in ACCURATE if p in entry["paths"]]
    if ok:
        rank = "whole_ms" if whole is not None else "kernel_ms"
        entry["auto"] = min(ok, key=lambda p: entry["paths"][p][rank])
    cache[key] = entry
    if save:
        save_cache(cache)
    return entry


def lookup(n: int, k: int, n_perms: int, cache: dict | None = None, device=None) -> dict | None:
    cache = load_cache() if cache is None else cache
    return cache.get(shape_key(n, k, n_perms, device))


def apply(n: int, k: int, n_perms: int, path: str | None = None, cache: dict | None = None,
          device=None) -> str | None:
    """Sets this thread's path and tuning from the cache; returns the path used
    (None when the shape has not been tuned: the library's defaults stay)."""
    entry = lookup(n, k, n_perms, cache, device)
    if entry is None:
        return None
    chosen = path or entry.get("auto")
    if chosen is None or chosen not in entry["paths"]:
        return None
    best = entry["paths"][chosen]
    ps.pstat_set_path(chosen)
    ps.pstat_set_tuning(chosen, best["tile"], best["batch"])
    return chosen
