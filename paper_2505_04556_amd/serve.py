"""Serving loop: many PERMANOVA tests of different n, k and permutation counts
on one GPU with continuous batching.

* Admission by HBM footprint: a request is admitted when its matrix, its job
  scratch and its labels fit in the remaining budget and a job slot is free;
  the oldest waiting request goes first, and smaller ones behind it may start
  while it waits for memory (first fit).
* Resident matrices: an admitted request's matrix is materialised on the device
  (its ``make_matrix`` callback stands in for the upload) and stays until the
  test finishes.
* Rounds: every round takes work units from the admitted jobs, oldest job
  first, up to a work budget, and runs them in one launch of the library's
  work-list kernel replayed from a captured hipGraph
  (``pstat_serve_round``).  Requests that arrive while a round runs join the
  next one, so their work overlaps other requests' on the device.
* A job whose last units ran is finished (FP64 reduction, recheck, F, p) and
  released; its latency is result time minus arrival time.

A job's numbers depend only on its own work units and a fixed reduction order,
so every result is bit-identical alone and in any mix.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Callable

import numpy as np


@dataclass
class Request:
    id: int
    n: int
    k: int
    grouping: np.ndarray            # int32 [n], labels 0..k-1
    n_perms: int
    seed: int
    arrival: float = 0.0            # seconds after the trace starts
    make_matrix: Callable | None = None   # device -> float32 [n, n] tensor, or the
                                          # packed strict upper triangle [n (n - 1) / 2]
    packed: bool = False            # make_matrix returns the packed layout

    @property
    def pair_perms(self) -> int:
        return self.n * (self.n - 1) // 2 * self.n_perms


@dataclass
class Outcome:
    id: int
    result: list | None = None      # [F_obs, p, s_W_obs, s_T]
    sW_all: np.ndarray | None = None
    rechecked: int = 0
    arrival: float = 0.0
    admitted: float = math.nan
    finished: float = math.nan
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Executor:
    """Device operations the scheduler needs (the GPU one is below; tests use
    a stand-in)."""

    def footprint(self, req: Request) -> int: ...
    def create(self, req: Request): ...            # -> (handle, n_units, unit_cost)
    def run_round(self, pairs: np.ndarray) -> None: ...
    def finish(self, handle, keep_sW: bool): ...   # -> (result, sW_all or None, rechecked)
    def release(self, handle) -> None: ...
    def close(self) -> None: ...


class GpuExecutor(Executor):
    """Executor on the pstat C ABI; all work on one created stream.

    ``path`` picks each job's form: "plain_f32", "mfma_split_bf16" or "auto"
    (the library's choice by n and k).  Unit costs are in plain-kernel
    pair-permutations, so one round budget covers both forms: an MFMA unit's
    pair-permutations count ``mfma_speedup`` times less."""

    mfma_speedup = 3.5     # split-BF16 MFMA vs plain FP32 throughput, n >= 5,000, k = 5

    def __init__(self, max_jobs: int = 64, max_units: int = 8192, device=None,
                 path: str = "auto"):
        import torch

        import paper_2505_04556_amd as ps
        self.ps, self.torch = ps, torch
        self.path = path
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = torch.cuda.Stream(self.device)     # default priority
        self.max_units = max_units
        self.max_jobs = max_jobs         # job slots of the device server
        with torch.cuda.stream(self.stream):
            self.server = ps.pstat_serve_create(max_jobs, max_units)
        self.live = {}

    def footprint(self, req: Request) -> int:
        ps = self.ps
        mat = 2 * req.n * (req.n - 1) if req.packed else 4 * req.n * req.n
        return mat + ps.pstat_job_bytes(req.n, req.n_perms, req.k, self.path) + 4 * req.n

    def form(self, req: Request) -> str:
        return self.ps.resolve_path(self.path, req.n, req.k)

    def create(self, req: Request):
        torch, ps = self.torch, self.ps
        with torch.cuda.stream(self.stream):
            mat = req.make_matrix(self.device)
            g = torch.from_numpy(np.ascontiguousarray(req.grouping, dtype=np.int32)).to(self.device)
            scratch = torch.empty(ps.pstat_job_bytes(req.n, req.n_perms, req.k, self.path),
                                  dtype=torch.uint8, device=self.device)
            job, units = ps.pstat_job_create(self.server, mat, g, req.k, req.n_perms, req.seed,
                                             scratch, self.path)
        # work of one unit in plain-kernel pair-permutations; used only to
        # size rounds
        pairs = req.n * (req.n - 1) / 2
        unit_cost = pairs * (req.n_perms + 1) / max(1, units)
        if self.form(req) == "mfma_split_bf16":
            unit_cost /= self.mfma_speedup
        self.live[job] = (mat, g, scratch, req.n_perms + 1)
        return job, units, unit_cost

    def run_round(self, pairs: np.ndarray) -> None:
        with self.torch.cuda.stream(self.stream):
            self.ps.pstat_serve_round(self.server, pairs)

    def finish(self, handle, keep_sW: bool = False):
        torch, ps = self.torch, self.ps
        R = self.live[handle][3]
        with torch.cuda.stream(self.stream):
            sw = torch.empty(R, dtype=torch.float64, device=self.device) if keep_sW else None
            res, rech = ps.pstat_job_finish(self.server, handle, sw)   # synchronises the stream
        return res, (sw.cpu().numpy() if keep_sW else None), rech

    def release(self, handle) -> None:
        with self.torch.cuda.stream(self.stream):
            self.ps.pstat_job_release(self.server, handle)
        self.live.pop(handle, None)

    def warmup(self, reserve_bytes: int = 0) -> None:
        """Start-up work that would otherwise land on the first requests: one
        small job of each form through create, a round and finish (loads the
        kernels and captures the round graphs), and, with reserve_bytes, one
        allocation of that size returned to torch's caching allocator so that
        job scratch is later carved from it instead of fresh device
        allocations."""
        torch = self.torch
        if reserve_bytes > 0:
            with torch.cuda.stream(self.stream):
                block = torch.empty(int(reserve_bytes), dtype=torch.uint8, device=self.device)
                del block
        rng = np.random.default_rng(0)
        # split BF16 with 512- and 256-column work-groups (k = 3, 2; k <= 16)
        # and plain (k = 40) under "auto"
        for k in (3, 2, 40):
            n = 640
            g = np.concatenate([np.arange(k), rng.integers(0, k, size=n - k)]).astype(np.int32)

            def make(dev, n=n):
                d = torch.rand(n, n, device=dev)
                d = (d + d.T) * 0.5
                d.fill_diagonal_(0.0)
                return d
            req = Request(id=-1, n=n, k=k, grouping=g, n_perms=63, seed=1, make_matrix=make)
            handle, n_units, _ = self.create(req)
            self.run_round(np.asarray([(handle, u) for u in range(n_units)], dtype=np.int64))
            self.finish(handle)
            self.release(handle)
        self.stream.synchronize()

    def close(self) -> None:
        self.stream.synchronize()
        self.ps.pstat_serve_destroy(self.server)


@dataclass
class _Active:
    req: Request
    handle: object
    n_units: int
    unit_cost: float
    next_unit: int = 0
    footprint: int = 0


@dataclass
class Server:
    executor: Executor
    hbm_budget: int
    max_jobs: int = 64
    round_work: float = 1.5e11      # pair-permutations per round (~20 ms of plain kernel)
    # a request that has waited this long for memory is passed by no later one
    aging_s: float = 0.5
    max_units: int = 8192
    keep_sW: bool = False
    clock: Callable[[], float] = time.perf_counter
    sleep: Callable[[float], None] = time.sleep
    log: list = field(default_factory=list)

    def run(self, requests: list[Request], realtime: bool = True) -> dict:
        """Serves the trace (arrivals at req.arrival seconds after start, or all
        at once when realtime is False); returns outcomes and statistics."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.id))
        out = {r.id: Outcome(id=r.id, arrival=r.arrival) for r in reqs}
        pending: collections.deque[Request] = collections.deque()
        active: list[_Active] = []
        used = 0
        peak = 0
        nxt = 0
        rounds = 0
        t0 = self.clock()
        now = lambda: self.clock() - t0  # noqa: E731
        # no more resident jobs than the executor has slots for
        max_jobs = min(self.max_jobs, getattr(self.executor, "max_jobs", self.max_jobs))
        if not realtime:
            for r in reqs:
                out[r.id].arrival = 0.0
        while nxt < len(reqs) or pending or active:
            t = now()
            while nxt < len(reqs) and (not realtime or reqs[nxt].arrival <= t):
                pending.append(reqs[nxt])
                nxt += 1
            # admission: oldest first; later ones may pass a request that waits
            # for memory (first fit) until it has waited aging_s, after which
            # admission stops at it (no starvation of large requests)
            for req in list(pending):
                fp = self.executor.footprint(req)
                if fp > self.hbm_budget:
                    pending.remove(req)
                    out[req.id].error = f"footprint {fp} exceeds the budget {self.hbm_budget}"
                    continue
                if len(active) >= max_jobs or used + fp > self.hbm_budget:
                    if realtime and t - req.arrival >= self.aging_s:
                        break
                    continue
                try:
                    handle, n_units, unit_cost = self.executor.create(req)
                except Exception as e:             # a bad request fails alone
                    pending.remove(req)
                    out[req.id].error = str(e)
                    continue
                pending.remove(req)
                used += fp
                peak = max(peak, used)
                active.append(_Active(req, handle, n_units, unit_cost, 0, fp))
                out[req.id].admitted = now()
            if not active:
                if nxt < len(reqs) and realtime:
                    self.sleep(max(0.0, reqs[nxt].arrival - now()))
                continue
            # one round: units from the oldest jobs first, within the work
            # budget; each job contributes one contiguous run of its units
            runs = []
            count = 0
            work = 0.0
            completing = []
            for a in active:
                if count >= self.max_units or (work >= self.round_work and count):
                    break
                room = self.max_units - count
                by_work = max(1, int((self.round_work - work) // max(a.unit_cost, 1.0)))
                take = min(a.n_units - a.next_unit, room, by_work)
                if take <= 0:
                    continue
                runs.append((a.handle, a.next_unit, take))
                count += take
                a.next_unit += take
                work += take * a.unit_cost
                if a.next_unit == a.n_units:
                    completing.append(a)
            if runs:
                pairs = np.empty((count, 2), dtype=np.int64)
                at = 0
                for h, first, take in runs:
                    pairs[at:at + take, 0] = h
                    pairs[at:at + take, 1] = np.arange(first, first + take, dtype=np.int64)
                    at += take
                self.executor.run_round(pairs)
                rounds += 1
                self.log.append((now(), count, len(runs)))
            for a in completing:
                res, sw, rech = self.executor.finish(a.handle, self.keep_sW)
                o = out[a.req.id]
                o.result, o.sW_all, o.rechecked = res, sw, rech
                o.finished = now()
                self.executor.release(a.handle)
                active.remove(a)
                used -= a.footprint
        return {"outcomes": out, "rounds": rounds, "peak_bytes": peak,
                "makespan": now(), "stats": stats(list(out.values()), reqs)}


def nearest_rank(values: list[float], q: float) -> float:
    """Quantile by the nearest-rank method: the ceil(q * N)-th smallest value."""
    v = sorted(values)
    if not v:
        return math.nan
    return v[max(0, math.ceil(q * len(v)) - 1)]


def stats(outcomes: list[Outcome], reqs: list[Request]) -> dict:
    ok = [o for o in outcomes if o.error is None and o.result is not None]
    lat = [o.latency for o in ok]
    by_id = {r.id: r for r in reqs}
    if not ok:
        return {"completed": 0}
    start = min(o.arrival for o in ok)
    end = max(o.finished for o in ok)
    pp = sum(by_id[o.id].pair_perms for o in ok)
    return {
        "completed": len(ok),
        "failed": len(outcomes) - len(ok),
        "p50_s": nearest_rank(lat, 0.50),
        "p99_s": nearest_rank(lat, 0.99),
        "max_s": max(lat),
        "mean_s": sum(lat) / len(lat),
        "makespan_s": end - start,
        "G_pair_perms_per_s": pp / (end - start) / 1e9 if end > start else math.nan,
        "requests_per_s": len(ok) / (end - start) if end > start else math.nan,
    }
