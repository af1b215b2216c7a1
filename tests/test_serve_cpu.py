"""Scheduler logic of the serving loop on the CPU, with a stand-in executor
that keeps a virtual clock (work / rate) instead of touching a GPU."""
import math

import numpy as np
import pytest

from paper_2505_04556_amd.serve import Executor, Request, Server, nearest_rank


class FakeExecutor(Executor):
    """Footprint 4 n^2 + 16 n P bytes; units of 256 permutations x 8 tile chunks."""

    def __init__(self, clock, rate=1e12, fail_ids=()):
        self.clock = clock
        self.rate = rate
        self.fail_ids = set(fail_ids)
        self.units_run = {}
        self.jobs = {}
        self.live_bytes = 0
        self.peak_live = 0
        self.order = []
        self.finished_before_all_units = []

    def footprint(self, req):
        return 4 * req.n * req.n + 16 * req.n * (req.n_perms + 1)

    def create(self, req):
        if req.id in self.fail_ids:
            raise ValueError("bad request")
        units = 8 * math.ceil((req.n_perms + 1) / 256)
        h = len(self.jobs)
        self.jobs[h] = (req, units)
        self.units_run[h] = []
        self.live_bytes += self.footprint(req)
        self.peak_live = max(self.peak_live, self.live_bytes)
        self.order.append(req.id)
        cost = req.n * (req.n - 1) / 2 * (req.n_perms + 1) / units
        return h, units, cost

    def run_round(self, pairs):
        work = 0.0
        for h, u in pairs:
            self.units_run[int(h)].append(int(u))
            req, units = self.jobs[int(h)]
            work += req.n * (req.n - 1) / 2 * (req.n_perms + 1) / units
        self.clock.t += work / self.rate

    def finish(self, h, keep_sW=False):
        req, units = self.jobs[h]
        if sorted(self.units_run[h]) != list(range(units)):
            self.finished_before_all_units.append(h)
        self.clock.t += 1e-4
        return [float(req.id), 0.5, 1.0, 2.0], None, 0

    def release(self, h):
        req, _ = self.jobs[h]
        self.live_bytes -= self.footprint(req)


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


def trace(count=30, seed=0):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(0.05, size=count))
    reqs = []
    for i in range(count):
        n = int(rng.choice([500, 1000, 2000]))
        k = int(rng.integers(2, 6))
        g = np.repeat(np.arange(k, dtype=np.int32), n // k + 1)[:n]
        reqs.append(Request(id=i, n=n, k=k, grouping=g, n_perms=int(rng.choice([99, 999])),
                            seed=i, arrival=float(t[i])))
    return reqs


def run(reqs, budget, **kw):
    clock = Clock()
    ex = FakeExecutor(clock, **{k: v for k, v in kw.items() if k in ("rate", "fail_ids")})
    srv = Server(ex, hbm_budget=budget, clock=clock, sleep=clock.sleep, round_work=2e9,
                 **{k: v for k, v in kw.items() if k in ("max_jobs", "max_units", "aging_s")})
    return srv.run(reqs), ex


def test_every_unit_runs_once_before_finish():
    res, ex = run(trace(), budget=1 << 40)
    assert res["stats"]["completed"] == 30
    assert not ex.finished_before_all_units
    for h, (req, units) in ex.jobs.items():
        assert sorted(ex.units_run[h]) == list(range(units))


def test_admission_respects_the_budget():
    reqs = trace(40, seed=1)
    ex0 = FakeExecutor(Clock())
    biggest = max(ex0.footprint(r) for r in reqs)
    budget = int(biggest * 2.5)
    res, ex = run(reqs, budget)
    assert res["stats"]["completed"] == 40
    assert ex.peak_live <= budget
    assert res["peak_bytes"] <= budget


def test_fifo_when_memory_is_plentiful():
    reqs = trace(25, seed=2)
    res, ex = run(reqs, budget=1 << 40)
    assert ex.order == [r.id for r in sorted(reqs, key=lambda r: r.arrival)]


def test_requests_overlap_on_the_device():
    # arrivals faster than service: several jobs share rounds
    reqs = trace(20, seed=3)
    for r in reqs:
        r.arrival *= 0.01
    clock = Clock()
    ex = FakeExecutor(clock, rate=1e11)
    srv = Server(ex, hbm_budget=1 << 40, clock=clock, sleep=clock.sleep, round_work=5e10)
    srv.run(reqs)
    assert max(jobs for _, _, jobs in srv.log) >= 3


def test_oversized_and_failing_requests_fail_alone():
    reqs = trace(12, seed=4)
    reqs[3].n = 200_000                     # 160 GB matrix: never fits
    res, ex = run(reqs, budget=64 << 30, fail_ids={7})
    outs = res["outcomes"]
    assert outs[3].error and "budget" in outs[3].error
    assert outs[7].error == "bad request"
    done = [o for o in outs.values() if o.error is None]
    assert len(done) == 10 and all(o.result is not None for o in done)


def test_latency_accounting():
    res, ex = run(trace(10, seed=5), budget=1 << 40)
    for o in res["outcomes"].values():
        assert o.finished >= o.admitted >= o.arrival
    st = res["stats"]
    assert st["p50_s"] <= st["p99_s"] <= st["max_s"]


def test_nearest_rank_quantiles():
    v = list(range(1, 65))                  # 64 samples
    assert nearest_rank(v, 0.5) == 32
    assert nearest_rank(v, 0.99) == 64      # ceil(0.99 * 64) = 64: p99 is the maximum
    assert nearest_rank([5.0], 0.99) == 5.0
    assert math.isnan(nearest_rank([], 0.5))


def test_autotune_keys_and_cache(tmp_path):
    from paper_2505_04556_amd import autotune
    assert autotune.bucket(1) == 1 and autotune.bucket(1000) == 1024 and autotune.bucket(1024) == 1024
    k1 = autotune.shape_key(10_000, 5, 9_999)
    assert k1 == autotune.shape_key(9_000, 5, 9_000)       # same buckets
    assert k1 != autotune.shape_key(10_000, 6, 9_999)
    f = str(tmp_path / "c.json")
    autotune.save_cache({"a": {"x": 1}}, f)
    assert autotune.load_cache(f) == {"a": {"x": 1}}
    assert autotune.load_cache(str(tmp_path / "missing.json")) == {}


def test_aging_stops_small_requests_from_starving_a_large_one():
    # Small requests, each running 0.3 s and arriving every 0.2 s, overlap in
    # pairs; a large one (arriving at 0.5 s) fits only when no small job is
    # resident.  If later requests could always pass it, a new small job would
    # be admitted before the previous one ends and the large one would wait
    # for the whole stream.  Once it has waited aging_s, admission stops at
    # it, the resident small jobs drain and it runs.
    def reqs():
        out = [Request(id=i, n=1000, k=2, grouping=np.zeros(1000, np.int32), n_perms=5999,
                       seed=i, arrival=0.2 * i) for i in range(40)]
        out.append(Request(id=40, n=5000, k=3, grouping=np.zeros(5000, np.int32), n_perms=999,
                           seed=40, arrival=0.5))
        return out
    ex0 = FakeExecutor(Clock())
    small, large = ex0.footprint(reqs()[0]), ex0.footprint(reqs()[40])
    budget = large + int(0.9 * small)          # two small jobs fit, large only alone
    assert 2 * small <= budget < large + small
    res_no, _ = run(reqs(), budget, rate=1e10, aging_s=1e9)
    res_ag, _ = run(reqs(), budget, rate=1e10, aging_s=0.5)
    for res in (res_no, res_ag):
        assert res["stats"]["completed"] == 41
    last_small = max(res_no["outcomes"][i].admitted for i in range(40))
    assert res_no["outcomes"][40].admitted >= last_small       # starved behind the stream
    # aged at 1.0 s; the two resident small jobs end within 0.6 s
    assert res_ag["outcomes"][40].admitted <= 0.5 + 0.5 + 0.6 + 0.05


def test_admission_respects_the_executors_job_slots():
    # all requests at once; the executor has 5 job slots, the server allows more
    reqs = trace(30, seed=6)
    clock = Clock()
    ex = FakeExecutor(clock)
    ex.max_jobs = 5
    live = []
    orig = ex.create

    def create(req):
        live.append(req.id)
        assert len(live) - len(done) <= 5, "more resident jobs than slots"
        return orig(req)
    done = []
    orig_release = ex.release

    def release(h):
        done.append(h)
        orig_release(h)
    ex.create, ex.release = create, release
    srv = Server(ex, hbm_budget=1 << 40, clock=clock, sleep=clock.sleep, round_work=2e9,
                 max_jobs=64)
    res = srv.run(reqs, realtime=False)
    assert res["stats"]["completed"] == 30
