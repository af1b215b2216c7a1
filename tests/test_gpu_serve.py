"""Serving on the GPU: continuous batching of several permutation tests whose
work shares launches; every result must be bit-identical alone and in the mix,
equal to the whole-test call on the same form, and match the FP64 oracle.  Jobs
run on the plain FP32 form, the split-BF16 MFMA form, or a mix of both (auto:
the small test takes the plain form, so rounds launch both work-list kernels)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import load_pstat, max_rel

pytestmark = pytest.mark.gpu


def requests(device_gen=True):
    from paper_2505_04556_amd.serve import Request
    import synth.device as sd
    specs = [(600, [100, 200, 300], 199), (1000, [500, 500], 511), (1500, [300, 500, 700], 299),
             (800, [100, 150, 250, 300], 399), (1200, [600, 600], 255), (700, [350, 350], 1023),
             (400, [150, 250], 255)]
    reqs = []
    for i, (n, sizes, P) in enumerate(specs):
        base = synth.base_labels(sizes)
        reqs.append(Request(id=i, n=n, k=len(sizes), grouping=base, n_perms=P, seed=7000 + i,
                            arrival=0.0,
                            make_matrix=(lambda dev, n=n, s=6000 + i: sd.uniform_matrix(n, s, dev))))
    return reqs


@pytest.fixture(scope="module")
def ps(dev):
    return load_pstat()


def serve(reqs, budget=8 << 30, round_work=1e8, path="plain_f32"):
    from paper_2505_04556_amd.serve import GpuExecutor, Server
    ex = GpuExecutor(max_jobs=16, max_units=4096, path=path)
    try:
        srv = Server(ex, hbm_budget=budget, keep_sW=True, round_work=round_work, max_units=4096)
        return srv.run(reqs), srv
    finally:
        ex.close()


@pytest.mark.parametrize("path", ["plain_f32", "mfma_split_bf16", "auto"])
def test_mix_equals_alone_and_oracle(ps, path):
    import torch
    reqs = requests()
    # small rounds, so every job spans several (MFMA units are larger)
    rw = 1e8 if path == "plain_f32" else 4e6
    mixed, srv = serve(reqs, path=path, round_work=rw)
    assert mixed["stats"]["completed"] == len(reqs)
    # rounds carried work of several jobs
    assert max(jobs for _, _, jobs in srv.log) >= 2
    assert srv.log and len(srv.log) > len(reqs)
    for r in reqs:
        alone, _ = serve([r], path=path, round_work=rw)
        a = alone["outcomes"][r.id]
        m = mixed["outcomes"][r.id]
        assert a.result == m.result, r.id
        assert np.array_equal(a.sW_all, m.sW_all), r.id
        # same numbers as the whole-test entry point on the same form
        form = ps.resolve_path(path, r.n, r.k)
        ps.pstat_set_path(form)
        D = r.make_matrix(torch.device("cuda"))
        sw = torch.empty(r.n_perms + 1, dtype=torch.float64, device="cuda")
        res, _ = ps.pstat_permanova(D, torch.from_numpy(r.grouping).cuda(), r.k, r.n_perms,
                                    r.seed, sW_all=sw)
        assert np.array_equal(sw.cpu().numpy(), m.sW_all), r.id
        assert list(res.cpu().numpy()) == m.result, r.id
        # and the FP64 oracle
        ref = oracle.permanova(D.cpu().numpy(), r.grouping, r.n_perms, r.seed)
        assert max_rel(m.sW_all[1:], ref["sW_perm"]) <= 1e-5
        assert abs(m.result[0] - ref["F_obs"]) <= 1e-5 * abs(ref["F_obs"])
        assert m.result[1] == ref["p"]
    ps.pstat_set_path(ps.PSTAT_PATH_AUTO)


def test_admission_under_a_small_budget(ps):
    reqs = requests()
    from paper_2505_04556_amd.serve import GpuExecutor
    ex = GpuExecutor(max_jobs=4, max_units=512)
    try:
        fps = [ex.footprint(r) for r in reqs]
    finally:
        ex.close()
    budget = int(max(fps) * 1.5)            # at most one or two tests resident
    res, _ = serve(reqs, budget=budget)
    assert res["stats"]["completed"] == len(reqs)
    assert res["peak_bytes"] <= budget


def test_executor_warmup_leaves_nothing_behind(ps):
    from paper_2505_04556_amd.serve import GpuExecutor
    ex = GpuExecutor(max_jobs=4, max_units=512)
    try:
        ex.warmup(reserve_bytes=1 << 28)
        assert not ex.live
        # the server still serves afterwards
        res, _ = serve(requests()[:3])
        assert res["stats"]["completed"] == 3
    finally:
        ex.close()


@pytest.mark.parametrize("path", ["plain_f32", "mfma_split_bf16"])
def test_jobs_count_ties_like_the_oracle(ps, path):
    # two equal groups at n = 12 (seed 12 reaches the observed partition
    # under swapped labels) and a constant matrix with inexact weights:
    # a served job's p equals the oracle's, ties counted at the tolerance
    import torch
    from paper_2505_04556_amd.serve import Request
    const = np.full((300, 300), 0.3, dtype=np.float32)
    np.fill_diagonal(const, 0.0)
    cases = [(synth.uniform_matrix(12, 52), [6, 6], 999, 12),
             (synth.uniform_matrix(20, 60), [10, 10], 999, 12),
             (const, [60, 100, 140], 299, 5)]
    reqs = [Request(id=i, n=D.shape[0], k=len(sizes), grouping=synth.base_labels(sizes),
                    n_perms=P, seed=seed, arrival=0.0,
                    make_matrix=(lambda dev, D=D: torch.from_numpy(D).to(dev)))
            for i, (D, sizes, P, seed) in enumerate(cases)]
    res, _ = serve(reqs, path=path, round_work=4e6)
    for r, (D, sizes, P, seed) in zip(reqs, cases):
        o = res["outcomes"][r.id]
        assert o.error is None, o.error
        ref = oracle.permanova(D, synth.base_labels(sizes), P, seed)
        assert o.result[1] == ref["p"], (r.id, o.result[1], ref["p"])
        assert max_rel(o.sW_all[1:], ref["sW_perm"]) <= 1e-5


@pytest.mark.slow
def test_serving_trace_matches_oracle_on_a_subset(ps):
    """The 64-request serving trace (n in 1k..20k, k in 2..12, 999 or 9,999
    permutations), served with all arrivals at once under an 8 GB budget on the
    library's own choice of form.  Every request must complete, and each one's
    s_W (all permutations) and result must equal pstat_permanova's on the
    same form bit for bit; every request with n <= 2,000 (the ones the FP64
    oracle finishes in about a second) is also checked against the oracle:
    s_W of every permutation within 1e-5, F_obs within 1e-5, p identical."""
    import synth.device as sd
    from paper_2505_04556_amd.serve import GpuExecutor, Request, Server
    specs = synth.serving_requests(64, 4.0, 4000)
    reqs = [Request(id=t["id"], n=t["n"], k=t["k"], grouping=synth.base_labels(t["sizes"]),
                    n_perms=t["n_perms"], seed=t["perm_seed"], arrival=t["arrival"],
                    make_matrix=(lambda dev, n=t["n"], s=t["matrix_seed"]:
                                 sd.uniform_matrix(n, s, dev)))
            for t in specs]
    ex = GpuExecutor(max_jobs=32, max_units=8192, path="auto")
    try:
        srv = Server(ex, hbm_budget=8 << 30, keep_sW=True, round_work=1.5e11, max_units=8192)
        res = srv.run(reqs, realtime=False)
    finally:
        ex.close()
    errors = {i: o.error for i, o in res["outcomes"].items() if o.error}
    assert not errors, errors
    assert res["stats"]["completed"] == 64
    import torch
    for r in reqs:
        o = res["outcomes"][r.id]
        ps.pstat_set_path(ps.resolve_path("auto", r.n, r.k))
        D = r.make_matrix(torch.device("cuda"))
        sw = torch.empty(r.n_perms + 1, dtype=torch.float64, device="cuda")
        whole, _ = ps.pstat_permanova(D, torch.from_numpy(r.grouping).cuda(), r.k, r.n_perms,
                                      r.seed, sW_all=sw)
        assert np.array_equal(sw.cpu().numpy(), o.sW_all), r.id
        assert list(whole.cpu().numpy()) == o.result, r.id
        del D, sw
    ps.pstat_set_path(ps.PSTAT_PATH_AUTO)
    checked = 0
    for t in specs:
        if t["n"] > 2000:
            continue
        o = res["outcomes"][t["id"]]
        ref = oracle.permanova(synth.uniform_matrix(t["n"], t["matrix_seed"]),
                               synth.base_labels(t["sizes"]), t["n_perms"], t["perm_seed"])
        assert max_rel(o.sW_all[1:], ref["sW_perm"]) <= 1e-5, t["id"]
        assert abs(o.result[0] - ref["F_obs"]) <= 1e-5 * abs(ref["F_obs"]), t["id"]
        assert o.result[1] == ref["p"], t["id"]
        checked += 1
    assert checked >= 16


@pytest.mark.parametrize("path", ["plain_f32", "mfma_split_bf16"])
def test_packed_matrix_jobs_equal_square(ps, path):
    # the same requests with D given as its packed strict upper triangle
    import torch
    from paper_2505_04556_amd.serve import Request

    def pack(D):
        iu = torch.triu_indices(D.shape[0], D.shape[0], 1, device=D.device)
        return D[iu[0], iu[1]].contiguous()

    reqs = requests()[:4]
    square, _ = serve(reqs, path=path, round_work=4e6)
    preqs = [Request(id=r.id, n=r.n, k=r.k, grouping=r.grouping, n_perms=r.n_perms, seed=r.seed,
                     arrival=0.0, packed=True,
                     make_matrix=(lambda dev, r=r: pack(r.make_matrix(dev))))
             for r in reqs]
    packed, _ = serve(preqs, path=path, round_work=4e6)
    for r in reqs:
        a, b = square["outcomes"][r.id], packed["outcomes"][r.id]
        assert a.result == b.result, r.id
        assert np.array_equal(a.sW_all, b.sW_all), r.id
