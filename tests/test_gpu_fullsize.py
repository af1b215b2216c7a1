"""Parity at the full workloads, in the launch configuration bench.py times
(pstat_permanova with the default tuning):

* n = 10,000 (Euclidean, k = 5, 9,999 permutations): every s_W against the
  FP64 oracle, F_obs, and the p-value (identical); every s_W also against the
  Euclidean closed form computed from the points.
* n = 25,000 (Euclidean, k = 10 uneven groups, 3,999 permutations): every
  computation form against the oracle on all permutations -- the per-dtype
  precision table -- and p identical for the forms that meet 1e-5.
* n = 100,000 (40 GB matrix, k = 3, 999 permutations): 64-bit offsets; sampled
  permutations against the oracle fed by row blocks copied from the device,
  F_obs against the oracle, and the p-value consistent with the returned s_W;
  the same varied matrix in the packed layout gives the same bits.
* n = 229,376 in the packed layout (only the strict upper triangle): a size
  whose square layout would not fit beside the MFMA tiles; closed form.
* n = 1,000 with 199,999 permutations: every s_W and the p-value against the
  oracle on both forms.
"""
import json
import os
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, load_pstat, max_rel

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def ps(dev):
    return load_pstat()


def record(name, payload):
    # the tables also go to $PSTAT_RESULTS_DIR when it names a directory
    d = os.environ.get("PSTAT_RESULTS_DIR", "")
    if d and os.path.isdir(d):
        with open(os.path.join(d, f"fullsize_{name}.json"), "w") as f:
            json.dump(payload, f, indent=1)
    print(name, json.dumps(payload), flush=True)


def whole_test(ps, D, cfg, path):
    import torch
    ps.pstat_set_path(path)
    base = torch.from_numpy(synth.base_labels(cfg["sizes"])).cuda()
    P = cfg["n_perms"]
    sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    res, rech = ps.pstat_permanova(D, base, cfg["k"], P, cfg["perm_seed"], sW_all=sw)
    torch.cuda.synchronize()
    return res.cpu().numpy(), sw.cpu().numpy(), rech


def huygens(points, labels, scale):
    """Closed form of s_W for Euclidean distances: sum over groups of the
    squared deviations from the group mean, for every row of labels."""
    x = points
    sq = (x * x).sum(1)
    out = np.zeros(labels.shape[0])
    for g in range(int(labels.max()) + 1):
        M = (labels == g).astype(np.float64)
        ng = M.sum(1)
        sx = M @ x
        out += (M @ sq) - (sx * sx).sum(1) / ng
    return out / (scale * scale)


def test_n10000_all_permutations(ps):
    import synth.device as sd
    cfg = synth.config(1)
    D = sd.matrix(cfg)
    Dh = D.cpu().numpy()
    base = synth.base_labels(cfg["sizes"])
    t0 = time.perf_counter()
    ref = oracle.permanova(Dh, base, cfg["n_perms"], cfg["perm_seed"])
    t_oracle = time.perf_counter() - t0
    import torch
    x = synth.euclid_points(cfg["n"], cfg["matrix_seed"])
    assert float(np.max(Dh)) == 1.0   # entries are d / dmax
    # dmax of the points (the generator's scale), for the closed form; on the
    # host (torch's device cdist returned a wrong maximum at this size)
    xt = torch.from_numpy(x)
    scale = float(torch.cdist(xt, xt, compute_mode="donot_use_mm_for_euclid_dist").max())
    del xt
    closed = huygens(x, np.vstack([base, ref["perms"]]), scale)
    assert max_rel(np.concatenate([[ref["sW_obs"]], ref["sW_perm"]]), closed) < 2e-7
    rows = {}
    g = torch.from_numpy(np.vstack([base, ref["perms"]])).cuda()
    w = torch.from_numpy(synth.inv_group_sizes(cfg["sizes"])).cuda()
    oracle_all = np.concatenate([[ref["sW_obs"]], ref["sW_perm"]])
    for path in ("plain_f32", "mfma_split_bf16", "mfma_f16", "mfma_bf16"):
        res, sw, rech = whole_test(ps, D, cfg, path)
        e_sw = max_rel(sw[1:], ref["sW_perm"])
        e_F = abs(res[0] - ref["F_obs"]) / abs(ref["F_obs"])
        # the form's own s_W before the FP64 recheck
        raw = ps.pstat_sW_k(D, g, cfg["k"], w).cpu().numpy()
        rows[path] = dict(max_rel_sW=e_sw, max_rel_sW_form_only=max_rel(raw, oracle_all),
                          rel_F_obs=e_F, p=res[1], p_oracle=ref["p"], rechecked=rech,
                          max_rel_vs_closed_form=max_rel(sw, closed))
        assert max_rel(raw, oracle_all) <= TOL[path], (path, rows[path])
        assert e_F <= 1e-5, (path, e_F)
        assert res[1] == ref["p"], (path, res[1], ref["p"])
        if path in ("plain_f32", "mfma_split_bf16"):
            assert e_sw <= 1e-5, (path, e_sw)
            assert max_rel(sw, closed) < 2e-7
    record("n10000", dict(oracle_seconds=t_oracle, forms=rows, F_obs=ref["F_obs"], p=ref["p"]))


def test_n25000_precision_table(ps):
    import synth.device as sd
    cfg = synth.config(2)
    D = sd.matrix(cfg)
    Dh = D.cpu().numpy()
    base = synth.base_labels(cfg["sizes"])
    t0 = time.perf_counter()
    ref = oracle.permanova(Dh, base, cfg["n_perms"], cfg["perm_seed"])
    t_oracle = time.perf_counter() - t0
    del Dh
    n, k = cfg["n"], cfg["k"]
    kappa = ref["sT"] / (ref["sT"] - ref["sW_obs"])
    table = {}
    for path in ("plain_f32", "mfma_split_bf16", "mfma_f16", "mfma_bf16"):
        res, sw, rech = whole_test(ps, D, cfg, path)
        # the form's own s_W before any FP64 recheck: pstat_sW_k on the same groupings
        import torch
        g = torch.from_numpy(np.vstack([base, ref["perms"]])).cuda()
        w = torch.from_numpy(synth.inv_group_sizes(cfg["sizes"])).cuda()
        raw = ps.pstat_sW_k(D, g, k, w).cpu().numpy()
        oracle_all = np.concatenate([[ref["sW_obs"]], ref["sW_perm"]])
        F_raw = oracle.F(raw[:1], ref["sT"], n, k)[0]
        table[path] = dict(max_rel_sW=max_rel(raw, oracle_all),
                           mean_rel_sW=float(np.mean(np.abs(raw - oracle_all) / oracle_all)),
                           rel_F_obs_form_only=abs(F_raw - ref["F_obs"]) / abs(ref["F_obs"]),
                           rel_F_obs_after_recheck=abs(res[0] - ref["F_obs"]) / abs(ref["F_obs"]),
                           p=res[1], p_identical=bool(res[1] == ref["p"]), rechecked=rech)
        assert max_rel(raw, oracle_all) <= TOL[path], (path, table[path])
        assert abs(res[0] - ref["F_obs"]) <= 1e-5 * abs(ref["F_obs"])
        assert res[1] == ref["p"], (path, res[1], ref["p"])
    record("n25000", dict(oracle_seconds=t_oracle, kappa_obs=kappa, F_obs=ref["F_obs"],
                          p=ref["p"], forms=table))


def test_n100000_sampled(ps):
    import torch

    import synth.device as sd
    cfg = synth.config(3)
    n, k, P = cfg["n"], cfg["k"], cfg["n_perms"]
    D = sd.uniform_matrix(n, cfg["matrix_seed"])          # 40 GB, 64-bit offsets
    base = synth.base_labels(cfg["sizes"])
    perms = oracle.permute(base, P, cfg["perm_seed"])
    sample = [0, 1, 2, 3, 250, 500, 750, P - 1]           # permutation indices
    rows = np.vstack([base, perms[sample]])
    w = synth.inv_group_sizes(cfg["sizes"])
    sums = oracle.new_group_sums(rows.shape[0], k)
    sq = np.zeros(2)
    block = 1000
    host = torch.empty((block, n), dtype=torch.float32, pin_memory=True)
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        host[: r1 - r0].copy_(D[r0:r1])
        blk = host[: r1 - r0].numpy()
        oracle.group_sums(blk, r0, n, rows, sums)
        oracle.sq_sum(blk, r0, n, sq)
    acc = oracle.sW_from_sums(sums, w)
    sT = sq.sum() / n
    F_obs = oracle.F(acc[:1], sT, n, k)[0]
    out = {}
    g = torch.from_numpy(rows).cuda()
    wd = torch.from_numpy(w).cuda()
    square = {}
    for path in ("mfma_split_bf16", "plain_f32", "mfma_f16", "mfma_bf16"):
        res, sw, rech = whole_test(ps, D, cfg, path)
        got = np.concatenate([sw[:1], sw[1:][sample]])
        raw = ps.pstat_sW_k(D, g, k, wd).cpu().numpy()   # the form alone, sampled rows
        square[path] = (res, sw, raw)
        out[path] = dict(max_rel_sW_sample=max_rel(got, acc),
                         max_rel_sW_form_only=max_rel(raw, acc),
                         rel_F_obs=abs(res[0] - F_obs) / abs(F_obs), rechecked=rech, p=res[1])
        assert max_rel(raw, acc) <= TOL[path], (path, out[path])
        if path in ("plain_f32", "mfma_split_bf16"):
            assert max_rel(got, acc) <= 1e-5, (path, out[path])
        assert abs(res[0] - F_obs) <= 1e-5 * abs(F_obs)
        assert abs(res[3] - sT) <= 1e-12 * sT
        # p is the count of the returned s_W at or below the observed one
        # (ties within the tolerance included)
        assert res[1] == oracle.pvalue(sw[0], sw[1:])
    # The same matrix given as its packed strict upper triangle (varied
    # values, element offsets past 2^32 in both layouts): every s_W, the
    # whole test's and the sampled rows' alone, equal to the square
    # layout's bit for bit -- and so within the tolerance of the row-block
    # oracle above.
    del D
    ps.pstat_free_workspace()
    torch.cuda.empty_cache()
    Dp = sd.uniform_packed(n, cfg["matrix_seed"])
    packed = {}
    for path in ("mfma_split_bf16", "plain_f32"):
        res, sw, _ = whole_test(ps, Dp, cfg, path)
        raw = ps.pstat_sW_k(Dp, g, k, wd).cpu().numpy()
        s_res, s_sw, s_raw = square[path]
        packed[path] = dict(whole_test_identical=bool(np.array_equal(sw, s_sw)),
                            sampled_rows_identical=bool(np.array_equal(raw, s_raw)),
                            result_identical=bool(np.array_equal(res, s_res)),
                            max_rel_sW_sample=max_rel(np.concatenate([sw[:1], sw[1:][sample]]),
                                                      acc))
        assert np.array_equal(sw, s_sw), path
        assert np.array_equal(raw, s_raw), path
        assert np.array_equal(res, s_res), path
        assert max_rel(raw, acc) <= TOL[path]
    ps.pstat_set_path("auto")
    del Dp
    ps.pstat_free_workspace()
    torch.cuda.empty_cache()
    record("n100000", dict(sample=sample, F_obs=F_obs, forms=out, packed_layout=packed))


def test_n229376_packed_closed_form(ps):
    """n = 229,376 in the packed layout: D (105 GB) and the split-BF16 tiles
    (105 GB) fit on the device together, where the square layout (210 GB) and
    its tiles would not.  Constant distances d = 1/2 make every s_W the closed
    form (1/8)(n - k) (each group contributes (n_g - 1) / 8); power-of-two
    group sizes make the weights exact, so every sum, the FP64 recheck's
    included, is exact: s_T = (1/8)(n - 1), F = 1 and p = 1."""
    import torch
    torch.cuda.empty_cache()
    ps.pstat_free_workspace()
    sizes, P, seed = [32_768, 65_536, 131_072], 99, 5
    n = sum(sizes)
    k = len(sizes)
    free, _ = torch.cuda.mem_get_info()
    need = 4 * n * n + (8 << 30)
    if free < need:
        pytest.skip(f"needs {need / 1e9:.0f} GB free, {free / 1e9:.0f} GB are")
    D = torch.full((n * (n - 1) // 2,), 0.5, dtype=torch.float32, device="cuda")
    base = torch.from_numpy(synth.base_labels(sizes)).cuda()
    sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    ps.pstat_set_path("mfma_split_bf16")
    try:
        t0 = time.time()
        res, rech = ps.pstat_permanova(D, base, k, P, seed, sW_all=sw)
        torch.cuda.synchronize()
        seconds = time.time() - t0
    finally:
        ps.pstat_set_path("auto")
        del D
        ps.pstat_free_workspace()
        torch.cuda.empty_cache()
    sw, res = sw.cpu().numpy(), res.cpu().numpy()
    record("n229376_packed", dict(seconds_first_call=seconds, rechecked=rech, result=list(res)))
    assert np.all(sw == 0.125 * (n - k))
    assert res[0] == 1.0 and res[1] == 1.0
    assert res[3] == 0.125 * (n - 1)


def test_many_permutations(ps):
    """n = 1,000 (k = 4, the 100/200/300/400 workload) with 199,999
    permutations -- the paper's range reaches 10^6 -- on both forms: every
    s_W against the oracle, p identical (hundreds of column blocks, label
    tables of 0.4 GB, several FP64 recheck passes)."""
    import torch
    cfg = synth.config(0)
    n, sizes, k = cfg["n"], cfg["sizes"], cfg["k"]
    P, seed = 199_999, 77
    D = synth.uniform_matrix(n, cfg["matrix_seed"])
    ref = oracle.permanova(D, synth.base_labels(sizes), P, seed)
    Dd = torch.from_numpy(D).cuda()
    base = torch.from_numpy(synth.base_labels(sizes)).cuda()
    out = {}
    for path in ("plain_f32", "mfma_split_bf16"):
        ps.pstat_set_path(path)
        sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
        t0 = time.perf_counter()
        res, rech = ps.pstat_permanova(Dd, base, k, P, seed, sW_all=sw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        r, s = res.cpu().numpy(), sw.cpu().numpy()
        err = max_rel(s[1:], ref["sW_perm"])
        out[path] = dict(p=float(r[1]), rechecked=rech, max_rel_err=err, seconds=round(dt, 4))
        assert err <= TOL[path], (path, err)
        assert s[0] == r[2]
        assert r[1] == ref["p"], (path, r[1], ref["p"])
    ps.pstat_set_path("auto")
    record("n1000_P199999", dict(oracle_p=ref["p"], forms=out))
