"""GPU parity: every computation form of the HIP library against the FP64 CPU
oracle on the same seeded inputs, through the C ABI (Python binding = argument
marshalling only).  Small and ragged sizes that span several tiles, plus the
degenerate cases; the full workloads are in test_gpu_fullsize.py."""
import ctypes

import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, load_pstat, max_rel, problem, to_dev

pytestmark = pytest.mark.gpu

ALL_PATHS = ["plain_f32", "plain_f64", "mfma_split_bf16", "mfma_split3_bf16", "mfma_f16", "mfma_bf16"]


@pytest.fixture(scope="module")
def ps(dev):
    return load_pstat()


def run_sW(ps, path, D, perms, w, validate=True, k=None, tuning=None):
    import torch
    ps.pstat_set_path(path)
    if tuning:
        ps.pstat_set_tuning(path, *tuning)
    Dd, gd, wd = to_dev(D, perms, w)
    out = (ps.pstat_sW(Dd, gd, wd) if validate else ps.pstat_sW_k(Dd, gd, k, wd))
    torch.cuda.synchronize()
    if tuning:
        ps.pstat_set_tuning(path, 0, 0)
    return out.cpu().numpy()


# --- input generators: device copy == host copy ----------------------------
def test_device_generators_match_host(ps):
    import synth.device as sd
    for n in (1, 2, 77, 300):
        a = sd.uniform_matrix(n, 1234).cpu().numpy()
        assert np.array_equal(a, synth.uniform_matrix(n, 1234))
    b = sd.euclid_matrix(150, 99).cpu().numpy()
    h = synth.euclid_matrix(150, 99)
    assert np.max(np.abs(b.astype(np.float64) - h)) <= 2.0 ** -24


# --- permutation generator: bit-exact with the oracle's ---------------------
@pytest.mark.parametrize("n,maxlab,P,seed", [
    (16, 2, 4, 3000), (2, 1, 7, 1), (1000, 3, 999, 3000), (500, 300, 64, 77),
    (90_000, 299, 3, 5),          # u16 labels that do not fit in LDS: in-place path
    (20_000, 4, 130, 9),          # u8 labels, several permutations per work-group
    # batched shuffle with 16 and 64 lanes per permutation, labels packed four
    # bits to an entry (below 16) or one byte (below 256); each of these
    # inputs has draws that Lemire's method rejects (asserted below), so the
    # in-order replay of a batch is exercised
    (10_000, 4, 400, 13), (12_000, 4, 200, 13), (60_000, 6, 24, 13),
    (10_000, 40, 400, 13), (60_000, 100, 24, 13), (10_003, 15, 256, 13),
    # labels below 4 packed two bits to an entry: a whole wave per
    # permutation while every permutation fits on the device at once, 16
    # lanes each beyond that; nibbles and bytes with 16 lanes each
    (100_000, 2, 40, 13), (60_000, 3, 24, 13), (10_000, 3, 400, 13),
    (5_000, 3, 5_000, 13), (5_000, 9, 5_000, 13), (5_000, 100, 5_000, 13),
    # a whole wave per permutation over partners above 2^16, where partners
    # that agree in their low 16 bits also count as conflicting (a few
    # percent of batches)
    (216_000, 3, 300, 13), (216_000, 3, 520, 13),
    # more permutations than the device runs at once with 16 lanes each: the
    # last partial round with a whole wave per permutation (9,999), and a
    # rest too large for that, left with 16 lanes (13,192)
    (10_000, 5, 9_999, 13), (10_000, 5, 13_192, 13),
])
def test_permute_bit_exact(ps, n, maxlab, P, seed):
    import torch
    rng = np.random.default_rng(seed)
    base = np.sort(rng.integers(0, maxlab + 1, size=n)).astype(np.int32)
    base[-1] = maxlab
    got = ps.pstat_permute(torch.from_numpy(base).cuda(), P, seed).cpu().numpy()
    assert np.array_equal(got, oracle.permute(base, P, seed))
    if seed == 13:
        assert oracle.count_rejections(n, P, seed) > 0


def test_permute_golden_fixture(ps):
    import os
    import torch
    path = os.path.join(os.path.dirname(__file__), "golden", "permute_n16_P4_seed3000.txt")
    rows = [list(map(int, l.split())) for l in open(path) if l.strip() and not l.startswith("#")]
    got = ps.pstat_permute(torch.tensor(rows[0], dtype=torch.int32).cuda(), 4, 3000)
    assert got.cpu().numpy().tolist() == rows[1:]


# --- s_W: every path, ragged sizes ---------------------------------------
SHAPES = [(2, [2], 1), (3, [1, 2], 5), (33, [10, 23], 63), (65, [20, 20, 25], 65),
          (100, [10, 20, 30, 40], 300), (257, [57, 100, 100], 129), (1000, [100, 200, 300, 400], 999)]


@pytest.mark.parametrize("path", ALL_PATHS)
@pytest.mark.parametrize("n,sizes,P", SHAPES)
def test_sW_matches_oracle(ps, path, n, sizes, P):
    D, base, perms, w = problem(n, sizes, P, mseed=n, pseed=P)
    ref = oracle.sW(D, perms, w)
    got = run_sW(ps, path, D, perms, w)
    err = max_rel(got, ref)
    assert err <= TOL[path], f"{path} n={n} P={P}: max rel err {err:.3e}"


@pytest.mark.parametrize("tile,lanes", [(32, 64), (32, 128), (64, 64), (64, 128), (64, 256)])
def test_plain_tunings(ps, tile, lanes):
    D, base, perms, w = problem(300, [50, 100, 150], 200, mseed=4, pseed=5)
    ref = oracle.sW(D, perms, w)
    got = run_sW(ps, "plain_f32", D, perms, w, tuning=(tile, lanes))
    assert max_rel(got, ref) <= TOL["plain_f32"]


@pytest.mark.parametrize("path", ["mfma_split_bf16", "mfma_split3_bf16", "mfma_f16", "mfma_bf16"])
@pytest.mark.parametrize("kcols,ncols", [(64, 256), (128, 512), (512, 256), (0, 512)])
def test_mfma_tunings(ps, path, kcols, ncols):
    D, base, perms, w = problem(700, [100, 250, 350], 50, mseed=6, pseed=7)
    ref = oracle.sW(D, perms, w)
    got = run_sW(ps, path, D, perms, w, tuning=(kcols, ncols))
    assert max_rel(got, ref) <= TOL[path]


def test_many_groups(ps):
    # k = 40 groups: 10,240 columns of G for 256 permutations
    sizes = [5 + (g % 7) for g in range(40)]
    n = sum(sizes)
    D, base, perms, w = problem(n, sizes, 256, mseed=8, pseed=9)
    ref = oracle.sW(D, perms, w)
    for path in ALL_PATHS:
        assert max_rel(run_sW(ps, path, D, perms, w), ref) <= TOL[path], path


# --- exactness and degenerate cases ---------------------------------------
@pytest.mark.parametrize("path", ALL_PATHS)
def test_dyadic_inputs_bit_exact(ps, path):
    # d = m/16: d^2 exact in every input type; power-of-two group sizes make
    # every weight exact, so every path must reproduce the oracle bit for bit
    sizes = [16, 32, 64, 16]
    D, base, perms, w = problem(sum(sizes), sizes, 70, mseed=3, pseed=4, matrix="dyadic")
    ref = oracle.sW(D, perms, w)
    got = run_sW(ps, path, D, perms, w)
    assert np.array_equal(got, ref), f"{path}: max rel err {max_rel(got, ref):.3e}"


@pytest.mark.parametrize("kcols", [0, 128])
def test_split3_carries_24_bit_squares_exactly(ps, kcols):
    # Squares with 24 significant bits (odd m^2 / 2^24, m = 4095, 4093): BF16
    # hi + lo keeps 16 of them, hi + mid + lo all.  One non-zero pair per
    # (panel, K chunk) work item, so no FP32 sum ever adds two of them; group
    # sizes of 128 make the weights exact.  The three-part form must match
    # the oracle bit for bit, the two-part one cannot.
    n = 256
    D = np.zeros((n, n), dtype=np.float32)
    for i, j, m in ((3, 200, 4095), (150, 250, 4093)):
        D[i, j] = D[j, i] = np.float32(m / 4096)
    base = synth.base_labels([128, 128])
    perms = np.vstack([base, oracle.permute(base, 63, 21)])
    w = synth.inv_group_sizes([128, 128])
    ref = oracle.sW(D, perms, w)
    assert np.count_nonzero(ref) > 10
    got = run_sW(ps, "mfma_split3_bf16", D, perms, w, tuning=(kcols, 0))
    assert np.array_equal(got, ref), f"max rel err {max_rel(got, ref):.3e}"
    two = run_sW(ps, "mfma_split_bf16", D, perms, w)
    assert not np.array_equal(two, ref)
    assert max_rel(two, ref) <= 2.0 ** -16


@pytest.mark.parametrize("path", ALL_PATHS)
@pytest.mark.parametrize("scale", [1e3, 3e-4, 2.0 ** 50, 0.0])
def test_distance_range(ps, path, scale):
    # Squares far outside FP16's range: up to 1e6 (FP16 overflows past
    # 65,504), about 1e-9 (FP16 flushes below 6e-8), 2^100; the FP16 form
    # scales them by a power of two first.  An all-zero matrix gives zeros.
    D, base, perms, w = problem(300, [100, 200], 40, mseed=31, pseed=32)
    D = (D.astype(np.float64) * scale).astype(np.float32)
    ref = oracle.sW(D, perms, w)
    got = run_sW(ps, path, D, perms, w)
    if scale == 0.0:
        assert np.all(got == 0.0)
    else:
        assert max_rel(got, ref) <= TOL[path], f"{path} x{scale}: {max_rel(got, ref):.3e}"


@pytest.mark.parametrize("path", ALL_PATHS)
def test_all_singletons_exact_zero(ps, path):
    n = 64
    D = synth.uniform_matrix(n, 3)
    g = np.arange(n, dtype=np.int32)[None, :].repeat(3, 0)
    got = run_sW(ps, path, D, g, np.ones(n))
    assert np.all(got == 0.0)


@pytest.mark.parametrize("path", ALL_PATHS)
def test_single_group_is_frobenius(ps, path):
    n = 190
    D = synth.uniform_matrix(n, 12)
    g = np.zeros((2, n), dtype=np.int32)
    got = run_sW(ps, path, D, g, np.array([1.0 / n]))
    fro = np.linalg.norm(D.astype(np.float64)) ** 2 / (2 * n)
    assert max_rel(got, [fro, fro]) <= TOL[path]


@pytest.mark.parametrize("path", ALL_PATHS)
def test_only_strict_upper_triangle_is_read(ps, path):
    D, base, perms, w = problem(150, [50, 100], 20, mseed=2, pseed=3)
    E = D.copy()
    E[np.tril_indices(150)] = np.nan
    a = run_sW(ps, path, D, perms, w)
    b = run_sW(ps, path, E, perms, w)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("path", ALL_PATHS)
def test_constant_matrix_closed_form(ps, path):
    sizes = [8, 16, 32, 8]
    n, k = sum(sizes), 4
    D = np.full((n, n), 0.5, dtype=np.float32)
    np.fill_diagonal(D, 0)
    perms = oracle.permute(synth.base_labels(sizes), 10, 1)
    got = run_sW(ps, path, D, perms, synth.inv_group_sizes(sizes))
    assert np.all(got == 0.25 * (n - k) / 2)


def test_results_are_deterministic(ps):
    D, base, perms, w = problem(500, [100, 400], 300, mseed=5, pseed=6)
    for path in ALL_PATHS:
        a = run_sW(ps, path, D, perms, w)
        b = run_sW(ps, path, D, perms, w)
        assert np.array_equal(a, b), path


# --- boundary: error codes --------------------------------------------------
def test_bad_labels_rejected_and_out_untouched(ps):
    import torch
    D, base, perms, w = problem(40, [20, 20], 5)
    perms = perms.copy()
    perms[3, 7] = -1
    Dd, gd, wd = to_dev(D, perms, w)
    out = torch.full((5,), 7.0, dtype=torch.float64, device="cuda")
    ps.pstat_set_path("plain_f32")
    with pytest.raises(ps.PstatError) as e:
        ps.pstat_sW(Dd, gd, wd, out)
    assert e.value.code == ps.PSTAT_ELABEL
    assert torch.all(out == 7.0)
    perms[3, 7] = 70000
    with pytest.raises(ps.PstatError):
        ps.pstat_sW(Dd, to_dev(perms)[0], wd, out)


def test_async_label_check_marks_nan(ps):
    import torch
    D, base, perms, w = problem(40, [20, 20], 5)
    perms = perms.copy()
    perms[2, 0] = 2                       # >= n_groups
    for path in ("plain_f32", "mfma_split_bf16"):
        ps.pstat_set_path(path)
        Dd, gd, wd = to_dev(D, perms, w)
        out = ps.pstat_sW_k(Dd, gd, 2, wd).cpu().numpy()
        assert np.isnan(out[2]) and np.all(np.isfinite(np.delete(out, 2)))
        with pytest.raises(ps.PstatError) as e:
            ps.pstat_check_labels()
        assert e.value.code == ps.PSTAT_ELABEL
        ps.pstat_check_labels()            # the flag was cleared


def test_host_pointers_and_bad_sizes(ps):
    import torch
    ps.pstat_set_path("plain_f32")
    lib = ps._lib
    D, base, perms, w = problem(20, [10, 10], 2)
    out = np.zeros(2)
    rc = lib.pstat_sW(D.ctypes.data, 20, perms.ctypes.data, 2, w.ctypes.data, out.ctypes.data)
    assert rc == ps.PSTAT_EPTR
    Dd, gd, wd = to_dev(D, perms, w)
    od = torch.zeros(2, dtype=torch.float64, device="cuda")
    assert lib.pstat_sW(Dd.data_ptr(), 1, gd.data_ptr(), 2, wd.data_ptr(), od.data_ptr()) == ps.PSTAT_EINVAL
    assert lib.pstat_sW(Dd.data_ptr(), 20, gd.data_ptr(), -1, wd.data_ptr(), od.data_ptr()) == ps.PSTAT_EINVAL
    assert lib.pstat_sW(Dd.data_ptr(), 20, gd.data_ptr(), 0, wd.data_ptr(), od.data_ptr()) == ps.PSTAT_OK
    assert lib.pstat_set_path(17) == ps.PSTAT_EINVAL
    assert lib.pstat_set_tuning(0, 48, 0) == ps.PSTAT_EINVAL
    assert lib.pstat_F(od.data_ptr(), 2, od.data_ptr(), 20, 1, od.data_ptr()) == ps.PSTAT_EDOMAIN
    assert lib.pstat_F(od.data_ptr(), 2, od.data_ptr(), 20, 20, od.data_ptr()) == ps.PSTAT_EDOMAIN


def test_user_workspace(ps):
    import torch
    D, base, perms, w = problem(300, [100, 200], 100)
    ref = oracle.sW(D, perms, w)
    for path in ("plain_f32", "mfma_split_bf16"):
        ps.pstat_set_path(path)
        need = ps.pstat_workspace_bytes(300, 100, 2, path)
        assert need > 0
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        ps.pstat_set_workspace(ws)
        try:
            Dd, gd, wd = to_dev(D, perms, w)
            got = ps.pstat_sW_k(Dd, gd, 2, wd).cpu().numpy()
            assert max_rel(got, ref) <= TOL[path]
            ps.pstat_set_workspace(ws[: need // 4])
            with pytest.raises(ps.PstatError) as e:
                ps.pstat_sW_k(Dd, gd, 2, wd)
            assert e.value.code == ps.PSTAT_ENOMEM
        finally:
            ps.pstat_set_workspace(None)


def test_registered_matrix(ps):
    D, base, perms, w = problem(400, [150, 250], 64)
    Dd, gd, wd = to_dev(D, perms, w)
    for path in ("plain_f32", "mfma_split_bf16", "mfma_bf16"):
        ps.pstat_set_path(path)
        direct = ps.pstat_sW_k(Dd, gd, 2, wd).cpu().numpy()
        h = ps.pstat_matrix_register(Dd, path)
        try:
            a = ps.pstat_sW_registered(h, gd, 2, wd).cpu().numpy()
            b = ps.pstat_sW_registered(h, gd, 2, wd).cpu().numpy()
        finally:
            ps.pstat_matrix_release(h)
        assert np.array_equal(a, direct) and np.array_equal(b, direct)


# --- s_T, F, p-value and the whole test ---------------------------------------
def test_sT_F_pvalue_kernels(ps):
    import torch
    D, base, perms, w = problem(500, [100, 150, 250], 199)
    sW = oracle.sW(D, np.vstack([base, perms]), w)
    sT = oracle.sT(D)
    Dd, swd = to_dev(D, sW)
    sTd = ps.pstat_sT(Dd)
    assert max_rel(sTd.cpu().numpy(), [sT]) <= 1e-13
    # the F kernel on the oracle's s_T (F near 0 would amplify the last-bit
    # difference between the two s_T sums)
    Fd = ps.pstat_F(swd, to_dev(np.array([sT]))[0], 500, 3).cpu().numpy()
    Fo = oracle.F(sW, sT, 500, 3)
    assert np.max(np.abs(Fd - Fo) / np.maximum(np.abs(Fo), 1.0)) <= 1e-13
    p = ps.pstat_pvalue(swd[:1], swd[1:]).item()
    assert p == oracle.pvalue(sW[0], sW[1:])
    empty = torch.empty(0, dtype=torch.float64, device="cuda")
    assert np.isnan(ps.pstat_pvalue(swd[:1], empty).item())


def test_group_weights(ps):
    import torch
    g = np.array([0, 2, 2, 1, 2, 0, 4], dtype=np.int32)
    got = ps.pstat_group_weights(torch.from_numpy(g).cuda(), 5).cpu().numpy()
    assert np.array_equal(got, [0.5, 1.0, 1 / 3, 0.0, 1.0])


def test_precision_table_n1000(ps):
    """Per-form error against the FP64 oracle on the n=1000 uniform workload
    (k=4, 999 permutations): every s_W of every form before any recheck."""
    import json
    import torch
    cfg = synth.config(0)
    D = synth.host_matrix(cfg)
    base = synth.base_labels(cfg["sizes"])
    P, seed, k = cfg["n_perms"], cfg["perm_seed"], cfg["k"]
    perms = oracle.permute(base, P, seed)
    rows = np.vstack([base, perms])
    w = synth.inv_group_sizes(cfg["sizes"])
    ref = oracle.sW(D, rows, w)
    Dd, gd, wd = to_dev(D, rows, w)
    table = {}
    for path in ("plain_f64", "plain_f32", "mfma_split_bf16", "mfma_split3_bf16", "mfma_f16",
                 "mfma_bf16"):
        ps.pstat_set_path(path)
        got = ps.pstat_sW_k(Dd, gd, k, wd).cpu().numpy()
        table[path] = dict(max_rel_sW=max_rel(got, ref),
                           mean_rel_sW=float(np.mean(np.abs(got - ref) / ref)))
        assert max_rel(got, ref) <= TOL[path], (path, table[path])
    ps.pstat_set_path(ps.PSTAT_PATH_AUTO)
    out = os.environ.get("PSTAT_RESULTS_DIR", "")
    if out and os.path.isdir(out):
        with open(os.path.join(out, "precision_n1000.json"), "w") as f:
            json.dump(table, f, indent=1)
    print("n1000", json.dumps(table), flush=True)


@pytest.mark.parametrize("path", ["plain_f32", "mfma_split_bf16", "mfma_split3_bf16", "mfma_bf16"])
def test_permanova_matches_oracle(ps, path):
    import torch
    cfg = synth.config(0)
    D = synth.host_matrix(cfg)
    base = synth.base_labels(cfg["sizes"])
    P, seed = cfg["n_perms"], cfg["perm_seed"]
    ref = oracle.permanova(D, base, P, seed)
    ps.pstat_set_path(path)
    Dd, bd = to_dev(D, base)
    sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    res, rechecked = ps.pstat_permanova(Dd, bd, cfg["k"], P, seed, sW_all=sw)
    res = res.cpu().numpy()
    sw = sw.cpu().numpy()
    assert max_rel(sw[1:], ref["sW_perm"]) <= TOL[path]
    assert max_rel([res[0]], [ref["F_obs"]]) <= 1e-5
    assert res[1] == ref["p"], (res[1], ref["p"], rechecked)
    assert max_rel([res[3]], [ref["sT"]]) <= 1e-13


# Whole test on both forms with labels of every shuffle storage width (four
# bits below 16, one byte below 256, u16 above) and without permutations.
@pytest.mark.parametrize("path", ["plain_f32", "mfma_split_bf16"])
@pytest.mark.parametrize("n,k,P", [(700, 20, 300), (700, 300, 100), (600, 3, 0), (650, 16, 64)])
def test_permanova_label_widths(ps, path, n, k, P):
    import torch
    rng = np.random.default_rng(n + k)
    # uneven group sizes, every group non-empty
    base = np.concatenate([np.arange(k), rng.integers(0, k, size=n - k)]).astype(np.int32)
    rng.shuffle(base)
    D = synth.uniform_matrix(n, 11 + k)
    seed = 4242 + P
    ref = oracle.permanova(D, base, P, seed)
    ps.pstat_set_path(path)
    Dd, bd = to_dev(D, base)
    sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    res, rechecked = ps.pstat_permanova(Dd, bd, k, P, seed, sW_all=sw)
    ps.pstat_set_path("auto")
    res = res.cpu().numpy()
    sw = sw.cpu().numpy()
    if P:
        assert max_rel(sw[1:], ref["sW_perm"]) <= TOL[path]
        assert res[1] == ref["p"], (res[1], ref["p"], rechecked)
    else:
        assert np.isnan(res[1]) and np.isnan(ref["p"])   # no permutations: p undefined
    assert max_rel([res[0]], [ref["F_obs"]]) <= 1e-5
    assert max_rel([res[3]], [ref["sT"]]) <= 1e-13


# Whole test on the MFMA forms: the largest group gets no columns; its block
# is the matrix total minus the other groups' rows.  Largest group first, in
# the middle, last and tied; k from 2 to 16 (one or two columns per
# permutation take 256-column work-groups; the three-part split with k = 2
# keeps all columns).  The fast values (rows past the 8 FP64 samples) meet
# the form's tolerance and agree with the same rows through pstat_sW, which
# always uses every column.
MFMA_PATHS = ["mfma_split_bf16", "mfma_split3_bf16", "mfma_f16", "mfma_bf16"]


@pytest.mark.parametrize("path", MFMA_PATHS)
@pytest.mark.parametrize("sizes", [[400, 100], [100, 400], [60, 300, 120], [120, 120, 60],
                                   [50, 70, 300, 90, 40], [30] * 16])
def test_permanova_complement_form(ps, path, sizes):
    import torch
    n, k, P = sum(sizes), len(sizes), 200
    D = synth.uniform_matrix(n, 900 + n)
    base = synth.base_labels(sizes)
    seed = 31 + k
    ref = oracle.permanova(D, base, P, seed)
    ps.pstat_set_path(path)
    Dd, bd = to_dev(D, base)
    sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    res, rechecked = ps.pstat_permanova(Dd, bd, k, P, seed, sW_all=sw)
    rows = np.vstack([base, oracle.permute(base, P, seed)])
    full = ps.pstat_sW_k(Dd, to_dev(rows)[0], k, to_dev(synth.inv_group_sizes(sizes))[0])
    ps.pstat_set_path("auto")
    sw, full, res = sw.cpu().numpy(), full.cpu().numpy(), res.cpu().numpy()
    assert max_rel(sw[1:], ref["sW_perm"]) <= TOL[path]
    assert max_rel(sw[8:], full[8:]) <= 2 * TOL[path]
    assert res[1] == ref["p"], (res[1], ref["p"], rechecked)
    assert max_rel([res[0]], [ref["F_obs"]]) <= 1e-5


# Dyadic inputs and power-of-two group sizes keep every sum exact, the
# complement's subtraction included: the whole test's s_W equal the oracle's
# bit for bit on every MFMA form.
@pytest.mark.parametrize("path", MFMA_PATHS)
def test_permanova_complement_dyadic_bit_exact(ps, path):
    import torch
    sizes = [16, 64, 32, 16]
    n, k, P, seed = sum(sizes), len(sizes), 90, 8
    D = synth.dyadic_matrix(n, 5)
    base = synth.base_labels(sizes)
    rows = np.vstack([base, oracle.permute(base, P, seed)])
    ref = oracle.sW(D, rows, synth.inv_group_sizes(sizes))
    ps.pstat_set_path(path)
    Dd, bd = to_dev(D, base)
    sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    ps.pstat_permanova(Dd, bd, k, P, seed, sW_all=sw)
    ps.pstat_set_path("auto")
    sw = sw.cpu().numpy()
    assert np.array_equal(sw, ref), f"max rel err {max_rel(sw, ref):.3e}"


# The observed grouping and the first 7 permutations are recomputed in FP64
# (inside the pre-pass on the MFMA forms, by the recheck kernel on the plain
# ones) and written back into sW_all: those entries match the oracle to FP64
# rounding, not just to the form's tolerance.
@pytest.mark.parametrize("path", ["plain_f32", "mfma_split_bf16", "mfma_bf16"])
@pytest.mark.parametrize("n,sizes,P", [(1000, [100, 200, 300, 400], 999), (700, [300, 400], 9),
                                       (2100, [500, 600, 1000], 40)])
def test_fp64_samples_exact(ps, path, n, sizes, P):
    import torch
    D = synth.uniform_matrix(n, 77 + n)
    base = synth.base_labels(sizes)
    seed = 515 + P
    ref = oracle.permanova(D, base, P, seed)
    ps.pstat_set_path(path)
    Dd, bd = to_dev(D, base)
    sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    ps.pstat_permanova(Dd, bd, len(sizes), P, seed, sW_all=sw)
    ps.pstat_set_path("auto")
    sw = sw.cpu().numpy()
    S = min(P, 7) + 1
    exact = np.concatenate([[ref["sW_obs"]], ref["sW_perm"][:S - 1]])
    assert max_rel(sw[:S], exact) <= 1e-12


# An empty group among the n_groups labels: it gets weight 0 and F counts only
# the non-empty groups, as the oracle does.
@pytest.mark.parametrize("path", ["plain_f32", "mfma_split_bf16"])
def test_permanova_with_an_empty_group(ps, path):
    import torch
    n, P, seed = 800, 199, 31
    base = synth.base_labels([200, 0, 250, 350])      # label 1 unused
    D = synth.uniform_matrix(n, 808)
    ref = oracle.permanova(D, base, P, seed)
    assert ref["k"] == 3
    ps.pstat_set_path(path)
    Dd, bd = to_dev(D, base)
    sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    res, _ = ps.pstat_permanova(Dd, bd, 4, P, seed, sW_all=sw)
    ps.pstat_set_path("auto")
    res = res.cpu().numpy()
    assert max_rel(sw.cpu().numpy()[1:], ref["sW_perm"]) <= TOL[path]
    assert max_rel([res[0]], [ref["F_obs"]]) <= 1e-5
    assert res[1] == ref["p"]


# Tiny and ragged whole tests on every form (n around one 128-row panel and
# one 64-column block, n not a multiple of 4, fewer permutations than the 15
# samples).
@pytest.mark.parametrize("path", ALL_PATHS)
@pytest.mark.parametrize("n,sizes,P", [(3, [1, 2], 5), (5, [2, 3], 40), (66, [30, 36], 17),
                                       (131, [40, 41, 50], 63), (257, [100, 157], 8)])
def test_permanova_tiny_and_ragged(ps, path, n, sizes, P):
    import torch
    D = synth.uniform_matrix(n, 900 + n)
    base = synth.base_labels(sizes)
    seed = 77 + n
    ref = oracle.permanova(D, base, P, seed)
    ps.pstat_set_path(path)
    Dd, bd = to_dev(D, base)
    sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    res, _ = ps.pstat_permanova(Dd, bd, len(sizes), P, seed, sW_all=sw)
    ps.pstat_set_path("auto")
    res = res.cpu().numpy()
    assert max_rel(sw.cpu().numpy()[1:], ref["sW_perm"]) <= TOL[path]
    assert max_rel([res[0]], [ref["F_obs"]]) <= 1e-5
    assert res[1] == ref["p"]
    assert max_rel([res[3]], [ref["sT"]]) <= 1e-13


# Ties are counted with a relative tolerance on both sides (the library's
# PSTAT_TIE_RTOL, the oracle's TIE_RTOL).  (1) Two equal groups: a shuffle
# that reproduces the observed partition under swapped labels has the
# observed s_W in exact arithmetic, whichever kernel computed each value
# (on the MFMA forms the observed value comes from the pre-pass, the flagged
# rows from the recheck kernel); seed 12 at n = 12 reaches it.  (2) A
# constant matrix: every grouping has the same s_W in exact arithmetic, so
# p = 1, also when the weights 1/n_g are not exact.
@pytest.mark.parametrize("path", ALL_PATHS)
@pytest.mark.parametrize("n,half", [(12, 6), (20, 10)])
def test_permanova_swapped_partition_ties(ps, path, n, half):
    import torch
    D = synth.uniform_matrix(n, 40 + n)
    base = synth.base_labels([half, half])
    P, seed = 999, 12
    ref = oracle.permanova(D, base, P, seed)
    same = sum(np.array_equal(p, base) or np.array_equal(p, 1 - base) for p in ref["perms"])
    if n == 12:
        assert same >= 1
    ps.pstat_set_path(path)
    Dd, bd = to_dev(D, base)
    sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    res, rechecked = ps.pstat_permanova(Dd, bd, 2, P, seed, sW_all=sw)
    ps.pstat_set_path("auto")
    res = res.cpu().numpy()
    assert res[1] == ref["p"], (res[1], ref["p"], rechecked, same)
    assert max_rel(sw.cpu().numpy()[1:], ref["sW_perm"]) <= TOL[path]


@pytest.mark.parametrize("path", ALL_PATHS)
@pytest.mark.parametrize("sizes,c", [([60, 100, 140], 0.5), ([3, 5, 7, 11], 0.3),
                                     ([8, 16, 32, 8], 0.5)])
def test_permanova_constant_matrix_ties(ps, path, sizes, c):
    import torch
    n, k, P, seed = sum(sizes), len(sizes), 299, 5
    D = np.full((n, n), c, dtype=np.float32)
    np.fill_diagonal(D, 0.0)
    base = synth.base_labels(sizes)
    ref = oracle.permanova(D, base, P, seed)
    assert ref["p"] == 1.0
    ps.pstat_set_path(path)
    Dd, bd = to_dev(D, base)
    sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    res, rechecked = ps.pstat_permanova(Dd, bd, k, P, seed, sW_all=sw)
    ps.pstat_set_path("auto")
    res, sw = res.cpu().numpy(), sw.cpu().numpy()
    assert res[1] == 1.0, (res[1], rechecked)
    assert max_rel(sw, np.full(P + 1, ref["sW_obs"])) <= 1e-12
    assert max_rel([res[0]], [ref["F_obs"]]) <= 1e-9


# More groups than the FP64 pass keeps weights for in LDS (1,024): the
# samples and the recheck then read each column label's weight from global
# memory, before the next tile's loads are issued.  Group sizes 1..3, so many
# shuffles land near the observed statistic's neighbourhood only by chance;
# p, F and every s_W must still match the oracle.
@pytest.mark.parametrize("path", ["plain_f32", "mfma_split_bf16"])
def test_permanova_more_groups_than_lds_weights(ps, path):
    import torch
    k, P, seed = 1100, 99, 77
    rng = np.random.default_rng(1100)
    sizes = rng.integers(1, 4, size=k)
    n = int(sizes.sum())
    base = np.repeat(np.arange(k, dtype=np.int32), sizes)
    rng.shuffle(base)
    D = synth.uniform_matrix(n, 31)
    ref = oracle.permanova(D, base, P, seed)
    ps.pstat_set_path(path)
    Dd, bd = to_dev(D, base)
    sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    res, rechecked = ps.pstat_permanova(Dd, bd, k, P, seed, sW_all=sw)
    ps.pstat_set_path("auto")
    res = res.cpu().numpy()
    assert max_rel(sw.cpu().numpy()[1:], ref["sW_perm"]) <= TOL[path]
    assert max_rel([res[0]], [ref["F_obs"]]) <= 1e-5
    assert res[1] == ref["p"], (path, res[1], ref["p"], rechecked)
    assert max_rel([res[3]], [ref["sT"]]) <= 1e-13


# (3) Near ties in bulk: entries of 0.5 and its FP32 neighbours, so every
# permutation's s_W lies within a few units of 1e-8 (relative) of every
# other -- about the MFMA forms' own error -- and most of the shuffles fall
# inside the recheck band: many FP64 recheck passes, and every one of them
# must land on the oracle's side of the edge.
@pytest.mark.parametrize("path", ["mfma_split_bf16", "mfma_bf16", "plain_f32"])
def test_permanova_bulk_near_ties(ps, path):
    import torch
    n, sizes, P, seed = 500, [150, 150, 200], 999, 21
    rng = np.random.default_rng(8)
    up = np.nextafter(np.float32(0.5), np.float32(1.0))
    dn = np.nextafter(np.float32(0.5), np.float32(0.0))
    choice = rng.integers(0, 3, size=(n, n))
    D = np.where(choice == 0, np.float32(0.5), np.where(choice == 1, up, dn)).astype(np.float32)
    D = np.triu(D, 1)
    D = D + D.T
    base = synth.base_labels(sizes)
    ref = oracle.permanova(D, base, P, seed)
    spread = (ref["sW_perm"].max() - ref["sW_perm"].min()) / ref["sW_obs"]
    assert spread < 1e-6
    ps.pstat_set_path(path)
    Dd, bd = to_dev(D, base)
    sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    res, rechecked = ps.pstat_permanova(Dd, bd, len(sizes), P, seed, sW_all=sw)
    ps.pstat_set_path("auto")
    res = res.cpu().numpy()
    assert res[1] == ref["p"], (path, res[1], ref["p"], rechecked, spread)
    assert max_rel(sw.cpu().numpy()[1:], ref["sW_perm"]) <= TOL[path]


# The library keeps its state (stream, workspace, flags, form) per host
# thread: two threads running whole tests on their own streams at once get
# exactly what each gets alone.
def test_two_threads_on_their_own_streams(ps):
    import threading
    import torch
    cases = [(900, [300, 600], 255, 41, "mfma_split_bf16"), (1100, [200, 400, 500], 127, 42, "plain_f32")]
    inputs = []
    for n, sizes, P, seed, path in cases:
        D = synth.uniform_matrix(n, 3000 + n)
        inputs.append((to_dev(D, synth.base_labels(sizes)), len(sizes), P, seed, path))

    def one(i, out):
        (Dd, bd), k, P, seed, path = inputs[i]
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            ps.pstat_set_path(path)
            sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
            for _ in range(3):
                res, _ = ps.pstat_permanova(Dd, bd, k, P, seed, sW_all=sw)
            st.synchronize()
            out[i] = (res.cpu().numpy(), sw.cpu().numpy())

    alone = {}
    for i in range(2):
        one(i, alone)
    both = {}
    ts = [threading.Thread(target=one, args=(i, both)) for i in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    ps.pstat_set_path("auto")
    for i in range(2):
        assert np.array_equal(alone[i][0], both[i][0])
        assert np.array_equal(alone[i][1], both[i][1])


# --- the packed strict-upper-triangle layout ----------------------------------
def packed(D):
    """The strict upper triangle of a square device tensor, row after row."""
    import torch
    n = D.shape[0]
    iu = torch.triu_indices(n, n, 1, device=D.device)
    return D[iu[0], iu[1]].contiguous()


# Only addresses change: every form gives the same bits from either layout.
@pytest.mark.parametrize("path", ALL_PATHS)
@pytest.mark.parametrize("n,sizes,P", [(2, [2], 3), (257, [57, 100, 100], 129),
                                       (1000, [100, 200, 300, 400], 300)])
def test_packed_layout_bit_identical(ps, path, n, sizes, P):
    import torch
    D, base, perms, w = problem(n, sizes, P, mseed=n + 1, pseed=P + 1)
    Dd, gd, wd = to_dev(D, perms, w)
    ps.pstat_set_path(path)
    a = ps.pstat_sW(Dd, gd, wd).cpu().numpy()
    b = ps.pstat_sW(packed(Dd), gd, wd).cpu().numpy()
    ps.pstat_set_path("auto")
    assert np.array_equal(a, b)
    assert max_rel(b, oracle.sW(D, perms, w)) <= TOL[path]
    assert ps.pstat_sT(Dd).item() == ps.pstat_sT(packed(Dd)).item()


@pytest.mark.parametrize("path", ["plain_f32", "mfma_split_bf16", "mfma_f16"])
def test_packed_layout_whole_test(ps, path):
    import torch
    sizes = [300, 450, 250]
    n, k, P, seed = sum(sizes), len(sizes), 999, 4
    D = synth.uniform_matrix(n, 17)
    base = synth.base_labels(sizes)
    Dd, bd = to_dev(D, base)
    ps.pstat_set_path(path)
    out = []
    for M in (Dd, packed(Dd)):
        sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
        res, rechecked = ps.pstat_permanova(M, bd, k, P, seed, sW_all=sw)
        out.append((res.cpu().numpy(), sw.cpu().numpy(), rechecked))
    # a registered matrix in the packed layout
    h = ps.pstat_matrix_register(packed(Dd), path)
    rows = to_dev(np.vstack([base, oracle.permute(base, 20, 3)]))[0]
    wd = to_dev(synth.inv_group_sizes(sizes))[0]
    reg = ps.pstat_sW_registered(h, rows, k, wd).cpu().numpy()
    ps.pstat_matrix_release(h)
    direct = ps.pstat_sW_k(Dd, rows, k, wd).cpu().numpy()
    ps.pstat_set_path("auto")
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]
    assert np.array_equal(reg, direct)
    ref = oracle.permanova(D, base, P, seed)
    assert out[1][0][1] == ref["p"]


def test_device_packed_generator_matches_square(ps):
    import synth.device as sd
    for n in (2, 3, 300):
        a = sd.uniform_packed(n, 77).cpu().numpy()
        b = packed(sd.uniform_matrix(n, 77)).cpu().numpy()
        assert np.array_equal(a, b)


def test_free_workspace_between_calls(ps):
    # the library-managed workspace is returned and allocated again
    D, base, perms, w = problem(400, [100, 300], 64, mseed=41, pseed=42)
    a = run_sW(ps, "mfma_split_bf16", D, perms, w)
    ps.pstat_free_workspace()
    ps.pstat_free_workspace()
    b = run_sW(ps, "mfma_split_bf16", D, perms, w)
    assert np.array_equal(a, b)
