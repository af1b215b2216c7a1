"""Generated problems (Hypothesis, derandomized: the same examples on every
run) through the library's forms against the FP64 oracle: sizes, group
counts, label patterns (empty groups, one group, all groups interleaved,
contiguous blocks) and permutation counts beyond the fixed shapes of
test_gpu_parity.py.  The scaled-FP16 form is left out: its error bound is
relative to the largest entry, not to s_W (test_gpu_parity.py covers it)."""
import numpy as np
import pytest
from hypothesis import HealthCheck, assume, given, settings, strategies as st

import oracle
import synth
from gpu_util import TOL, load_pstat, max_rel, to_dev

pytestmark = pytest.mark.gpu

PATHS = ["plain_f32", "plain_f64", "mfma_split_bf16", "mfma_split3_bf16", "mfma_bf16"]
SETTINGS = dict(derandomize=True, deadline=None, database=None,
                suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])


@pytest.fixture(scope="module")
def ps(dev):
    return load_pstat()


def labels(rng, pattern, P, n, k):
    if pattern == "random":
        return rng.integers(0, k, size=(P, n))
    if pattern == "one":
        return np.zeros((P, n), dtype=np.int64)
    if pattern == "interleaved":
        return np.stack([rng.permutation(np.arange(n) % k) for _ in range(P)])
    cuts = np.sort(rng.integers(0, n + 1, size=k - 1))         # contiguous blocks
    row = np.searchsorted(cuts, np.arange(n), side="right")
    return np.stack([row] * P)


@st.composite
def problems(draw):
    n = draw(st.integers(2, 300))
    k = draw(st.integers(1, 8))
    P = draw(st.integers(1, 70))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    pattern = draw(st.sampled_from(["random", "one", "interleaved", "blocks"]))
    rng = np.random.default_rng(seed)
    g = labels(rng, pattern, P, n, k).astype(np.int32)
    D = synth.uniform_matrix(n, seed % 997 + 1)
    w = rng.uniform(0.01, 2.0, size=k)
    return D, g, w


@settings(max_examples=150, **SETTINGS)
@given(prob=problems())
def test_generated_sW_every_form(ps, prob):
    import torch
    D, g, w = prob
    ref = oracle.sW(D, g, w)
    Dd, gd, wd = to_dev(D, g, w)
    for path in PATHS:
        ps.pstat_set_path(path)
        got = ps.pstat_sW(Dd, gd, wd).cpu().numpy()
        assert max_rel(got, ref) <= TOL[path], (path, D.shape[0], g.shape, max_rel(got, ref))
    ps.pstat_set_path("auto")
    torch.cuda.synchronize()


@st.composite
def whole_cases(draw):
    sizes = draw(st.lists(st.integers(1, 60), min_size=2, max_size=6))
    assume(sum(sizes) > len(sizes))       # F needs n > k
    P = draw(st.integers(1, 200))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    return sizes, P, seed


@settings(max_examples=80, **SETTINGS)
@given(case=whole_cases())
def test_generated_whole_test_p_equals_oracle(ps, case):
    sizes, P, seed = case
    n, k = sum(sizes), len(sizes)
    D = synth.uniform_matrix(n, seed % 991 + 1)
    base = synth.base_labels(sizes)
    ref = oracle.permanova(D, base, P, seed)
    Dd, bd = to_dev(D, base)
    for path in ("plain_f32", "mfma_split_bf16"):
        ps.pstat_set_path(path)
        res, _ = ps.pstat_permanova(Dd, bd, k, P, seed)
        r = res.cpu().numpy()
        assert r[1] == ref["p"], (path, sizes, P, seed, r[1], ref["p"])
        # F_obs comes from the FP64 recheck of the observed grouping
        assert abs(r[0] - ref["F_obs"]) <= 1e-8 * abs(ref["F_obs"]), (path, r[0], ref["F_obs"])
    ps.pstat_set_path("auto")
