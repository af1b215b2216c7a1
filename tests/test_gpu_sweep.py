"""GPU parity over seeded random shapes: sizes, label ranges, group counts and
permutation counts drawn from fixed seeds, so that the launch plans the
library picks by size (entry widths, lanes per permutation, a split last
pass, tile edges, K chunks) meet combinations the hand-picked cases do not.
Every case is checked against the FP64 CPU oracle: the shuffles bit for bit,
the whole test by s_W within the form's bound, F, the exact p and s_T, and
the same whole test on the packed strict upper triangle bit for bit."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL, load_pstat, max_rel, to_dev

pytestmark = pytest.mark.gpu

LABEL_MAX = [1, 2, 3, 4, 7, 15, 16, 100, 255, 256, 1000, 60000]


def shuffle_case(i):
    rng = np.random.default_rng(9000 + i)
    n = int(math.exp(rng.uniform(math.log(2), math.log(250_000))))
    maxlab = int(rng.choice(LABEL_MAX))
    P = max(1, int(min(20_000, 2e8 / n) * rng.uniform(0.02, 1.0)))
    return n, maxlab, P, 9000 + i


def whole_case(i):
    rng = np.random.default_rng(7000 + i)
    n = int(rng.integers(20, 2501))
    k = int(rng.integers(2, min(12, n) + 1))
    cut = np.sort(rng.choice(np.arange(1, n), size=k - 1, replace=False))
    sizes = np.diff(np.concatenate([[0], cut, [n]]))
    P = int(rng.integers(1, 601))
    return n, [int(s) for s in sizes], P, 7000 + i


@pytest.fixture(scope="module")
def ps(dev):
    return load_pstat()


@pytest.mark.parametrize("i", range(40))
def test_shuffle_random_shapes(ps, i):
    import torch
    n, maxlab, P, seed = shuffle_case(i)
    print(f"shuffle case {i}: n={n} max_label={maxlab} P={P} seed={seed}", flush=True)
    rng = np.random.default_rng(seed)
    base = np.sort(rng.integers(0, maxlab + 1, size=n)).astype(np.int32)
    base[-1] = maxlab
    got = ps.pstat_permute(torch.from_numpy(base).cuda(), P, seed).cpu().numpy()
    assert np.array_equal(got, oracle.permute(base, P, seed))


@pytest.mark.parametrize("path", ["plain_f32", "mfma_split_bf16"])
@pytest.mark.parametrize("i", range(24))
def test_permanova_random_shapes(ps, i, path):
    import torch
    n, sizes, P, seed = whole_case(i)
    print(f"whole-test case {i} ({path}): n={n} sizes={sizes} P={P} seed={seed}", flush=True)
    base = synth.base_labels(sizes)
    rng = np.random.default_rng(seed)
    rng.shuffle(base)
    D = synth.uniform_matrix(n, seed)
    ref = oracle.permanova(D, base, P, seed)
    ps.pstat_set_path(path)
    Dd, bd = to_dev(D, base)
    sw = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    res, rechecked = ps.pstat_permanova(Dd, bd, len(sizes), P, seed, sW_all=sw)
    ps.pstat_set_path("auto")
    res = res.cpu().numpy()
    sw = sw.cpu().numpy()
    assert max_rel(sw[1:], ref["sW_perm"]) <= TOL[path]
    assert max_rel([res[0]], [ref["F_obs"]]) <= 1e-5
    assert res[1] == ref["p"], (path, res[1], ref["p"], rechecked)
    assert max_rel([res[3]], [ref["sT"]]) <= 1e-13
    # the same test on the packed strict upper triangle: the same bits
    packed = torch.from_numpy(D[np.triu_indices(n, 1)].copy()).cuda()
    sw2 = torch.empty(P + 1, dtype=torch.float64, device="cuda")
    ps.pstat_set_path(path)
    res2, _ = ps.pstat_permanova(packed, bd, len(sizes), P, seed, sW_all=sw2)
    ps.pstat_set_path("auto")
    assert np.array_equal(sw2.cpu().numpy(), sw)
    assert np.array_equal(res2.cpu().numpy(), res)
