"""The autotuner on the GPU: every candidate runs, the chosen form meets the
accuracy bar, applying the cache reproduces the tuned kernel's results."""
import json

import numpy as np
import pytest

import oracle
from gpu_util import TOL, load_pstat, max_rel, problem, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps(dev):
    return load_pstat()


def test_tune_apply_roundtrip(ps, tmp_path):
    from paper_2505_04556_amd import autotune
    D, base, perms, w = problem(900, [200, 300, 400], 300, mseed=3, pseed=4)
    ref = oracle.sW(D, perms, w)
    Dd, gd, wd = to_dev(D, perms, w)
    cache_file = str(tmp_path / "tune.json")
    cache = {}
    entry = autotune.tune(Dd, gd, 3, wd, reps=1, cache=cache, save=False)
    autotune.save_cache(cache, cache_file)
    assert set(entry["paths"]) == set(autotune.ALL_PATHS)
    for path, best in entry["paths"].items():
        assert (best["tile"], best["batch"]) in autotune.space_for(path)
        assert best["kernel_ms"] > 0
        assert all("kernel_ms" in t or "error" in t for t in best["trials"])
    assert entry["auto"] in autotune.ACCURATE
    loaded = autotune.load_cache(cache_file)
    assert json.dumps(loaded, sort_keys=True) == json.dumps(cache, sort_keys=True)
    chosen = autotune.apply(900, 3, 300, cache=loaded)
    assert chosen == entry["auto"]
    got = ps.pstat_sW_k(Dd, gd, 3, wd).cpu().numpy()
    assert max_rel(got, ref) <= TOL[chosen]
    for path in autotune.ALL_PATHS:
        autotune.apply(900, 3, 300, path=path, cache=loaded)
        assert max_rel(ps.pstat_sW_k(Dd, gd, 3, wd).cpu().numpy(), ref) <= TOL[path]
        ps.pstat_set_tuning(path, 0, 0)
    ps.pstat_set_path(ps.PSTAT_PATH_AUTO)


def test_untuned_shape_keeps_defaults(ps):
    from paper_2505_04556_amd import autotune
    assert autotune.apply(12345, 7, 77, cache={}) is None
