"""pstat_sW_k_noalloc -- pstat_sW_k for callers that cannot allocate, with a
static device array as scratch -- called through the C ABI, against
pstat_sW_k on the same inputs: bit-identical on two calls in a row, the
second with a smaller input (the array keeps the first call's contents), and
a clear error with the output untouched when a shape needs more scratch than
the array holds."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_util import load_pstat, problem, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps(dev):
    return load_pstat()


def noalloc(ps, D, g, k, w, out):
    """The C entry point itself (ctypes); returns (status, scratch bytes)."""
    import torch
    ps._ready(D.device)
    ps._check(ps._lib.pstat_set_matrix_layout(ps.PSTAT_LAYOUT_SQUARE))
    used = ctypes.c_size_t(0)
    rc = ps._lib.pstat_sW_k_noalloc(D.data_ptr(), D.shape[0], g.data_ptr(), g.shape[0], k,
                                    w.data_ptr(), out.data_ptr(), ctypes.byref(used))
    torch.cuda.synchronize()
    return rc, int(used.value)


@pytest.mark.parametrize("path", ["plain_f32", "mfma_split_bf16", "plain_f64", "mfma_bf16"])
def test_noalloc_equals_sW_k_twice_then_smaller(ps, path):
    import torch
    ps.pstat_set_path(path)
    try:
        for n, sizes, P, seed in [(1500, [300, 500, 700], 700, 1), (700, [200, 500], 130, 2)]:
            D, base, perms, w = problem(n, sizes, P, mseed=seed, pseed=seed + 10)
            Dd, gd, wd = to_dev(D, perms, w)
            ref = ps.pstat_sW_k(Dd, gd, len(sizes), wd).cpu().numpy()
            out = torch.full((P,), -1.0, dtype=torch.float64, device="cuda")
            rc, used = noalloc(ps, Dd, gd, len(sizes), wd, out)
            assert rc == ps.PSTAT_OK, ps._lib.pstat_last_error()
            assert 0 < used <= ps.pstat_noalloc_scratch_bytes()
            assert np.array_equal(out.cpu().numpy(), ref), (path, n)
        ps.pstat_check_labels()
    finally:
        ps.pstat_set_path("auto")


def test_noalloc_rejects_shapes_beyond_the_array(ps):
    import torch
    ps.pstat_set_path("plain_f32")
    try:
        n, P = 4000, 8000          # labels 4000 x 8192 x 2 B and partials: > 64 MiB
        D = torch.zeros((n, n), dtype=torch.float32, device="cuda")
        g = torch.zeros((P, n), dtype=torch.int32, device="cuda")
        w = torch.ones(1, dtype=torch.float64, device="cuda")
        out = torch.full((P,), 7.0, dtype=torch.float64, device="cuda")
        rc, used = noalloc(ps, D, g, 1, w, out)
        assert rc == ps.PSTAT_ENOMEM
        assert used > ps.pstat_noalloc_scratch_bytes()
        assert b"static scratch" in ps._lib.pstat_last_error()
        assert torch.all(out == 7.0)
    finally:
        ps.pstat_set_path("auto")
