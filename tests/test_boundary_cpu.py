"""The C-ABI library loads without a GPU and exports every entry point that
include/pstat.h declares; the oracle and input generators are importable."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pstat.h")
LIB = os.path.join(ROOT, "paper_2505_04556_amd", "libpstat.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pstat_[A-Za-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from gpu_util import load_build_module
        load_build_module().build_pstat()
    return ctypes.CDLL(LIB)


def test_header_declares_the_papers_calls():
    syms = declared_symbols()
    for name in ("pstat_sW", "pstat_F", "pstat_pvalue", "pstat_permute", "pstat_sT"):
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_exports_match_nm():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\b(pstat_[A-Za-z0-9_]+)\b", out))
    assert set(declared_symbols()) <= exported


def test_no_device_calls_without_init(lib):
    # Before pstat_init every compute call must refuse with PSTAT_ESTATE (-7)
    # without touching a device.
    lib.pstat_sW.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                             ctypes.c_void_p, ctypes.c_void_p]
    assert lib.pstat_sW(None, 10, None, 1, None, None) == -7
    lib.pstat_last_error.restype = ctypes.c_char_p
    assert b"pstat_init" in lib.pstat_last_error()
    assert lib.pstat_version() >= 10000


def test_binding_names_match_header():
    import importlib
    try:
        mod = importlib.import_module("paper_2505_04556_amd")
    except ImportError:
        pytest.skip("library not built")
    assert sorted(mod.exported_symbols()) == declared_symbols()


def test_packed_n():
    import paper_2505_04556_amd as ps
    for n in (2, 3, 10, 1000, 380_000):
        assert ps.packed_n(n * (n - 1) // 2) == n
    for bad in (0, 2, 4, 5, 4949):
        with pytest.raises(ps.PstatError):
            ps.packed_n(bad)


def test_host_only_settings(lib):
    # thread settings that need no device: layouts, path names and their
    # resolution (PSTAT_EINVAL = -1 for unknown values)
    assert lib.pstat_set_matrix_layout(0) == 0
    assert lib.pstat_set_matrix_layout(1) == 0
    assert lib.pstat_set_matrix_layout(2) == -1
    assert lib.pstat_set_matrix_layout(0) == 0
    lib.pstat_resolve_path.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int32]
    assert lib.pstat_resolve_path(5, 1000, 3) == 5          # three-part split BF16
    assert lib.pstat_resolve_path(-1, 10000, 5) == 3        # auto: split BF16
    assert lib.pstat_resolve_path(-1, 10000, 40) == 0       # auto: plain FP32 above 16 groups
    assert lib.pstat_resolve_path(6, 1000, 3) == -1
    assert lib.pstat_free_workspace() == 0                  # none held
