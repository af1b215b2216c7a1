"""PERMANOVA's permuted within-group statistic s_W on AMD MI355X (gfx950).

Thin Python binding of ``libpstat.so`` (C ABI in ``include/pstat.h``).  Every
function has the C entry point's name and only marshals arguments: torch CUDA
tensors in, device pointers and sizes out, the library's status code turned
into an exception.  All computation runs in the library's HIP kernels; there
is no CPU fallback, and importing this package fails loudly if the library has
not been built (``python paper_2505_04556_amd/build.py``).

torch supplies device memory and the current stream only.
"""
from __future__ import annotations

import ctypes
import math
import os
import threading

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpstat.so")

PSTAT_OK = 0
PSTAT_EINVAL = -1
PSTAT_ELABEL = -2
PSTAT_EDOMAIN = -3
PSTAT_ENOMEM = -4
PSTAT_EHIP = -5
PSTAT_EPTR = -6
PSTAT_ESTATE = -7

PSTAT_LAYOUT_SQUARE = 0
PSTAT_LAYOUT_UPPER_PACKED = 1

PSTAT_PATH_AUTO = -1
PSTAT_PATH_PLAIN_F32 = 0
PSTAT_PATH_MFMA_BF16 = 1
PSTAT_PATH_MFMA_F16 = 2
PSTAT_PATH_MFMA_SPLIT_BF16 = 3
PSTAT_PATH_PLAIN_F64 = 4
PSTAT_PATH_MFMA_SPLIT3_BF16 = 5
PATH_NAMES = {
    PSTAT_PATH_PLAIN_F32: "plain_f32",
    PSTAT_PATH_MFMA_BF16: "mfma_bf16",
    PSTAT_PATH_MFMA_F16: "mfma_f16",
    PSTAT_PATH_MFMA_SPLIT_BF16: "mfma_split_bf16",
    PSTAT_PATH_PLAIN_F64: "plain_f64",
    PSTAT_PATH_MFMA_SPLIT3_BF16: "mfma_split3_bf16",
}
PATH_IDS = {v: k for k, v in PATH_NAMES.items()}
PATH_IDS["auto"] = PSTAT_PATH_AUTO

_CODE_NAMES = {
    PSTAT_EINVAL: "EINVAL", PSTAT_ELABEL: "ELABEL", PSTAT_EDOMAIN: "EDOMAIN",
    PSTAT_ENOMEM: "ENOMEM", PSTAT_EHIP: "EHIP", PSTAT_EPTR: "EPTR", PSTAT_ESTATE: "ESTATE",
}


class PstatError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_CODE_NAMES.get(code, code)}: {message}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2505_04556_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_i64, _i32, _u64, _int, _size = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int,
                                 ctypes.c_size_t)
_SIGS = {
    "pstat_version": ([], _int),
    "pstat_last_error": ([], ctypes.c_char_p),
    "pstat_init": ([_int], _int),
    "pstat_set_stream": ([_P], _int),
    "pstat_set_matrix_layout": ([_int], _int),
    "pstat_free_workspace": ([], _int),
    "pstat_set_path": ([_int], _int),
    "pstat_set_tuning": ([_int, _int, _int], _int),
    "pstat_set_workspace": ([_P, _size], _int),
    "pstat_workspace_bytes": ([_i64, _i64, _i32, _int], _size),
    "pstat_sW": ([_P, _i64, _P, _i64, _P, _P], _int),
    "pstat_sW_k": ([_P, _i64, _P, _i64, _i32, _P, _P], _int),
    "pstat_sW_k_noalloc": ([_P, _i64, _P, _i64, _i32, _P, _P, ctypes.POINTER(_size)], _int),
    "pstat_noalloc_scratch_bytes": ([], _size),
    "pstat_check_labels": ([], _int),
    "pstat_sT": ([_P, _i64, _P], _int),
    "pstat_F": ([_P, _i64, _P, _i64, _i32, _P], _int),
    "pstat_pvalue": ([_P, _P, _i64, _P], _int),
    "pstat_group_weights": ([_P, _i64, _i32, _P], _int),
    "pstat_permute": ([_P, _i64, _i64, _u64, _P], _int),
    "pstat_permanova": ([_P, _i64, _P, _i32, _i64, _u64, _P, _P, ctypes.POINTER(_i64)], _int),
    "pstat_matrix_register": ([_P, _i64, _int, ctypes.POINTER(_i64)], _int),
    "pstat_matrix_release": ([_i64], _int),
    "pstat_sW_registered": ([_i64, _P, _i64, _i32, _P, _P], _int),
    "pstat_serve_create": ([_i64, _i64, ctypes.POINTER(_i64)], _int),
    "pstat_serve_destroy": ([_i64], _int),
    "pstat_resolve_path": ([_int, _i64, _i32], _int),
    "pstat_job_bytes": ([_i64, _i64, _i32, _int], _size),
    "pstat_job_create": ([_i64, _P, _i64, _P, _i32, _i64, _u64, _int, _P, _size,
                          ctypes.POINTER(_i64), ctypes.POINTER(_i64)], _int),
    "pstat_serve_round": ([_i64, _P, _i64], _int),
    "pstat_job_finish": ([_i64, _i64, ctypes.POINTER(ctypes.c_double), _P, ctypes.POINTER(_i64)],
                         _int),
    "pstat_job_release": ([_i64, _i64], _int),
    "pstat_profile": ([_int], _int),
    "pstat_profile_read": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)], _int),
}
for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res

_tls = threading.local()


def _check(rc: int) -> None:
    if rc != PSTAT_OK:
        raise PstatError(rc, _lib.pstat_last_error().decode(errors="replace"))


def _ready(device: torch.device) -> None:
    """pstat_init once per thread and device; current torch stream every call."""
    idx = device.index if device.index is not None else torch.cuda.current_device()
    if getattr(_tls, "device", None) != idx:
        _check(_lib.pstat_init(idx))
        _tls.device = idx
    _check(_lib.pstat_set_stream(ctypes.c_void_p(torch.cuda.current_stream(idx).cuda_stream)))


def _dev(t: torch.Tensor, dtype: torch.dtype, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise PstatError(PSTAT_EPTR, f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise PstatError(PSTAT_EINVAL, f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise PstatError(PSTAT_EINVAL, f"{name} must be contiguous")
    return t.data_ptr()


def _need(t, count: int, name: str) -> None:
    """Size check before any launch: t must be a tensor of at least `count`
    elements (the library reads or writes that many through its pointer)."""
    if not isinstance(t, torch.Tensor):
        raise PstatError(PSTAT_EINVAL, f"{name} must be a tensor")
    if t.numel() < count:
        raise PstatError(PSTAT_EINVAL, f"{name} holds {t.numel()} elements, {count} needed")


def _rows(groupings: torch.Tensor, n: int, name: str = "groupings") -> int:
    """Number of grouping rows of a [P, n] (or one [n]) label tensor."""
    if not isinstance(groupings, torch.Tensor):
        raise PstatError(PSTAT_EINVAL, f"{name} must be a tensor")
    if groupings.dim() == 1 and groupings.shape[0] == n:
        return 1
    if groupings.dim() == 2 and groupings.shape[1] == n:
        return int(groupings.shape[0])
    raise PstatError(PSTAT_EINVAL, f"{name} must be [P, {n}] or [{n}], got {tuple(groupings.shape)}")


def _mat_n(mat: torch.Tensor) -> int:
    """n of a matrix argument (square n x n, or packed strict upper triangle)."""
    if not isinstance(mat, torch.Tensor):
        raise PstatError(PSTAT_EINVAL, "mat must be a tensor")
    if mat.dim() == 2 and mat.shape[0] == mat.shape[1]:
        return int(mat.shape[0])
    if mat.dim() == 1:
        return packed_n(mat.numel())
    raise PstatError(PSTAT_EINVAL, f"mat must be n x n or packed 1-D, got {tuple(mat.shape)}")


def packed_n(length: int) -> int:
    """n of a strict upper triangle packed into `length` = n (n - 1) / 2 floats."""
    n = (1 + math.isqrt(1 + 8 * int(length))) // 2
    if n < 2 or n * (n - 1) // 2 != length:
        raise PstatError(PSTAT_EINVAL, f"{length} is not n (n - 1) / 2 for any n >= 2")
    return n


def _mat(mat: torch.Tensor) -> tuple[int, int]:
    """Pointer and n of a matrix argument, setting this thread's layout: an
    n x n tensor is the square layout, a 1-D tensor of n (n - 1) / 2 floats
    the packed strict upper triangle."""
    n = _mat_n(mat)
    ptr = _dev(mat, torch.float32, "mat")
    layout = PSTAT_LAYOUT_UPPER_PACKED if mat.dim() == 1 else PSTAT_LAYOUT_SQUARE
    _check(_lib.pstat_set_matrix_layout(layout))
    return ptr, n


def pstat_version() -> int:
    return int(_lib.pstat_version())


def pstat_set_path(path) -> None:
    p = PATH_IDS[path] if isinstance(path, str) else int(path)
    _ready(torch.device("cuda", torch.cuda.current_device()))
    _check(_lib.pstat_set_path(p))


def pstat_resolve_path(path, n: int, n_groups: int) -> str:
    """Name of the form `path` ("auto" included) runs at this shape; host only."""
    p = PATH_IDS[path] if isinstance(path, str) else int(path)
    r = int(_lib.pstat_resolve_path(p, int(n), int(n_groups)))
    if r < 0:                       # a resolved path is never AUTO
        _check(r)
    return PATH_NAMES[r]


resolve_path = pstat_resolve_path


def pstat_set_tuning(path, tile: int = 0, batch: int = 0) -> None:
    p = PATH_IDS[path] if isinstance(path, str) else int(path)
    _ready(torch.device("cuda", torch.cuda.current_device()))
    _check(_lib.pstat_set_tuning(p, int(tile), int(batch)))


def pstat_set_workspace(ws: torch.Tensor | None) -> None:
    if ws is None:
        _check(_lib.pstat_set_workspace(None, 0))
        return
    _ready(ws.device)
    _check(_lib.pstat_set_workspace(_dev(ws, torch.uint8, "workspace"), ws.numel()))


def pstat_free_workspace() -> None:
    """Return the library-managed workspace of this thread to the device."""
    _check(_lib.pstat_free_workspace())


def pstat_workspace_bytes(n: int, n_perms: int, n_groups: int, path=PSTAT_PATH_AUTO) -> int:
    p = PATH_IDS[path] if isinstance(path, str) else int(path)
    _ready(torch.device("cuda", torch.cuda.current_device()))
    return int(_lib.pstat_workspace_bytes(n, n_perms, n_groups, p))


def pstat_sW(mat: torch.Tensor, groupings: torch.Tensor, inv_group_sizes: torch.Tensor,
             out: torch.Tensor | None = None) -> torch.Tensor:
    """s_W of every grouping row (validates labels; synchronises once).  The
    library takes k = 1 + the largest label and reads that many weights."""
    P = _rows(groupings, _mat_n(mat))
    if out is not None:
        _need(out, P, "out")
    _need(inv_group_sizes, 1, "inv_group_sizes")
    if groupings.numel() and isinstance(groupings, torch.Tensor) and groupings.is_cuda:
        # argument check: the weights must cover the largest label (one
        # reduction; the call synchronises anyway)
        _need(inv_group_sizes, int(groupings.max().item()) + 1, "inv_group_sizes")
    if out is None:
        out = torch.empty(P, dtype=torch.float64, device=mat.device)
    _ready(mat.device)
    mp, n = _mat(mat)
    _check(_lib.pstat_sW(mp, n,
                         _dev(groupings, torch.int32, "groupings"), P,
                         _dev(inv_group_sizes, torch.float64, "inv_group_sizes"),
                         _dev(out, torch.float64, "out")))
    return out


def pstat_sW_k(mat, groupings, n_groups: int, inv_group_sizes, out=None) -> torch.Tensor:
    """s_W with the number of groups given; asynchronous."""
    P = _rows(groupings, _mat_n(mat))
    _need(inv_group_sizes, int(n_groups), "inv_group_sizes")
    if out is not None:
        _need(out, P, "out")
    if out is None:
        out = torch.empty(P, dtype=torch.float64, device=mat.device)
    _ready(mat.device)
    mp, n = _mat(mat)
    _check(_lib.pstat_sW_k(mp, n,
                           _dev(groupings, torch.int32, "groupings"), P, int(n_groups),
                           _dev(inv_group_sizes, torch.float64, "inv_group_sizes"),
                           _dev(out, torch.float64, "out")))
    return out


def pstat_sW_k_noalloc(mat, groupings, n_groups: int, inv_group_sizes, out) -> int:
    """pstat_sW_k with the library's static scratch (allocates nothing; out
    must be given).  Returns the scratch bytes the shape used."""
    P = _rows(groupings, _mat_n(mat))
    _need(inv_group_sizes, int(n_groups), "inv_group_sizes")
    _need(out, P, "out")
    _ready(mat.device)
    mp, n = _mat(mat)
    used = _size(0)
    _check(_lib.pstat_sW_k_noalloc(mp, n, _dev(groupings, torch.int32, "groupings"), P,
                                   int(n_groups),
                                   _dev(inv_group_sizes, torch.float64, "inv_group_sizes"),
                                   _dev(out, torch.float64, "out"), ctypes.byref(used)))
    return int(used.value)


def pstat_noalloc_scratch_bytes() -> int:
    return int(_lib.pstat_noalloc_scratch_bytes())


def pstat_check_labels() -> None:
    _ready(torch.device("cuda", torch.cuda.current_device()))
    _check(_lib.pstat_check_labels())


def pstat_sT(mat: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    _mat_n(mat)
    if out is not None:
        _need(out, 1, "s_T")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=mat.device)
    _ready(mat.device)
    mp, n = _mat(mat)
    _check(_lib.pstat_sT(mp, n,
                         _dev(out, torch.float64, "s_T")))
    return out


def pstat_F(s_W: torch.Tensor, s_T: torch.Tensor, n: int, k: int,
            out: torch.Tensor | None = None) -> torch.Tensor:
    _need(s_W, 0, "s_W")
    _need(s_T, 1, "s_T")
    if out is not None:
        _need(out, s_W.numel(), "F")
    if out is None:
        out = torch.empty_like(s_W)
    _ready(s_W.device)
    _check(_lib.pstat_F(_dev(s_W, torch.float64, "s_W"), s_W.numel(),
                        _dev(s_T, torch.float64, "s_T"), int(n), int(k),
                        _dev(out, torch.float64, "F")))
    return out


def pstat_pvalue(s_W_obs: torch.Tensor, s_W_perm: torch.Tensor,
                 out: torch.Tensor | None = None) -> torch.Tensor:
    _need(s_W_obs, 1, "s_W_obs")
    _need(s_W_perm, 0, "s_W_perm")
    if out is not None:
        _need(out, 1, "p")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=s_W_obs.device)
    _ready(s_W_obs.device)
    perm_ptr = _dev(s_W_perm, torch.float64, "s_W_perm") if s_W_perm.numel() else None
    _check(_lib.pstat_pvalue(_dev(s_W_obs, torch.float64, "s_W_obs"), perm_ptr,
                             s_W_perm.numel(), _dev(out, torch.float64, "p")))
    return out


def pstat_group_weights(grouping: torch.Tensor, n_groups: int,
                        out: torch.Tensor | None = None) -> torch.Tensor:
    _need(grouping, 1, "grouping")
    if out is not None:
        _need(out, int(n_groups), "inv")
    if out is None:
        out = torch.empty(n_groups, dtype=torch.float64, device=grouping.device)
    _ready(grouping.device)
    _check(_lib.pstat_group_weights(_dev(grouping, torch.int32, "grouping"), grouping.numel(),
                                    int(n_groups), _dev(out, torch.float64, "inv")))
    return out


def pstat_permute(base: torch.Tensor, n_perms: int, seed: int,
                  out: torch.Tensor | None = None) -> torch.Tensor:
    _need(base, 1, "base")
    n = base.numel()
    if out is not None:
        _need(out, int(n_perms) * n, "groupings")
    if out is None:
        out = torch.empty((n_perms, n), dtype=torch.int32, device=base.device)
    _ready(base.device)
    _check(_lib.pstat_permute(_dev(base, torch.int32, "base"), n, int(n_perms),
                              int(seed) & 0xFFFFFFFFFFFFFFFF, _dev(out, torch.int32, "groupings")))
    return out


def pstat_permanova(mat: torch.Tensor, grouping: torch.Tensor, n_groups: int, n_perms: int,
                    seed: int, result: torch.Tensor | None = None,
                    sW_all: torch.Tensor | None = None) -> tuple[torch.Tensor, int]:
    """The whole test.  Returns (result = [F_obs, p, s_W_obs, s_T], n_rechecked)."""
    n = _mat_n(mat)
    _need(grouping, n, "grouping")
    if grouping.numel() != n:
        raise PstatError(PSTAT_EINVAL, f"grouping must hold n = {n} labels")
    if result is not None:
        _need(result, 4, "result")
    if sW_all is not None:
        _need(sW_all, int(n_perms) + 1, "sW_all")
    if result is None:
        result = torch.empty(4, dtype=torch.float64, device=mat.device)
    _ready(mat.device)
    rechecked = _i64(0)
    sw_ptr = _dev(sW_all, torch.float64, "sW_all") if sW_all is not None else None
    mp, n = _mat(mat)
    _check(_lib.pstat_permanova(mp, n,
                                _dev(grouping, torch.int32, "grouping"), int(n_groups),
                                int(n_perms), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                _dev(result, torch.float64, "result"), sw_ptr,
                                ctypes.byref(rechecked)))
    return result, int(rechecked.value)


# n of each registered matrix (argument checks of pstat_sW_registered)
_registered_n: dict[int, int] = {}
# grouping rows (n_perms + 1) of each live serving job, by (server, job)
_job_rows: dict[tuple[int, int], int] = {}


def pstat_matrix_register(mat: torch.Tensor, path=PSTAT_PATH_AUTO) -> int:
    p = PATH_IDS[path] if isinstance(path, str) else int(path)
    _ready(mat.device)
    h = _i64(0)
    mp, n = _mat(mat)
    _check(_lib.pstat_matrix_register(mp, n, p,
                                      ctypes.byref(h)))
    _registered_n[int(h.value)] = n
    return int(h.value)


def pstat_matrix_release(handle: int) -> None:
    _check(_lib.pstat_matrix_release(int(handle)))
    _registered_n.pop(int(handle), None)


def pstat_sW_registered(handle: int, groupings: torch.Tensor, n_groups: int,
                        inv_group_sizes: torch.Tensor, out: torch.Tensor | None = None):
    n = _registered_n.get(int(handle))
    if n is None:
        raise PstatError(PSTAT_EINVAL, f"unknown handle {handle}")
    P = _rows(groupings, n)
    _need(inv_group_sizes, int(n_groups), "inv_group_sizes")
    if out is not None:
        _need(out, P, "out")
    if out is None:
        out = torch.empty(P, dtype=torch.float64, device=groupings.device)
    _ready(groupings.device)
    _check(_lib.pstat_sW_registered(int(handle), _dev(groupings, torch.int32, "groupings"), P,
                                    int(n_groups),
                                    _dev(inv_group_sizes, torch.float64, "inv_group_sizes"),
                                    _dev(out, torch.float64, "out")))
    return out


def pstat_serve_create(max_jobs: int, max_units: int) -> int:
    _ready(torch.device("cuda", torch.cuda.current_device()))
    h = _i64(0)
    _check(_lib.pstat_serve_create(int(max_jobs), int(max_units), ctypes.byref(h)))
    return int(h.value)


def pstat_serve_destroy(server: int) -> None:
    _check(_lib.pstat_serve_destroy(int(server)))


def pstat_job_bytes(n: int, n_perms: int, n_groups: int, path=PSTAT_PATH_PLAIN_F32) -> int:
    p = PATH_IDS[path] if isinstance(path, str) else int(path)
    _ready(torch.device("cuda", torch.cuda.current_device()))
    return int(_lib.pstat_job_bytes(int(n), int(n_perms), int(n_groups), p))


def pstat_job_create(server: int, mat: torch.Tensor, grouping: torch.Tensor, n_groups: int,
                     n_perms: int, seed: int, scratch: torch.Tensor,
                     path=PSTAT_PATH_PLAIN_F32) -> tuple[int, int]:
    """Returns (job id, number of work units)."""
    p = PATH_IDS[path] if isinstance(path, str) else int(path)
    n = _mat_n(mat)
    _need(grouping, n, "grouping")
    if grouping.numel() != n:
        raise PstatError(PSTAT_EINVAL, f"grouping must hold n = {n} labels")
    _ready(mat.device)
    job, units = _i64(0), _i64(0)
    mp, n = _mat(mat)
    _check(_lib.pstat_job_create(int(server), mp, n,
                                 _dev(grouping, torch.int32, "grouping"), int(n_groups),
                                 int(n_perms), int(seed) & 0xFFFFFFFFFFFFFFFF, p,
                                 _dev(scratch, torch.uint8, "scratch"), scratch.numel(),
                                 ctypes.byref(job), ctypes.byref(units)))
    _job_rows[(int(server), int(job.value))] = int(n_perms) + 1
    return int(job.value), int(units.value)


def pstat_serve_round(server: int, pairs) -> None:
    """pairs: int64 numpy array of shape (count, 2) = (job, unit) per row."""
    import numpy as np
    arr = np.ascontiguousarray(pairs, dtype=np.int64).reshape(-1, 2)
    _ready(torch.device("cuda", torch.cuda.current_device()))
    _check(_lib.pstat_serve_round(int(server), arr.ctypes.data if len(arr) else None, len(arr)))


def pstat_job_finish(server: int, job: int, sW_all: torch.Tensor | None = None):
    """Returns ([F_obs, p, s_W_obs, s_T], n_rechecked)."""
    if sW_all is not None:
        rows = _job_rows.get((int(server), int(job)))
        if rows is None:
            raise PstatError(PSTAT_EINVAL, f"unknown job {job}")
        _need(sW_all, rows, "sW_all")
    _ready(torch.device("cuda", torch.cuda.current_device()))
    res = (ctypes.c_double * 4)()
    rech = _i64(0)
    sw = _dev(sW_all, torch.float64, "sW_all") if sW_all is not None else None
    _check(_lib.pstat_job_finish(int(server), int(job), res, sw, ctypes.byref(rech)))
    return [float(v) for v in res], int(rech.value)


def pstat_job_release(server: int, job: int) -> None:
    _check(_lib.pstat_job_release(int(server), int(job)))
    _job_rows.pop((int(server), int(job)), None)


def pstat_profile(on: bool) -> None:
    _check(_lib.pstat_profile(1 if on else 0))


def pstat_profile_read() -> tuple[float, int]:
    """(summed main-kernel milliseconds, launches) since pstat_profile(True)."""
    ms = ctypes.c_double(0.0)
    cnt = _i64(0)
    _check(_lib.pstat_profile_read(ctypes.byref(ms), ctypes.byref(cnt)))
    return float(ms.value), int(cnt.value)


def exported_symbols() -> list[str]:
    return sorted(_SIGS)
