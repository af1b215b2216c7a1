"""Device-memory copies of the synthetic matrices (same values as the numpy
generators in ``synth``), produced on the GPU by ``libsynth.so`` so that
40 GB matrices never exist on the host."""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

import synth

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsynth.so")
_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} missing: run `python paper_2505_04556_amd/build.py`")
        L = ctypes.CDLL(_LIB_PATH)
        L.synth_uniform.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p]
        L.synth_uniform_packed.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64,
                                           ctypes.c_void_p]
        L.synth_euclid.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p]
        _lib = L
    return _lib


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def uniform_matrix(n: int, seed: int, device="cuda", out: torch.Tensor | None = None,
                   rows: tuple[int, int] | None = None) -> torch.Tensor:
    """Rows [r0, r1) (all by default) of the hash-uniform matrix, on the device."""
    r0, r1 = rows if rows is not None else (0, n)
    if out is None:
        out = torch.empty((r1 - r0, n), dtype=torch.float32, device=device)
    assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
    assert out.numel() == (r1 - r0) * n
    rc = lib().synth_uniform(out.data_ptr(), n, r0, r1 - r0, synth.mix64(int(seed)),
                             _stream(out.device))
    if rc != 0:
        raise RuntimeError("synth_uniform launch failed")
    return out


def uniform_packed(n: int, seed: int, device="cuda") -> torch.Tensor:
    """The hash-uniform matrix's strict upper triangle, packed row after row
    (n (n - 1) / 2 floats), on the device; equal to the square's entries."""
    out = torch.empty(n * (n - 1) // 2, dtype=torch.float32, device=device)
    rc = lib().synth_uniform_packed(out.data_ptr(), n, synth.mix64(int(seed)), _stream(out.device))
    if rc != 0:
        raise RuntimeError("synth_uniform_packed launch failed")
    return out


def euclid_matrix(n: int, seed: int, device="cuda", dims: int = 32,
                  points: np.ndarray | None = None) -> torch.Tensor:
    x = synth.euclid_points(n, seed, dims) if points is None else points
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(device)
    out = torch.empty((n, n), dtype=torch.float32, device=device)
    scratch = torch.empty(1, dtype=torch.int64, device=device)
    rc = lib().synth_euclid(out.data_ptr(), xd.data_ptr(), n, x.shape[1], scratch.data_ptr(),
                            _stream(out.device))
    if rc != 0:
        raise RuntimeError("synth_euclid launch failed")
    torch.cuda.current_stream(out.device).synchronize()
    del xd, scratch
    return out


def matrix(cfg: dict, device="cuda") -> torch.Tensor:
    if cfg["matrix"] == "uniform":
        return uniform_matrix(cfg["n"], cfg["matrix_seed"], device)
    return euclid_matrix(cfg["n"], cfg["matrix_seed"], device)
