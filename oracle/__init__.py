"""Python face of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the package smoke check and the
benchmark's CPU-baseline leg are the only callers.  Nothing here is part of the
HIP product path, and nothing here imports the product package.

All functions take and return numpy arrays; matrices are float32 row-major,
labels int32, weights and results float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
           "-shared", "-fPIC", "-Wall", "-Wextra"]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (no GPU code involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", *_CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, u64, f64, c_int = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                     ctypes.c_double, ctypes.c_int)
        L.oracle_sW_rows.argtypes = [P, i64, i64, i64, P, i64, P, P, c_int]
        L.oracle_sW.argtypes = [P, i64, P, i64, P, P, c_int]
        L.oracle_sW_tiled.argtypes = [P, i64, P, i64, P, i64, P, c_int]
        L.oracle_sq_rows.argtypes = [P, i64, i64, i64, P]
        L.oracle_sT.argtypes = [P, i64]
        L.oracle_sT.restype = f64
        L.oracle_between_unweighted.argtypes = [P, i64, P]
        L.oracle_between_unweighted.restype = f64
        L.oracle_F.argtypes = [P, i64, f64, i64, i32, P]
        L.oracle_pvalue.argtypes = [f64, P, i64]
        L.oracle_pvalue.restype = f64
        L.oracle_pvalue_sW.argtypes = [f64, P, i64]
        L.oracle_pvalue_sW.restype = f64
        L.oracle_splitmix64_next.argtypes = [P]
        L.oracle_splitmix64_next.restype = u64
        L.oracle_stream_start.argtypes = [u64, u64]
        L.oracle_stream_start.restype = u64
        L.oracle_bounded.argtypes = [P, ctypes.c_uint32]
        L.oracle_bounded.restype = ctypes.c_uint32
        L.oracle_permute.argtypes = [P, i64, i64, u64, P, c_int]
        L.oracle_count_rejections.argtypes = [i64, i64, u64]
        L.oracle_count_rejections.restype = i64
        L.oracle_max_threads.restype = c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _mat(mat) -> np.ndarray:
    mat = np.ascontiguousarray(mat, dtype=np.float32)
    if mat.ndim != 2 or mat.shape[0] != mat.shape[1]:
        raise ValueError("matrix must be square")
    return mat


def _groupings(groupings, n: int) -> np.ndarray:
    g = np.ascontiguousarray(groupings, dtype=np.int32)
    if g.ndim == 1:
        g = g[None, :]
    if g.shape[1] != n:
        raise ValueError("groupings must have n columns")
    return g


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def sW(mat, groupings, inv, nthreads: int = 0) -> np.ndarray:
    """s_W for every grouping row (Algorithm 1, FP64)."""
    mat = _mat(mat)
    n = mat.shape[0]
    g = _groupings(groupings, n)
    inv = np.ascontiguousarray(inv, dtype=np.float64)
    out = np.zeros(g.shape[0], dtype=np.float64)
    lib().oracle_sW(_ptr(mat), n, _ptr(g), g.shape[0], _ptr(inv), _ptr(out), nthreads)
    return out


def sW_rows(rows, row0: int, n: int, groupings, inv, acc: np.ndarray, nthreads: int = 0) -> None:
    """Continue acc[p] over matrix rows [row0, row0 + rows.shape[0])."""
    rows = np.ascontiguousarray(rows, dtype=np.float32)
    assert rows.ndim == 2 and rows.shape[1] == n
    g = _groupings(groupings, n)
    inv = np.ascontiguousarray(inv, dtype=np.float64)
    assert acc.dtype == np.float64 and acc.flags.c_contiguous and acc.shape[0] == g.shape[0]
    lib().oracle_sW_rows(_ptr(rows), row0, rows.shape[0], n, _ptr(g), g.shape[0], _ptr(inv),
                         _ptr(acc), nthreads)


def sW_tiled(mat, groupings, inv, tile: int, nthreads: int = 0) -> np.ndarray:
    """s_W in Algorithm 2's tiled traversal (FP64)."""
    mat = _mat(mat)
    n = mat.shape[0]
    g = _groupings(groupings, n)
    inv = np.ascontiguousarray(inv, dtype=np.float64)
    out = np.zeros(g.shape[0], dtype=np.float64)
    lib().oracle_sW_tiled(_ptr(mat), n, _ptr(g), g.shape[0], _ptr(inv), int(tile), _ptr(out),
                          nthreads)
    return out


def sq_rows(rows, row0: int, n: int, acc: float) -> float:
    rows = np.ascontiguousarray(rows, dtype=np.float32)
    a = np.array([acc], dtype=np.float64)
    lib().oracle_sq_rows(_ptr(rows), row0, rows.shape[0], n, _ptr(a))
    return float(a[0])


def sT(mat) -> float:
    mat = _mat(mat)
    return float(lib().oracle_sT(_ptr(mat), mat.shape[0]))


def between_unweighted(mat, grouping) -> float:
    mat = _mat(mat)
    g = _groupings(grouping, mat.shape[0])[0]
    g = np.ascontiguousarray(g)
    return float(lib().oracle_between_unweighted(_ptr(mat), mat.shape[0], _ptr(g)))


def F(sW_values, sT_value: float, n: int, k: int) -> np.ndarray:
    s = np.ascontiguousarray(np.atleast_1d(sW_values), dtype=np.float64)
    out = np.empty_like(s)
    lib().oracle_F(_ptr(s), s.shape[0], float(sT_value), int(n), int(k), _ptr(out))
    return out


def pvalue(F_obs: float, F_perm) -> float:
    f = np.ascontiguousarray(F_perm, dtype=np.float64)
    return float(lib().oracle_pvalue(float(F_obs), _ptr(f), f.shape[0]))


def pvalue_sW(sW_obs: float, sW_perm) -> float:
    s = np.ascontiguousarray(sW_perm, dtype=np.float64)
    return float(lib().oracle_pvalue_sW(float(sW_obs), _ptr(s), s.shape[0]))


def splitmix64_stream(state: int, count: int) -> list[int]:
    st = np.array([state], dtype=np.uint64)
    return [int(lib().oracle_splitmix64_next(_ptr(st))) for _ in range(count)]


def stream_start(seed: int, p: int) -> int:
    return int(lib().oracle_stream_start(seed, p))


def bounded(state: int, s: int, count: int) -> list[int]:
    st = np.array([state], dtype=np.uint64)
    return [int(lib().oracle_bounded(_ptr(st), s)) for _ in range(count)]


def permute(base, n_perms: int, seed: int, nthreads: int = 0) -> np.ndarray:
    """n_perms Fisher-Yates shuffles of base, int32 [n_perms, n]."""
    base = np.ascontiguousarray(base, dtype=np.int32)
    out = np.empty((n_perms, base.shape[0]), dtype=np.int32)
    lib().oracle_permute(_ptr(base), base.shape[0], n_perms, seed, _ptr(out), nthreads)
    return out


def count_rejections(n: int, n_perms: int, seed: int) -> int:
    """Draws discarded by the bounded draws of permute(base of length n, ...)
    (test helper: which inputs exercise a generator's rejection path)."""
    return int(lib().oracle_count_rejections(int(n), int(n_perms), int(seed) & 0xFFFFFFFFFFFFFFFF))


def group_sizes(grouping, k: int | None = None) -> np.ndarray:
    g = np.asarray(grouping)
    return np.bincount(g, minlength=k or 0)


def permanova(mat, grouping, n_perms: int, seed: int, nthreads: int = 0) -> dict:
    """The whole test: weights 1/n_g from the observed grouping, n_perms
    shuffles, s_W for the observed grouping and every shuffle, s_T, F, p."""
    mat = _mat(mat)
    n = mat.shape[0]
    grouping = np.ascontiguousarray(grouping, dtype=np.int32)
    sizes = group_sizes(grouping)
    k = int((sizes > 0).sum())
    inv = np.where(sizes > 0, 1.0 / np.maximum(sizes, 1), 0.0).astype(np.float64)
    perms = permute(grouping, n_perms, seed, nthreads)
    allg = np.vstack([grouping[None, :], perms])
    s = sW(mat, allg, inv, nthreads)
    t = sT(mat)
    f = F(s, t, n, k)
    return dict(sW_obs=float(s[0]), sW_perm=s[1:], sT=t, F_obs=float(f[0]), F_perm=f[1:],
                p=pvalue(float(f[0]), f[1:]), k=k, inv=inv, perms=perms)
