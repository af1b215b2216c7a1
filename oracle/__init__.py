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

# Relative tie tolerance of the p-value count (a reading of the permutation
# test of section 1): permutation q counts as at least as extreme as the
# observed grouping when s_W[q] <= s_W_obs + TIE_RTOL * |s_W_obs|.  Groupings
# whose statistics are equal in exact arithmetic (the same partition under
# other labels, or any grouping of a constant matrix) then tie whatever the
# FP64 summation order; 1e-10 sits far above FP64 rounding of s_W (~1e-13 at
# n = 10^5) and far below the spread of s_W across permutations.
TIE_RTOL = 1e-10


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, u64, f64, c_int = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                     ctypes.c_double, ctypes.c_int)
        L.oracle_group_sums.argtypes = [P, i64, i64, i64, P, i64, i32, P, c_int]
        L.oracle_group_sums.restype = c_int
        L.oracle_sW_from_sums.argtypes = [P, i64, i32, P, P]
        L.oracle_sW.argtypes = [P, i64, P, i64, i32, P, P, c_int]
        L.oracle_sW.restype = c_int
        L.oracle_sq_sum.argtypes = [P, i64, i64, i64, P]
        L.oracle_sT.argtypes = [P, i64]
        L.oracle_sT.restype = f64
        L.oracle_between_unweighted.argtypes = [P, i64, P]
        L.oracle_between_unweighted.restype = f64
        L.oracle_F.argtypes = [P, i64, f64, i64, i32, P]
        L.oracle_pvalue_F.argtypes = [f64, P, i64]
        L.oracle_pvalue_F.restype = f64
        L.oracle_pvalue.argtypes = [f64, P, i64, f64]
        L.oracle_pvalue.restype = f64
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
        L.oracle_pin_threads.argtypes = [P, c_int, c_int, c_int]
        L.oracle_pin_threads.restype = c_int
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
    if g.ndim != 2 or g.shape[1] != n:
        raise ValueError("groupings must have n columns")
    return g


def _k_of(g: np.ndarray, k: int | None) -> int:
    if k is None:
        k = int(g.max()) + 1 if g.size else 1
    if g.size and (int(g.min()) < 0 or int(g.max()) >= k):
        raise ValueError(f"labels must lie in [0, {k})")
    return int(k)


def _weights(inv, k: int) -> np.ndarray:
    w = np.ascontiguousarray(inv, dtype=np.float64).reshape(-1)
    if w.shape[0] < k:
        raise ValueError(f"need {k} weights, got {w.shape[0]}")
    return w


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def pin_threads(cpus, nthreads: int, one_each: bool) -> None:
    """CPU affinity of a team of nthreads (measurement helper): thread t on
    cpus[t] alone (one_each), else every thread on all of cpus."""
    arr = np.ascontiguousarray(cpus, dtype=np.int32)
    if lib().oracle_pin_threads(_ptr(arr), arr.shape[0], int(nthreads), int(bool(one_each))):
        raise OSError("sched_setaffinity failed")


def sW(mat, groupings, inv, nthreads: int = 0, k: int | None = None) -> np.ndarray:
    """s_W of every grouping row: the weighted within-group sums of squared
    distances (the quantity of section 2, Algorithm 1), FP64."""
    mat = _mat(mat)
    n = mat.shape[0]
    g = _groupings(groupings, n)
    k = _k_of(g, k)
    w = _weights(inv, k)
    out = np.zeros(g.shape[0], dtype=np.float64)
    if lib().oracle_sW(_ptr(mat), n, _ptr(g), g.shape[0], k, _ptr(w), _ptr(out), nthreads):
        raise RuntimeError("oracle_sW failed")
    return out


def new_group_sums(n_groupings: int, k: int) -> np.ndarray:
    """Zeroed compensated accumulators for group_sums: [groupings, k, 2]."""
    return np.zeros((n_groupings, k, 2), dtype=np.float64)


def group_sums(rows, row0: int, n: int, groupings, sums: np.ndarray, nthreads: int = 0) -> None:
    """Continue the within-group sums over matrix rows [row0, row0 + rows.shape[0])
    (so a matrix too large for the host can be fed in row blocks, in order)."""
    rows = np.ascontiguousarray(rows, dtype=np.float32)
    assert rows.ndim == 2 and rows.shape[1] == n
    g = _groupings(groupings, n)
    k = sums.shape[1]
    _k_of(g, k)
    assert sums.dtype == np.float64 and sums.flags.c_contiguous
    assert sums.shape == (g.shape[0], k, 2)
    if lib().oracle_group_sums(_ptr(rows), row0, rows.shape[0], n, _ptr(g), g.shape[0], k,
                               _ptr(sums), nthreads):
        raise RuntimeError("oracle_group_sums failed")


def sW_from_sums(sums: np.ndarray, inv) -> np.ndarray:
    """s_W = sum_c w_c S_c from group_sums' accumulators."""
    k = sums.shape[1]
    w = _weights(inv, k)
    out = np.zeros(sums.shape[0], dtype=np.float64)
    lib().oracle_sW_from_sums(_ptr(np.ascontiguousarray(sums)), sums.shape[0], k, _ptr(w),
                              _ptr(out))
    return out


def sq_sum(rows, row0: int, n: int, acc: np.ndarray) -> None:
    """Continue the compensated sum acc (2 doubles) of d^2 above the diagonal
    over matrix rows [row0, row0 + rows.shape[0]); s_T = acc.sum() / n."""
    rows = np.ascontiguousarray(rows, dtype=np.float32)
    assert acc.dtype == np.float64 and acc.shape == (2,)
    lib().oracle_sq_sum(_ptr(rows), row0, rows.shape[0], n, _ptr(acc))


def sT(mat) -> float:
    mat = _mat(mat)
    return float(lib().oracle_sT(_ptr(mat), mat.shape[0]))


def between_unweighted(mat, grouping) -> float:
    mat = _mat(mat)
    g = np.ascontiguousarray(_groupings(grouping, mat.shape[0])[0])
    return float(lib().oracle_between_unweighted(_ptr(mat), mat.shape[0], _ptr(g)))


def F(sW_values, sT_value: float, n: int, k: int) -> np.ndarray:
    s = np.ascontiguousarray(np.atleast_1d(sW_values), dtype=np.float64)
    out = np.empty_like(s)
    lib().oracle_F(_ptr(s), s.shape[0], float(sT_value), int(n), int(k), _ptr(out))
    return out


def pvalue_F(F_obs: float, F_perm) -> float:
    """Textbook count: (1 + #{F_q >= F_obs}) / (1 + P)."""
    f = np.ascontiguousarray(F_perm, dtype=np.float64)
    return float(lib().oracle_pvalue_F(float(F_obs), _ptr(f), f.shape[0]))


def pvalue(sW_obs: float, sW_perm, rtol: float = TIE_RTOL) -> float:
    """(1 + #{s_W[q] <= s_W_obs + rtol |s_W_obs|}) / (1 + P)."""
    s = np.ascontiguousarray(sW_perm, dtype=np.float64)
    return float(lib().oracle_pvalue(float(sW_obs), _ptr(s), s.shape[0], float(rtol)))


def splitmix64_stream(state: int, count: int) -> list[int]:
    st = np.array([state], dtype=np.uint64)
    return [int(lib().oracle_splitmix64_next(_ptr(st))) for _ in range(count)]


def stream_start(seed: int, p: int) -> int:
    m = (1 << 64) - 1
    return int(lib().oracle_stream_start(int(seed) & m, int(p) & m))


def bounded(state: int, s: int, count: int) -> list[int]:
    st = np.array([state], dtype=np.uint64)
    return [int(lib().oracle_bounded(_ptr(st), s)) for _ in range(count)]


def permute(base, n_perms: int, seed: int, nthreads: int = 0) -> np.ndarray:
    """n_perms Fisher-Yates shuffles of base, int32 [n_perms, n]."""
    base = np.ascontiguousarray(base, dtype=np.int32)
    out = np.empty((n_perms, base.shape[0]), dtype=np.int32)
    lib().oracle_permute(_ptr(base), base.shape[0], n_perms, int(seed) & 0xFFFFFFFFFFFFFFFF,
                         _ptr(out), nthreads)
    return out


def count_rejections(n: int, n_perms: int, seed: int) -> int:
    """Draws discarded by the bounded draws of permute(base of length n, ...)
    (test helper: which inputs exercise a generator's rejection path)."""
    return int(lib().oracle_count_rejections(int(n), int(n_perms), int(seed) & 0xFFFFFFFFFFFFFFFF))


def group_sizes(grouping, k: int | None = None) -> np.ndarray:
    g = np.asarray(grouping)
    return np.bincount(g, minlength=k or 0)


def permanova(mat, grouping, n_perms: int, seed: int, nthreads: int = 0,
              rtol: float = TIE_RTOL) -> dict:
    """The whole test: weights 1/n_g from the observed grouping, n_perms
    shuffles, s_W for the observed grouping and every shuffle, s_T, F, and p
    (tie tolerance rtol; p_F is the textbook count on F, without it)."""
    mat = _mat(mat)
    n = mat.shape[0]
    grouping = np.ascontiguousarray(grouping, dtype=np.int32)
    sizes = group_sizes(grouping)
    k = int((sizes > 0).sum())
    inv = np.where(sizes > 0, 1.0 / np.maximum(sizes, 1), 0.0).astype(np.float64)
    perms = permute(grouping, n_perms, seed, nthreads)
    allg = np.vstack([grouping[None, :], perms])
    s = sW(mat, allg, inv, nthreads, k=len(sizes))
    t = sT(mat)
    f = F(s, t, n, k)
    return dict(sW_obs=float(s[0]), sW_perm=s[1:], sT=t, F_obs=float(f[0]), F_perm=f[1:],
                p=pvalue(float(s[0]), s[1:], rtol), p_F=pvalue_F(float(f[0]), f[1:]), k=k,
                inv=inv, perms=perms)
