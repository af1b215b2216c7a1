"""Seeded synthetic inputs for PERMANOVA's within-group statistic.

This module only *produces inputs*: distance matrices, group sizes, base
labels and the per-group weights the caller passes in.  It holds none of the
statistic's arithmetic (no s_W, s_T, F, p-value and no permutation
generator), so both the FP64 oracle (``oracle/``) and the HIP library can take
their inputs from it without sharing any of the method.

The paper measures on a 25,145 x 25,145 Unweighted UniFrac matrix of the Earth
Microbiome Project (section 3).  That data is not available here; the
workloads below are synthetic stand-ins with the paper's sizes, value range
[0, 1], zero diagonal and exact symmetry.

Host generators (numpy) are defined here.  ``synth.device`` produces the same
matrices directly in device memory for sizes where a host copy is impractical
(n = 100,000 is 40 GB); the two are bit-identical by construction
(integer hashing, exactly representable values, sequential FP64 sums with
correctly rounded sqrt and division).
"""
from __future__ import annotations

import numpy as np

MASK64 = np.uint64(0xFFFFFFFFFFFFFFFF)
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def mix64(z):
    """SplitMix64 finaliser (Steele, Lea & Flood, OOPSLA 2014), vectorised.

    Accepts a Python int or a numpy uint64 array; arithmetic is modulo 2^64.
    """
    if isinstance(z, (int, np.integer)) and not isinstance(z, np.ndarray):
        m = (1 << 64) - 1
        z = int(z) & m
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
        return z ^ (z >> 31)
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


# --------------------------------------------------------------------------
# Distance matrices
# --------------------------------------------------------------------------

def uniform_entry_keys(rows: np.ndarray, cols: np.ndarray, n: int) -> np.ndarray:
    """Key of entry (i, j): min(i,j) * n + max(i,j), so the matrix is symmetric."""
    lo = np.minimum(rows, cols).astype(np.uint64)
    hi = np.maximum(rows, cols).astype(np.uint64)
    return lo * np.uint64(n) + hi


def uniform_values(keys: np.ndarray, seed: int) -> np.ndarray:
    """Hash-uniform value in (0, 1) for each key, exactly representable in fp32.

    h = mix64(key XOR mix64(seed)); value = (2 * (h >> 41) + 1) * 2^-24, an odd
    multiple of 2^-24 below 1 (at most 24 significant bits).
    """
    s = np.uint64(mix64(int(seed)))
    h = mix64(keys.astype(np.uint64) ^ s)
    m = ((h >> np.uint64(41)) << np.uint64(1)) | np.uint64(1)
    return (m.astype(np.float64) * 2.0 ** -24).astype(np.float32)


def uniform_matrix(n: int, seed: int, rows: slice | None = None) -> np.ndarray:
    """Symmetric n x n fp32 matrix, zero diagonal, entries hash-uniform in (0, 1).

    ``rows`` selects a block of rows (so very large matrices can be produced in
    pieces); the full matrix is returned when it is None.
    """
    r0, r1 = (0, n) if rows is None else (rows.start or 0, rows.stop)
    ri = np.arange(r0, r1, dtype=np.int64)[:, None]
    cj = np.arange(n, dtype=np.int64)[None, :]
    out = uniform_values(uniform_entry_keys(ri, cj, n), seed)
    out[ri == cj] = 0.0
    return out


def euclid_points(n: int, seed: int, dims: int = 32) -> np.ndarray:
    """n seeded N(0, 1) points in ``dims`` dimensions (FP64)."""
    return np.random.default_rng(seed).standard_normal((n, dims))


def _pair_dist(xa: np.ndarray, xb: np.ndarray) -> np.ndarray:
    """FP64 Euclidean distances, squared differences summed in dimension order."""
    acc = np.zeros((xa.shape[0], xb.shape[0]), dtype=np.float64)
    for d in range(xa.shape[1]):
        t = xa[:, d][:, None] - xb[:, d][None, :]
        acc += t * t
    return np.sqrt(acc)


def euclid_matrix(n: int, seed: int, dims: int = 32, points: np.ndarray | None = None,
                  block: int = 1024) -> np.ndarray:
    """Euclidean distances between seeded points, divided by the largest one, fp32.

    d_ij = RN_fp32( ||x_i - x_j|| / max_{a != b} ||x_a - x_b|| ), FP64 before
    the final rounding; symmetric with an exactly zero diagonal.
    """
    x = euclid_points(n, seed, dims) if points is None else points
    dmax = 0.0
    for a in range(0, n, block):
        for b in range(a, n, block):
            dmax = max(dmax, float(_pair_dist(x[a:a + block], x[b:b + block]).max()))
    out = np.empty((n, n), dtype=np.float32)
    for a in range(0, n, block):
        d = _pair_dist(x[a:a + block], x)
        out[a:a + block] = (d / dmax).astype(np.float32)
    np.fill_diagonal(out, 0.0)
    return out


def dyadic_matrix(n: int, seed: int, levels: int = 16) -> np.ndarray:
    """Symmetric matrix of 4-bit dyadic values m/16 (m in 0..15), zero diagonal.

    d^2 = m^2/256 has at most 8 significant bits, so it is exact in BF16, FP16,
    FP32 and FP64, and short sums of such values are exact too.
    """
    rng = np.random.default_rng(seed)
    m = rng.integers(0, levels, size=(n, n))
    m = np.triu(m, 1)
    m = m + m.T
    return (m.astype(np.float64) / levels).astype(np.float32)


# --------------------------------------------------------------------------
# Groups
# --------------------------------------------------------------------------

def dirichlet_sizes(n: int, k: int, min_size: int, seed: int) -> list[int]:
    """Uneven group sizes: min_size + floor(prop_g * (n - k*min_size)).

    prop ~ Dirichlet(1, ..., 1) from ``default_rng(seed)``; the remainder goes
    one each to the groups with the largest fractional parts (ties to lower g).
    """
    if k * min_size > n:
        raise ValueError("k * min_size exceeds n")
    prop = np.random.default_rng(seed).dirichlet(np.ones(k))
    free = n - k * min_size
    raw = prop * free
    base = np.floor(raw).astype(np.int64)
    rem = free - int(base.sum())
    frac = raw - base
    order = sorted(range(k), key=lambda g: (-frac[g], g))
    for g in order[:rem]:
        base[g] += 1
    return [int(min_size + b) for b in base]


def base_labels(sizes) -> np.ndarray:
    """Contiguous blocks: sizes[0] objects of group 0, then sizes[1] of group 1, ..."""
    return np.repeat(np.arange(len(sizes), dtype=np.int32), np.asarray(sizes, dtype=np.int64))


def inv_group_sizes(sizes) -> np.ndarray:
    """Per-group weight 1/n_g in FP64 (correctly rounded division)."""
    return 1.0 / np.asarray(sizes, dtype=np.float64)


# --------------------------------------------------------------------------
# The benchmark workloads (seeds: matrix 1000+c, sizes 2000+c, perms 3000+c)
# --------------------------------------------------------------------------

CONFIGS = {
    0: dict(name="n1000_k4_P999_uniform", n=1000, sizes=[100, 200, 300, 400], n_perms=999,
            matrix="uniform"),
    1: dict(name="n10000_k5_P9999_euclid32", n=10_000, sizes=[1000, 1500, 2000, 2500, 3000],
            n_perms=9999, matrix="euclid"),
    2: dict(name="n25000_k10_P3999_euclid32", n=25_000, k=10, min_size=500, n_perms=3999,
            matrix="euclid"),
    3: dict(name="n100000_k3_P999_uniform", n=100_000, sizes=[20_000, 30_000, 50_000],
            n_perms=999, matrix="uniform"),
}


def config(c: int) -> dict:
    """Resolved workload c: n, sizes, k, n_perms, matrix kind and the three seeds."""
    cfg = dict(CONFIGS[c])
    cfg["matrix_seed"] = 1000 + c
    cfg["sizes_seed"] = 2000 + c
    cfg["perm_seed"] = 3000 + c
    if "sizes" not in cfg:
        cfg["sizes"] = dirichlet_sizes(cfg["n"], cfg["k"], cfg["min_size"], cfg["sizes_seed"])
    cfg["k"] = len(cfg["sizes"])
    assert sum(cfg["sizes"]) == cfg["n"]
    return cfg


def host_matrix(cfg: dict) -> np.ndarray:
    """Host copy of a workload's matrix (only sensible for n up to ~25k)."""
    if cfg["matrix"] == "uniform":
        return uniform_matrix(cfg["n"], cfg["matrix_seed"])
    return euclid_matrix(cfg["n"], cfg["matrix_seed"])


def serving_requests(count: int = 64, rate: float = 4.0, seed: int = 4000) -> list[dict]:
    """The serving trace: Poisson arrivals, per-request n, k, sizes and permutations.

    n in {1k, 2k, 5k, 10k, 20k}, k uniform in 2..12 with Dirichlet sizes
    (min = max(2, n // (4k))), permutations in {999, 9999}; request i draws its
    own parameters from seed 5000 + i.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(count):
        r = np.random.default_rng(5000 + i)
        n = int(r.choice([1000, 2000, 5000, 10_000, 20_000]))
        k = int(r.integers(2, 13))
        min_size = max(2, n // (4 * k))
        sizes = dirichlet_sizes(n, k, min_size, 5000 + i)
        n_perms = int(r.choice([999, 9999]))
        reqs.append(dict(id=i, arrival=float(t[i]), n=n, k=k, sizes=sizes, n_perms=n_perms,
                         matrix_seed=5000 + i, perm_seed=5000 + i))
    return reqs
