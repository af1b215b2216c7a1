"""Shared helpers for the GPU tests: building/loading the library, inputs on
both sides, error measures.  Inputs come from ``synth`` (generators) and
expected values from ``oracle`` only."""
from __future__ import annotations

import os

import numpy as np

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_build_module():
    """The build script, loaded by path (importing the package needs the
    library it builds)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "pstat_build", os.path.join(ROOT, "paper_2505_04556_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def load_pstat():
    lib = os.path.join(ROOT, "paper_2505_04556_amd", "libpstat.so")
    slib = os.path.join(ROOT, "synth", "libsynth.so")
    if not (os.path.exists(lib) and os.path.exists(slib)):
        load_build_module().build_all()
    import paper_2505_04556_amd as pstat
    return pstat


def problem(n, sizes, P, mseed=1, pseed=2, matrix="uniform"):
    """Host inputs: matrix, base labels, P oracle permutations, weights."""
    if matrix == "uniform":
        D = synth.uniform_matrix(n, mseed)
    elif matrix == "dyadic":
        D = synth.dyadic_matrix(n, mseed)
    else:
        D = synth.euclid_matrix(n, mseed)
    base = synth.base_labels(sizes)
    perms = oracle.permute(base, P, pseed) if P > 0 else np.zeros((0, n), np.int32)
    return D, base, perms, synth.inv_group_sizes(sizes)


def to_dev(*arrays, device="cuda"):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in arrays]


def max_rel(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.maximum(np.abs(ref), 1e-300)
    return float(np.max(np.abs(got - ref) / den)) if ref.size else 0.0


# Stated accuracy of each path against the FP64 oracle (relative, per s_W).
# FP32 and split-BF16 meet the 1e-5 bar; plain BF16/FP16 carry their input
# rounding (2^-9 and 2^-11 per element, worst case when all errors align).
TOL = {"plain_f32": 1e-5, "plain_f64": 1e-12, "mfma_split_bf16": 1e-5, "mfma_split3_bf16": 1e-5,
       "mfma_f16": 2 ** -10, "mfma_bf16": 2 ** -8}
