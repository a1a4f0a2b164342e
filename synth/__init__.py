"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package draws graphs and query sources only. It contains none of the
similarity method's arithmetic, so the oracle and the GPU library can both
read its output without sharing any method code.

The graphs stand in for the paper's real datasets (Sec. 5, Tables 1 and 2),
which are not available here. Their shapes follow the paper's user-item and
click graphs: power-law degrees on both sides, many low-degree nodes, a few
hubs, positive edge weights.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chunglu.c")
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C sampler into ``libsynth.so`` next to this file."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_chung_lu.restype = ctypes.c_int
        lib.synth_chung_lu.argtypes = [
            ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
            ctypes.c_int32, ctypes.c_uint64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


WEIGHT_KINDS = {"int10": 0, "lognormal": 1}


@dataclass(frozen=True)
class EdgeList:
    n_u: int
    n_v: int
    u: np.ndarray  # int32[n_e]
    v: np.ndarray  # int32[n_e]
    w: np.ndarray  # float64[n_e]; values exactly representable in FP32

    @property
    def n_e(self) -> int:
        return int(self.u.shape[0])

    def degrees_u(self) -> np.ndarray:
        return np.bincount(self.u, minlength=self.n_u).astype(np.int64)

    def degrees_v(self) -> np.ndarray:
        return np.bincount(self.v, minlength=self.n_v).astype(np.int64)


def chung_lu(n_u: int, n_v: int, n_e: int, gamma: float, weights: str, seed: int) -> EdgeList:
    """Bipartite Chung-Lu graph with exactly ``n_e`` distinct (u, v) pairs."""
    lib = _load()
    u = np.empty(n_e, dtype=np.int32)
    v = np.empty(n_e, dtype=np.int32)
    w = np.empty(n_e, dtype=np.float64)
    rc = lib.synth_chung_lu(n_u, n_v, n_e, gamma, WEIGHT_KINDS[weights], seed,
                            u.ctypes.data, v.ctypes.data, w.ctypes.data)
    if rc != 0:
        raise ValueError(f"synth_chung_lu failed with code {rc}")
    return EdgeList(n_u, n_v, u, v, w)


def sample_sources(el: EdgeList, n: int, mode: str, seed: int) -> np.ndarray:
    """Query sources among non-isolated U nodes.

    mode 'uniform': distinct nodes, uniform (the paper's 100 random queries,
    Sec. 5.4 settings). mode 'degree': distinct nodes with probability
    proportional to degree, so frontiers differ widely between sources.
    """
    deg = el.degrees_u()
    cand = np.nonzero(deg > 0)[0]
    rng = np.random.default_rng(seed)
    if n > cand.size:
        raise ValueError("more sources requested than non-isolated U nodes")
    if mode == "uniform":
        pick = rng.choice(cand.size, size=n, replace=False)
    elif mode == "degree":
        p = deg[cand].astype(np.float64)
        pick = rng.choice(cand.size, size=n, replace=False, p=p / p.sum())
    else:
        raise ValueError(mode)
    return cand[pick].astype(np.int32)


@dataclass(frozen=True)
class Workload:
    """A named synthetic workload: graph recipe plus query recipe."""
    name: str
    n_u: int
    n_v: int
    n_e: int
    gamma: float
    weights: str
    graph_seed: int
    n_sources: int
    source_mode: str
    source_seed: int
    alpha: float
    eps: float
    k: int
    dtype: str  # arithmetic type of the GPU path: "f64" or "f32"

    def graph(self) -> EdgeList:
        return chung_lu(self.n_u, self.n_v, self.n_e, self.gamma, self.weights, self.graph_seed)

    def sources(self, el: EdgeList) -> np.ndarray:
        return sample_sources(el, self.n_sources, self.source_mode, self.source_seed)


# DBLP-sized graph (Table 2 scale), FP64 single-source queries.
SMALL = Workload("cl2.2_2kx3k_20k_int10", 2000, 3000, 20000, 2.2, "int10", 2313,
                 16, "uniform", 7001, 0.15, 1e-7, 50, "f64")
# Last.fm-sized graph (Table 2 scale), 64 FP32 sources run together.
MEDIUM = Workload("cl2.1_1Mx2M_20M_lognormal", 1_000_000, 2_000_000, 20_000_000, 2.1,
                  "lognormal", 2314, 64, "uniform", 7002, 0.15, 1e-6, 100, "f32")
# 100M-edge graph, 1024 degree-proportional FP32 sources.
LARGE = Workload("cl2.1_5Mx10M_100M_lognormal", 5_000_000, 10_000_000, 100_000_000, 2.1,
                 "lognormal", 2315, 1024, "degree", 7003, 0.15, 1e-6, 100, "f32")

WORKLOADS = {w.name: w for w in (SMALL, MEDIUM, LARGE)}
