"""Seeded synthetic graph inputs for the tests and the benchmark.

This module only generates inputs: R-MAT graphs, 2D / 3D random geometric
graphs, and seeded integer weights. It contains none of the clustering,
contraction or compression arithmetic, so the CPU oracle and the GPU library
can both consume its graphs without sharing code.

The heavy lifting is in ``synth.c`` (OpenMP C, built into ``libsynth.so`` by
``build()``). Every draw comes from a counter-indexed SplitMix64 stream, so the
output is identical for any thread count.

Workload recipes (sizes, radii, R-MAT parameters) follow the shapes of the
paper's synthetic families (random geometric and power-law graphs, Section VI
"Instances") at the sizes the benchmark configurations name.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


class _CSR(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("two_m", ctypes.c_uint64),
        ("xadj", ctypes.POINTER(ctypes.c_uint64)),
        ("adjncy", ctypes.POINTER(ctypes.c_int32)),
    ]


def build() -> str:
    """Compile libsynth.so (always recompiles)."""
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.synth_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(_CSR)]
    lib.synth_rmat.restype = ctypes.c_int
    lib.synth_rgg.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                              ctypes.POINTER(_CSR)]
    lib.synth_rgg.restype = ctypes.c_int
    lib.synth_free.argtypes = [ctypes.POINTER(_CSR)]
    lib.synth_copy.argtypes = [ctypes.POINTER(_CSR), ctypes.c_void_p, ctypes.c_void_p]
    lib.synth_weights.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                  ctypes.c_void_p]
    lib.synth_edge_weights.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p]
    lib.synth_unit.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.synth_unit.restype = ctypes.c_double
    lib.synth_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.synth_draw.restype = ctypes.c_uint64
    _lib = lib
    return lib


@dataclass
class Graph:
    """Symmetric CSR: neighbours of u are adjncy[xadj[u]:xadj[u+1]], sorted."""
    n: int
    xadj: np.ndarray          # uint64[n+1]
    adjncy: np.ndarray        # int32[2m]
    adjwgt: np.ndarray | None = None  # int32[2m] or None (unit)
    vwgt: np.ndarray | None = None    # int32[n] or None (unit)
    name: str = ""

    @property
    def two_m(self) -> int:
        return int(self.xadj[-1])


def _take(csr: _CSR) -> tuple[np.ndarray, np.ndarray]:
    lib = _load()
    n, two_m = int(csr.n), int(csr.two_m)
    xadj = np.empty(n + 1, dtype=np.uint64)
    adj = np.empty(two_m, dtype=np.int32)
    lib.synth_copy(ctypes.byref(csr), xadj.ctypes.data, adj.ctypes.data)
    lib.synth_free(ctypes.byref(csr))
    return xadj, adj


def rmat(scale: int, nsamples: int, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, n_limit: int = 0, name: str = "") -> Graph:
    """R-MAT graph over 2^scale IDs (or n_limit IDs, rejecting larger endpoints)."""
    lib = _load()
    csr = _CSR()
    rc = lib.synth_rmat(scale, nsamples, a, b, c, seed, n_limit, ctypes.byref(csr))
    if rc != 0:
        raise RuntimeError(f"synth_rmat failed ({rc})")
    xadj, adj = _take(csr)
    return Graph(len(xadj) - 1, xadj, adj, name=name or f"rmat{scale}")


def rgg(dim: int, n: int, r: float, seed: int = 1, name: str = "") -> Graph:
    """Random geometric graph in the unit square (dim=2) or cube (dim=3)."""
    lib = _load()
    csr = _CSR()
    rc = lib.synth_rgg(dim, n, r, seed, ctypes.byref(csr))
    if rc != 0:
        raise RuntimeError(f"synth_rgg failed ({rc})")
    xadj, adj = _take(csr)
    return Graph(n, xadj, adj, name=name or f"rgg{dim}d")


def rgg_radius(dim: int, n: int, avg_deg: float) -> float:
    """Radius giving the requested expected degree away from the boundary."""
    if dim == 2:
        return math.sqrt(avg_deg / (math.pi * (n - 1)))
    return (3.0 * avg_deg / (4.0 * math.pi * (n - 1))) ** (1.0 / 3.0)


def vertex_weights(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    _load().synth_weights(n, lo, hi, seed, out.ctypes.data)
    return out


def edge_weights(g: Graph, lo: int, hi: int, seed: int) -> np.ndarray:
    """Seeded weights that are symmetric: w(u,v) == w(v,u)."""
    out = np.empty(g.two_m, dtype=np.int32)
    _load().synth_edge_weights(g.n, g.xadj.ctypes.data, g.adjncy.ctypes.data, lo, hi, seed,
                               out.ctypes.data)
    return out


def unit(seed: int, k: int) -> float:
    return float(_load().synth_unit(seed, k))


def draw(seed: int, k: int) -> int:
    return int(_load().synth_draw(seed, k))


# ----------------------------------------------------------------- recipes --

def rgg2d_16k(seed: int = 1) -> Graph:
    """2D RGG, n = 16384, radius for expected degree 8, unit weights."""
    n = 16384
    return rgg(2, n, rgg_radius(2, n, 8.0), seed, name="rgg2d-n16384")


def rmat_scale(scale: int, edge_factor: int, seed: int = 1) -> Graph:
    """R-MAT (0.57, 0.19, 0.19, 0.05), edge_factor * 2^scale samples, no ID permutation."""
    return rmat(scale, edge_factor << scale, 0.57, 0.19, 0.19, seed,
                name=f"rmat-s{scale}-ef{edge_factor}")


def rgg3d(n: int, avg_deg: float = 27.0, seed: int = 1) -> Graph:
    return rgg(3, n, rgg_radius(3, n, avg_deg), seed, name=f"rgg3d-n{n}")


def random_small(n: int, p_edge: float, seed: int) -> Graph:
    """Erdos-Renyi-style small graph from a pair-indexed stream (for exhaustive tests)."""
    edges = []
    k = 0
    for u in range(n):
        for v in range(u + 1, n):
            if unit(seed, k) < p_edge:
                edges.append((u, v))
            k += 1
    return from_edges(n, edges)


def from_edges(n: int, edges, weights=None) -> Graph:
    """Symmetric CSR from an undirected edge list (u != v, no duplicates);
    every neighbourhood sorted by (neighbour, weight)."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    w = np.ones(len(e), dtype=np.int64) if weights is None else np.asarray(weights, dtype=np.int64)
    src = np.concatenate([e[:, 0], e[:, 1]])
    dst = np.concatenate([e[:, 1], e[:, 0]])
    ww = np.concatenate([w, w])
    order = np.lexsort((ww, dst, src))
    xadj = np.zeros(n + 1, dtype=np.uint64)
    xadj[1:] = np.cumsum(np.bincount(src, minlength=n)[:n], dtype=np.uint64)
    g = Graph(n, xadj, dst[order].astype(np.int32))
    if weights is not None:
        g.adjwgt = ww[order].astype(np.int32)
    return g


def batch_recipe(count: int = 512, base_seed: int = 1000):
    """Sizes and kinds of the many-graph batch: n log-uniform in [1e3, 1e6],
    RGG-2D (degree 8) or R-MAT (edge factor 8..16) by a fair coin."""
    out = []
    for i in range(count):
        s = base_seed + i
        n = int(math.exp(math.log(1e3) + unit(s, 0) * (math.log(1e6) - math.log(1e3))))
        if unit(s, 1) < 0.5:
            out.append(("rgg2d", n, 8, s))
        else:
            ef = 8 + int(draw(s, 2) % 9)
            out.append(("rmat", n, ef, s))
    return out


def batch_graph(kind: str, n: int, param: int, seed: int) -> Graph:
    if kind == "rgg2d":
        return rgg(2, n, rgg_radius(2, n, float(param)), seed, name=f"rgg2d-n{n}-s{seed}")
    scale = max(1, math.ceil(math.log2(n)))
    return rmat(scale, param * n, 0.57, 0.19, 0.19, seed, n_limit=n, name=f"rmat-n{n}-ef{param}-s{seed}")


def serve_pool(count: int = 24, base_seed: int = 5000):
    """Resident graphs of the serving workload: directed edge counts
    log-uniform in [1e4, 1e8] (the first two graphs at the two ends of the
    range), RGG-2D (degree 8) or R-MAT (edge factor 8..16) by a fair coin;
    entries as in batch_recipe."""
    out = []
    for i in range(count):
        s = base_seed + i
        u = 0.0 if i == 0 else 1.0 if i == 1 else unit(s, 0)
        m2 = math.exp(math.log(1e4) + u * (math.log(1e8) - math.log(1e4)))
        if unit(s, 1) < 0.5:
            out.append(("rgg2d", max(64, int(m2 / 8)), 8, s))
        else:
            ef = 8 + int(draw(s, 2) % 9)
            out.append(("rmat", max(64, int(m2 / (2 * ef))), ef, s))
    return out


def serve_trace(rate: float, count: int, pool_size: int, seed: int = 7):
    """Arrival trace of the serving workload: (arrival seconds, pool graph,
    job seed) with exponential gaps at `rate` per second."""
    t = 0.0
    out = []
    for i in range(count):
        u = unit(seed, 3 * i)
        t += -math.log(max(u, 1e-300)) / rate
        out.append((t, int(draw(seed, 3 * i + 1) % pool_size), int(draw(seed, 3 * i + 2) % 1000003)))
    return out
