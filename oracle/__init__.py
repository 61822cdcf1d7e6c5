"""CPU ORACLE — test infrastructure only.

Plain, slow, obviously correct reference implementations of what the GPU
library computes (see ``oracle.c`` for the rules and the paper passages each
function follows). Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package. The GPU library never
loads it and shares no code with it.

The C part is built into ``liboracle.so`` by :func:`build` (gcc, OpenMP).
The coarsening loop and the multilevel partition driver are plain Python on
top of the C cluster / refine / contract calls; projection, block weights and
the affinities of Section V are numpy written out from their definitions.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, ENOMEM, EOVERFLOW, EFORMAT = 0, -1, -2, -3, -4
CHUNK_THRESHOLD = 10000
CHUNK_LEN = 1000

_P = ctypes.c_void_p


class _Stats(ctypes.Structure):
    _fields_ = [("rounds_run", ctypes.c_int32),
                ("proposals", ctypes.c_int64 * 64),
                ("moves", ctypes.c_int64 * 64)]


def build() -> str:
    """Compile liboracle.so (always recompiles)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", _SRC,
           "-o", _LIB_PATH + ".tmp"]
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
    lib.orc_varint_put.argtypes = [_P, ctypes.c_uint64]
    lib.orc_varint_put.restype = ctypes.c_size_t
    lib.orc_varint_get.argtypes = [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64),
                                   ctypes.POINTER(ctypes.c_uint64)]
    lib.orc_zigzag.argtypes = [ctypes.c_int64]
    lib.orc_zigzag.restype = ctypes.c_uint64
    lib.orc_unzigzag.argtypes = [ctypes.c_uint64]
    lib.orc_unzigzag.restype = ctypes.c_int64
    lib.orc_compress_bound.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int]
    lib.orc_compress_bound.restype = ctypes.c_uint64
    lib.orc_compress.argtypes = [ctypes.c_int32, _P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_uint64)]
    lib.orc_decompress.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int, _P, _P, _P, _P, _P]
    lib.orc_compress_ex.argtypes = [ctypes.c_int32, _P, _P, _P, ctypes.c_int, _P, _P, ctypes.POINTER(ctypes.c_uint64)]
    lib.orc_decompress_ex.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, _P, _P, _P, _P,
                                      _P]
    lib.orc_tiebreak_key.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
    lib.orc_tiebreak_key.restype = ctypes.c_uint64
    lib.orc_lp_cluster.argtypes = [ctypes.c_int32, _P, _P, _P, _P, ctypes.c_int64, ctypes.c_int32,
                                   ctypes.c_uint64, _P, ctypes.POINTER(_Stats)]
    lib.orc_lp_cluster_sub.argtypes = [ctypes.c_int32, _P, _P, _P, _P, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_uint64, _P, ctypes.POINTER(_Stats)]
    lib.orc_lp_rounds_from.argtypes = [ctypes.c_int32, _P, _P, _P, _P, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_uint64, _P, ctypes.POINTER(_Stats)]
    lib.orc_lp_cluster_async.argtypes = [ctypes.c_int32, _P, _P, _P, _P, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.c_uint64, _P, ctypes.POINTER(_Stats)]
    lib.orc_lp_refine.argtypes = [ctypes.c_int32, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, _P, ctypes.POINTER(_Stats)]
    lib.orc_initial_partition.argtypes = [ctypes.c_int32, _P, ctypes.c_int32, _P]
    lib.orc_subround.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.orc_subround.restype = ctypes.c_uint32
    lib.orc_lp_proposals.argtypes = [ctypes.c_int32, _P, _P, _P, _P, _P, _P, ctypes.c_int64,
                                     ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, _P, _P, _P]
    lib.orc_contract.argtypes = [ctypes.c_int32, _P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                 ctypes.POINTER(_P), _P]
    lib.orc_free.argtypes = [_P]
    lib.orc_edge_cut.argtypes = [ctypes.c_int32, _P, _P, _P, _P]
    lib.orc_edge_cut.restype = ctypes.c_int64
    _lib = lib
    return lib


def set_threads(k: int) -> None:
    """OpenMP thread count of the rating loop (results do not depend on it)."""
    lib = ctypes.CDLL(None)
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(k))
    except OSError:
        pass
    del lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Args:
    """Converted copies of array arguments, kept alive for one C call (a
    pointer taken from a temporary copy would dangle once the copy is freed)."""

    def __init__(self):
        self._keep = []

    def __call__(self, a, dtype):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dtype)
        self._keep.append(a)
        return a.ctypes.data


def _arr(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------- codec ----

def varint(x: int) -> bytes:
    buf = (ctypes.c_uint8 * 16)()
    k = _load().orc_varint_put(buf, x)
    return bytes(buf[:k])


def varint_decode(b: bytes) -> tuple[int, int]:
    """(value, length) of the VarInt at the start of b; raises on a bad one."""
    buf = (ctypes.c_uint8 * max(1, len(b))).from_buffer_copy(b if b else b"\0")
    pos, val = ctypes.c_uint64(0), ctypes.c_uint64(0)
    if not _load().orc_varint_get(buf, len(b), ctypes.byref(pos), ctypes.byref(val)):
        raise ValueError("malformed VarInt")
    return int(val.value), int(pos.value)


def zigzag(x: int) -> int:
    return int(_load().orc_zigzag(x))


def unzigzag(z: int) -> int:
    return int(_load().orc_unzigzag(z))


def compress(n: int, xadj, adjncy, adjwgt=None, intervals: bool = False) -> tuple[np.ndarray, np.ndarray]:
    """(offs uint64[n+1], bytes uint8[...]) of the compressed neighbourhoods
    (gap encoding, plus interval encoding if `intervals`)."""
    lib = _load()
    xadj = _arr(xadj, np.uint64)
    adjncy = _arr(adjncy, np.int32)
    adjwgt = _arr(adjwgt, np.int32)
    two_m = int(xadj[-1])
    bound = int(lib.orc_compress_bound(n, two_m, adjwgt is not None))
    offs = np.empty(n + 1, dtype=np.uint64)
    out = np.empty(bound, dtype=np.uint8)
    nb = ctypes.c_uint64(0)
    rc = lib.orc_compress_ex(n, _ptr(xadj), _ptr(adjncy), _ptr(adjwgt), int(bool(intervals)), _ptr(offs), _ptr(out),
                             ctypes.byref(nb))
    if rc != OK:
        raise RuntimeError(f"orc_compress: {rc}")
    return offs, out[: nb.value].copy()


def decompress(n: int, two_m: int, weighted: bool, offs, data, intervals: bool = False):
    """(xadj, adjncy, adjwgt or None); raises ValueError on a malformed stream."""
    lib = _load()
    offs = _arr(offs, np.uint64)
    data = _arr(data, np.uint8)
    xadj = np.empty(n + 1, dtype=np.uint64)
    adjncy = np.empty(max(two_m, 1), dtype=np.int32)
    adjwgt = np.empty(max(two_m, 1), dtype=np.int32) if weighted else None
    rc = lib.orc_decompress_ex(n, two_m, int(weighted), int(bool(intervals)), _ptr(offs), _ptr(data), _ptr(xadj),
                               _ptr(adjncy), _ptr(adjwgt))
    if rc == EFORMAT:
        raise ValueError("malformed compressed graph")
    if rc != OK:
        raise RuntimeError(f"orc_decompress: {rc}")
    return xadj, adjncy[:two_m], (adjwgt[:two_m] if weighted else None)


# ------------------------------------------------------- clustering ----

def tiebreak_key(seed: int, rnd: int, c: int) -> int:
    return int(_load().orc_tiebreak_key(seed, rnd, c))


@dataclass
class LPStats:
    rounds_run: int
    proposals: list
    moves: list


def subround(u: int, S: int) -> int:
    """Sub-round of vertex u among S (fixed for a whole call)."""
    return int(_load().orc_subround(u, S))


def lp_cluster(g, cap: int, rounds: int, seed: int, subrounds: int = 1):
    """Labels (int32[n]) of synchronous size-constrained LP, plus per-round stats.
    With subrounds = S > 1 every round is split into S sub-rounds over the
    vertices of each sub-round (see orc_lp_cluster_sub)."""
    A = _Args()
    lib = _load()
    labels = np.empty(max(g.n, 1), dtype=np.int32)
    st = _Stats()
    rc = lib.orc_lp_cluster_sub(g.n, A(g.xadj, np.uint64), A(g.adjncy, np.int32),
                                A(g.adjwgt, np.int32), A(g.vwgt, np.int32), cap, rounds,
                                subrounds, seed, _ptr(labels), ctypes.byref(st))
    if rc != OK:
        raise ValueError(f"orc_lp_cluster: {rc}")
    k = min(st.rounds_run, 64)
    return labels[: g.n], LPStats(st.rounds_run, list(st.proposals[:k]), list(st.moves[:k]))


def lp_rounds_from(g, cap: int, seed: int, labels, first_round: int, rounds: int = 1):
    """Synchronous LP rounds first_round .. first_round + rounds - 1 resumed
    from `labels` (a clustering a previous call produced); new labels and the
    statistics of these rounds. Rounds 0..R-1 run in pieces give the labels of
    lp_cluster(g, cap, R, seed)."""
    A = _Args()
    lib = _load()
    out = np.array(labels, dtype=np.int32, copy=True)
    if out.shape != (g.n,):
        raise ValueError("labels must hold one label per vertex")
    st = _Stats()
    rc = lib.orc_lp_rounds_from(g.n, A(g.xadj, np.uint64), A(g.adjncy, np.int32), A(g.adjwgt, np.int32),
                                A(g.vwgt, np.int32), cap, first_round, rounds, seed, _ptr(out), ctypes.byref(st))
    if rc != OK:
        raise ValueError(f"orc_lp_rounds_from: {rc}")
    k = min(st.rounds_run, 64)
    return out, LPStats(st.rounds_run, list(st.proposals[:k]), list(st.moves[:k]))


def lp_cluster_async(g, cap: int, rounds: int, seed: int):
    """The paper's asynchronous LP (sequential, random vertex order per round,
    moves applied at once) as a quality reference; labels and per-round moves."""
    A = _Args()
    lib = _load()
    labels = np.empty(max(g.n, 1), dtype=np.int32)
    st = _Stats()
    rc = lib.orc_lp_cluster_async(g.n, A(g.xadj, np.uint64), A(g.adjncy, np.int32),
                                  A(g.adjwgt, np.int32), A(g.vwgt, np.int32), cap, rounds,
                                  seed, _ptr(labels), ctypes.byref(st))
    if rc != OK:
        raise ValueError(f"orc_lp_cluster_async: {rc}")
    k = min(st.rounds_run, 64)
    return labels[: g.n], LPStats(st.rounds_run, list(st.proposals[:k]), list(st.moves[:k]))


def lp_proposals(g, C0, W0, cap: int, seed: int, rnd: int, vertices):
    """Best move (target or -1, gain) of each listed vertex under snapshot (C0, W0)."""
    A = _Args()
    lib = _load()
    vertices = _arr(vertices, np.int32)
    tgt = np.empty(len(vertices), dtype=np.int32)
    gain = np.empty(len(vertices), dtype=np.int64)
    C0 = _arr(C0, np.int32)
    W0 = _arr(W0, np.int64)
    rc = lib.orc_lp_proposals(g.n, A(g.xadj, np.uint64), A(g.adjncy, np.int32),
                              A(g.adjwgt, np.int32), A(g.vwgt, np.int32), _ptr(C0),
                              _ptr(W0), cap, seed, rnd, len(vertices), _ptr(vertices), _ptr(tgt),
                              _ptr(gain))
    if rc != OK:
        raise RuntimeError(f"orc_lp_proposals: {rc}")
    return tgt, gain


@dataclass
class Coarse:
    n: int
    xadj: np.ndarray
    adjncy: np.ndarray
    adjwgt: np.ndarray
    vwgt: np.ndarray

    @property
    def two_m(self) -> int:
        return int(self.xadj[-1])


def contract(g, labels):
    """(coarse graph, map int32[n]); raises OverflowError on a coarse weight > INT32_MAX."""
    A = _Args()
    lib = _load()
    labels = _arr(labels, np.int32)
    m = np.empty(max(g.n, 1), dtype=np.int32)
    nc = ctypes.c_int32(0)
    px, pa, pw, pv = _P(), _P(), _P(), _P()
    rc = lib.orc_contract(g.n, A(g.xadj, np.uint64), A(g.adjncy, np.int32),
                          A(g.adjwgt, np.int32), A(g.vwgt, np.int32), _ptr(labels),
                          ctypes.byref(nc), ctypes.byref(px), ctypes.byref(pa), ctypes.byref(pw),
                          ctypes.byref(pv), _ptr(m))
    if rc == EINVAL:
        raise ValueError("labels out of range")
    if rc == ENOMEM:
        raise MemoryError("orc_contract")
    k = nc.value
    xadj = np.ctypeslib.as_array(ctypes.cast(px, ctypes.POINTER(ctypes.c_uint64)), (k + 1,)).copy()
    two_m = int(xadj[-1])
    if two_m:
        adjncy = np.ctypeslib.as_array(ctypes.cast(pa, ctypes.POINTER(ctypes.c_int32)), (two_m,)).copy()
        adjwgt = np.ctypeslib.as_array(ctypes.cast(pw, ctypes.POINTER(ctypes.c_int32)), (two_m,)).copy()
    else:
        adjncy = np.empty(0, dtype=np.int32)
        adjwgt = np.empty(0, dtype=np.int32)
    vwgt = np.ctypeslib.as_array(ctypes.cast(pv, ctypes.POINTER(ctypes.c_int32)), (max(k, 1),))[:k].copy()
    for p in (px, pa, pw, pv):
        lib.orc_free(p)
    if rc == EOVERFLOW:
        raise OverflowError("coarse weight exceeds INT32_MAX")
    return Coarse(k, xadj, adjncy, adjwgt, vwgt), m[: g.n]


def edge_cut(g, labels) -> int:
    A = _Args()
    lib = _load()
    return int(lib.orc_edge_cut(g.n, A(g.xadj, np.uint64), A(g.adjncy, np.int32),
                                A(g.adjwgt, np.int32), A(labels, np.int32)))


# ----------------------------------------------------------- coarsening ----

def coarsen_params(n0: int, total_weight: int):
    """Target size and the (level-constant) cluster-weight cap of the loop."""
    n_target = min(1 << 14, max(256, -(-n0 // 64)))
    cap = -(-3 * total_weight // n_target)
    return n_target, cap


def coarsen(g, seed: int, rounds: int = 5, max_levels: int = 32, cluster=None, cap=None):
    """Cluster-and-contract until the graph has at most n_target vertices, the
    graph shrinks by less than 5 % in a level (stall), or max_levels levels.
    Level l clusters with seed + l (by `cluster(graph, cap, rounds, seed)`,
    default the synchronous lp_cluster); `cap`, if given, replaces the
    loop's cluster-weight cap. Returns the list of levels
    [(graph, labels, map)] and the final graph."""
    cluster = cluster or lp_cluster
    total = int(g.n if g.vwgt is None else int(np.asarray(g.vwgt, dtype=np.int64).sum()))
    n_target, cap0 = coarsen_params(g.n, total)
    cap = cap0 if cap is None else int(cap)
    levels = []
    cur = g
    lvl = 0
    while lvl < max_levels and cur.n > n_target:
        labels, _ = cluster(cur, cap, rounds, seed + lvl)
        nxt, mp = contract(cur, labels)
        levels.append((cur, labels, mp))
        prev_n = cur.n
        cur = nxt
        lvl += 1
        if 100 * cur.n > 95 * prev_n:
            break
    return levels, cur, n_target, cap


# --------------------------------------------------------- uncoarsening ----

def max_block_weight(total_weight: int, k: int, eps_permille: int = 30) -> int:
    """Balance bound of a k-way partition: the paper's (1 + eps) * c(V) / k
    (Section I; eps = 3 % in its experiments), with c(V) / k rounded up to a
    whole weight so that a perfectly balanced partition always fits, and eps
    in thousandths: L = ceil(c(V) / k) + floor(L0 * eps_permille / 1000)."""
    base = -(-int(total_weight) // int(k))
    return base + base * int(eps_permille) // 1000


def partition_cap(n0: int, total_weight: int, k: int, eps_permille: int = 30) -> int:
    """Cluster-weight cap of the coarsening that precedes a k-way partition:
    the coarsening loop's own cap, but no more than the balance slack
    L - ceil(c(V) / k) (at least 1), so that no coarse vertex is heavier than
    what a block may exceed its share by. The contiguous initial partition of
    the coarsest graph then respects L."""
    _, cap = coarsen_params(n0, total_weight)
    return min(cap, max(1, max_block_weight(total_weight, k, eps_permille) - (-(-int(total_weight) // int(k)))))


def initial_partition(g, k: int):
    """Contiguous-weight initial partition (see orc_initial_partition)."""
    A = _Args()
    labels = np.empty(max(g.n, 1), dtype=np.int32)
    rc = _load().orc_initial_partition(g.n, A(g.vwgt, np.int32), k, _ptr(labels))
    if rc != OK:
        raise ValueError(f"orc_initial_partition: {rc}")
    return labels[: g.n]


def lp_refine(g, blocks, k: int, max_weight: int, rounds: int, seed: int, subrounds: int = 1):
    """Refined blocks (int32[n]) and per-round stats: synchronous
    size-constrained LP started from `blocks` (see orc_lp_refine)."""
    A = _Args()
    lib = _load()
    labels = np.array(blocks, dtype=np.int32, copy=True)
    if labels.size == 0:
        labels = np.zeros(1, dtype=np.int32)
    st = _Stats()
    rc = lib.orc_lp_refine(g.n, A(g.xadj, np.uint64), A(g.adjncy, np.int32),
                           A(g.adjwgt, np.int32), A(g.vwgt, np.int32), k, max_weight, rounds,
                           subrounds, seed, _ptr(labels), ctypes.byref(st))
    if rc != OK:
        raise ValueError(f"orc_lp_refine: {rc}")
    r = min(st.rounds_run, 64)
    return labels[: g.n], LPStats(st.rounds_run, list(st.proposals[:r]), list(st.moves[:r]))


def project(fine_to_coarse, coarse_blocks):
    """Blocks of the finer graph: every vertex takes the block of the coarse
    vertex it was contracted into (Section II-A, uncoarsening)."""
    return np.asarray(coarse_blocks, dtype=np.int32)[np.asarray(fine_to_coarse, dtype=np.int64)]


def block_weights(g, blocks, k: int):
    w = np.ones(g.n, dtype=np.int64) if g.vwgt is None else np.asarray(g.vwgt, dtype=np.int64)
    return np.bincount(np.asarray(blocks, dtype=np.int64), weights=w, minlength=k).astype(np.int64)


def partition(g, k: int, seed: int = 1, rounds: int = 5, eps_permille: int = 30, subrounds: int = 1,
              refine_subrounds: int = 1):
    """Multilevel k-way partition (Section II-A): coarsen with LP clustering
    under partition_cap, partition the coarsest graph (initial_partition, then lp_refine there),
    then project to each finer level and refine it. Level l (0 = the input)
    refines with seed + l. Returns (blocks int32[n], per-level list of
    (n, cut after refinement) from the coarsest to the input)."""
    total = int(g.n if g.vwgt is None else int(np.asarray(g.vwgt, dtype=np.int64).sum()))
    lmax = max_block_weight(total, k, eps_permille)
    cl = None
    if subrounds > 1:
        def cl(gr, cap, rnd, sd):
            return lp_cluster(gr, cap, rnd, sd, subrounds=subrounds)
    levels, coarsest, _, _ = coarsen(g, seed, rounds, cluster=cl, cap=partition_cap(g.n, total, k, eps_permille))
    depth = len(levels)
    blocks = initial_partition(coarsest, k)
    blocks, _ = lp_refine(coarsest, blocks, k, lmax, rounds, seed + depth, refine_subrounds)
    trace = [(coarsest.n, edge_cut(coarsest, blocks))]
    for lvl in range(depth - 1, -1, -1):
        fine, _, mp = levels[lvl]
        blocks = project(mp, blocks)
        blocks, _ = lp_refine(fine, blocks, k, lmax, rounds, seed + lvl, refine_subrounds)
        trace.append((fine.n, edge_cut(fine, blocks)))
    return blocks, trace


# ------------------------------------------------------------ gain table ----

def affinity(g, blocks, k: int):
    """Affinities of every vertex to every block (Section V): A[u, b] = total
    weight of the edges from u to vertices of block b. Dense int64[n, k],
    by the definition (small graphs only)."""
    blocks = np.asarray(blocks, dtype=np.int64)
    deg = np.diff(np.asarray(g.xadj, dtype=np.int64))
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    dst = np.asarray(g.adjncy, dtype=np.int64)
    w = np.ones(g.two_m, dtype=np.int64) if g.adjwgt is None else np.asarray(g.adjwgt, dtype=np.int64)
    A = np.zeros((g.n, k), dtype=np.int64)
    np.add.at(A, (src, blocks[dst]), w)
    return A


def move_gains(g, blocks, k: int):
    """Gain of moving every vertex to every block: A[u, b] - A[u, block(u)]
    (Section V)."""
    A = affinity(g, blocks, k)
    own = A[np.arange(g.n), np.asarray(blocks, dtype=np.int64)]
    return A - own[:, None]
