"""Python binding of the MI355X label-propagation coarsening library.

Argument marshalling only: every step runs in the HIP kernels of
``liblpgpu.so`` (built by :func:`build`), reached through the C ABI declared
in ``include/lp.h``. PyTorch provides device memory and streams. There is no
CPU fallback: importing works without a GPU, but every call needs the built
library and a HIP device and raises otherwise.

Entry points mirror the C names: :func:`lp_compress`, :func:`lp_graph_from_csr`,
:func:`lp_decompress`, :func:`lp_cluster`, :func:`lp_contract`,
:func:`lp_edge_cut`, plus the multilevel loop :func:`coarsen`.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

from ._build import LIB as _LIB_PATH
from ._build import build as _build_lib

LP_OK, LP_EINVAL, LP_ENOMEM, LP_EOVERFLOW, LP_EDEVICE, LP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
LP_CHUNK_THRESHOLD = 10000
LP_CHUNK_LEN = 1000

_P = ctypes.c_void_p
_lib = None


class LPError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _load().lp_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {msg} ({status})")


PHASES = ("setup", "lane", "tile", "block", "hub", "accept", "round", "hub_whole", "hub_pieces", "hub_reduce")


class lp_config(ctypes.Structure):
    _fields_ = [("t_lane", ctypes.c_int32), ("t_tile", ctypes.c_int32),
                ("t_block", ctypes.c_int32), ("hub_part", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("subrounds", ctypes.c_int32), ("gain_table", ctypes.c_int32), ("overlap", ctypes.c_int32),
                ("reorder", ctypes.c_int32)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class lp_allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


class lp_cluster_stats(ctypes.Structure):
    _fields_ = [("rounds_run", ctypes.c_int32), ("n_lane", ctypes.c_int32), ("n_tile", ctypes.c_int32),
                ("n_block", ctypes.c_int32), ("n_hub", ctypes.c_int32),
                ("proposals", ctypes.c_int64 * 64), ("moves", ctypes.c_int64 * 64),
                ("bucket_edges", ctypes.c_uint64 * 4), ("bucket_bytes", ctypes.c_uint64 * 4),
                ("phase_ms", ctypes.c_float * len(PHASES)), ("phase_launches", ctypes.c_int32 * len(PHASES)),
                ("round_ms", ctypes.c_float * 64)]


def build() -> str:
    """Compile the HIP library for gfx950 (always recompiles)."""
    return _build_lib()


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run paper_2410_19119_amd.build()")
    # torch first: its HIP runtime then satisfies the library's libamdhip64.so.7
    # dependency, so one runtime serves both (two runtimes in one process do
    # not share devices, memory or streams).
    import torch  # noqa: F401
    lib = ctypes.CDLL(_LIB_PATH)
    S = ctypes.c_int32
    lib.lp_strerror.argtypes = [S]
    lib.lp_strerror.restype = ctypes.c_char_p
    lib.lp_version.restype = ctypes.c_char_p
    lib.lp_compress.argtypes = [ctypes.c_int32, _P, _P, _P, _P, _P, ctypes.POINTER(_P)]
    lib.lp_compress.restype = S
    lib.lp_compress_ex.argtypes = [ctypes.c_int32, _P, _P, _P, _P, ctypes.c_int32, _P, ctypes.POINTER(_P)]
    lib.lp_compress_ex.restype = S
    lib.lp_graph_from_csr.argtypes = [ctypes.c_int32, _P, _P, _P, _P, _P, ctypes.POINTER(_P)]
    lib.lp_graph_from_csr.restype = S
    lib.lp_graph_info.argtypes = [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint64),
                                  ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
    lib.lp_graph_info.restype = S
    lib.lp_graph_export.argtypes = [_P, _P, _P, _P]
    lib.lp_graph_export.restype = S
    lib.lp_decompress.argtypes = [_P, _P, _P, _P, _P, _P]
    lib.lp_decompress.restype = S
    lib.lp_cluster.argtypes = [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, _P, _P]
    lib.lp_cluster.restype = S
    lib.lp_cluster_ex.argtypes = [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, _P,
                                  ctypes.POINTER(lp_config), ctypes.POINTER(lp_cluster_stats), _P]
    lib.lp_cluster_ex.restype = S
    lib.lp_contract.argtypes = [_P, _P, _P, _P, ctypes.POINTER(_P)]
    lib.lp_contract.restype = S
    lib.lp_edge_cut.argtypes = [_P, _P, ctypes.POINTER(ctypes.c_int64), _P]
    lib.lp_edge_cut.restype = S
    lib.lp_edge_cut_noalloc.argtypes = [_P, _P, _P, _P]
    lib.lp_edge_cut_noalloc.restype = S
    lib.lp_graph_free.argtypes = [_P]
    lib.lp_graph_free.restype = None
    lib.lp_trim_memory.argtypes = []
    lib.lp_trim_memory.restype = None
    lib.lp_set_allocator.argtypes = [ctypes.POINTER(lp_allocator)]
    lib.lp_set_allocator.restype = S
    lib.lp_memory_info.argtypes = [ctypes.POINTER(ctypes.c_uint64)] * 3
    lib.lp_memory_info.restype = S
    lib.lp_batch_create.argtypes = [ctypes.c_int32, _P, _P, ctypes.POINTER(_P)]
    lib.lp_batch_create.restype = S
    lib.lp_batch_info.argtypes = [_P, ctypes.POINTER(ctypes.c_int32), _P]
    lib.lp_batch_info.restype = S
    lib.lp_batch_cluster_ex.argtypes = [_P, _P, ctypes.c_int32, _P, _P, ctypes.POINTER(lp_config),
                                        ctypes.POINTER(lp_cluster_stats), _P]
    lib.lp_batch_cluster_ex.restype = S
    lib.lp_batch_cluster.argtypes = [ctypes.c_int32, _P, _P, ctypes.c_int32, _P, _P, _P]
    lib.lp_batch_cluster.restype = S
    lib.lp_initial_partition.argtypes = [_P, ctypes.c_int32, _P, _P]
    lib.lp_initial_partition.restype = S
    lib.lp_project.argtypes = [ctypes.c_int32, _P, ctypes.c_int32, _P, _P, _P]
    lib.lp_project.restype = S
    lib.lp_refine.argtypes = [_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, _P, _P]
    lib.lp_refine.restype = S
    lib.lp_refine_ex.argtypes = [_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, _P,
                                 ctypes.POINTER(lp_config), ctypes.POINTER(lp_cluster_stats), _P]
    lib.lp_refine_ex.restype = S
    lib.lp_gain_table_create.argtypes = [_P, _P, ctypes.c_int32, _P, ctypes.POINTER(_P)]
    lib.lp_gain_table_create.restype = S
    lib.lp_gain_table_affinity.argtypes = [_P, ctypes.c_int64, _P, _P, _P, _P]
    lib.lp_gain_table_affinity.restype = S
    lib.lp_gain_table_move.argtypes = [_P, ctypes.c_int64, _P, _P, _P]
    lib.lp_gain_table_move.restype = S
    lib.lp_gain_table_info.argtypes = [_P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.lp_gain_table_info.restype = S
    lib.lp_gain_table_free.argtypes = [_P]
    lib.lp_gain_table_free.restype = None
    _lib = lib
    return lib


def _torch_alloc(nbytes, stream, ctx):
    try:
        return _torch()._C._cuda_cudaCachingAllocator_raw_alloc(int(nbytes), int(stream or 0))
    except RuntimeError:  # out of memory: the library call fails with LP_ENOMEM
        return None


def _torch_free(ptr, stream, ctx):
    _torch()._C._cuda_cudaCachingAllocator_raw_delete(int(ptr))


_TORCH_ALLOCATOR = None  # keeps the callbacks alive while installed


def use_torch_allocator(on: bool = True) -> None:
    """Route the library's scratch memory through torch's caching allocator
    (lp_set_allocator), or back to the library's own memory cache. Every
    allocation then costs a Python callback (a few microseconds)."""
    global _TORCH_ALLOCATOR
    lib = _load()
    if on:
        a = lp_allocator(_ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free), None)
        _check(lib.lp_set_allocator(ctypes.byref(a)), "lp_set_allocator")
        _TORCH_ALLOCATOR = a
    else:
        _check(lib.lp_set_allocator(None), "lp_set_allocator")
        _TORCH_ALLOCATOR = None


def memory_info() -> dict:
    """Device memory the library holds (lp_memory_info): cache blocks in use,
    cache blocks kept for reuse, and blocks from the caller's allocator."""
    live, cached, ext = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(_load().lp_memory_info(ctypes.byref(live), ctypes.byref(cached), ctypes.byref(ext)), "lp_memory_info")
    return {"live": live.value, "cached": cached.value, "external": ext.value}


def exported_symbols() -> list[str]:
    return ["lp_strerror", "lp_version", "lp_compress", "lp_compress_ex", "lp_graph_from_csr", "lp_graph_info",
            "lp_graph_export", "lp_decompress", "lp_cluster", "lp_cluster_ex", "lp_contract",
            "lp_edge_cut", "lp_edge_cut_noalloc", "lp_graph_free", "lp_batch_create", "lp_batch_info", "lp_batch_cluster_ex",
            "lp_batch_cluster", "lp_trim_memory", "lp_set_allocator", "lp_memory_info", "lp_initial_partition", "lp_project", "lp_refine",
            "lp_refine_ex", "lp_gain_table_create", "lp_gain_table_affinity", "lp_gain_table_move",
            "lp_gain_table_info", "lp_gain_table_free"]


def _check(st: int, where: str) -> None:
    if st != LP_OK:
        raise LPError(st, where)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("a HIP device is required (no CPU fallback)")
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(a, dtype):
    """Device tensor of `dtype` (copies numpy / host tensors; None stays None)."""
    if a is None:
        return None
    torch = _torch()
    if isinstance(a, np.ndarray):
        a = torch.from_numpy(np.ascontiguousarray(a))
    t = a.to(device="cuda", dtype=dtype)
    return t.contiguous()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Graph:
    """Owns an ``lp_graph`` handle (device-resident, immutable)."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        n = ctypes.c_int32()
        two_m = ctypes.c_uint64()
        nb = ctypes.c_uint64()
        comp = ctypes.c_int32()
        wt = ctypes.c_int32()
        tot = ctypes.c_int64()
        _check(_load().lp_graph_info(handle, n, two_m, nb, comp, wt, tot), "lp_graph_info")
        self.n = n.value
        self.two_m = two_m.value
        self.nbytes = nb.value
        self.compressed = bool(comp.value)
        self.intervals = comp.value == 2
        self.weighted = bool(wt.value)
        self.total_vwgt = tot.value

    @property
    def handle(self):
        return self._h

    def free(self) -> None:
        if self._h is not None and _lib is not None:
            _lib.lp_graph_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __repr__(self):
        kind = "compressed" if self.compressed else "plain"
        return f"Graph(n={self.n}, 2m={self.two_m}, {kind}, bytes={self.nbytes})"


def _make(fn_name: str, n, xadj, adjncy, adjwgt=None, vwgt=None, stream=None, flags=None) -> Graph:
    torch = _torch()
    lib = _load()
    x = _dev(xadj, torch.int64)  # uint64 bit pattern
    a = _dev(adjncy, torch.int32)
    if a.numel() == 0:
        a = torch.zeros(1, dtype=torch.int32, device="cuda")
    w = _dev(adjwgt, torch.int32)
    v = _dev(vwgt, torch.int32)
    h = _P()
    if flags is None:
        st = getattr(lib, fn_name)(int(n), _ptr(x), _ptr(a), _ptr(w), _ptr(v), _stream(stream), ctypes.byref(h))
    else:
        st = getattr(lib, fn_name)(int(n), _ptr(x), _ptr(a), _ptr(w), _ptr(v), int(flags), _stream(stream),
                                   ctypes.byref(h))
    _check(st, fn_name)
    return Graph(h)


LP_COMPRESS_INTERVALS = 1


def lp_compress(n, xadj, adjncy, adjwgt=None, vwgt=None, stream=None, intervals: bool = False) -> Graph:
    """Compressed handle from a CSR (numpy or tensors; copied to the device);
    with intervals=True runs of consecutive IDs are interval encoded."""
    if intervals:
        return _make("lp_compress_ex", n, xadj, adjncy, adjwgt, vwgt, stream, flags=LP_COMPRESS_INTERVALS)
    return _make("lp_compress", n, xadj, adjncy, adjwgt, vwgt, stream)


def lp_graph_from_csr(n, xadj, adjncy, adjwgt=None, vwgt=None, stream=None) -> Graph:
    """Plain CSR handle."""
    return _make("lp_graph_from_csr", n, xadj, adjncy, adjwgt, vwgt, stream)


def lp_graph_export(g: Graph, stream=None):
    """(offs, bytes) device tensors of a compressed handle."""
    torch = _torch()
    offs = torch.empty(g.n + 1, dtype=torch.int64, device="cuda")
    data = torch.empty(max(g.nbytes, 1), dtype=torch.uint8, device="cuda")
    _check(_load().lp_graph_export(g.handle, _ptr(offs), _ptr(data), _stream(stream)), "lp_graph_export")
    return offs, data[: g.nbytes]


def lp_decompress(g: Graph, stream=None):
    """(xadj, adjncy, adjwgt, vwgt) device tensors (int64 / int32)."""
    torch = _torch()
    xadj = torch.empty(g.n + 1, dtype=torch.int64, device="cuda")
    adj = torch.empty(max(g.two_m, 1), dtype=torch.int32, device="cuda")
    wgt = torch.empty(max(g.two_m, 1), dtype=torch.int32, device="cuda")
    vw = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda")
    _check(_load().lp_decompress(g.handle, _ptr(xadj), _ptr(adj), _ptr(wgt), _ptr(vw), _stream(stream)),
           "lp_decompress")
    return xadj, adj[: g.two_m], wgt[: g.two_m], vw[: g.n]


@dataclass
class ClusterStats:
    rounds_run: int
    buckets: tuple
    proposals: list = field(default_factory=list)
    moves: list = field(default_factory=list)
    bucket_edges: tuple = ()
    bucket_bytes: tuple = ()
    phase_ms: dict = field(default_factory=dict)
    phase_launches: dict = field(default_factory=dict)
    round_ms: list = field(default_factory=list)  # per timed round (first 64)


def lp_cluster(g: Graph, max_cluster_weight: int, rounds: int = 5, seed: int = 1, labels=None,
               config: dict | None = None, stats: bool = False, stream=None):
    """Size-constrained LP labels (int32 device tensor); with stats=True also ClusterStats."""
    torch = _torch()
    if labels is None:
        labels = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda")
    cfg = None
    if config:
        cfg = lp_config(**{k: int(v) for k, v in config.items()})
    st_obj = lp_cluster_stats() if stats else None
    st = _load().lp_cluster_ex(g.handle, int(max_cluster_weight), int(rounds), int(seed) & (2**64 - 1),
                               _ptr(labels), ctypes.byref(cfg) if cfg else None,
                               ctypes.byref(st_obj) if st_obj is not None else None, _stream(stream))
    _check(st, "lp_cluster")
    out = labels[: g.n]
    return (out, _stats_of(st_obj)) if stats else out


def _stats_of(st_obj) -> ClusterStats:
    k = min(st_obj.rounds_run, 64)
    return ClusterStats(st_obj.rounds_run, (st_obj.n_lane, st_obj.n_tile, st_obj.n_block, st_obj.n_hub),
                        list(st_obj.proposals[:k]), list(st_obj.moves[:k]),
                        tuple(st_obj.bucket_edges), tuple(st_obj.bucket_bytes),
                        dict(zip(PHASES, st_obj.phase_ms)), dict(zip(PHASES, st_obj.phase_launches)),
                        list(st_obj.round_ms[:min(st_obj.phase_launches[PHASES.index("round")], 64)]))


class Batch(Graph):
    """Disjoint union of several graph handles (lp_batch_create); graph i owns
    vertices [vbase[i], vbase[i + 1]) of the union."""

    def __init__(self, handle):
        super().__init__(handle)
        G = ctypes.c_int32()
        _check(_load().lp_batch_info(self.handle, ctypes.byref(G), None), "lp_batch_info")
        vb = (ctypes.c_int32 * (G.value + 1))()
        _check(_load().lp_batch_info(self.handle, None, vb), "lp_batch_info")
        self.G = G.value
        self.vbase = list(vb)

    def split(self, labels):
        """Per-graph views of a union-sized array."""
        return [labels[self.vbase[i]: self.vbase[i + 1]] for i in range(self.G)]


def lp_batch_create(graphs, stream=None) -> Batch:
    """One batch handle over the given graph handles (they stay usable)."""
    arr = (_P * len(graphs))(*[g.handle for g in graphs])
    h = _P()
    _check(_load().lp_batch_create(len(graphs), arr, _stream(stream), ctypes.byref(h)), "lp_batch_create")
    return Batch(h)


def lp_batch_cluster_ex(b: Batch, caps, rounds: int, seeds, labels=None, config: dict | None = None,
                        stats: bool = False, stream=None):
    """Labels of every graph of a batch (union-sized int32 tensor, local IDs per graph)."""
    torch = _torch()
    if labels is None:
        labels = torch.empty(max(b.n, 1), dtype=torch.int32, device="cuda")
    c = (ctypes.c_int64 * b.G)(*[int(v) for v in caps])
    sd = (ctypes.c_uint64 * b.G)(*[int(v) & (2**64 - 1) for v in seeds])
    cfg = lp_config(**{k: int(v) for k, v in config.items()}) if config else None
    st_obj = lp_cluster_stats() if stats else None
    st = _load().lp_batch_cluster_ex(b.handle, c, int(rounds), sd, _ptr(labels), ctypes.byref(cfg) if cfg else None,
                                     ctypes.byref(st_obj) if st_obj is not None else None, _stream(stream))
    _check(st, "lp_batch_cluster_ex")
    out = labels[: b.n]
    return (out, _stats_of(st_obj)) if stats else out


def lp_batch_cluster(graphs, caps, rounds: int, seeds, labels=None, stream=None):
    """G handles in, G label tensors out (one batched run)."""
    torch = _torch()
    G = len(graphs)
    if labels is None:
        labels = [torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda") for g in graphs]
    arr = (_P * G)(*[g.handle for g in graphs])
    outs = (_P * G)(*[_ptr(t) for t in labels])
    c = (ctypes.c_int64 * G)(*[int(v) for v in caps])
    sd = (ctypes.c_uint64 * G)(*[int(v) & (2**64 - 1) for v in seeds])
    _check(_load().lp_batch_cluster(G, arr, c, int(rounds), sd, outs, _stream(stream)), "lp_batch_cluster")
    return [t[: g.n] for t, g in zip(labels, graphs)]


def lp_contract(g: Graph, labels, want_map: bool = True, stream=None):
    """(coarse Graph, map int32 device tensor or None)."""
    torch = _torch()
    lab = _dev(labels, torch.int32)
    mp = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda") if want_map else None
    h = _P()
    _check(_load().lp_contract(g.handle, _ptr(lab), _ptr(mp), _stream(stream), ctypes.byref(h)), "lp_contract")
    return Graph(h), (mp[: g.n] if mp is not None else None)


def lp_trim_memory() -> None:
    """Returns the library's cached device memory to HIP (waits for the device)."""
    _load().lp_trim_memory()


def lp_edge_cut(g: Graph, labels, stream=None) -> int:
    torch = _torch()
    lab = _dev(labels, torch.int32)
    out = ctypes.c_int64()
    _check(_load().lp_edge_cut(g.handle, _ptr(lab), ctypes.byref(out), _stream(stream)), "lp_edge_cut")
    return out.value


def lp_edge_cut_noalloc(g: Graph, labels, cut_out, stream=None) -> None:
    """The cut written into cut_out (int64 device tensor of one element) with
    no allocation and no synchronisation; the handle's plan must exist."""
    torch = _torch()
    lab = _dev(labels, torch.int32)
    if cut_out.dtype != torch.int64 or not cut_out.is_cuda or cut_out.numel() < 1:
        raise ValueError("cut_out must be an int64 device tensor")
    _check(_load().lp_edge_cut_noalloc(g.handle, _ptr(lab), _ptr(cut_out), _stream(stream)), "lp_edge_cut_noalloc")


def coarsen_params(n0: int, total_weight: int):
    """Target size and the level-constant cluster-weight cap of the multilevel loop."""
    n_target = min(1 << 14, max(256, -(-n0 // 64)))
    cap = -(-3 * total_weight // n_target)
    return n_target, cap


def coarsen(g: Graph, seed: int = 1, rounds: int = 5, max_levels: int = 32, stream=None, subrounds: int = 1):
    """Repeated lp_cluster + lp_contract (all on the device; the host reads n' only).
    Stops at n' <= n_target, when a level shrinks by less than 5 %, or after
    max_levels levels. Level l clusters with seed + l (and `subrounds`
    sub-rounds per round). Returns
    (levels: list of (Graph, labels, map), final Graph, n_target, cap)."""
    n_target, cap = coarsen_params(g.n, g.total_vwgt)
    levels = []
    cur = g
    lvl = 0
    cfg = dict(subrounds=subrounds) if subrounds > 1 else None
    while lvl < max_levels and cur.n > n_target:
        labels = lp_cluster(cur, cap, rounds, seed + lvl, stream=stream, config=cfg)
        nxt, mp = lp_contract(cur, labels, stream=stream)
        levels.append((cur, labels, mp))
        prev_n = cur.n
        cur = nxt
        lvl += 1
        if 100 * cur.n > 95 * prev_n:
            break
    return levels, cur, n_target, cap


# ------------------------------------------------------------ uncoarsening ----

def max_block_weight(total_weight: int, k: int, eps_permille: int = 30) -> int:
    """Balance bound (1 + eps) * c(V) / k of Section I, with c(V) / k rounded up
    to a whole weight and eps in thousandths:
    ceil(c(V) / k) + floor(ceil(c(V) / k) * eps_permille / 1000)."""
    base = -(-int(total_weight) // int(k))
    return base + base * int(eps_permille) // 1000


def partition_cap(n0: int, total_weight: int, k: int, eps_permille: int = 30) -> int:
    """Cluster-weight cap of the coarsening before a k-way partition: the
    coarsening loop's cap, but at most the balance slack (at least 1), so that
    no coarse vertex outweighs what a block may exceed its share by."""
    _, cap = coarsen_params(n0, total_weight)
    slack = max_block_weight(total_weight, k, eps_permille) - (-(-int(total_weight) // int(k)))
    return min(cap, max(1, slack))


def lp_initial_partition(g: Graph, k: int, labels=None, stream=None):
    """Contiguous-weight k-way partition (int32 device tensor)."""
    torch = _torch()
    if labels is None:
        labels = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda")
    _check(_load().lp_initial_partition(g.handle, int(k), _ptr(labels), _stream(stream)), "lp_initial_partition")
    return labels[: g.n]


def lp_project(fine_to_coarse, coarse_labels, stream=None):
    """Blocks of the finer graph: labels[u] = coarse_labels[map[u]]."""
    torch = _torch()
    mp = _dev(fine_to_coarse, torch.int32)
    cl = _dev(coarse_labels, torch.int32)
    n = int(mp.numel())
    out = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    _check(_load().lp_project(n, _ptr(mp), int(cl.numel()), _ptr(cl), _ptr(out), _stream(stream)), "lp_project")
    return out[:n]


def lp_refine(g: Graph, blocks, k: int, max_block_weight: int, rounds: int = 5, seed: int = 1,
              config: dict | None = None, stats: bool = False, stream=None):
    """Size-constrained LP refinement of a k-way partition; returns the refined
    blocks (a new int32 device tensor) and, with stats=True, ClusterStats."""
    torch = _torch()
    labels = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda")
    if g.n:
        labels[: g.n].copy_(_dev(blocks, torch.int32)[: g.n])
    cfg = lp_config(**{kk: int(v) for kk, v in config.items()}) if config else None
    st_obj = lp_cluster_stats() if stats else None
    st = _load().lp_refine_ex(g.handle, int(k), int(max_block_weight), int(rounds), int(seed) & (2**64 - 1),
                              _ptr(labels), ctypes.byref(cfg) if cfg else None,
                              ctypes.byref(st_obj) if st_obj is not None else None, _stream(stream))
    _check(st, "lp_refine")
    out = labels[: g.n]
    return (out, _stats_of(st_obj)) if stats else out


def partition(g: Graph, k: int, seed: int = 1, rounds: int = 5, eps_permille: int = 30, subrounds: int = 1,
              refine_subrounds: int = 1, gain_table: bool = False, stream=None, trace: bool = False):
    """Multilevel k-way partition (Section II-A), all steps on the device:
    coarsen with LP clustering under partition_cap, partition the coarsest
    graph (lp_initial_partition, then lp_refine there), then project to each
    finer level and refine it; level l (0 = the input) refines with seed + l.
    Returns the blocks of g (int32 device tensor); with trace=True also the
    list of (n, cut after refinement) from the coarsest level to g. With
    gain_table=True every refinement rates from a sparse gain table (same
    result)."""
    cap = partition_cap(g.n, g.total_vwgt, k, eps_permille)
    lmax = max_block_weight(g.total_vwgt, k, eps_permille)
    n_target, _ = coarsen_params(g.n, g.total_vwgt)
    cfg = dict(subrounds=subrounds) if subrounds > 1 else None
    rcfg = dict(subrounds=refine_subrounds, gain_table=int(bool(gain_table)))
    levels = []
    cur = g
    while len(levels) < 32 and cur.n > n_target:
        labels = lp_cluster(cur, cap, rounds, seed + len(levels), stream=stream, config=cfg)
        nxt, mp = lp_contract(cur, labels, stream=stream)
        levels.append((cur, mp))
        prev_n, cur = cur.n, nxt
        if 100 * cur.n > 95 * prev_n:
            break
    blocks = lp_initial_partition(cur, k, stream=stream)
    blocks = lp_refine(cur, blocks, k, lmax, rounds, seed + len(levels), config=rcfg, stream=stream)
    steps = [(cur.n, lp_edge_cut(cur, blocks, stream=stream))] if trace else None
    for lvl in range(len(levels) - 1, -1, -1):
        fine, mp = levels[lvl]
        if cur is not g:
            cur.free()
        blocks = lp_project(mp, blocks, stream=stream)
        blocks = lp_refine(fine, blocks, k, lmax, rounds, seed + lvl, config=rcfg, stream=stream)
        cur = fine
        if trace:
            steps.append((fine.n, lp_edge_cut(fine, blocks, stream=stream)))
    return (blocks, steps) if trace else blocks


class GainTable:
    """Owns an ``lp_gain_table``: the affinity of every vertex to every block
    adjacent to it (Section V), for a partition of `g` into k blocks."""

    def __init__(self, g: Graph, blocks, k: int, stream=None):
        torch = _torch()
        b = _dev(blocks, torch.int32)
        h = _P()
        _check(_load().lp_gain_table_create(g.handle, _ptr(b), int(k), _stream(stream), ctypes.byref(h)),
               "lp_gain_table_create")
        self._h = h
        self.g = g
        self.k = int(k)

    def affinity(self, vertices, blocks, stream=None):
        """int64 device tensor of the affinities of the (vertex, block) pairs."""
        torch = _torch()
        v = _dev(vertices, torch.int32)
        b = _dev(blocks, torch.int32)
        out = torch.empty(max(int(v.numel()), 1), dtype=torch.int64, device="cuda")
        _check(_load().lp_gain_table_affinity(self._h, int(v.numel()), _ptr(v), _ptr(b), _ptr(out),
                                              _stream(stream)), "lp_gain_table_affinity")
        return out[: v.numel()]

    def move(self, vertices, to, stream=None) -> None:
        """Moves distinct vertices to new blocks at once."""
        torch = _torch()
        v = _dev(vertices, torch.int32)
        t = _dev(to, torch.int32)
        _check(_load().lp_gain_table_move(self._h, int(v.numel()), _ptr(v), _ptr(t), _stream(stream)),
               "lp_gain_table_move")

    def info(self):
        """(slots, device bytes, missing entries met by updates, slices rebuilt)."""
        e, b, m, r = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_int64(), ctypes.c_int64()
        _check(_load().lp_gain_table_info(self._h, ctypes.byref(e), ctypes.byref(b), ctypes.byref(m),
                                          ctypes.byref(r)), "lp_gain_table_info")
        return e.value, b.value, m.value, r.value

    def free(self) -> None:
        if self._h is not None and _lib is not None:
            _lib.lp_gain_table_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
