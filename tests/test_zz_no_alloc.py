"""lp_edge_cut_noalloc, the entry point for callers that cannot allocate:
called through the C ABI, it must give exactly lp_edge_cut's result, call
after call on the one scratch array it keeps per device (the second call
with a smaller graph), on compressed graphs with every rating path (lanes,
tiles, hub pieces), on weighted and on plain (coarse) handles, and refuse a
handle whose plan no earlier call has built."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _noalloc(lp, G, lab):
    import torch
    out = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    st = lp._load().lp_edge_cut_noalloc(G.handle, ctypes.c_void_p(lab.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                        None)
    assert st == lp.LP_OK, st
    torch.cuda.synchronize()
    return int(out.item())


def _case(lp, g, cap, seed, compressed=True):
    if compressed:
        G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy, g.adjwgt, g.vwgt)
    else:
        G = lp.lp_graph_from_csr(g.n, g.xadj.view(np.int64), g.adjncy, g.adjwgt, g.vwgt)
    lab = lp.lp_cluster(G, cap, 3, seed)  # default thresholds: builds the handle's plan
    return G, lab


def test_noalloc_cut_equals_cut_call_after_call(lp, synth_mod):
    big = synth_mod.rmat_scale(15, 16, seed=4)
    small = synth_mod.rgg2d_16k(seed=1)
    G1, lab1 = _case(lp, big, 64, 3)
    G2, lab2 = _case(lp, small, 32, 1)
    assert G2.two_m < G1.two_m
    ref1, ref2 = lp.lp_edge_cut(G1, lab1), lp.lp_edge_cut(G2, lab2)
    assert ref1 > 0 and ref2 > 0
    assert _noalloc(lp, G1, lab1) == ref1
    assert _noalloc(lp, G2, lab2) == ref2  # the second call, on a smaller graph, starts from a clear array
    assert _noalloc(lp, G1, lab1) == ref1
    G1.free()
    G2.free()


@pytest.mark.parametrize("kind", ["star-hub", "weighted", "plain"])
def test_noalloc_cut_other_handles(lp, synth_mod, kind):
    if kind == "star-hub":  # a hub of degree 25000 takes the chunked piece path
        g = synth_mod.from_edges(25001, [(0, i) for i in range(1, 25001)])
        G, lab = _case(lp, g, 100, 2)
    elif kind == "weighted":
        g = synth_mod.rmat_scale(12, 8, seed=9)
        g.adjwgt = synth_mod.edge_weights(g, 1, 1000, 9)
        G, lab = _case(lp, g, 40, 5)
    else:
        g = synth_mod.rmat_scale(13, 16, seed=2)
        G, lab = _case(lp, g, 64, 7, compressed=False)
    assert _noalloc(lp, G, lab) == lp.lp_edge_cut(G, lab)
    G.free()


def test_noalloc_cut_needs_the_plan(lp, synth_mod):
    import torch
    g = synth_mod.rgg2d_16k(seed=2)
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
    lab = torch.arange(g.n, dtype=torch.int32, device="cuda")
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = lp._load().lp_edge_cut_noalloc(G.handle, ctypes.c_void_p(lab.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                        None)
    assert st == lp.LP_EINVAL
    assert lp.lp_edge_cut(G, lab) == g.two_m // 2  # builds the plan; singletons cut every edge
    assert _noalloc(lp, G, lab) == g.two_m // 2
    G.free()
