"""Handles made inside a call on a stream (coarse graphs, batches) live in the
device's stream-ordered pool and are released in that stream's order: their
contents must be right when used on another stream after ordering, and
memory released by one handle and taken by the next must not leak values."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _np(t):
    return t.cpu().numpy()


def test_coarse_graph_made_on_a_stream(lp, oracle_mod, synth_mod):
    import torch

    g = synth_mod.rmat_scale(12, 8, seed=3)
    exp_lab, _ = oracle_mod.lp_cluster(g, 64, 5, 1)
    cg, mp = oracle_mod.contract(g, exp_lab)
    exp_lab2, _ = oracle_mod.lp_cluster(cg, 256, 5, 2)
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for it in range(3):  # later iterations reuse memory the earlier ones released
        with torch.cuda.stream(s1):
            lab = lp.lp_cluster(G, 64, 5, 1)
            C, M = lp.lp_contract(G, lab)
        s2.wait_stream(s1)
        with torch.cuda.stream(s2):
            lab2 = lp.lp_cluster(C, 256, 5, 2)
            x, a, w, v = lp.lp_decompress(C)
        s1.wait_stream(s2)  # the caller orders s2's use before the release on s1
        C.free()
        s1.synchronize()
        assert np.array_equal(_np(lab), exp_lab), it
        assert np.array_equal(_np(M), mp), it
        assert np.array_equal(_np(x).view(np.uint64), cg.xadj), it
        assert np.array_equal(_np(a), cg.adjncy) and np.array_equal(_np(w), cg.adjwgt), it
        assert np.array_equal(_np(v), cg.vwgt), it
        assert np.array_equal(_np(lab2), exp_lab2), it


def test_batch_made_on_a_stream(lp, oracle_mod, synth_mod):
    import torch

    recipe = [("rgg2d", 900, 8, 21), ("rmat", 700, 10, 22), ("rmat", 3000, 9, 23)]
    gs = [synth_mod.batch_graph(*r) for r in recipe]
    hs = [lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy) for g in gs]
    caps, seeds = [40, 17, 90], [5, 6, 7]
    exp = [oracle_mod.lp_cluster(g, c, 5, sd)[0] for g, c, sd in zip(gs, caps, seeds)]
    s = torch.cuda.Stream()
    for it in range(3):
        with torch.cuda.stream(s):
            outs = lp.lp_batch_cluster(hs, caps, 5, seeds)
            B = lp.lp_batch_create(hs)
            lab = lp.lp_batch_cluster_ex(B, caps, 5, seeds)
            shift = torch.tensor(np.repeat(B.vbase[:-1], np.diff(B.vbase)), device="cuda", dtype=torch.int32)
            cut = lp.lp_edge_cut(B, lab + shift)
            B.free()
        s.synchronize()
        for o, e, part in zip(outs, exp, B.split(_np(lab))):
            assert np.array_equal(_np(o), e) and np.array_equal(part, e), it
        assert cut == sum(oracle_mod.edge_cut(g, e) for g, e in zip(gs, exp)), it


def test_results_stable_across_cache_reuse_and_trim(lp, oracle_mod, synth_mod):
    # calls reuse cached blocks that still hold earlier calls' data; emptying
    # the cache in between must not change anything either
    g = synth_mod.rmat_scale(13, 12, seed=9)
    exp_lab, _ = oracle_mod.lp_cluster(g, 100, 5, 3)
    cg, mp = oracle_mod.contract(g, exp_lab)
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
    for it in range(4):
        lab = lp.lp_cluster(G, 100, 5, 3)
        C, M = lp.lp_contract(G, lab)
        x, a, w, v = lp.lp_decompress(C)
        assert np.array_equal(_np(lab), exp_lab), it
        assert np.array_equal(_np(x).view(np.uint64), cg.xadj) and np.array_equal(_np(a), cg.adjncy), it
        assert np.array_equal(_np(w), cg.adjwgt) and np.array_equal(_np(M), mp), it
        assert lp.lp_edge_cut(G, lab) == oracle_mod.edge_cut(g, exp_lab), it
        C.free()
        if it == 1:
            lp.lp_trim_memory()
