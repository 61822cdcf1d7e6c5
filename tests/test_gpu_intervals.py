"""Interval encoding on the GPU (Section III-A; layout in include/lp.h):
compressed bytes equal the oracle's encoder byte for byte, decompression
gives back the sorted CSR, and every step that decodes neighbourhoods -
clustering on every rating path (lanes, small and large tiles, hub pieces,
split and unsplit records), contraction, the cut, sub-rounds, batches and
the gain table's refinement - gives exactly the results of the oracle, which
works on the plain CSR (results never depend on the format)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _np(t):
    return t.cpu().numpy()


def _star(synth_mod, d, center, weights=False):
    n = d + 1
    edges = [(center, v) for v in range(n) if v != center]
    w = [1 + (i * 7919) % 1000 for i in range(len(edges))] if weights else None
    return synth_mod.from_edges(n, edges, w)


def _graphs(synth_mod):
    out = {"rgg2d-16k": synth_mod.rgg2d_16k(seed=2), "rgg3d-2^14": synth_mod.rgg3d(1 << 14, 27.0, seed=2),
           "rmat-s12": synth_mod.rmat_scale(12, 8, seed=3)}
    g = synth_mod.rgg3d(1 << 13, 27.0, seed=4)
    g.adjwgt = synth_mod.edge_weights(g, 1, 50, 4)
    g.vwgt = synth_mod.vertex_weights(g.n, 1, 3, 4)
    out["rgg3d-weighted"] = g
    out["star-4000"] = _star(synth_mod, 4000, 2000)     # the largest unsplit record
    out["star-4001-w"] = _star(synth_mod, 4001, 17, True)  # split into five chunks
    out["star-25000"] = _star(synth_mod, 25000, 12345)
    # consecutive runs across chunk boundaries and mixed with gaps
    edges = [(0, v) for v in range(1, 9000) if v % 7 != 3] + [(v, v + 1) for v in range(1, 8999, 2)]
    out["runs-9000"] = synth_mod.from_edges(9000, edges)
    return out


@pytest.fixture(scope="module")
def graphs(synth_mod):
    return _graphs(synth_mod)


NAMES = ["rgg2d-16k", "rgg3d-2^14", "rmat-s12", "rgg3d-weighted", "star-4000", "star-4001-w", "star-25000",
         "runs-9000"]


@pytest.mark.parametrize("name", NAMES)
def test_bytes_match_oracle_and_roundtrip(lp, oracle_mod, graphs, name):
    g = graphs[name]
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy, g.adjwgt, g.vwgt, intervals=True)
    assert G.intervals and G.compressed
    offs, data = lp.lp_graph_export(G)
    eo, ed = oracle_mod.compress(g.n, g.xadj, g.adjncy, g.adjwgt, intervals=True)
    assert np.array_equal(_np(offs).view(np.uint64), eo) and np.array_equal(_np(data), ed)
    x, a, w, v = lp.lp_decompress(G)
    assert np.array_equal(_np(x).view(np.uint64), g.xadj) and np.array_equal(_np(a), g.adjncy)
    if g.adjwgt is not None:
        assert np.array_equal(_np(w), g.adjwgt)
    G.free()


KNOBS = [None, dict(t_lane=1, t_tile=1, t_block=1, hub_part=256), dict(t_lane=4, t_tile=64, t_block=64),
         dict(t_lane=16, t_tile=16, t_block=16, hub_part=512, overlap=1)]


@pytest.mark.parametrize("knobs", KNOBS)
@pytest.mark.parametrize("name", NAMES)
def test_labels_match_oracle(lp, oracle_mod, graphs, name, knobs):
    g = graphs[name]
    cap = 40 if "star" not in name else 300
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy, g.adjwgt, g.vwgt, intervals=True)
    exp, ost = oracle_mod.lp_cluster(g, cap, 4, 5)
    lab, st = lp.lp_cluster(G, cap, 4, 5, config=knobs, stats=True)
    assert np.array_equal(_np(lab), exp)
    assert st.proposals == ost.proposals and st.moves == ost.moves
    G.free()


@pytest.mark.parametrize("name", NAMES)
def test_contraction_and_cut_match_oracle(lp, oracle_mod, graphs, name):
    g = graphs[name]
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy, g.adjwgt, g.vwgt, intervals=True)
    lab = lp.lp_cluster(G, 40, 4, 7)
    exp, _ = oracle_mod.lp_cluster(g, 40, 4, 7)
    assert np.array_equal(_np(lab), exp)
    C, mp = lp.lp_contract(G, lab)
    cg, emp = oracle_mod.contract(g, exp)
    x, a, w, v = lp.lp_decompress(C)
    assert C.n == cg.n and np.array_equal(_np(mp), emp)
    assert np.array_equal(_np(x).view(np.uint64), cg.xadj) and np.array_equal(_np(a), cg.adjncy)
    assert np.array_equal(_np(w), cg.adjwgt) and np.array_equal(_np(v), cg.vwgt)
    assert lp.lp_edge_cut(G, lab) == oracle_mod.edge_cut(g, exp)
    C.free()
    G.free()


@pytest.mark.parametrize("S", [2, 4])
def test_subrounds_match_oracle(lp, oracle_mod, graphs, S):
    g = graphs["rgg3d-2^14"]
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy, intervals=True)
    exp, _ = oracle_mod.lp_cluster(g, 64, 5, 3, subrounds=S)
    assert np.array_equal(_np(lp.lp_cluster(G, 64, 5, 3, config=dict(subrounds=S))), exp)
    G.free()


def test_batch_of_interval_graphs(lp, graphs):
    names = ["rgg2d-16k", "rgg3d-2^14", "star-25000", "runs-9000"]
    hs = [lp.lp_compress(graphs[k].n, graphs[k].xadj.view(np.int64), graphs[k].adjncy, intervals=True)
          for k in names]
    caps, seeds = [32, 48, 300, 20], [1, 2, 3, 4]
    outs = lp.lp_batch_cluster(hs, caps, 4, seeds)
    for h, c, sd, o in zip(hs, caps, seeds, outs):
        assert np.array_equal(_np(o), _np(lp.lp_cluster(h, c, 4, sd)))
    # a batch mixes formats only in the same encoding
    plain = lp.lp_compress(graphs["rmat-s12"].n, graphs["rmat-s12"].xadj.view(np.int64), graphs["rmat-s12"].adjncy)
    with pytest.raises(lp.LPError):
        lp.lp_batch_create([hs[0], plain])
    for h in hs + [plain]:
        h.free()


@pytest.mark.parametrize("name", ["rgg3d-2^14", "rgg3d-weighted", "star-25000"])
def test_gain_table_refinement_matches_oracle(lp, oracle_mod, graphs, name):
    g = graphs[name]
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy, g.adjwgt, g.vwgt, intervals=True)
    k = 4
    start = oracle_mod.initial_partition(g, k)
    lmax = lp.max_block_weight(G.total_vwgt, k)
    exp, _ = oracle_mod.lp_refine(g, start, k, lmax, 5, 11)
    for cfg in (None, dict(gain_table=1)):
        got = lp.lp_refine(G, start, k, lmax, 5, 11, config=cfg)
        assert np.array_equal(_np(got), exp), cfg
    G.free()


def test_interval_bytes_smaller_on_geometric_graphs(lp, graphs):
    g = graphs["rgg3d-2^14"]
    a = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
    b = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy, intervals=True)
    assert b.nbytes < a.nbytes and not a.intervals
    a.free()
    b.free()


def test_unknown_flags_rejected(lp, graphs):
    import ctypes
    import torch
    g = graphs["rgg2d-16k"]
    x = torch.from_numpy(g.xadj.view(np.int64)).cuda()
    a = torch.from_numpy(g.adjncy).cuda()
    h = ctypes.c_void_p()
    st = lp._load().lp_compress_ex(g.n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(a.data_ptr()), None, None, 6,
                                   None, ctypes.byref(h))
    assert st == lp.LP_EINVAL
