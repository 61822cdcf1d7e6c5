"""Batched form vs each graph alone (GPU) and vs the CPU oracle: the labels of
every graph of a batch must equal, element by element, those of the graph
clustered on its own (all-integer work: tolerance zero)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _np(t):
    return t.cpu().numpy()


def _h(lp, g, compressed=True):
    make = lp.lp_compress if compressed else lp.lp_graph_from_csr
    return make(g.n, g.xadj.view(np.int64), g.adjncy, g.adjwgt, g.vwgt)


def _mix(synth_mod, weighted=False, count=12, seed=40):
    out = []
    for i in range(count):
        n = [300, 1000, 2500, 5000][i % 4]
        if i % 3 == 0:
            g = synth_mod.rgg(2, n, synth_mod.rgg_radius(2, n, 8.0), seed=seed + i)
        else:
            g = synth_mod.rmat_scale(int(np.ceil(np.log2(n))), 8 + i % 9, seed=seed + i)
        if weighted:
            g.adjwgt = synth_mod.edge_weights(g, 1, 50, seed + i)
            g.vwgt = synth_mod.vertex_weights(g.n, 1, 3, seed + i)
        out.append(g)
    return out


@pytest.mark.parametrize("compressed", [True, False])
@pytest.mark.parametrize("weighted", [False, True])
def test_batch_matches_oracle_and_alone(lp, oracle_mod, synth_mod, compressed, weighted):
    gs = _mix(synth_mod, weighted)
    hs = [_h(lp, g, compressed) for g in gs]
    caps = [3 * int(np.ceil(g.two_m / max(g.n, 1))) + (7 * i) % 11 for i, g in enumerate(gs)]
    seeds = [1000 + 17 * i for i in range(len(gs))]
    b = lp.lp_batch_create(hs)
    assert b.G == len(gs) and b.vbase[-1] == sum(g.n for g in gs)
    lab = lp.lp_batch_cluster_ex(b, caps, 5, seeds)
    for i, (g, h) in enumerate(zip(gs, hs)):
        got = _np(b.split(lab)[i])
        alone = _np(lp.lp_cluster(h, caps[i], 5, seeds[i]))
        exp, _ = oracle_mod.lp_cluster(g, caps[i], 5, seeds[i])
        assert np.array_equal(got, alone), i
        assert np.array_equal(got, exp), i


@pytest.mark.parametrize("knobs", [dict(t_lane=1, t_tile=64, t_block=256, hub_part=256),
                                   dict(t_lane=1, t_tile=2048, t_block=4096),
                                   dict(t_lane=16, t_tile=16, t_block=16, hub_part=512)])
def test_batch_knobs_and_tile_boundaries(lp, oracle_mod, synth_mod, knobs):
    # t_lane=1 packs up to 80 vertices in a tile: tiles must stop at graph ends
    gs = _mix(synth_mod, count=9, seed=70)
    hs = [_h(lp, g) for g in gs]
    caps = [40] * len(gs)
    seeds = list(range(len(gs)))
    b = lp.lp_batch_create(hs)
    lab = lp.lp_batch_cluster_ex(b, caps, 4, seeds, config=knobs)
    for i, g in enumerate(gs):
        exp, _ = oracle_mod.lp_cluster(g, caps[i], 4, seeds[i])
        assert np.array_equal(_np(b.split(lab)[i]), exp), i


def test_batch_with_hubs_and_degenerate_graphs(lp, oracle_mod, synth_mod):
    star = synth_mod.from_edges(25001, [(7, v) for v in range(25001) if v != 7])
    gs = [synth_mod.from_edges(1, []), synth_mod.from_edges(50, []), star,
          synth_mod.rmat_scale(12, 16, seed=2), synth_mod.from_edges(2, [(0, 1)])]
    hs = [_h(lp, g) for g in gs]
    caps = [5, 5, 300, 64, 2]
    seeds = [3, 4, 5, 6, 7]
    outs = lp.lp_batch_cluster(hs, caps, 3, seeds)
    for i, g in enumerate(gs):
        exp, _ = oracle_mod.lp_cluster(g, caps[i], 3, seeds[i])
        assert np.array_equal(_np(outs[i]), exp), i


def test_batch_many_small_graphs(lp, oracle_mod, synth_mod):
    gs = [synth_mod.random_small(5 + i % 23, 0.3, seed=i) for i in range(200)]
    hs = [_h(lp, g) for g in gs]
    caps = [2 + i % 5 for i in range(len(gs))]
    seeds = [i * 31 for i in range(len(gs))]
    outs = lp.lp_batch_cluster(hs, caps, 5, seeds)
    for i, g in enumerate(gs):
        exp, _ = oracle_mod.lp_cluster(g, caps[i], 5, seeds[i])
        assert np.array_equal(_np(outs[i]), exp), i


def test_batch_contract_and_cut_see_the_union(lp, oracle_mod, synth_mod):
    gs = _mix(synth_mod, count=6, seed=90)
    hs = [_h(lp, g) for g in gs]
    caps = [30] * len(gs)
    seeds = [9] * len(gs)
    b = lp.lp_batch_create(hs)
    lab = lp.lp_batch_cluster_ex(b, caps, 5, seeds)
    glob = lab.clone()
    for i in range(b.G):
        glob[b.vbase[i]: b.vbase[i + 1]] += b.vbase[i]
    C, mp = lp.lp_contract(b, glob)
    xa, ad, wt, vw = lp.lp_decompress(C)
    xa, ad, wt, vw, mp = _np(xa).view(np.uint64), _np(ad), _np(wt), _np(vw), _np(mp)
    cb = 0
    cut_total = 0
    for i, g in enumerate(gs):
        loc = _np(b.split(lab)[i])
        oc, omap = oracle_mod.contract(g, loc)
        assert np.array_equal(mp[b.vbase[i]: b.vbase[i + 1]], omap + cb)
        sub_x = xa[cb: cb + oc.n + 1] - xa[cb]
        assert np.array_equal(sub_x, oc.xadj)
        e0 = int(xa[cb])
        assert np.array_equal(ad[e0: e0 + oc.two_m], oc.adjncy + cb)
        assert np.array_equal(vw[cb: cb + oc.n], oc.vwgt)
        cb += oc.n
        cut_total += oracle_mod.edge_cut(g, loc)
    assert C.n == cb
    assert lp.lp_edge_cut(b, glob) == cut_total


def test_batch_errors(lp, synth_mod):
    g = synth_mod.rgg2d_16k()
    a, p = _h(lp, g, True), _h(lp, g, False)
    with pytest.raises(lp.LPError):
        lp.lp_batch_create([a, p])  # mixed representations
    b = lp.lp_batch_create([a, a])
    with pytest.raises(lp.LPError):
        lp.lp_cluster(b, 32, 5, 1)  # a batch needs per-graph caps and seeds
    with pytest.raises(lp.LPError):
        lp.lp_decompress(b)
    with pytest.raises(lp.LPError):
        lp.lp_batch_cluster_ex(b, [32, 0], 5, [1, 1])
    with pytest.raises(lp.LPError):
        lp.lp_batch_create([b, a])  # batches do not nest
