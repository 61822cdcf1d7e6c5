"""GPU library vs CPU oracle, element by element (all-integer work: the
tolerance is zero). Every call goes through the C ABI of liblpgpu.so."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _np(t):
    return t.cpu().numpy()


def _gpu_graph(lp, g, compressed=True):
    make = lp.lp_compress if compressed else lp.lp_graph_from_csr
    return make(g.n, g.xadj.view(np.int64), g.adjncy, g.adjwgt, g.vwgt)


def _star(synth_mod, d, center=0, weights=False):
    n = d + 1
    edges = [(center, v) for v in range(n) if v != center]
    w = [1 + (i * 7919) % 1000 for i in range(len(edges))] if weights else None
    return synth_mod.from_edges(n, edges, w)


def _graphs(synth_mod):
    out = {}
    out["rgg2d-16k"] = synth_mod.rgg2d_16k()
    out["rmat-s13-ef16"] = synth_mod.rmat_scale(13, 16, seed=3)
    g = synth_mod.rmat_scale(12, 8, seed=5)
    g.adjwgt = synth_mod.edge_weights(g, 1, 100, 5)
    g.vwgt = synth_mod.vertex_weights(g.n, 1, 4, 5)
    out["rmat-s12-weighted"] = g
    out["star-25000"] = _star(synth_mod, 25000, center=7)
    out["star-10001-w"] = _star(synth_mod, 10001, center=5000, weights=True)
    out["bip-5x2048"] = _bipartite(synth_mod, 5, 2048)
    out["bip-5x2048-heavy"] = _bipartite(synth_mod, 5, 2048, heavy=True)
    out["bip-3x9000-w"] = _bipartite(synth_mod, 3, 9000, small=True)  # unsplit hubs cut into pieces
    return out


def _bipartite(synth_mod, a, b, heavy=False, small=False):
    # complete bipartite K_{a,b} plus a path over the b side: the a side has
    # degree b exactly (the largest degree rated in tiles); with heavy random
    # weights each of its records takes about 6 bytes per neighbour, so tiles
    # are cut by their byte budget
    edges = [(i, a + j) for i in range(a) for j in range(b)]
    edges += [(a + j, a + j + 1) for j in range(b - 1)]
    w = None
    if heavy:
        w = [2**29 + (k * 2654435761) % (2**31 - 2**29 - 1) for k in range(len(edges))]
    elif small:
        w = [1 + (k * 7919) % 100 for k in range(len(edges))]
    return synth_mod.from_edges(a + b, edges, w)


@pytest.fixture(scope="module")
def graphs(synth_mod):
    return _graphs(synth_mod)


# ------------------------------------------------------------------ codec --

@pytest.mark.parametrize("name", ["rgg2d-16k", "rmat-s13-ef16", "rmat-s12-weighted", "star-25000", "star-10001-w"])
def test_compress_bytes_match_oracle(lp, oracle_mod, graphs, name):
    g = graphs[name]
    G = _gpu_graph(lp, g)
    offs, data = lp.lp_graph_export(G)
    o_offs, o_data = oracle_mod.compress(g.n, g.xadj, g.adjncy, g.adjwgt)
    assert np.array_equal(_np(offs).view(np.uint64), o_offs)
    assert np.array_equal(_np(data), o_data)


@pytest.mark.parametrize("name", ["rgg2d-16k", "rmat-s13-ef16", "rmat-s12-weighted", "star-25000", "star-10001-w"])
def test_decompress_roundtrip(lp, graphs, name):
    g = graphs[name]
    G = _gpu_graph(lp, g)
    x, a, w, v = lp.lp_decompress(G)
    assert np.array_equal(_np(x).view(np.uint64), g.xadj)
    assert np.array_equal(_np(a), g.adjncy)
    assert np.array_equal(_np(w), g.adjwgt if g.adjwgt is not None else np.ones(g.two_m, np.int32))
    assert np.array_equal(_np(v), g.vwgt if g.vwgt is not None else np.ones(g.n, np.int32))


@pytest.mark.parametrize("case", ["hub-then-isolated", "isolated-only", "weighted-hubs-first"])
def test_codec_work_blocks(lp, oracle_mod, synth_mod, case):
    # the codec kernels take vertices in blocks of 16384 units of work (degree
    # plus one per vertex): hubs spanning many blocks, long runs of isolated
    # vertices, and a work total that is an exact multiple of the block
    if case == "hub-then-isolated":
        edges = [(0, v) for v in range(1, 40001)] + [(90001 + i, 90002 + i) for i in range(999)]
        g = synth_mod.from_edges(91001, edges)
    elif case == "isolated-only":
        g = synth_mod.from_edges(16384, [])
    else:
        hubs = [(h, v) for h in range(3) for v in range(3, 30003) if (v * 7 + h) % 3]
        g = synth_mod.from_edges(30003 + 70000, hubs, [1 + (i * 7919) % 50 for i in range(len(hubs))])
    G = _gpu_graph(lp, g)
    offs, data = lp.lp_graph_export(G)
    o_offs, o_data = oracle_mod.compress(g.n, g.xadj, g.adjncy, g.adjwgt)
    assert np.array_equal(_np(offs).view(np.uint64), o_offs)
    assert np.array_equal(_np(data), o_data)
    x, a, w, v = lp.lp_decompress(G)
    assert np.array_equal(_np(x).view(np.uint64), g.xadj) and np.array_equal(_np(a), g.adjncy)
    if g.adjwgt is not None:
        assert np.array_equal(_np(w), g.adjwgt)


def test_compress_rejects_bad_input(lp, synth_mod):
    g = synth_mod.from_edges(3, [(0, 1), (1, 2)])
    adj = g.adjncy.copy()
    adj[0] = 7  # out of range
    with pytest.raises(lp.LPError):
        lp.lp_compress(g.n, g.xadj.view(np.int64), adj)
    adj = g.adjncy.copy()
    adj[0] = 0  # self-loop
    with pytest.raises(lp.LPError):
        lp.lp_compress(g.n, g.xadj.view(np.int64), adj)
    with pytest.raises(lp.LPError):
        lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy, np.array([1, 0, 1, 1], np.int32))
    h = synth_mod.from_edges(4, [(0, 1), (0, 2)])
    adj = h.adjncy.copy()
    adj[0], adj[1] = adj[1], adj[0]  # unsorted neighbourhood
    with pytest.raises(lp.LPError):
        lp.lp_compress(h.n, h.xadj.view(np.int64), adj)
    x = g.xadj.copy()
    x[1], x[2] = x[2], x[1]  # offsets that decrease
    for make in (lp.lp_compress, lp.lp_graph_from_csr):
        with pytest.raises(lp.LPError) as e:
            make(g.n, x.view(np.int64), g.adjncy)
        assert e.value.status == lp.LP_EINVAL


# ----------------------------------------------------------------- cluster --

CASES = [
    ("rgg2d-16k", 32, 5, 1),
    ("rmat-s13-ef16", 256, 5, 1),
    ("rmat-s13-ef16", 20, 5, 7),
    ("rmat-s12-weighted", 60, 5, 3),
    ("star-25000", 300, 3, 2),
    ("star-10001-w", 5000, 3, 2),
    ("bip-5x2048", 700, 4, 3),
    ("bip-5x2048-heavy", 900, 4, 4),
    ("bip-3x9000-w", 30000, 4, 5),
]


@pytest.mark.parametrize("name,cap,rounds,seed", CASES)
@pytest.mark.parametrize("compressed", [True, False])
def test_cluster_matches_oracle(lp, oracle_mod, graphs, name, cap, rounds, seed, compressed):
    g = graphs[name]
    G = _gpu_graph(lp, g, compressed)
    lab, st = lp.lp_cluster(G, cap, rounds, seed, stats=True)
    exp, ost = oracle_mod.lp_cluster(g, cap, rounds, seed)
    assert np.array_equal(_np(lab), exp)
    assert st.rounds_run == ost.rounds_run
    assert st.proposals == ost.proposals and st.moves == ost.moves


KNOBS = [
    dict(t_lane=1, t_tile=1, t_block=1, hub_part=256),        # almost everything on the hub path
    dict(t_lane=16, t_tile=16, t_block=16, hub_part=512),
    dict(t_lane=4, t_tile=64, t_block=64, hub_part=1024),
    dict(t_lane=16, t_tile=512, t_block=4096, hub_part=8192),
    dict(t_lane=8, t_tile=100, t_block=1000, hub_part=300),
    dict(t_lane=1, t_tile=2048, t_block=2048, hub_part=4096),   # tiles of up to 128 vertices
    dict(overlap=1),                                            # rating paths on concurrent streams
    dict(t_lane=4, t_tile=64, t_block=64, hub_part=1024, overlap=1),
]


@pytest.mark.parametrize("knobs", KNOBS)
@pytest.mark.parametrize("name", ["rmat-s13-ef16", "rmat-s12-weighted", "star-25000", "bip-5x2048-heavy",
                                  "bip-3x9000-w"])
@pytest.mark.parametrize("compressed", [True, False])
def test_bucket_thresholds_do_not_change_results(lp, oracle_mod, graphs, knobs, name, compressed):
    g = graphs[name]
    G = _gpu_graph(lp, g, compressed)
    exp, _ = oracle_mod.lp_cluster(g, 64, 4, 11)
    lab = lp.lp_cluster(G, 64, 4, 11, config=knobs)
    assert np.array_equal(_np(lab), exp)


def test_wide_ratings_path(lp, oracle_mod, synth_mod):
    # weighted degrees above 2^31 switch the LDS tables to 64-bit ratings
    g = synth_mod.rmat_scale(12, 8, seed=9)
    g.adjwgt = synth_mod.edge_weights(g, 2**29, 2**31 - 1, 9)
    G = _gpu_graph(lp, g)
    exp, _ = oracle_mod.lp_cluster(g, 40, 5, 2)
    assert np.array_equal(_np(lp.lp_cluster(G, 40, 5, 2)), exp)


@pytest.mark.parametrize("case", ["single", "no-edges", "cap1", "zero-rounds", "matching"])
def test_degenerate_cases(lp, oracle_mod, synth_mod, case):
    if case == "single":
        g, cap, r = synth_mod.from_edges(1, []), 5, 5
    elif case == "no-edges":
        g, cap, r = synth_mod.from_edges(100, []), 5, 5
    elif case == "cap1":
        g, cap, r = synth_mod.rgg2d_16k(), 1, 5
    elif case == "zero-rounds":
        g, cap, r = synth_mod.rgg2d_16k(), 32, 0
    else:
        g, cap, r = synth_mod.from_edges(200, [(2 * i, 2 * i + 1) for i in range(100)]), 2, 3
    G = _gpu_graph(lp, g)
    exp, _ = oracle_mod.lp_cluster(g, cap, r, 1)
    assert np.array_equal(_np(lp.lp_cluster(G, cap, r, 1)), exp)


def test_cluster_argument_errors(lp, graphs):
    G = _gpu_graph(lp, graphs["rgg2d-16k"])
    with pytest.raises(lp.LPError):
        lp.lp_cluster(G, 0, 5, 1)
    with pytest.raises(lp.LPError):
        lp.lp_cluster(G, 5, -1, 1)
    with pytest.raises(lp.LPError):
        lp.lp_cluster(G, 5, 1, 1, config=dict(t_lane=17))
    with pytest.raises(lp.LPError):
        lp.lp_cluster(G, 5, 1, 1, config=dict(t_block=8192))
    with pytest.raises(lp.LPError):
        lp.lp_cluster(G, 5, 1, 1, config=dict(t_tile=4096, t_block=4096))
    with pytest.raises(lp.LPError):
        lp.lp_cluster(G, 5, 1, 1, config=dict(t_tile=64, t_block=32))


def test_repeatable(lp, graphs):
    G = _gpu_graph(lp, graphs["rmat-s13-ef16"])
    a = _np(lp.lp_cluster(G, 100, 5, 5))
    for _ in range(3):
        assert np.array_equal(_np(lp.lp_cluster(G, 100, 5, 5)), a)


# ---------------------------------------------------------------- contract --

@pytest.mark.parametrize("name,cap", [("rgg2d-16k", 32), ("rmat-s13-ef16", 256), ("rmat-s13-ef16", 5000),
                                      ("rmat-s12-weighted", 200), ("star-25000", 30000)])
@pytest.mark.parametrize("compressed", [True, False])
def test_contract_matches_oracle(lp, oracle_mod, graphs, name, cap, compressed):
    g = graphs[name]
    exp_lab, _ = oracle_mod.lp_cluster(g, cap, 5, 1)
    cg, mp = oracle_mod.contract(g, exp_lab)
    G = _gpu_graph(lp, g, compressed)
    C, M = lp.lp_contract(G, exp_lab)
    assert C.n == cg.n and C.two_m == cg.two_m and not C.compressed
    x, a, w, v = lp.lp_decompress(C)
    assert np.array_equal(_np(M), mp)
    assert np.array_equal(_np(x).view(np.uint64), cg.xadj)
    assert np.array_equal(_np(a), cg.adjncy)
    assert np.array_equal(_np(w), cg.adjwgt)
    assert np.array_equal(_np(v), cg.vwgt)
    assert lp.lp_edge_cut(G, exp_lab) == oracle_mod.edge_cut(g, exp_lab)


def test_contract_identity_and_all_in_one(lp, oracle_mod, graphs):
    g = graphs["rmat-s13-ef16"]
    G = _gpu_graph(lp, g)
    C, M = lp.lp_contract(G, np.arange(g.n, dtype=np.int32))
    x, a, w, v = lp.lp_decompress(C)
    assert np.array_equal(_np(a), g.adjncy) and (_np(w) == 1).all()
    C, M = lp.lp_contract(G, np.full(g.n, 3, dtype=np.int32))
    assert C.n == 1 and C.two_m == 0 and int(_np(lp.lp_decompress(C)[3])[0]) == g.n


def test_contract_heavy_windows(lp, oracle_mod, synth_mod):
    # random labels with few clusters: every cluster is heavy (large member
    # degree) and has many distinct coarse neighbours
    g = synth_mod.rmat_scale(14, 16, seed=8)
    rng = np.random.default_rng(3)
    lab = rng.integers(0, 20000, g.n).astype(np.int32) % g.n
    cg, mp = oracle_mod.contract(g, lab)
    C, M = lp.lp_contract(_gpu_graph(lp, g), lab)
    x, a, w, v = lp.lp_decompress(C)
    assert np.array_equal(_np(a), cg.adjncy) and np.array_equal(_np(w), cg.adjwgt)
    assert np.array_equal(_np(x).view(np.uint64), cg.xadj)


def test_contract_errors(lp, synth_mod):
    g = synth_mod.from_edges(4, [(0, 2), (1, 3)], [2**31 - 1, 2**31 - 1])
    G = _gpu_graph(lp, g)
    with pytest.raises(lp.LPError) as e:
        lp.lp_contract(G, np.array([0, 0, 2, 2], dtype=np.int32))
    assert e.value.status == lp.LP_EOVERFLOW
    with pytest.raises(lp.LPError) as e:
        lp.lp_contract(G, np.array([0, 9, 2, 2], dtype=np.int32))
    assert e.value.status == lp.LP_EINVAL


@pytest.mark.parametrize("compressed", [True, False])
def test_contract_wide_weighted_degrees(lp, oracle_mod, synth_mod, compressed):
    # a centre whose summed weight exceeds 2^31 (records keep one per edge,
    # no per-vertex sums) next to low-degree vertices, leaves grouped in
    # threes so every coarse edge weight still fits 32 bits; also a hub
    # wider than the whole-hub limit
    k = 40000
    edges = [(0, 1 + j) for j in range(k)] + [(1 + j, 2 + j) for j in range(k - 1)]
    w = [2**29 + (j * 7919) % 1000 for j in range(k)] + [1 + j % 5 for j in range(k - 1)]
    g = synth_mod.from_edges(k + 1, edges, w)
    lab = np.concatenate([[0], 1 + 3 * (np.arange(k) // 3)]).astype(np.int32)
    cg, mp = oracle_mod.contract(g, lab)
    C, M = lp.lp_contract(_gpu_graph(lp, g, compressed), lab)
    x, a, w_, v = lp.lp_decompress(C)
    assert np.array_equal(_np(M), mp)
    assert np.array_equal(_np(x).view(np.uint64), cg.xadj)
    assert np.array_equal(_np(a), cg.adjncy) and np.array_equal(_np(w_), cg.adjwgt)


def _hot_cluster(synth_mod, weighted=False):
    # cluster A (10^6 vertices, label 0) joined to both vertices of cluster B
    # and to 8 of 200000 singleton clusters C each: 10^7 records in A, so its
    # partitions are as many as the splitter sample allows (about 4900
    # records, over 1024 distinct: several windows), and the partition of B's
    # coarse vertex holds its 10^6 summed records plus the spread ones that
    # follow in ID order (over 16384 records and 4096 distinct: the wide
    # reduction with its own window retries)
    na, nb, nc = 1_000_000, 2, 200_000
    a = np.arange(na, dtype=np.int64)
    e = [np.stack([a, np.full(na, na + j, np.int64)], 1) for j in range(nb)]
    e += [np.stack([a, na + nb + (7 * a + 25_000 * k) % nc], 1) for k in range(8)]
    e = np.concatenate(e)
    w = (1 + (e[:, 0] * 7 + e[:, 1]) % 5).astype(np.int64) if weighted else None
    g = synth_mod.from_edges(na + nb + nc, e, w)
    lab = np.concatenate([np.zeros(na), np.full(nb, na), na + nb + np.arange(nc)]).astype(np.int32)
    return g, lab


@pytest.mark.parametrize("compressed,weighted", [(True, False), (False, False), (True, True)])
def test_contract_hot_neighbour_and_wide_reduction(lp, oracle_mod, synth_mod, compressed, weighted):
    # weighted: 64-bit table sums in every reduction configuration
    g, lab = _hot_cluster(synth_mod, weighted)
    cg, mp = oracle_mod.contract(g, lab)
    C, M = lp.lp_contract(_gpu_graph(lp, g, compressed), lab)
    x, a, w, v = lp.lp_decompress(C)
    assert np.array_equal(_np(M), mp)
    assert np.array_equal(_np(x).view(np.uint64), cg.xadj)
    assert np.array_equal(_np(a), cg.adjncy) and np.array_equal(_np(w), cg.adjwgt)
    assert np.array_equal(_np(v), cg.vwgt)


def test_cut_matches_oracle(lp, oracle_mod, graphs):
    for name in ("rgg2d-16k", "rmat-s12-weighted", "star-10001-w"):
        g = graphs[name]
        lab = (np.arange(g.n) * 2654435761 % 97).astype(np.int32)
        for comp in (True, False):
            assert lp.lp_edge_cut(_gpu_graph(lp, g, comp), lab) == oracle_mod.edge_cut(g, lab)


# ---------------------------------------------------------------- coarsen --

@pytest.mark.parametrize("which", ["rgg2d", "rmat"])
def test_coarsening_matches_oracle(lp, oracle_mod, synth_mod, which):
    if which == "rgg2d":
        g = synth_mod.rgg(2, 1 << 16, synth_mod.rgg_radius(2, 1 << 16, 8.0), 4)
    else:
        g = synth_mod.rmat_scale(15, 16, seed=4)
    levels, final, n_target, cap = oracle_mod.coarsen(g, 1)
    glev, gfinal, gt, gcap = lp.coarsen(_gpu_graph(lp, g), 1)
    assert (gt, gcap) == (n_target, cap)
    assert [G.n for G, _, _ in glev] == [lv[0].n for lv in levels]
    for (G, lab, mp), (og, olab, omp) in zip(glev, levels):
        assert np.array_equal(_np(lab), olab) and np.array_equal(_np(mp), omp)
    x, a, w, v = lp.lp_decompress(gfinal)
    assert np.array_equal(_np(a), final.adjncy) and np.array_equal(_np(w), final.adjwgt)
    assert np.array_equal(_np(v), final.vwgt)


@pytest.mark.parametrize("labels_kind", ["star-identity", "blocks-64", "blocks-4096"])
def test_contract_light_to_heavy_handover(lp, oracle_mod, synth_mod, labels_kind):
    # star-identity: one cluster with 3000 distinct coarse neighbours and
    # member degree 3000 (large light class, handed to the heavy path);
    # blocks-k: clusters of k consecutive R-MAT vertices (many members each)
    if labels_kind == "star-identity":
        g = _star(synth_mod, 3000, center=11)
        lab = np.arange(g.n, dtype=np.int32)
    else:
        g = synth_mod.rmat_scale(14, 16, seed=6)
        k = int(labels_kind.split("-")[1])
        lab = ((np.arange(g.n) // k) * k).astype(np.int32)
    cg, mp = oracle_mod.contract(g, lab)
    for comp in (True, False):
        C, M = lp.lp_contract(_gpu_graph(lp, g, comp), lab)
        x, a, w, v = lp.lp_decompress(C)
        assert np.array_equal(_np(x).view(np.uint64), cg.xadj)
        assert np.array_equal(_np(a), cg.adjncy) and np.array_equal(_np(w), cg.adjwgt)
        assert np.array_equal(_np(v), cg.vwgt) and np.array_equal(_np(M), mp)


@pytest.mark.parametrize("knobs,compressed", [(None, True), (dict(t_lane=1, t_tile=1, t_block=1, hub_part=256), True),
                                              (None, False)])
def test_packed_hub_records_split_large_ratings(lp, oracle_mod, synth_mod, knobs, compressed):
    # 2^27 vertex IDs leave 5 bits of a packed 32-bit hub record for the
    # partial rating (at most 31): once the leaves of a star gather in one
    # cluster, each 4000-neighbour piece of the centre rates it up to 4000,
    # which takes many records per cluster
    n = 1 << 27
    c = n - 25001
    g = synth_mod.from_edges(n, [(c, v) for v in range(c + 1, n)])
    G = _gpu_graph(lp, g, compressed)
    exp, ost = oracle_mod.lp_cluster(g, 30000, 4, 3)
    lab, st = lp.lp_cluster(G, 30000, 4, 3, config=knobs, stats=True)
    assert np.array_equal(_np(lab), exp)
    assert st.proposals == ost.proposals and st.moves == ost.moves
    G.free()


def _giant_hubs(synth_mod):
    # hub 0 joined to every leaf (1.1M neighbours: more than 256 pieces, so
    # its partitions are summed over several piece batches), hub 1 to every
    # other leaf, and a ring over the leaves so that later rounds see mixed
    # labels around the hubs
    leaves = 1_100_000
    n = leaves + 2
    lv = np.arange(2, n, dtype=np.int64)
    e = [np.stack([np.zeros(leaves, np.int64), lv], 1),
         np.stack([np.ones(leaves // 2, np.int64), lv[::2]], 1),
         np.stack([lv[:-1], lv[1:]], 1)]
    return synth_mod.from_edges(n, np.concatenate(e))


@pytest.fixture(scope="module")
def giant_hubs(synth_mod):
    return _giant_hubs(synth_mod)


@pytest.mark.parametrize("knobs", [None,
                                   dict(hub_part=256),    # 1024 partitions of ~1100 records: two label sub-passes
                                   dict(hub_part=8192)])  # ~8200 records per partition: four owner-map windows
@pytest.mark.parametrize("compressed", [True, False])
def test_giant_hub_partitions(lp, oracle_mod, giant_hubs, knobs, compressed):
    g = giant_hubs
    G = _gpu_graph(lp, g, compressed)
    exp, _ = oracle_mod.lp_cluster(g, 3000, 4, 21)
    lab = lp.lp_cluster(G, 3000, 4, 21, config=knobs)
    assert np.array_equal(_np(lab), exp)


def _kab_ring(synth_mod, a, b):
    # K_{a,b} plus a ring over the b side: the a side has degree b exactly
    # (b = 16000: the largest hub rated whole with 16-bit ratings, sixteen
    # chunks; b = 16001: cut into pieces)
    edges = [(i, a + j) for i in range(a) for j in range(b)]
    edges += [(a + j, a + (j + 1) % b) for j in range(b)]
    return synth_mod.from_edges(a + b, edges)


@pytest.mark.parametrize("a,b", [(3, 16000), (2, 16001), (4, 12000)])
@pytest.mark.parametrize("fmt", ["gap", "intervals", "plain"])
def test_whole_hub_bounds(lp, oracle_mod, synth_mod, a, b, fmt):
    g = _kab_ring(synth_mod, a, b)
    if fmt == "plain":
        G = lp.lp_graph_from_csr(g.n, g.xadj.view(np.int64), g.adjncy, g.adjwgt, g.vwgt)
    else:
        G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy, g.adjwgt, g.vwgt, intervals=fmt == "intervals")
    for cap, rounds, seed in ((50, 4, 3), (20000, 3, 5)):
        exp, _ = oracle_mod.lp_cluster(g, cap, rounds, seed)
        assert np.array_equal(_np(lp.lp_cluster(G, cap, rounds, seed)), exp)
    # the edge visits (cut, contraction records) take the same whole / cut split
    lab = (np.arange(g.n, dtype=np.int64) * 7919 % 101).astype(np.int32)
    assert lp.lp_edge_cut(G, lab) == oracle_mod.edge_cut(g, lab)
    cg, mp = oracle_mod.contract(g, lab)
    C, M = lp.lp_contract(G, lab)
    x, adj, w, v = lp.lp_decompress(C)
    assert np.array_equal(_np(M), mp) and np.array_equal(_np(adj), cg.adjncy) and np.array_equal(_np(w), cg.adjwgt)


REORDER_KNOBS = [dict(reorder=1), dict(reorder=1, t_lane=1, t_tile=1, t_block=1, hub_part=256),
                 dict(reorder=1, t_lane=4, t_tile=64, t_block=64, hub_part=1024, overlap=1)]


@pytest.mark.parametrize("name", ["rgg2d-16k", "rmat-s13-ef16", "rmat-s12-weighted", "star-25000", "star-10001-w",
                                  "bip-5x2048-heavy", "bip-3x9000-w"])
@pytest.mark.parametrize("fmt", ["gap", "intervals", "plain"])
def test_degree_ordered_copy_gives_identical_results(lp, oracle_mod, graphs, name, fmt):
    # rating on the degree-ordered copy: labels valued by the original IDs,
    # proposals at the original vertices, so labels and per-round counts equal
    # the oracle's on the graph as given
    g = graphs[name]
    if fmt == "plain":
        G = lp.lp_graph_from_csr(g.n, g.xadj.view(np.int64), g.adjncy, g.adjwgt, g.vwgt)
    else:
        G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy, g.adjwgt, g.vwgt, intervals=fmt == "intervals")
    exp, ost = oracle_mod.lp_cluster(g, 64, 4, 11)
    for knobs in REORDER_KNOBS:
        lab, st = lp.lp_cluster(G, 64, 4, 11, config=knobs, stats=True)
        assert np.array_equal(_np(lab), exp), knobs
        assert st.rounds_run == ost.rounds_run and st.proposals == ost.proposals and st.moves == ost.moves
    # once the copy exists, the cut and the contraction records visit the
    # copy (labels permuted to it, records at the original vertices): the
    # cut, the fine-to-coarse map and the coarse graph equal the oracle's
    lab = lp.lp_cluster(G, 64, 4, 11, config=dict(reorder=1))
    assert lp.lp_edge_cut(G, lab) == oracle_mod.edge_cut(g, exp)
    try:
        cg, mp = oracle_mod.contract(g, exp)
    except OverflowError:  # a coarse edge weight beyond 32 bits: the library reports it too
        with pytest.raises(lp.LPError) as e:
            lp.lp_contract(G, lab)
        assert e.value.status == lp.LP_EOVERFLOW
        return
    C, M = lp.lp_contract(G, lab)
    x, a, w, v = lp.lp_decompress(C)
    assert np.array_equal(_np(M), mp)
    assert np.array_equal(_np(x).view(np.uint64), cg.xadj)
    assert np.array_equal(_np(a), cg.adjncy) and np.array_equal(_np(w), cg.adjwgt)
    assert np.array_equal(_np(v), cg.vwgt)


def test_degree_ordered_copy_giant_hubs(lp, oracle_mod, giant_hubs):
    g = giant_hubs
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
    exp, ost = oracle_mod.lp_cluster(g, 3000, 4, 21)
    for knobs in (dict(reorder=0), dict(reorder=2), dict(reorder=1, hub_part=256)):
        lab, st = lp.lp_cluster(G, 3000, 4, 21, config=knobs, stats=True)
        assert np.array_equal(_np(lab), exp), knobs
        assert st.proposals == ost.proposals and st.moves == ost.moves
    # cut and contraction on the copy (hub pieces and whole hubs in record mode)
    assert lp.lp_edge_cut(G, lab) == oracle_mod.edge_cut(g, exp)
    cg, mp = oracle_mod.contract(g, exp)
    C, M = lp.lp_contract(G, lab)
    x, a, w, v = lp.lp_decompress(C)
    assert np.array_equal(_np(M), mp) and np.array_equal(_np(x).view(np.uint64), cg.xadj)
    assert np.array_equal(_np(a), cg.adjncy) and np.array_equal(_np(w), cg.adjwgt)


def test_reorder_option_errors(lp, graphs):
    G = _gpu_graph(lp, graphs["rgg2d-16k"])
    with pytest.raises(lp.LPError):
        lp.lp_cluster(G, 5, 1, 1, config=dict(reorder=3))
