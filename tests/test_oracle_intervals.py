"""Pins of the oracle's interval encoding (paper Section III-A: a run
x, x+1, ..., x+l-1 of at least three consecutive neighbour IDs is stored as
the pair (x, l); weights stay gap + VarInt coded). Reading of the layout per
chunk: VarInt(k intervals); per interval VarInt(zigzag(x - u)),
VarInt(l - 3); the interval neighbours' weights; then the other neighbours
gap encoded as in the plain format, weights continuing the same chain.
Interval-coded neighbourhoods are split into chunks of 1000 above 4000
neighbours (10 000 without intervals)."""
import numpy as np
import pytest


def _graph(synth_mod, n, edges, weights=None):
    return synth_mod.from_edges(n, edges, weights)


def test_hand_case_unweighted(oracle_mod, synth_mod):
    # vertex 0: neighbours 1 2 3 4 | 7 | 9 10 11 -> intervals (1, 4) and
    # (9, 3), residual 7. Record: fe 0, k 2, zz(1)=2 l-3=1, zz(9)=18 l-3=0,
    # zz(7)=14. Vertex 1 (neighbour 0): fe 8, k 0, zz(0-1)=1.
    g = _graph(synth_mod, 12, [(0, v) for v in (1, 2, 3, 4, 7, 9, 10, 11)])
    offs, data = oracle_mod.compress(g.n, g.xadj, g.adjncy, intervals=True)
    rec0 = data[offs[0]:offs[1]].tobytes().hex()
    rec1 = data[offs[1]:offs[2]].tobytes().hex()
    assert rec0 == "00020201120" + "00e"
    assert rec1 == "080001"


def test_hand_case_weighted(oracle_mod, synth_mod):
    # vertex 0: neighbours 1 2 3 (weights 4 4 6) form an interval, 5 (weight 2)
    # is a residual: fe 0, k 1, zz(1)=2, 0, weights zz(4)=8 zz(0)=0 zz(2)=4,
    # then zz(5)=10 with weight zz(2-6)=7
    g = _graph(synth_mod, 6, [(0, 1), (0, 2), (0, 3), (0, 5)], [4, 4, 6, 2])
    offs, data = oracle_mod.compress(g.n, g.xadj, g.adjncy, g.adjwgt, intervals=True)
    assert data[offs[0]:offs[1]].tobytes().hex() == "000102000800040a07"


@pytest.mark.parametrize("nbrs,runs", [
    ([3, 4], []),                    # a run of two is not an interval
    ([3, 4, 5], [(3, 3)]),           # exactly three is
    ([2, 3, 4, 6, 7, 8, 9], [(2, 3), (6, 4)]),
    ([5, 6, 7, 9], [(5, 3)]),
])
def test_run_detection(oracle_mod, synth_mod, nbrs, runs):
    n = max(nbrs) + 1
    g = _graph(synth_mod, n, [(0, v) for v in nbrs])
    offs, data = oracle_mod.compress(g.n, g.xadj, g.adjncy, intervals=True)
    rec = data[offs[0]:offs[1]].tobytes()
    pos = 1  # after fe = 0
    k, d = oracle_mod.varint_decode(rec[pos:])
    pos += d
    got = []
    for _ in range(k):
        zs, d = oracle_mod.varint_decode(rec[pos:])
        pos += d
        lm3, d = oracle_mod.varint_decode(rec[pos:])
        pos += d
        got.append((oracle_mod.unzigzag(zs), lm3 + 3))
    assert got == runs


def test_duplicates_break_runs(oracle_mod, synth_mod):
    # neighbourhood 5 5 6 7 (a parallel edge): the first 5 is a residual, the
    # run 5 6 7 that follows is an interval; the round trip keeps both 5s
    g = synth_mod.Graph(8, np.array([0, 4, 4, 4, 4, 4, 6, 7, 8], dtype=np.uint64),
                        np.array([5, 5, 6, 7, 0, 0, 0, 0], dtype=np.int32))
    offs, data = oracle_mod.compress(g.n, g.xadj, g.adjncy, intervals=True)
    assert data[offs[0]:offs[1]].tobytes().hex() == "00010a000a"
    x, a, _ = oracle_mod.decompress(g.n, g.two_m, False, offs, data, intervals=True)
    assert np.array_equal(a, g.adjncy) and np.array_equal(x, g.xadj)


def test_chunks_restart_intervals(oracle_mod, synth_mod):
    # centre 0 with leaves 1..10001: eleven chunks of 1000; chunk k holds the
    # run 1000k+1 .. 1000k+1000 as one interval (the last chunk one residual)
    g = _graph(synth_mod, 10002, [(0, v) for v in range(1, 10002)])
    offs, data = oracle_mod.compress(g.n, g.xadj, g.adjncy, intervals=True)
    rec = data[offs[0]:offs[1]].tobytes()
    table = [int.from_bytes(rec[1 + 4 * i: 5 + 4 * i], "little") for i in range(10)]
    for k, rel in enumerate([1 + 40] + table):
        kk, d = oracle_mod.varint_decode(rec[rel:])
        if k < 10:
            assert kk == 1
            zs, d2 = oracle_mod.varint_decode(rec[rel + d:])
            lm3, _ = oracle_mod.varint_decode(rec[rel + d + d2:])
            assert (oracle_mod.unzigzag(zs), lm3 + 3) == (1000 * k + 1, 1000)
        else:
            assert kk == 0  # one neighbour left: a residual
    assert len(rec) < 200  # 10001 neighbours in a few bytes per chunk


def test_chunk_threshold_4000(oracle_mod, synth_mod):
    # 4000 neighbours: one chunk; 4001: five chunks, so a table of four offsets
    for d, table in ((4000, 0), (4001, 4)):
        g = _graph(synth_mod, d + 1, [(0, v) for v in range(1, d + 1)])
        offs, data = oracle_mod.compress(g.n, g.xadj, g.adjncy, intervals=True)
        rec = data[offs[0]:offs[1]].tobytes()
        k, _ = oracle_mod.varint_decode(rec[1 + 4 * table:])
        assert k == 1  # the first chunk holds one interval
        if table:
            rels = [int.from_bytes(rec[1 + 4 * i: 5 + 4 * i], "little") for i in range(table)]
            assert rels == sorted(rels) and rels[0] > 1 + 4 * table


@pytest.mark.parametrize("d", [0, 1, 3999, 4000, 4001, 9999, 10000, 10001, 25000])
@pytest.mark.parametrize("weighted", [False, True])
def test_roundtrip_stars(oracle_mod, synth_mod, d, weighted):
    # stars with the centre inside the leaf range: long consecutive runs
    for center in (0, d // 2, d):
        n = d + 1
        edges = [(center, v) for v in range(n) if v != center]
        w = [1 + (i * 7919) % 1000 for i in range(len(edges))] if weighted else None
        g = _graph(synth_mod, max(n, 1), edges, w)
        offs, data = oracle_mod.compress(g.n, g.xadj, g.adjncy, g.adjwgt, intervals=True)
        x, a, ww = oracle_mod.decompress(g.n, g.two_m, weighted, offs, data, intervals=True)
        assert np.array_equal(x, g.xadj) and np.array_equal(a, g.adjncy)
        if weighted:
            assert np.array_equal(ww, g.adjwgt)


@pytest.mark.parametrize("kind", ["rgg2d", "rgg3d", "rmat"])
@pytest.mark.parametrize("weighted", [False, True])
def test_roundtrip_random_graphs(oracle_mod, synth_mod, kind, weighted):
    if kind == "rgg2d":
        g = synth_mod.rgg2d_16k(seed=3)
    elif kind == "rgg3d":
        g = synth_mod.rgg3d(1 << 14, 27.0, seed=3)
    else:
        g = synth_mod.rmat_scale(12, 8, seed=3)
    wts = synth_mod.edge_weights(g, 1, 2**31 - 1, 4) if weighted else None
    offs, data = oracle_mod.compress(g.n, g.xadj, g.adjncy, wts, intervals=True)
    x, a, w = oracle_mod.decompress(g.n, g.two_m, weighted, offs, data, intervals=True)
    assert np.array_equal(x, g.xadj) and np.array_equal(a, g.adjncy)
    if weighted:
        assert np.array_equal(w, wts)


def test_intervals_shrink_geometric_graphs_only(oracle_mod, synth_mod):
    # cell-ordered geometric graphs have runs of consecutive IDs; R-MAT
    # neighbourhoods almost never do, so there each chunk pays its count byte
    for g, smaller in ((synth_mod.rgg3d(1 << 16, 27.0, seed=1), True), (synth_mod.rmat_scale(14, 16, seed=1), False)):
        _, gap = oracle_mod.compress(g.n, g.xadj, g.adjncy)
        _, itv = oracle_mod.compress(g.n, g.xadj, g.adjncy, intervals=True)
        assert (len(itv) < len(gap)) == smaller


def test_malformed_interval_stream_rejected(oracle_mod, synth_mod):
    g = _graph(synth_mod, 12, [(0, v) for v in (1, 2, 3, 4, 7, 9, 10, 11)])
    offs, data = oracle_mod.compress(g.n, g.xadj, g.adjncy, intervals=True)
    bad = data.copy()
    bad[offs[0] + 3] = 0x7f  # first interval length 130: more neighbours than the vertex has
    with pytest.raises(ValueError):
        oracle_mod.decompress(g.n, g.two_m, False, offs, bad, intervals=True)
    # the same bytes read as the plain format are not a valid graph either
    with pytest.raises(ValueError):
        oracle_mod.decompress(g.n, g.two_m, False, offs, data, intervals=False)
