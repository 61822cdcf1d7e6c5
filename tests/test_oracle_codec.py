"""Pins of the oracle's codec against the compressed format's definition
(paper Section III-A: gap encoding, VarInt with 7 payload bits and a
continuation bit, first-edge-ID headers, chunks of 1 000 neighbours for
degrees above 10 000, weights as zigzag differences interleaved with the
neighbour codes)."""
import numpy as np
import pytest

pytestmark = []


# LEB128 / VarInt textbook vectors (low 7-bit group first, 0x80 = more).
VARINT_VECTORS = [
    (0, "00"),
    (1, "01"),
    (127, "7f"),
    (128, "8001"),
    (300, "ac02"),
    (16383, "ff7f"),
    (16384, "808001"),
    (2**32 - 1, "ffffffff0f"),
    (2**63, "80808080808080808001"),
    (2**64 - 1, "ffffffffffffffffff01"),
]


@pytest.mark.parametrize("value,hexstr", VARINT_VECTORS)
def test_varint_vectors(oracle_mod, value, hexstr):
    assert oracle_mod.varint(value).hex() == hexstr
    v, k = oracle_mod.varint_decode(bytes.fromhex(hexstr) + b"\x55")
    assert (v, k) == (value, len(hexstr) // 2)


def test_varint_truncated_rejected(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.varint_decode(bytes.fromhex("8080"))


@pytest.mark.parametrize("x,z", [(0, 0), (-1, 1), (1, 2), (-2, 3), (2, 4),
                                 (2**31 - 1, 2**32 - 2), (-(2**31), 2**32 - 1)])
def test_zigzag(oracle_mod, x, z):
    assert oracle_mod.zigzag(x) == z
    assert oracle_mod.unzigzag(z) == x


def _path3(weights=None):
    import synth
    return synth.from_edges(3, [(0, 1), (1, 2)], weights)


def test_format_hand_case_unweighted(oracle_mod):
    # path 0-1-2. Records: [fe=0][zz(1-0)=2] | [fe=1][zz(0-1)=1][gap 2-0=2] | [fe=3][zz(1-2)=1]
    g = _path3()
    offs, data = oracle_mod.compress(g.n, g.xadj, g.adjncy)
    assert data.tobytes().hex() == "00020101020301"
    assert list(offs) == [0, 2, 5, 7]


def test_format_hand_case_weighted(oracle_mod):
    # w(0,1)=5, w(1,2)=3: vertex 1 codes: nbr 0 zz(-1)=1, weight zz(5-0)=10,
    # nbr 2 gap 2, weight zz(3-5)=3
    g = _path3([5, 3])
    offs, data = oracle_mod.compress(g.n, g.xadj, g.adjncy, g.adjwgt)
    assert data.tobytes().hex() == "00020a01010a0203030106"
    assert list(offs) == [0, 3, 8, 11]


def _star(oracle_mod, synth_mod, d, center=0, weights=False):
    n = d + 1
    edges = [(center, v) for v in range(n) if v != center]
    w = None
    if weights:
        w = [1 + (i * 7919) % 1000 for i in range(len(edges))]
    return synth_mod.from_edges(n, edges, w)


def test_chunk_table_points_at_chunk_starts(oracle_mod, synth_mod):
    # centre 0 with 10001 leaves: split into chunks of 1000; chunk k starts
    # with zigzag(v - u) of its first neighbour v = 1000k + 1.
    g = _star(oracle_mod, synth_mod, 10001)
    offs, data = oracle_mod.compress(g.n, g.xadj, g.adjncy)
    rec = data[offs[0]:offs[1]].tobytes()
    assert rec[0] == 0  # first edge id 0
    nchunks = 11
    table = [int.from_bytes(rec[1 + 4 * i: 5 + 4 * i], "little") for i in range(nchunks - 1)]
    assert rec[1 + 4 * (nchunks - 1)] == 2  # chunk 0 starts with zz(1 - 0)
    for k, rel in enumerate(table, start=1):
        v, _ = oracle_mod.varint_decode(rec[rel:rel + 10])
        assert oracle_mod.unzigzag(v) == 1000 * k + 1
    # the 10000 and 10001 boundary: exactly 10000 neighbours is not split
    g2 = _star(oracle_mod, synth_mod, 10000)
    offs2, data2 = oracle_mod.compress(g2.n, g2.xadj, g2.adjncy)
    rec2 = data2[offs2[0]:offs2[1]].tobytes()
    assert rec2[1] == 2 and len(rec2) == 1 + 1 + 9999


@pytest.mark.parametrize("d", [1, 9999, 10000, 10001, 25000])
@pytest.mark.parametrize("weighted", [False, True])
def test_roundtrip_stars(oracle_mod, synth_mod, d, weighted):
    for center in (0, d // 2, d):
        g = _star(oracle_mod, synth_mod, d, center, weighted)
        offs, data = oracle_mod.compress(g.n, g.xadj, g.adjncy, g.adjwgt)
        x, a, w = oracle_mod.decompress(g.n, g.two_m, weighted, offs, data)
        assert np.array_equal(x, g.xadj)
        assert np.array_equal(a, g.adjncy)
        if weighted:
            assert np.array_equal(w, g.adjwgt)


def test_roundtrip_random_graphs(oracle_mod, synth_mod):
    for seed in range(3):
        g = synth_mod.rmat_scale(11, 8, seed=seed + 5)
        g.adjwgt = synth_mod.edge_weights(g, 1, 2**31 - 1, seed)
        for wts in (None, g.adjwgt):
            offs, data = oracle_mod.compress(g.n, g.xadj, g.adjncy, wts)
            x, a, w = oracle_mod.decompress(g.n, g.two_m, wts is not None, offs, data)
            assert np.array_equal(x, g.xadj) and np.array_equal(a, g.adjncy)
            if wts is not None:
                assert np.array_equal(w, wts)


def test_compress_sorts_neighbourhoods(oracle_mod, synth_mod):
    g = synth_mod.rgg2d_16k()
    rng = np.random.default_rng(0)
    adj = g.adjncy.copy()
    for u in range(0, g.n, 97):
        b, e = int(g.xadj[u]), int(g.xadj[u + 1])
        adj[b:e] = rng.permutation(adj[b:e])
    o1, d1 = oracle_mod.compress(g.n, g.xadj, g.adjncy)
    o2, d2 = oracle_mod.compress(g.n, g.xadj, adj)
    assert np.array_equal(o1, o2) and np.array_equal(d1, d2)


def test_malformed_stream_rejected(oracle_mod):
    g = _path3()
    offs, data = oracle_mod.compress(g.n, g.xadj, g.adjncy)
    bad = data.copy()
    bad[1] = 0x80  # continuation into the next record
    with pytest.raises(ValueError):
        oracle_mod.decompress(g.n, g.two_m, False, offs, bad)
