"""Sparse gain table on the GPU (paper Section V) against the oracle's
affinity definition, element by element: after building it for a partition
and after batches of moves (enough of them that hash slices fill with stale
zero entries and get rebuilt), on graphs that reach every slice kind (dense
rows, hash slices, chunked hubs), plain and compressed, weighted; argument
errors; and LP refinement rated from the table, bit-exact against the
oracle's refinement (labels and per-round counts)."""
import numpy as np
import pytest

from test_gpu_parity import _graphs, _gpu_graph

pytestmark = pytest.mark.gpu


def _np(t):
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def graphs(synth_mod):
    return _graphs(synth_mod)


def _total(g):
    return g.n if g.vwgt is None else int(np.asarray(g.vwgt, dtype=np.int64).sum())


def _check_all(lp, oracle_mod, T, g, blocks, k, rows=None):
    A = oracle_mod.affinity(g, blocks, k)
    rows = np.arange(g.n) if rows is None else rows
    us = np.repeat(rows, k).astype(np.int32)
    bs = np.tile(np.arange(k), len(rows)).astype(np.int32)
    got = _np(T.affinity(us, bs)).reshape(len(rows), k)
    assert np.array_equal(got, A[rows])


@pytest.mark.parametrize("compressed", [True, False])
@pytest.mark.parametrize("name,k", [("rgg2d-16k", 8), ("rmat-s13-ef16", 64), ("rmat-s12-weighted", 300),
                                    ("star-25000", 5), ("star-10001-w", 64), ("bip-3x9000-w", 2),
                                    ("bip-5x2048-heavy", 3)])  # weighted degrees above 2^31: int64 slots
def test_table_matches_definition_through_moves(lp, oracle_mod, graphs, name, k, compressed):
    g = graphs[name]
    G = _gpu_graph(lp, g, compressed)
    rng = np.random.default_rng(k)
    blocks = rng.integers(0, k, g.n).astype(np.int32)
    T = lp.GainTable(G, blocks, k)
    rows = None if g.n * k <= 4_000_000 else np.unique(np.concatenate(
        [rng.integers(0, g.n, 2000), np.argsort(np.diff(g.xadj.astype(np.int64)))[-20:]]))
    _check_all(lp, oracle_mod, T, g, blocks, k, rows)
    for it in range(12):
        m = int(rng.integers(1, max(2, g.n // 5)))
        us = rng.choice(g.n, m, replace=False).astype(np.int32)
        to = rng.integers(0, k, m).astype(np.int32)
        T.move(us, to)
        blocks[us] = to
        if it % 4 == 3:
            _check_all(lp, oracle_mod, T, g, blocks, k, rows)
    _check_all(lp, oracle_mod, T, g, blocks, k, rows)
    slots, nbytes, missing, rebuilds = T.info()
    assert missing == 0 and slots > 0 and nbytes > 4 * slots
    if name == "rmat-s12-weighted":  # many short hash slices, k = 300: stale zeros fill some
        assert rebuilds > 0
    T.free()


def test_table_memory_is_linear_in_edges(lp, graphs):
    # hash slices of pow2(2 deg) slots, dense rows of k: at most 4 slots per edge
    g = graphs["rmat-s13-ef16"]
    G = _gpu_graph(lp, g)
    for k in (2, 64, 4096):
        T = lp.GainTable(G, np.arange(g.n, dtype=np.int32) % k, k)
        slots = T.info()[0]
        deg = np.diff(g.xadj.astype(np.int64))
        assert slots <= 4 * g.two_m and slots <= int(np.minimum(4 * deg, k).sum()) + 1
        T.free()


def test_table_errors(lp, graphs):
    g = graphs["rgg2d-16k"]
    G = _gpu_graph(lp, g)
    with pytest.raises(lp.LPError):
        lp.GainTable(G, np.full(g.n, 3, dtype=np.int32), 3)
    with pytest.raises(lp.LPError):
        lp.GainTable(G, np.zeros(g.n, dtype=np.int32), 0)
    blocks = np.arange(g.n, dtype=np.int32) % 4
    T = lp.GainTable(G, blocks, 4)
    before = _np(T.affinity(np.arange(100, dtype=np.int32), np.zeros(100, dtype=np.int32)))
    for us, to in (([5, 5], [1, 2]), ([g.n], [0]), ([3], [4]), ([-1], [0])):
        with pytest.raises(lp.LPError):
            T.move(np.array(us, dtype=np.int32), np.array(to, dtype=np.int32))
    # rejected batches change nothing; out-of-range queries give -1
    assert np.array_equal(_np(T.affinity(np.arange(100, dtype=np.int32), np.zeros(100, dtype=np.int32))), before)
    assert _np(T.affinity(np.array([g.n, 0], dtype=np.int32), np.array([0, 4], dtype=np.int32))).tolist() == [-1, -1]
    T.free()


CASES = [("rgg2d-16k", 8), ("rmat-s13-ef16", 64), ("rmat-s12-weighted", 5), ("star-25000", 2),
         ("star-10001-w", 3), ("bip-5x2048", 4), ("bip-3x9000-w", 16), ("bip-5x2048-heavy", 4)]


@pytest.mark.parametrize("compressed", [True, False])
@pytest.mark.parametrize("name,k", CASES)
def test_refine_from_gain_table_matches_oracle(lp, oracle_mod, graphs, name, k, compressed):
    g = graphs[name]
    G = _gpu_graph(lp, g, compressed)
    lmax = oracle_mod.max_block_weight(_total(g), k)
    for start in (oracle_mod.initial_partition(g, k), np.random.default_rng(k).integers(0, k, g.n).astype(np.int32)):
        exp, ost = oracle_mod.lp_refine(g, start, k, lmax, 5, 11)
        got, st = lp.lp_refine(G, start, k, lmax, 5, 11, config=dict(gain_table=1), stats=True)
        assert np.array_equal(_np(got), exp)
        assert st.proposals == ost.proposals and st.moves == ost.moves


@pytest.mark.parametrize("S", [2, 4])
def test_refine_from_gain_table_subrounds(lp, oracle_mod, graphs, S):
    g = graphs["rmat-s12-weighted"]
    G = _gpu_graph(lp, g)
    lmax = oracle_mod.max_block_weight(_total(g), 6)
    start = np.random.default_rng(S).integers(0, 6, g.n).astype(np.int32)
    exp, ost = oracle_mod.lp_refine(g, start, 6, lmax, 5, 2, subrounds=S)
    got, st = lp.lp_refine(G, start, 6, lmax, 5, 2, config=dict(subrounds=S, gain_table=1), stats=True)
    assert np.array_equal(_np(got), exp) and st.moves == ost.moves


def test_gain_table_rejected_for_clustering(lp, graphs):
    G = _gpu_graph(lp, graphs["rgg2d-16k"])
    with pytest.raises(lp.LPError):
        lp.lp_cluster(G, 32, 5, 1, config=dict(gain_table=1))


def test_partition_driver_with_gain_table(lp, oracle_mod, graphs):
    g = graphs["rgg2d-16k"]
    exp, etrace = oracle_mod.partition(g, 16, seed=2)
    got, trace = lp.partition(_gpu_graph(lp, g), 16, seed=2, gain_table=True, trace=True)
    assert np.array_equal(_np(got), exp) and trace == etrace
