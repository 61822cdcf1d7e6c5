"""Uncoarsening slice on the GPU vs the oracle, bit-exact: the contiguous
initial partition, projection through a contraction, size-constrained LP
refinement (labels and per-round statistics, on graphs that reach every
rating path, plain and compressed, with sub-rounds), the multilevel k-way
partition driver, argument errors, and refinement at the benchmark's full
size (R-MAT scale 24, k = 64, rated from the graph and from a gain table)."""
import dataclasses

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


@pytest.mark.parametrize("name", ["rgg2d-16k", "rmat-s12-weighted", "star-25000"])
@pytest.mark.parametrize("k", [1, 3, 64, 1000])
def test_initial_partition_matches_oracle(lp, oracle_mod, graphs, name, k):
    g = graphs[name]
    G = _gpu_graph(lp, g)
    assert np.array_equal(_np(lp.lp_initial_partition(G, k)), oracle_mod.initial_partition(g, k))


def test_initial_partition_heavy_weights(lp, oracle_mod, synth_mod):
    # vertex weights near 2^31: prefixes need 64 bits
    g = synth_mod.rmat_scale(10, 8, seed=4)
    g = dataclasses.replace(g, vwgt=(2**31 - 1 - synth_mod.vertex_weights(g.n, 0, 1000, 4)).astype(np.int32))
    G = _gpu_graph(lp, g)
    for k in (2, 7, 1000):
        assert np.array_equal(_np(lp.lp_initial_partition(G, k)), oracle_mod.initial_partition(g, k))


def test_projection_matches_oracle(lp, oracle_mod, graphs):
    g = graphs["rmat-s13-ef16"]
    lab, _ = oracle_mod.lp_cluster(g, 40, 5, 3)
    cg, mp = oracle_mod.contract(g, lab)
    cb = np.random.default_rng(5).integers(0, 9, cg.n).astype(np.int32)
    out = _np(lp.lp_project(mp, cb))
    assert np.array_equal(out, oracle_mod.project(mp, cb))
    # a map entry outside the coarse graph gives -1
    bad = mp.copy()
    bad[[0, 17]] = [cg.n, -3]
    out = _np(lp.lp_project(bad, cb))
    assert out[0] == -1 and out[17] == -1 and np.array_equal(out[1:17], oracle_mod.project(mp, cb)[1:17])


CASES = [("rgg2d-16k", 8), ("rmat-s13-ef16", 64), ("rmat-s12-weighted", 5), ("star-25000", 2),
         ("star-10001-w", 3), ("bip-5x2048", 4), ("bip-3x9000-w", 16), ("bip-5x2048-heavy", 4)]


@pytest.mark.parametrize("compressed", [True, False])
@pytest.mark.parametrize("name,k", CASES)
def test_refine_matches_oracle(lp, oracle_mod, graphs, name, k, compressed):
    g = graphs[name]
    G = _gpu_graph(lp, g, compressed)
    lmax = oracle_mod.max_block_weight(_total(g), k)
    # from the contiguous split, and from a seeded random assignment
    starts = [oracle_mod.initial_partition(g, k),
              np.random.default_rng(k).integers(0, k, g.n).astype(np.int32)]
    for start in starts:
        exp, ost = oracle_mod.lp_refine(g, start, k, lmax, 5, 11)
        got, st = lp.lp_refine(G, start, k, lmax, 5, 11, stats=True)
        assert np.array_equal(_np(got), exp)
        assert st.rounds_run == ost.rounds_run
        assert st.proposals == ost.proposals and st.moves == ost.moves


@pytest.mark.parametrize("S", [2, 4])
@pytest.mark.parametrize("name,k", [("rgg2d-16k", 8), ("rmat-s12-weighted", 5), ("star-25000", 2)])
def test_refine_subrounds_match_oracle(lp, oracle_mod, graphs, name, k, S):
    g = graphs[name]
    G = _gpu_graph(lp, g)
    lmax = oracle_mod.max_block_weight(_total(g), k)
    start = np.random.default_rng(S).integers(0, k, g.n).astype(np.int32)
    exp, ost = oracle_mod.lp_refine(g, start, k, lmax, 5, 2, subrounds=S)
    got, st = lp.lp_refine(G, start, k, lmax, 5, 2, config=dict(subrounds=S), stats=True)
    assert np.array_equal(_np(got), exp)
    assert st.proposals == ost.proposals and st.moves == ost.moves


def test_refine_tight_and_loose_bounds(lp, oracle_mod, graphs):
    g = graphs["rmat-s13-ef16"]
    G = _gpu_graph(lp, g)
    start = oracle_mod.initial_partition(g, 4)
    for lmax in (1, g.n // 4, g.n // 4 + 7, g.n):
        exp, _ = oracle_mod.lp_refine(g, start, 4, lmax, 4, 5)
        assert np.array_equal(_np(lp.lp_refine(G, start, 4, lmax, 4, 5)), exp), lmax


def test_refine_from_singletons_is_clustering(lp, graphs):
    g = graphs["rmat-s13-ef16"]
    G = _gpu_graph(lp, g)
    lab = _np(lp.lp_cluster(G, 30, 5, 4))
    ref = _np(lp.lp_refine(G, np.arange(g.n, dtype=np.int32), g.n, 30, 5, 4))
    assert np.array_equal(lab, ref)


def test_refine_errors(lp, graphs):
    g = graphs["rgg2d-16k"]
    G = _gpu_graph(lp, g)
    good = np.zeros(g.n, dtype=np.int32)
    for blocks, k in ((np.full(g.n, 2, dtype=np.int32), 2), (np.full(g.n, -1, dtype=np.int32), 2),
                      (good, 0), (good, g.n + 1)):
        with pytest.raises(lp.LPError):
            lp.lp_refine(G, blocks, k, 100, 5, 1)
    with pytest.raises(lp.LPError):
        lp.lp_refine(G, good, 2, 0, 5, 1)
    with pytest.raises(lp.LPError):
        lp.lp_initial_partition(G, 0)
    # the handle and the device stay usable after a rejected call
    assert np.array_equal(_np(lp.lp_refine(G, good, 1, g.n, 5, 1)), good)


@pytest.mark.parametrize("name,k", [("rgg2d-16k", 2), ("rgg2d-16k", 8), ("rgg2d-16k", 64), ("rmat-s13-ef16", 16),
                                    ("rmat-s12-weighted", 4)])
def test_partition_driver_matches_oracle(lp, oracle_mod, graphs, name, k):
    g = graphs[name]
    exp, etrace = oracle_mod.partition(g, k, seed=3)
    G = _gpu_graph(lp, g)
    got, trace = lp.partition(G, k, seed=3, trace=True)
    assert np.array_equal(_np(got), exp)
    assert trace == etrace
    w = oracle_mod.block_weights(g, exp, k)
    assert w.max() <= oracle_mod.max_block_weight(_total(g), k)


def test_partition_driver_subrounds(lp, oracle_mod, graphs):
    g = graphs["rgg2d-16k"]
    exp, etrace = oracle_mod.partition(g, 8, seed=1, subrounds=4, refine_subrounds=2)
    got, trace = lp.partition(_gpu_graph(lp, g), 8, seed=1, subrounds=4, refine_subrounds=2, trace=True)
    assert np.array_equal(_np(got), exp) and trace == etrace


def test_refine_full_size(lp, oracle_mod, rmat24):
    # R-MAT scale 24, edge factor 16, k = 64 from the contiguous split
    g = rmat24
    k = 64
    lmax = oracle_mod.max_block_weight(g.n, k)
    start = oracle_mod.initial_partition(g, k)
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
    assert np.array_equal(_np(lp.lp_initial_partition(G, k)), start)
    exp, ost = oracle_mod.lp_refine(g, start, k, lmax, 5, 1)
    got, st = lp.lp_refine(G, start, k, lmax, 5, 1, stats=True)
    assert np.array_equal(_np(got), exp)
    assert st.proposals == ost.proposals and st.moves == ost.moves
    assert lp.lp_edge_cut(G, got) == oracle_mod.edge_cut(g, exp)
    # rated from the sparse gain table instead
    got, st = lp.lp_refine(G, start, k, lmax, 5, 1, config=dict(gain_table=1), stats=True)
    assert np.array_equal(_np(got), exp)
    assert st.proposals == ost.proposals and st.moves == ost.moves
    G.free()


def test_degenerate_inputs(lp, oracle_mod, synth_mod):
    # no vertices; no edges; zero rounds; isolated vertices and a vertex heavier than the bound
    import dataclasses
    empty = synth_mod.from_edges(0, [])
    E = lp.lp_compress(0, empty.xadj.view(np.int64), np.zeros(0, dtype=np.int32))
    assert lp.lp_initial_partition(E, 3).numel() == 0
    assert lp.lp_refine(E, np.zeros(0, dtype=np.int32), 1, 1, 5, 1).numel() == 0
    assert lp.lp_project(np.zeros(0, dtype=np.int32), np.zeros(0, dtype=np.int32)).numel() == 0
    g = synth_mod.from_edges(50, [])
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
    start = oracle_mod.initial_partition(g, 4)
    assert np.array_equal(_np(lp.lp_initial_partition(G, 4)), start)
    assert np.array_equal(_np(lp.lp_refine(G, start, 4, 13, 5, 1)), start)
    g = synth_mod.rmat_scale(11, 8, seed=9)
    vw = synth_mod.vertex_weights(g.n, 1, 3, 9)
    vw[7] = 10_000  # heavier than any bound below: never moves, never receives
    g = dataclasses.replace(g, vwgt=vw)
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy, None, g.vwgt)
    k = 6
    lmax = oracle_mod.max_block_weight(int(vw.astype(np.int64).sum()), k)
    start = oracle_mod.initial_partition(g, k)
    for rounds in (0, 1, 5):
        exp, _ = oracle_mod.lp_refine(g, start, k, lmax, rounds, 4)
        assert np.array_equal(_np(lp.lp_refine(G, start, k, lmax, rounds, 4)), exp), rounds
        got = _np(lp.lp_refine(G, start, k, lmax, rounds, 4, config=dict(gain_table=1)))
        assert np.array_equal(got, exp), rounds
    assert np.array_equal(_np(lp.lp_refine(G, start, k, lmax, 0, 4)), start)
