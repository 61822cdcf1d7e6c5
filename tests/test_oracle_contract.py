"""Pins of the oracle's contraction (paper Section IV-B: one coarse vertex
per cluster, coarse edge weight = summed weight of the fine edges between
the two clusters, intra-cluster edges dropped), edge cut (Section I) and the
multilevel loop parameters."""
import numpy as np
import pytest

import bruteforce as bf


def test_identity_clustering_gives_the_graph(oracle_mod, synth_mod):
    g = synth_mod.rgg2d_16k()
    cg, mp = oracle_mod.contract(g, np.arange(g.n))
    assert cg.n == g.n and np.array_equal(mp, np.arange(g.n))
    assert np.array_equal(cg.xadj, g.xadj) and np.array_equal(cg.adjncy, g.adjncy)
    assert (cg.adjwgt == 1).all() and (cg.vwgt == 1).all()


def test_all_in_one(oracle_mod, synth_mod):
    g = synth_mod.rmat_scale(10, 8, seed=1)
    cg, mp = oracle_mod.contract(g, np.full(g.n, 17))
    assert cg.n == 1 and cg.two_m == 0 and cg.vwgt[0] == g.n and (mp == 0).all()


@pytest.mark.parametrize("seed", range(8))
def test_matches_dense_enumeration(oracle_mod, synth_mod, seed):
    n = 8 + seed
    g = synth_mod.random_small(n, 0.5, seed)
    g.adjwgt = synth_mod.edge_weights(g, 1, 9, seed)
    g.vwgt = synth_mod.vertex_weights(n, 1, 4, seed)
    rng = np.random.default_rng(seed)
    labels = rng.integers(0, n, n).astype(np.int32)
    cg, mp = oracle_mod.contract(g, labels)
    k, A, vw = bf.dense_quotient(g, labels)
    assert cg.n == k
    assert np.array_equal(cg.vwgt, vw)
    D = np.zeros((k, k), dtype=np.int64)
    for a in range(k):
        nb = cg.adjncy[cg.xadj[a]:cg.xadj[a + 1]]
        assert (np.diff(nb) > 0).all()  # sorted, no duplicates
        D[a, nb] = cg.adjwgt[cg.xadj[a]:cg.xadj[a + 1]]
    assert np.array_equal(D, A)
    assert np.array_equal(D, D.T)
    used = sorted(set(labels.tolist()))
    assert np.array_equal(mp, [used.index(c) for c in labels])
    # coarse weight sums: total = 2 * cut; vertex weights preserved
    assert cg.adjwgt.sum() == 2 * oracle_mod.edge_cut(g, labels) == 2 * bf.cut_by_enumeration(g, labels)


def test_lp_then_contract_rmat(oracle_mod, synth_mod):
    g = synth_mod.rmat_scale(12, 16, seed=4)
    lab, _ = oracle_mod.lp_cluster(g, 50, 5, 1)
    cg, mp = oracle_mod.contract(g, lab)
    assert cg.vwgt.sum() == g.n
    assert cg.adjwgt.sum() == 2 * oracle_mod.edge_cut(g, lab)
    assert (cg.vwgt[np.bincount(mp) >= 2] <= 50).all()


def test_overflow_detected(oracle_mod, synth_mod):
    g = synth_mod.from_edges(4, [(0, 2), (1, 3)], [2**31 - 1, 2**31 - 1])
    with pytest.raises(OverflowError):
        oracle_mod.contract(g, np.array([0, 0, 2, 2], dtype=np.int32))


def test_bad_labels_rejected(oracle_mod, synth_mod):
    g = synth_mod.from_edges(3, [(0, 1)])
    with pytest.raises(ValueError):
        oracle_mod.contract(g, np.array([0, 5, 1], dtype=np.int32))


def test_cut_enumeration(oracle_mod, synth_mod):
    g = synth_mod.random_small(12, 0.4, 3)
    g.adjwgt = synth_mod.edge_weights(g, 1, 7, 3)
    lab = np.array([i % 3 for i in range(12)], dtype=np.int32)
    assert oracle_mod.edge_cut(g, lab) == bf.cut_by_enumeration(g, lab)


def test_coarsen_params():
    import oracle
    assert oracle.coarsen_params(1 << 26, 1 << 26) == (16384, 12288)
    assert oracle.coarsen_params(16384, 16384) == (256, 192)
    assert oracle.coarsen_params(100000, 100000) == (1563, 192)


def test_coarsen_levels_shrink(oracle_mod, synth_mod):
    g = synth_mod.rgg2d_16k()
    levels, final, n_target, cap = oracle_mod.coarsen(g, 1)
    assert levels and final.n < g.n
    sizes = [lv[0].n for lv in levels] + [final.n]
    assert all(b < a for a, b in zip(sizes, sizes[1:]))
    assert final.n <= n_target or 100 * final.n > 95 * levels[-1][0].n
    assert final.vwgt.sum() == g.n
