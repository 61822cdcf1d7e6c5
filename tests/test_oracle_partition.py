"""Pins of the oracle's uncoarsening slice (paper Section II-A: initial
partition of the coarsest graph, projection, size-constrained LP refinement as
in Section II-B; balance bound of Section I): hand-computed initial
partitions, refinement closed forms (a misplaced vertex, the synchronous swap,
a full block), the balance invariant, the cut-preservation property of
projection through a contraction, and the whole multilevel driver."""
import dataclasses

import numpy as np
import pytest


def _weighted(g, vw):
    return dataclasses.replace(g, vwgt=np.asarray(vw, dtype=np.int32))


# ------------------------------------------------------ initial partition --

def test_initial_partition_unit_weights_by_hand(oracle_mod, synth_mod):
    g = synth_mod.from_edges(10, [(i, i + 1) for i in range(9)])
    # block(u) = floor(3 u / 10)
    assert oracle_mod.initial_partition(g, 3).tolist() == [0, 0, 0, 0, 1, 1, 1, 2, 2, 2]
    assert oracle_mod.initial_partition(g, 1).tolist() == [0] * 10
    # k = n: one vertex per block
    assert oracle_mod.initial_partition(g, 10).tolist() == list(range(10))


def test_initial_partition_weighted_by_hand(oracle_mod, synth_mod):
    g = _weighted(synth_mod.from_edges(6, [(i, i + 1) for i in range(5)]), [5, 1, 1, 1, 1, 1])
    # c(V) = 10, prefixes 0 5 6 7 8 9 -> floor(2 P / 10)
    assert oracle_mod.initial_partition(g, 2).tolist() == [0, 1, 1, 1, 1, 1]
    # floor(4 P / 10) = 0 2 2 2 3 3
    assert oracle_mod.initial_partition(g, 4).tolist() == [0, 2, 2, 2, 3, 3]


@pytest.mark.parametrize("k", [1, 2, 7, 64, 300])
def test_initial_partition_bounds(oracle_mod, synth_mod, k):
    g = synth_mod.rgg2d_16k()
    g = _weighted(g, synth_mod.vertex_weights(g.n, 1, 40, 5))
    b = oracle_mod.initial_partition(g, k)
    assert b.min() >= 0 and b.max() < k
    assert np.all(np.diff(b) >= 0)  # contiguous in vertex order
    w = oracle_mod.block_weights(g, b, k)
    total = int(np.asarray(g.vwgt, dtype=np.int64).sum())
    assert w.sum() == total
    # every block weighs less than c(V)/k plus one vertex weight
    assert np.all(w * k < total + k * int(g.vwgt.max()))


def test_initial_partition_rejects_bad_k(oracle_mod, synth_mod):
    g = synth_mod.from_edges(4, [(0, 1)])
    with pytest.raises(ValueError):
        oracle_mod.initial_partition(g, 0)


# ------------------------------------------------------------- refinement --

def _two_triangles(synth_mod):
    return synth_mod.from_edges(6, [(0, 1), (0, 2), (1, 2), (3, 4), (3, 5), (4, 5), (2, 3)])


def test_refine_moves_a_misplaced_vertex(oracle_mod, synth_mod):
    # vertex 2 sits in block 1 with one edge there and two into block 0: it
    # moves (gain 2 - 1); 0 and 1 see a tie 1 : 1 with their own block and
    # stay; round 1 has no proposal
    g = _two_triangles(synth_mod)
    b, st = oracle_mod.lp_refine(g, [0, 0, 1, 1, 1, 1], 2, 6, 5, 1)
    assert b.tolist() == [0, 0, 0, 1, 1, 1]
    assert st.rounds_run == 1 and st.proposals == [1] and st.moves == [1]
    assert oracle_mod.edge_cut(g, b) == 1


def test_refine_respects_a_full_block(oracle_mod, synth_mod):
    g = _two_triangles(synth_mod)
    # block 0 weighs 2; with L = 3 vertex 2 fits, with L = 2 it does not
    b, _ = oracle_mod.lp_refine(g, [0, 0, 1, 1, 1, 1], 2, 3, 5, 1)
    assert b.tolist() == [0, 0, 0, 1, 1, 1]
    b, st = oracle_mod.lp_refine(g, [0, 0, 1, 1, 1, 1], 2, 2, 5, 1)
    assert b.tolist() == [0, 0, 1, 1, 1, 1] and st.rounds_run == 0


@pytest.mark.parametrize("rounds", [1, 2, 3])
def test_refine_synchronous_swap(oracle_mod, synth_mod, rounds):
    # matching {2i, 2i+1} with the partners in different blocks: every vertex
    # proposes its partner's block with gain 1 and, with room, all move at
    # once, so the blocks swap every round and the cut stays k
    k = 40
    g = synth_mod.from_edges(2 * k, [(2 * i, 2 * i + 1) for i in range(k)])
    start = np.arange(2 * k) % 2
    b, st = oracle_mod.lp_refine(g, start, 2, 2 * k, rounds, 9)
    assert np.array_equal(b, start ^ 1 if rounds % 2 else start)
    assert st.proposals == [2 * k] * rounds
    # exact balance (L = k): no block can take anyone
    b, st = oracle_mod.lp_refine(g, start, 2, k, rounds, 9)
    assert np.array_equal(b, start) and st.rounds_run == 0


def test_refine_from_singletons_is_clustering(oracle_mod, synth_mod):
    # with one block per vertex the refinement starts where clustering starts
    g = synth_mod.random_small(40, 0.15, 3)
    lab, st = oracle_mod.lp_cluster(g, 4, 5, 2)
    b, st2 = oracle_mod.lp_refine(g, np.arange(g.n), g.n, 4, 5, 2)
    assert np.array_equal(lab, b) and st.proposals == st2.proposals


@pytest.mark.parametrize("k,seed", [(2, 1), (8, 2), (33, 3)])
def test_refine_keeps_balance_and_weight(oracle_mod, synth_mod, k, seed):
    g = synth_mod.rmat_scale(12, 8, seed=seed)
    g = _weighted(g, synth_mod.vertex_weights(g.n, 1, 9, seed))
    total = int(np.asarray(g.vwgt, dtype=np.int64).sum())
    lmax = oracle_mod.max_block_weight(total, k)
    start = oracle_mod.initial_partition(g, k)
    w0 = oracle_mod.block_weights(g, start, k)
    b, st = oracle_mod.lp_refine(g, start, k, lmax, 5, seed)
    w = oracle_mod.block_weights(g, b, k)
    assert w.sum() == total
    # a block within the bound stays within it (admission against the
    # start-of-round weight, departures not credited)
    assert np.all(w[w0 <= lmax] <= lmax)
    assert sum(st.moves) > 0
    assert oracle_mod.edge_cut(g, b) < oracle_mod.edge_cut(g, start)


def test_refine_rejects_bad_blocks(oracle_mod, synth_mod):
    g = _two_triangles(synth_mod)
    for blocks, k in (([0, 0, 2, 1, 1, 1], 2), ([0, 0, -1, 1, 1, 1], 2), ([0] * 6, 0), ([0] * 6, 7)):
        with pytest.raises(ValueError):
            oracle_mod.lp_refine(g, blocks, k, 6, 5, 1)


def test_max_block_weight(oracle_mod):
    # L = ceil(c/k) + floor(ceil(c/k) * eps / 1000)
    assert oracle_mod.max_block_weight(1000, 8) == 125 + 3
    assert oracle_mod.max_block_weight(1001, 8) == 126 + 3
    assert oracle_mod.max_block_weight(16384, 64, 0) == 256
    assert oracle_mod.max_block_weight(10, 3, 500) == 4 + 2


# ------------------------------------------------------------- projection --

@pytest.mark.parametrize("seed", [1, 2])
def test_projection_preserves_cut_and_block_weights(oracle_mod, synth_mod, seed):
    # a partition of the quotient graph, projected to the fine graph, has the
    # same cut and the same block weights (every coarse edge weight is the
    # total weight of the fine edges between the two clusters)
    g = synth_mod.rmat_scale(11, 8, seed=seed)
    g = dataclasses.replace(g, adjwgt=synth_mod.edge_weights(g, 1, 5, seed))
    lab, _ = oracle_mod.lp_cluster(g, 12, 5, seed)
    cg, mp = oracle_mod.contract(g, lab)
    rng = np.random.default_rng(seed)
    k = 5
    cb = rng.integers(0, k, cg.n).astype(np.int32)
    fb = oracle_mod.project(mp, cb)
    assert oracle_mod.edge_cut(g, fb) == oracle_mod.edge_cut(cg, cb)
    assert np.array_equal(oracle_mod.block_weights(g, fb, k), oracle_mod.block_weights(cg, cb, k))


# ---------------------------------------------------------------- driver --

@pytest.mark.parametrize("k", [2, 8, 64])
def test_partition_driver(oracle_mod, synth_mod, k):
    g = synth_mod.rgg2d_16k()
    b, trace = oracle_mod.partition(g, k, seed=1)
    lmax = oracle_mod.max_block_weight(g.n, k)
    w = oracle_mod.block_weights(g, b, k)
    assert b.min() >= 0 and b.max() < k and w.sum() == g.n
    assert w.max() <= lmax
    assert trace[-1] == (g.n, oracle_mod.edge_cut(g, b))
    # the coarsest graph is small, and every coarse vertex fits the slack
    assert trace[0][0] < g.n // 4
    # far below the cut of the contiguous split of the input itself
    assert oracle_mod.edge_cut(g, b) < oracle_mod.edge_cut(g, oracle_mod.initial_partition(g, k))


def test_partition_cap(oracle_mod):
    # the loop's own cap (3 c(V) / n_target) unless the balance slack is smaller
    assert oracle_mod.partition_cap(16384, 16384, 2) == 192
    assert oracle_mod.partition_cap(16384, 16384, 8) == 61
    assert oracle_mod.partition_cap(16384, 16384, 64, 0) == 1
