"""Pins of the oracle's affinity / gain definition (paper Section V: the
affinity of a vertex to a block is the weight of its edges into the block,
the gain of a move is the affinity to the target minus the affinity to the
own block): a hand-computed example, row sums, the symmetry of block-pair
weights, the cut identity, and the effect of a single move."""
import dataclasses

import numpy as np


def _path_graph(synth_mod):
    # 0-1-2-3-4 with weights 1, 2, 3, 4
    return synth_mod.from_edges(5, [(0, 1), (1, 2), (2, 3), (3, 4)], [1, 2, 3, 4])


def test_affinity_by_hand(oracle_mod, synth_mod):
    g = _path_graph(synth_mod)
    A = oracle_mod.affinity(g, [0, 0, 1, 1, 2], 3)
    assert A.tolist() == [[1, 0, 0], [1, 2, 0], [2, 3, 0], [0, 3, 4], [0, 4, 0]]
    G = oracle_mod.move_gains(g, [0, 0, 1, 1, 2], 3)
    # vertex 2 (block 1): to block 0 gains 2 - 3, vertex 4 (block 2): to block 1 gains 4
    assert G[2].tolist() == [-1, 0, -3] and G[4].tolist() == [0, 4, 0]


def test_affinity_identities(oracle_mod, synth_mod):
    g = synth_mod.rmat_scale(10, 8, seed=6)
    g = dataclasses.replace(g, adjwgt=synth_mod.edge_weights(g, 1, 50, 6))
    k = 7
    blocks = np.random.default_rng(6).integers(0, k, g.n)
    A = oracle_mod.affinity(g, blocks, k)
    src = np.repeat(np.arange(g.n), np.diff(g.xadj.astype(np.int64)))
    wdeg = np.bincount(src, weights=g.adjwgt, minlength=g.n).astype(np.int64)
    assert np.array_equal(A.sum(axis=1), wdeg)  # every edge lands in exactly one block
    # block-pair weights are symmetric: the edges from b into c are those from c into b
    P = np.zeros((k, k), dtype=np.int64)
    np.add.at(P, blocks, A)
    assert np.array_equal(P, P.T)
    # the cut is half of what every vertex sends outside its own block
    own = A[np.arange(g.n), blocks]
    assert (wdeg - own).sum() == 2 * oracle_mod.edge_cut(g, blocks)


def test_single_move_changes_neighbours_only(oracle_mod, synth_mod):
    g = synth_mod.rmat_scale(9, 8, seed=2)
    k = 4
    blocks = np.random.default_rng(2).integers(0, k, g.n)
    A0 = oracle_mod.affinity(g, blocks, k)
    u = int(np.argmax(np.diff(g.xadj.astype(np.int64))))
    s, t = int(blocks[u]), (int(blocks[u]) + 1) % k
    b2 = blocks.copy()
    b2[u] = t
    A1 = oracle_mod.affinity(g, b2, k)
    D = A1 - A0
    nb = g.adjncy[g.xadj[u]: g.xadj[u + 1]]
    # each neighbour loses the edge weight to s and gains it to t; nobody else changes
    exp = np.zeros_like(D)
    np.add.at(exp, (nb, np.full(len(nb), s)), -1)
    np.add.at(exp, (nb, np.full(len(nb), t)), 1)
    assert np.array_equal(D, exp)
