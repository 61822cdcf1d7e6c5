"""Brute-force checks used to pin the oracle on tiny graphs.

These are deliberately written differently from the oracle: ratings are a
dense table over every cluster ID, computed from an edge list, and every
property is checked by enumeration. They check the rules of the synchronous
size-constrained label propagation (paper Section IV-A, read as rounds over a
snapshot with prefix admission per target) and of contraction (Section IV-B).
"""
from __future__ import annotations

import numpy as np


def edge_list(g):
    """Directed (u, v, w) triples of a CSR graph."""
    out = []
    for u in range(g.n):
        for e in range(int(g.xadj[u]), int(g.xadj[u + 1])):
            out.append((u, int(g.adjncy[e]), 1 if g.adjwgt is None else int(g.adjwgt[e])))
    return out


def vweights(g):
    return np.ones(g.n, dtype=np.int64) if g.vwgt is None else np.asarray(g.vwgt, dtype=np.int64)


def cluster_weights(g, labels):
    W = np.zeros(g.n, dtype=np.int64)
    w = vweights(g)
    for u in range(g.n):
        W[labels[u]] += w[u]
    return W


def dense_ratings(g, C0):
    """R[u][c] = total weight of edges from u to vertices in cluster c."""
    R = np.zeros((g.n, g.n), dtype=np.int64)
    for u, v, w in edge_list(g):
        R[u, C0[v]] += w
    return R


def expected_proposals(g, C0, cap, seed, rnd, key):
    """(target or -1, gain) per vertex by enumerating every cluster ID."""
    W0 = cluster_weights(g, C0)
    w = vweights(g)
    R = dense_ratings(g, C0)
    tgt = np.full(g.n, -1, dtype=np.int64)
    gain = np.zeros(g.n, dtype=np.int64)
    for u in range(g.n):
        own = R[u, C0[u]]
        best = None
        for c in range(g.n):
            if c == C0[u] or R[u, c] <= 0 or W0[c] + w[u] > cap:
                continue
            cand = (-R[u, c], key(seed, rnd, c), c)
            if best is None or cand < best:
                best = cand
        if best is not None and -best[0] > own:
            tgt[u] = best[2]
            gain[u] = -best[0] - own
    return tgt, gain


def expected_next(g, C0, cap, seed, rnd, key):
    """Labels after one synchronous round, admission by enumeration: for each
    target, walk its proposals in (gain desc, vertex asc) order and admit
    while the running weight fits; the first rejection closes the target."""
    tgt, gain = expected_proposals(g, C0, cap, seed, rnd, key)
    W0 = cluster_weights(g, C0)
    w = vweights(g)
    C = np.array(C0, dtype=np.int64).copy()
    for c in sorted(set(int(t) for t in tgt if t >= 0)):
        props = sorted((-int(gain[u]), u) for u in range(g.n) if tgt[u] == c)
        run = W0[c]
        for _, u in props:
            run += w[u]
            if run > cap:
                break
            C[u] = c
    return C, tgt, gain


def check_valid_clustering(g, labels, cap):
    labels = np.asarray(labels)
    assert labels.min() >= 0 and labels.max() < g.n
    W = cluster_weights(g, labels)
    sizes = np.bincount(labels, minlength=g.n)
    # every cluster that gained a member respects the cap
    for c in range(g.n):
        if sizes[c] >= 2:
            assert W[c] <= cap, (c, W[c], cap)
    assert W.sum() == vweights(g).sum()


def dense_quotient(g, labels):
    """(n', dense coarse adjacency, coarse vertex weights) by enumeration."""
    used = sorted(set(int(x) for x in labels))
    rank = {c: i for i, c in enumerate(used)}
    k = len(used)
    A = np.zeros((k, k), dtype=np.int64)
    for u, v, w in edge_list(g):
        a, b = rank[int(labels[u])], rank[int(labels[v])]
        if a != b:
            A[a, b] += w
    vw = np.zeros(k, dtype=np.int64)
    wts = vweights(g)
    for u in range(g.n):
        vw[rank[int(labels[u])]] += wts[u]
    return k, A, vw


def cut_by_enumeration(g, labels):
    s = 0
    for u, v, w in edge_list(g):
        if u < v and labels[u] != labels[v]:
            s += w
    return s
