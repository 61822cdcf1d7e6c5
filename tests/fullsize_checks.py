"""Checks shared by the full-size GPU tests: the oracle's rounds one call at
a time (so that each finished round is reported), and the coarse graph on
sampled coarse vertices recomputed from the definition of the quotient graph
(coarse ID = rank of the label among the nonempty labels; coarse edge weight
= sum of the weights of the fine edges between the two clusters)."""
import time

import numpy as np


def oracle_rounds(oracle_mod, g, cap: int, rounds: int, seed: int, progress, name: str):
    """Labels and per-round proposal / move counts of lp_cluster(g, cap, rounds, seed)."""
    lab = np.arange(g.n, dtype=np.int32)
    props, moves = [], []
    for r in range(rounds):
        t = time.time()
        lab, s = oracle_mod.lp_rounds_from(g, cap, seed, lab, r, 1)
        progress(f"{name}: oracle round {r} in {time.time() - t:.0f}s, proposals {s.proposals}")
        if s.rounds_run == 0:
            break
        props += s.proposals
        moves += s.moves
    return lab, props, moves


def coarse_map(lab: np.ndarray):
    n = len(lab)
    nonempty = np.zeros(n, dtype=bool)
    nonempty[lab] = True
    rank = np.cumsum(nonempty, dtype=np.int64) - 1
    return rank[lab].astype(np.int32), int(nonempty.sum())


def check_coarse_rows(g, cmap: np.ndarray, cn: int, cx, ca, cw, sample: int, seed: int, heaviest: int = 20):
    """Sampled coarse rows (plus the clusters with the largest member degree
    sums, which take the heavy contraction path) against the definition."""
    deg = np.diff(g.xadj.astype(np.int64))
    dsum = np.bincount(cmap, weights=deg, minlength=cn)
    rng = np.random.default_rng(seed)
    pick = np.unique(np.concatenate([rng.integers(0, cn, sample), np.argsort(dsum)[-heaviest:]]))
    order = np.argsort(cmap, kind="stable")
    starts = np.searchsorted(cmap[order], np.arange(cn + 1))
    for a in pick:
        members = order[starts[a]: starts[a + 1]]
        nb = np.concatenate([g.adjncy[g.xadj[u]: g.xadj[u + 1]] for u in members])
        wt = (np.concatenate([g.adjwgt[g.xadj[u]: g.xadj[u + 1]] for u in members])
              if g.adjwgt is not None else np.ones(len(nb), dtype=np.int64))
        b = cmap[nb]
        keep = b != a
        keys, inv = np.unique(b[keep], return_inverse=True)
        sums = np.bincount(inv, weights=wt[keep].astype(np.int64), minlength=len(keys)).astype(np.int64)
        row = slice(int(cx[a]), int(cx[a + 1]))
        assert np.array_equal(ca[row], keys), a
        assert np.array_equal(cw[row].astype(np.int64), sums), a
    return len(pick)
