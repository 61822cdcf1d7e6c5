"""Pins of the oracle's label propagation (paper Section IV-A, read as
synchronous rounds over a snapshot): closed forms, brute-force enumeration of the
per-round rule on tiny graphs, exhaustive small graphs, and thread-count
invariance."""
import itertools

import numpy as np
import pytest

import bruteforce as bf


def test_tiebreak_key_is_splitmix64(oracle_mod):
    # Published SplitMix64 outputs for seed 0 (Steele, Lea, Flood 2014):
    # draw k is mix(k * gamma); key(s, 0, 0) = mix(s + gamma), so s = 0,
    # gamma, 2 gamma give the first three outputs of the seed-0 stream.
    gamma = 0x9E3779B97F4A7C15
    assert oracle_mod.tiebreak_key(0, 0, 0) == 0xE220A8397B1DCDAF
    assert oracle_mod.tiebreak_key(gamma, 0, 0) == 0x6E789E6AA1B965F4
    assert oracle_mod.tiebreak_key((2 * gamma) % 2**64, 0, 0) == 0x06C45D188009454F
    # round and cluster enter by XOR: key(s, r, c) = key(s ^ (r << 32) ^ c, 0, 0)
    assert oracle_mod.tiebreak_key(5, 3, 7) == oracle_mod.tiebreak_key(5 ^ (3 << 32) ^ 7, 0, 0)
    keys = {oracle_mod.tiebreak_key(11, 2, c) for c in range(5000)}
    assert len(keys) == 5000  # a bijection of c: no secondary ties


def test_cap_one_and_zero_rounds_are_identity(oracle_mod, synth_mod):
    g = synth_mod.rgg2d_16k()
    lab, st = oracle_mod.lp_cluster(g, 1, 5, 1)
    assert np.array_equal(lab, np.arange(g.n))
    assert st.rounds_run == 0
    lab, _ = oracle_mod.lp_cluster(g, 32, 0, 1)
    assert np.array_equal(lab, np.arange(g.n))


@pytest.mark.parametrize("rounds", [1, 2, 3, 4, 5])
def test_perfect_matching_swaps(oracle_mod, synth_mod, rounds):
    # edges {2i, 2i+1}: every vertex proposes its partner's cluster (gain 1)
    # and all are admitted, so labels swap every round (synchronous swap).
    k = 50
    g = synth_mod.from_edges(2 * k, [(2 * i, 2 * i + 1) for i in range(k)])
    lab, st = oracle_mod.lp_cluster(g, 2, rounds, 3)
    ident = np.arange(2 * k)
    swapped = ident ^ 1
    assert np.array_equal(lab, swapped if rounds % 2 else ident)
    assert oracle_mod.edge_cut(g, lab) == k
    assert st.proposals[:rounds] == [2 * k] * rounds


@pytest.mark.parametrize("n,seed", [(3, 1), (5, 7), (9, 2), (20, 11)])
def test_complete_graph_two_rounds(oracle_mod, synth_mod, n, seed):
    # K_n, unit weights, cap >= n. Round 0: all ratings 1 -> everyone picks
    # the neighbour label with the smallest key: t for u != t, t2 for t.
    # Round 1: t sees rating n-1 for cluster t against own 0 -> returns.
    g = synth_mod.from_edges(n, list(itertools.combinations(range(n), 2)))
    keys = [oracle_mod.tiebreak_key(seed, 0, c) for c in range(n)]
    order = sorted(range(n), key=lambda c: keys[c])
    t, t2 = order[0], order[1]
    lab1, _ = oracle_mod.lp_cluster(g, n, 1, seed)
    exp = np.full(n, t)
    exp[t] = t2
    assert np.array_equal(lab1, exp)
    lab2, _ = oracle_mod.lp_cluster(g, n, 2, seed)
    assert np.array_equal(lab2, np.full(n, t))
    assert oracle_mod.edge_cut(g, lab2) == 0


@pytest.mark.parametrize("k,q", [(10, 1), (10, 3), (10, 9), (40, 17)])
def test_star_admits_lowest_ids(oracle_mod, synth_mod, k, q):
    # star centre 0, leaves 1..k, cap q+1: leaves propose cluster 0 with gain
    # 1 and are admitted in increasing ID until the cap (W0[0] = 1); the
    # centre moves to the leaf label with the smallest key.
    g = synth_mod.from_edges(k + 1, [(0, v) for v in range(1, k + 1)])
    seed = 4
    lab, _ = oracle_mod.lp_cluster(g, q + 1, 1, seed)
    keys = {c: oracle_mod.tiebreak_key(seed, 0, c) for c in range(1, k + 1)}
    centre_to = min(keys, key=keys.get)
    exp = np.arange(k + 1)
    exp[1:q + 1] = 0
    exp[0] = centre_to
    assert np.array_equal(lab, exp)


def _snapshots(oracle_mod, g, cap, rounds, seed):
    return [oracle_mod.lp_cluster(g, cap, r, seed)[0] for r in range(rounds + 1)]


@pytest.mark.parametrize("seed", range(12))
def test_rounds_match_enumeration_small_random(oracle_mod, synth_mod, seed):
    n = 6 + seed % 7
    g = synth_mod.random_small(n, 0.45, seed)
    if seed % 3 == 1:
        g.adjwgt = synth_mod.edge_weights(g, 1, 5, seed)
    if seed % 4 == 2:
        g.vwgt = synth_mod.vertex_weights(n, 1, 3, seed)
    cap = 2 + seed % 4
    snaps = _snapshots(oracle_mod, g, cap, 4, seed)
    for r in range(4):
        C0 = snaps[r]
        exp_next, exp_t, exp_g = bf.expected_next(g, C0, cap, seed, r, oracle_mod.tiebreak_key)
        tgt, gain = oracle_mod.lp_proposals(g, C0, bf.cluster_weights(g, C0), cap, seed, r, np.arange(n))
        assert np.array_equal(tgt, exp_t)
        assert np.array_equal(gain[tgt >= 0], exp_g[exp_t >= 0])
        if (exp_t >= 0).any():
            assert np.array_equal(snaps[r + 1], exp_next)
        else:  # fixed point: the run stops, later snapshots repeat
            assert np.array_equal(snaps[r + 1], C0)
        bf.check_valid_clustering(g, snaps[r + 1], cap)


def test_exhaustive_five_vertices(oracle_mod, synth_mod):
    # every labelled simple graph on 5 vertices x caps x rounds x seeds
    n = 5
    pairs = list(itertools.combinations(range(n), 2))
    count = 0
    for mask in range(1 << len(pairs)):
        edges = [p for i, p in enumerate(pairs) if mask >> i & 1]
        g = synth_mod.from_edges(n, edges)
        for cap in (1, 2, 3, 5):
            for seed in (1, 2):
                snaps = _snapshots(oracle_mod, g, cap, 3, seed)
                for r in range(3):
                    exp, exp_t, _ = bf.expected_next(g, snaps[r], cap, seed, r, oracle_mod.tiebreak_key)
                    if (exp_t >= 0).any():
                        assert np.array_equal(snaps[r + 1], exp), (mask, cap, seed, r)
                    else:
                        assert np.array_equal(snaps[r + 1], snaps[r])
                    bf.check_valid_clustering(g, snaps[r + 1], cap)
                    count += 1
    assert count == 1024 * 4 * 2 * 3


def test_heavy_vertex_never_moves(oracle_mod, synth_mod):
    g = synth_mod.from_edges(4, [(0, 1), (1, 2), (2, 3), (0, 3)])
    g.vwgt = np.array([10, 1, 1, 1], dtype=np.int32)
    lab, _ = oracle_mod.lp_cluster(g, 5, 5, 3)
    assert lab[0] == 0  # heavier than the cap: cannot move
    assert (lab[1:] != 0).all()  # and nobody can join it


def test_isolated_vertices_stay(oracle_mod, synth_mod):
    g = synth_mod.from_edges(6, [(0, 1), (1, 2)])
    lab, _ = oracle_mod.lp_cluster(g, 10, 5, 1)
    assert list(lab[3:]) == [3, 4, 5]


def test_weighted_rating_prefers_heavy_edge(oracle_mod, synth_mod):
    # vertex 0 has neighbours 1 (weight 1) and 2 (weight 5): rating of 2's
    # cluster wins regardless of the tie-break
    g = synth_mod.from_edges(3, [(0, 1), (0, 2)], [1, 5])
    for seed in range(10):
        tgt, gain = oracle_mod.lp_proposals(g, np.arange(3), np.ones(3), 3, seed, 0, [0])
        assert tgt[0] == 2 and gain[0] == 5


def test_thread_count_invariance(oracle_mod, synth_mod):
    g = synth_mod.rmat_scale(14, 16, seed=3)
    oracle_mod.set_threads(1)
    a, sa = oracle_mod.lp_cluster(g, 64, 5, 9)
    oracle_mod.set_threads(8)
    b, sb = oracle_mod.lp_cluster(g, 64, 5, 9)
    assert np.array_equal(a, b) and sa.proposals == sb.proposals


def test_invariants_rmat(oracle_mod, synth_mod):
    g = synth_mod.rmat_scale(12, 16, seed=2)
    lab, st = oracle_mod.lp_cluster(g, 40, 5, 3)
    bf.check_valid_clustering(g, lab, 40)
    assert all(m <= p for m, p in zip(st.moves, st.proposals))
    # every proposal at the last round's snapshot is a true maximum
    snap, _ = oracle_mod.lp_cluster(g, 40, 4, 3)
    W0 = bf.cluster_weights(g, snap)
    sample = np.arange(0, g.n, 7, dtype=np.int32)
    tgt, gain = oracle_mod.lp_proposals(g, snap, W0, 40, 3, 4, sample)
    w = bf.vweights(g)
    for i, u in enumerate(sample):
        nb = g.adjncy[g.xadj[u]:g.xadj[u + 1]]
        ratings = {}
        for v in nb:
            ratings[snap[v]] = ratings.get(snap[v], 0) + 1
        own = ratings.get(snap[u], 0)
        feas = {c: r for c, r in ratings.items() if c != snap[u] and W0[c] + w[u] <= 40}
        if not feas or max(feas.values()) <= own:
            assert tgt[i] == -1
        else:
            assert feas[tgt[i]] == max(feas.values()) and gain[i] == feas[tgt[i]] - own


# ----------------------------------------------------------- sub-rounds ----
# Each round is split into S sub-rounds; vertex u acts in sub-round sub(u),
# a fixed mix of u (the tie-break function, pinned above, on a constant
# salt), and every sub-round is one synchronous step over its vertices
# against the state left by the sub-rounds before it.

def test_subround_is_the_tiebreak_mix_of_a_fixed_salt(oracle_mod):
    salt = 0x6A09E667F3BCC909
    for S in (2, 3, 7, 64):
        subs = [oracle_mod.subround(u, S) for u in range(4000)]
        assert subs == [oracle_mod.tiebreak_key(salt, 0, u) % S for u in range(4000)]
        counts = np.bincount(subs, minlength=S)
        assert counts.min() > 0.7 * 4000 / S  # a balanced split


def _subround_runs(oracle_mod, g, cap, rounds, seed, S):
    """Labels after 0..rounds rounds by enumeration: every sub-round takes the
    enumerated best moves of its own vertices under the current labels and
    admits them per target like one synchronous round."""
    w = bf.vweights(g)
    C = np.arange(g.n, dtype=np.int64)
    out = [C.copy()]
    sub = np.array([oracle_mod.subround(u, S) for u in range(g.n)])
    for r in range(rounds):
        moved_any = False
        for s in range(S):
            tgt, gain = bf.expected_proposals(g, C, cap, seed, r, oracle_mod.tiebreak_key)
            tgt = np.where(sub == s, tgt, -1)
            if (tgt >= 0).any():
                moved_any = True
            W0 = bf.cluster_weights(g, C)
            nxt = C.copy()
            for c in sorted(set(int(t) for t in tgt if t >= 0)):
                run = W0[c]
                for _, u in sorted((-int(gain[u]), u) for u in range(g.n) if tgt[u] == c):
                    run += w[u]
                    if run > cap:
                        break
                    nxt[u] = c
            C = nxt
        out.append(C.copy())
        if not moved_any:  # a fixed point: later rounds repeat it
            out.extend(C.copy() for _ in range(rounds - r - 1))
            break
    return out


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("S", [2, 3])
def test_subrounds_match_enumeration_small_random(oracle_mod, synth_mod, seed, S):
    n = 6 + seed % 7
    g = synth_mod.random_small(n, 0.45, seed)
    if seed % 3 == 1:
        g.adjwgt = synth_mod.edge_weights(g, 1, 5, seed)
    if seed % 4 == 2:
        g.vwgt = synth_mod.vertex_weights(n, 1, 3, seed)
    cap = 2 + seed % 4
    exp = _subround_runs(oracle_mod, g, cap, 4, seed, S)
    for r in range(5):
        lab, _ = oracle_mod.lp_cluster(g, cap, r, seed, subrounds=S)
        assert np.array_equal(lab, exp[r]), (seed, S, r)
        bf.check_valid_clustering(g, lab, cap)


@pytest.mark.parametrize("rounds", [1, 2, 3])
@pytest.mark.parametrize("S", [1, 2, 5])
def test_perfect_matching_with_subrounds(oracle_mod, synth_mod, rounds, S):
    # pair (a, b): in the same sub-round both move at once and swap every
    # round (the synchronous pathology); in different sub-rounds the earlier
    # one joins the other's cluster, the later one then stays, and the pair
    # is merged under the label of its later member for good
    k = 60
    g = synth_mod.from_edges(2 * k, [(2 * i, 2 * i + 1) for i in range(k)])
    lab, _ = oracle_mod.lp_cluster(g, 2, rounds, 3, subrounds=S)
    exp = np.empty(2 * k, dtype=np.int64)
    for i in range(k):
        a, b = 2 * i, 2 * i + 1
        sa, sb = oracle_mod.subround(a, S), oracle_mod.subround(b, S)
        if S == 1 or sa == sb:
            exp[a], exp[b] = (b, a) if rounds % 2 else (a, b)
        else:
            exp[a] = exp[b] = b if sa < sb else a
    assert np.array_equal(lab, exp)
    if S > 1:
        merged = sum(oracle_mod.subround(2 * i, S) != oracle_mod.subround(2 * i + 1, S) for i in range(k))
        assert merged > 0 and oracle_mod.edge_cut(g, lab) == k - merged


def test_subround_argument_checks(oracle_mod, synth_mod):
    g = synth_mod.from_edges(4, [(0, 1), (2, 3)])
    for S in (0, 65):
        with pytest.raises(ValueError):
            oracle_mod.lp_cluster(g, 2, 1, 1, subrounds=S)


# ------------------------------------------------- asynchronous reference ----

def test_async_matching_merges_every_pair(oracle_mod, synth_mod):
    # in place: whichever member of a pair comes first joins the other's
    # cluster, and the other then stays (its neighbour is already with it)
    k = 80
    g = synth_mod.from_edges(2 * k, [(2 * i, 2 * i + 1) for i in range(k)])
    lab, st = oracle_mod.lp_cluster_async(g, 2, 5, 9)
    assert all(lab[2 * i] == lab[2 * i + 1] for i in range(k))
    assert oracle_mod.edge_cut(g, lab) == 0
    assert st.rounds_run == 1 and st.moves == [k]


@pytest.mark.parametrize("n,seed", [(5, 1), (12, 4), (30, 9)])
def test_async_complete_graph_one_cluster(oracle_mod, synth_mod, n, seed):
    # K_n, cap >= n: the first mover joins some cluster, which then has the
    # highest rating for every later vertex
    g = synth_mod.from_edges(n, [(a, b) for a in range(n) for b in range(a + 1, n)])
    lab, _ = oracle_mod.lp_cluster_async(g, n, 3, seed)
    assert len(set(lab.tolist())) == 1


@pytest.mark.parametrize("seed", range(6))
def test_async_valid_and_cap(oracle_mod, synth_mod, seed):
    g = synth_mod.random_small(40 + seed, 0.2, seed)
    if seed % 2:
        g.vwgt = synth_mod.vertex_weights(g.n, 1, 3, seed)
    cap = 3 + seed
    lab, _ = oracle_mod.lp_cluster_async(g, cap, 5, seed)
    bf.check_valid_clustering(g, lab, cap)
    # a fixed point of the in-place rule: after the last round nobody moves
    lab2, st2 = oracle_mod.lp_cluster_async(g, cap, 40, seed)
    assert st2.rounds_run < 40
    W = bf.cluster_weights(g, lab2)
    tgt, _ = bf.expected_proposals(g, lab2, cap, seed, st2.rounds_run, oracle_mod.tiebreak_key)
    assert (tgt < 0).all()
    assert W.sum() == bf.vweights(g).sum()


@pytest.mark.parametrize("seed", [1, 5])
def test_rounds_resumed_in_pieces_equal_one_call(oracle_mod, synth_mod, seed):
    # the state between synchronous rounds is the labelling alone, so rounds
    # run one call at a time (as the full-size tests do) give one call's result
    g = synth_mod.rmat_scale(12, 8, seed=seed)
    exp, st = oracle_mod.lp_cluster(g, 40, 6, seed)
    lab = np.arange(g.n, dtype=np.int32)
    props, moves = [], []
    for r in range(6):
        lab, s = oracle_mod.lp_rounds_from(g, 40, seed, lab, r, 1)
        props += s.proposals
        moves += s.moves
    assert np.array_equal(lab, exp)
    assert props == st.proposals and moves == st.moves
    # a fixed point (the matching after its swaps, cap 1) stays put
    m = synth_mod.from_edges(8, [(0, 1), (2, 3), (4, 5), (6, 7)])
    same, s = oracle_mod.lp_rounds_from(m, 1, 3, np.arange(8, dtype=np.int32), 4, 2)
    assert np.array_equal(same, np.arange(8)) and s.rounds_run == 0
