"""Sub-round LP on the GPU vs the oracle (labels and per-round statistics
bit-exact), on graphs that reach every rating path, with other thresholds,
on plain and compressed handles, and on batches (each graph's sub-rounds
come from its own vertex IDs)."""
import numpy as np
import pytest

from test_gpu_parity import _graphs, _gpu_graph

pytestmark = pytest.mark.gpu


def _np(t):
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def graphs(synth_mod):
    return _graphs(synth_mod)


CASES = [("rgg2d-16k", 32), ("rmat-s13-ef16", 64), ("rmat-s12-weighted", 40), ("star-25000", 300),
         ("star-10001-w", 5000), ("bip-5x2048", 600), ("bip-3x9000-w", 4000)]


@pytest.mark.parametrize("S", [2, 3, 4])
@pytest.mark.parametrize("name,cap", CASES)
def test_subrounds_match_oracle(lp, oracle_mod, graphs, name, cap, S):
    g = graphs[name]
    exp, ost = oracle_mod.lp_cluster(g, cap, 5, 7, subrounds=S)
    G = _gpu_graph(lp, g)
    lab, st = lp.lp_cluster(G, cap, 5, 7, config=dict(subrounds=S), stats=True)
    assert np.array_equal(_np(lab), exp)
    assert st.rounds_run == ost.rounds_run
    assert st.proposals == ost.proposals and st.moves == ost.moves


@pytest.mark.parametrize("knobs", [dict(t_lane=1, t_tile=1, t_block=1, hub_part=256),
                                   dict(t_lane=4, t_tile=64, t_block=64, hub_part=1024)])
def test_subrounds_with_other_thresholds_and_plain(lp, oracle_mod, graphs, knobs):
    g = graphs["rmat-s13-ef16"]
    exp, _ = oracle_mod.lp_cluster(g, 64, 4, 3, subrounds=3)
    for compressed in (True, False):
        G = _gpu_graph(lp, g, compressed)
        lab = lp.lp_cluster(G, 64, 4, 3, config=dict(knobs, subrounds=3))
        assert np.array_equal(_np(lab), exp), (knobs, compressed)
        # the cached sub-round plans of the default thresholds, twice
        for _ in range(2):
            assert np.array_equal(_np(lp.lp_cluster(G, 64, 4, 3, config=dict(subrounds=3))), exp)


def test_matching_merges_across_subrounds(lp, oracle_mod, synth_mod):
    k = 500
    g = synth_mod.from_edges(2 * k, [(2 * i, 2 * i + 1) for i in range(k)])
    G = _gpu_graph(lp, g)
    for S, rounds in ((1, 3), (2, 3), (4, 2)):
        lab = _np(lp.lp_cluster(G, 2, rounds, 3, config=dict(subrounds=S)))
        exp, _ = oracle_mod.lp_cluster(g, 2, rounds, 3, subrounds=S)
        assert np.array_equal(lab, exp)
        cut = lp.lp_edge_cut(G, lab)
        assert cut == (k if S == 1 else oracle_mod.edge_cut(g, exp)) and (S == 1 or cut < k)


def test_subrounds_in_batches(lp, oracle_mod, synth_mod):
    recipe = [("rgg2d", 900, 8, 31), ("rmat", 700, 10, 32), ("rmat", 3000, 9, 33), ("rgg2d", 2000, 8, 34)]
    gs = [synth_mod.batch_graph(*r) for r in recipe]
    hs = [lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy) for g in gs]
    caps, seeds = [40, 17, 90, 33], [5, 6, 7, 8]
    B = lp.lp_batch_create(hs)
    lab = _np(lp.lp_batch_cluster_ex(B, caps, 5, seeds, config=dict(subrounds=3)))
    for part, g, c, sd in zip(B.split(lab), gs, caps, seeds):
        exp, _ = oracle_mod.lp_cluster(g, c, 5, sd, subrounds=3)
        assert np.array_equal(part, exp)


def test_subround_argument_errors(lp, synth_mod):
    g = synth_mod.from_edges(4, [(0, 1), (2, 3)])
    G = _gpu_graph(lp, g)
    for S in (-1, 65):
        with pytest.raises(lp.LPError) as e:
            lp.lp_cluster(G, 2, 1, 1, config=dict(subrounds=S))
        assert e.value.status == lp.LP_EINVAL
