"""Coarsening quality of the three LP schedules on the 16k-vertex RGG-2D
graph, all from the oracle: plain synchronous rounds stall early on this
geometric graph (neighbours keep moving at once), while sub-rounds and the
paper's asynchronous in-place rounds coarsen it to the target size with a
far smaller cut of the composed clustering."""
import numpy as np
import pytest


def _left(x):
    return int(np.asarray(x.adjwgt, dtype=np.int64).sum()) // 2 if x.adjwgt is not None else x.two_m // 2


@pytest.fixture(scope="module")
def runs(oracle_mod, synth_mod):
    g = synth_mod.rgg2d_16k()
    out = {}
    for name, fn in (("sync", None),
                     ("sub4", lambda G, c, r, s: oracle_mod.lp_cluster(G, c, r, s, subrounds=4)),
                     ("async", oracle_mod.lp_cluster_async)):
        levels, final, n_target, _ = oracle_mod.coarsen(g, 1, 5, cluster=fn)
        out[name] = (len(levels), final.n, n_target, _left(final))
    return out


def test_subrounds_and_async_reach_the_target(runs):
    for name in ("sub4", "async"):
        _, n, n_target, _ = runs[name]
        assert n <= n_target, (name, n, n_target)
    _, n_sync, n_target, _ = runs["sync"]
    assert n_sync > n_target  # the synchronous schedule stalls first


def test_subrounds_and_async_cut_far_less(runs):
    cut_sync = runs["sync"][3]
    assert runs["sub4"][3] < cut_sync / 2
    assert runs["async"][3] < cut_sync / 2
