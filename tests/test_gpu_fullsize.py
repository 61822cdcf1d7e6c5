"""Full-size parity on the benchmark workload (R-MAT scale 24, edge factor 16,
cap 256, 5 rounds, seed 1), in the launch configuration bench.py times:
every label and the per-round proposal / move counts against the oracle;
the cut against the oracle; the coarse graph on sampled coarse vertices
(and the largest clusters, which take the heavy contraction path), each
recomputed from the definition of the quotient graph."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu_run(lp, rmat24):
    g = rmat24
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
    lab, st = lp.lp_cluster(G, 256, 5, 1, config=dict(timing=1), stats=True)
    C, mp = lp.lp_contract(G, lab)
    cut = lp.lp_edge_cut(G, lab)
    x, a, w, v = lp.lp_decompress(C)
    out = dict(labels=lab.cpu().numpy(), stats=st, map=mp.cpu().numpy(), cut=cut, cn=C.n,
               cx=x.cpu().numpy().view(np.uint64), ca=a.cpu().numpy(), cw=w.cpu().numpy(), cv=v.cpu().numpy())
    C.free()
    G.free()
    return out


def test_labels_and_counts_match_oracle(oracle_mod, rmat24, gpu_run):
    exp, ost = oracle_mod.lp_cluster(rmat24, 256, 5, 1)
    assert np.array_equal(gpu_run["labels"], exp)
    st = gpu_run["stats"]
    assert st.rounds_run == ost.rounds_run
    assert st.proposals == ost.proposals and st.moves == ost.moves


def test_cut_matches_oracle(oracle_mod, rmat24, gpu_run):
    assert gpu_run["cut"] == oracle_mod.edge_cut(rmat24, gpu_run["labels"])


def test_coarse_graph_sampled(rmat24, gpu_run):
    g, lab = rmat24, gpu_run["labels"]
    n = g.n
    # coarse ID = rank of the label among the nonempty labels
    nonempty = np.zeros(n, dtype=bool)
    nonempty[lab] = True
    rank = np.cumsum(nonempty, dtype=np.int64) - 1
    cmap = rank[lab].astype(np.int32)
    assert np.array_equal(gpu_run["map"], cmap)
    assert gpu_run["cn"] == int(nonempty.sum())
    # coarse vertex weights (unit fine weights): cluster sizes
    sizes = np.bincount(cmap, minlength=gpu_run["cn"])
    assert np.array_equal(gpu_run["cv"], sizes.astype(np.int32))
    # sampled coarse vertices plus the 20 largest clusters by member degree sum
    deg = np.diff(g.xadj.astype(np.int64))
    dsum = np.bincount(cmap, weights=deg, minlength=gpu_run["cn"])
    rng = np.random.default_rng(11)
    pick = np.unique(np.concatenate([rng.integers(0, gpu_run["cn"], 1500), np.argsort(dsum)[-20:]]))
    order = np.argsort(cmap, kind="stable")
    starts = np.searchsorted(cmap[order], np.arange(gpu_run["cn"] + 1))
    cx, ca, cw = gpu_run["cx"], gpu_run["ca"], gpu_run["cw"]
    for a in pick:
        members = order[starts[a]: starts[a + 1]]
        nb = np.concatenate([g.adjncy[g.xadj[u]: g.xadj[u + 1]] for u in members])
        b = cmap[nb]
        b = b[b != a]
        keys, cnt = np.unique(b, return_counts=True)
        row = slice(int(cx[a]), int(cx[a + 1]))
        assert np.array_equal(ca[row], keys), a
        assert np.array_equal(cw[row], cnt.astype(np.int32)), a
