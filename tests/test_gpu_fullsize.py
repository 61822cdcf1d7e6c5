"""Full-size parity on the benchmark workload (R-MAT scale 24, edge factor 16,
cap 256, 5 rounds, seed 1), in the launch configuration bench.py times:
every label and the per-round proposal / move counts against the oracle;
the cut against the oracle; the coarse graph element by element against the
oracle's contraction."""
import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


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


def test_coarse_graph_matches_oracle(oracle_mod, rmat24, gpu_run, progress):
    # element by element: offsets, adjacency, edge weights, vertex weights, map
    import time
    t = time.time()
    cg, mp = oracle_mod.contract(rmat24, gpu_run["labels"])
    progress(f"rmat-s24: oracle contraction in {time.time() - t:.0f}s (coarse n {cg.n}, 2m {cg.two_m})")
    assert gpu_run["cn"] == cg.n
    assert np.array_equal(gpu_run["map"], mp)
    assert np.array_equal(gpu_run["cx"], cg.xadj.astype(np.uint64))
    assert np.array_equal(gpu_run["ca"], cg.adjncy)
    assert np.array_equal(gpu_run["cw"], cg.adjwgt)
    assert np.array_equal(gpu_run["cv"], cg.vwgt)
