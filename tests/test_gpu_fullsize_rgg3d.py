"""Full-size parity on the geometric graph of the large coarsening workload:
RGG-3D with 2^26 vertices, average degree 27, cell-ordered IDs, level 0 of
the coarsening to 2^14 vertices (cap 12288, 5 rounds, seed 1). Every label
and the per-round proposal / move counts against the oracle; the cut against
the oracle; the coarse graph's map and vertex weights, total edge weight and
sampled rows against the definition of the quotient graph."""
import time

import numpy as np
import pytest

from fullsize_checks import check_coarse_rows, coarse_map, oracle_rounds

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

CAP, ROUNDS, SEED = 12288, 5, 1


@pytest.fixture(scope="module")
def rgg3d(synth_mod, progress):
    t = time.time()
    g = synth_mod.rgg3d(1 << 26, 27.0, seed=1)
    progress(f"rgg3d-2^26 generated: n={g.n} 2m={g.two_m} in {time.time() - t:.0f}s")
    return g


@pytest.fixture(scope="module")
def gpu_run(lp, rgg3d, progress):
    g = rgg3d
    t = time.time()
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
    lab, st = lp.lp_cluster(G, CAP, ROUNDS, SEED, config=dict(timing=1), stats=True)
    cut = lp.lp_edge_cut(G, lab)
    C, mp = lp.lp_contract(G, lab)
    out = dict(labels=lab.cpu().numpy(), stats=st, map=mp.cpu().numpy(), cut=cut, cn=C.n)
    G.free()
    x, a, w, v = lp.lp_decompress(C)
    out.update(cx=x.cpu().numpy().view(np.uint64), ca=a.cpu().numpy(), cw=w.cpu().numpy(), cv=v.cpu().numpy())
    del x, a, w, v
    C.free()
    progress(f"rgg3d-2^26: GPU run in {time.time() - t:.0f}s (coarse n {out['cn']})")
    return out


def test_labels_and_counts_match_oracle(oracle_mod, rgg3d, gpu_run, progress):
    exp, props, moves = oracle_rounds(oracle_mod, rgg3d, CAP, ROUNDS, SEED, progress, "rgg3d-2^26")
    assert np.array_equal(gpu_run["labels"], exp)
    st = gpu_run["stats"]
    assert st.rounds_run == len(props)
    assert st.proposals == props and st.moves == moves


def test_cut_matches_oracle(oracle_mod, rgg3d, gpu_run):
    assert gpu_run["cut"] == oracle_mod.edge_cut(rgg3d, gpu_run["labels"])


def test_coarse_graph(rgg3d, gpu_run):
    g, r = rgg3d, gpu_run
    cmap, cn = coarse_map(r["labels"])
    assert r["cn"] == cn and np.array_equal(r["map"], cmap)
    assert np.array_equal(r["cv"], np.bincount(cmap, minlength=cn).astype(np.int32))
    assert int(r["cw"].astype(np.int64).sum()) == 2 * r["cut"]
    check_coarse_rows(g, cmap, cn, r["cx"], r["ca"], r["cw"], sample=1500, seed=12)
