"""Full-size parity on the large coarsening workload: R-MAT scale 26, edge
factor 32, level 0 of the coarsening to 2^14 vertices (cap 12288, 5 rounds,
seed 1), in the launch configuration bench.py times. The graph has
4,157,283,128 adjacency entries (past any signed 32-bit edge index) and
9.2 GB of code bytes (past any 32-bit byte offset), so the 64-bit edge and
byte offset paths of compression, rating, contraction and the cut run. Every label and the per-round proposal / move counts against the
oracle, rated on the graph as given and on its degree-ordered copy; the cut against the oracle; the coarse graph: the fine-to-coarse map
and every coarse vertex weight, the total coarse edge weight (twice the
cut), and sampled coarse rows plus the 20 heaviest clusters recomputed from
the definition of the quotient graph."""
import time

import numpy as np
import pytest

from fullsize_checks import check_coarse_rows, coarse_map, oracle_rounds

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

CAP, ROUNDS, SEED = 12288, 5, 1


@pytest.fixture(scope="module")
def rmat26(synth_mod, progress):
    t = time.time()
    g = synth_mod.rmat_scale(26, 32, seed=1)
    progress(f"rmat-s26-ef32 generated: n={g.n} 2m={g.two_m} in {time.time() - t:.0f}s")
    return g


@pytest.fixture(scope="module")
def gpu_run(lp, rmat26, progress):
    g = rmat26
    t = time.time()
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
    lab, st = lp.lp_cluster(G, CAP, ROUNDS, SEED, config=dict(timing=1), stats=True)
    # rated again on the degree-ordered copy, as bench.py's timed steps are
    lab_ro, st_ro = lp.lp_cluster(G, CAP, ROUNDS, SEED, config=dict(timing=1, reorder=1), stats=True)
    same_ro = bool((lab_ro == lab).all().item()) and st_ro.proposals == st.proposals and st_ro.moves == st.moves
    del lab_ro
    cut = lp.lp_edge_cut(G, lab)
    C, mp = lp.lp_contract(G, lab)
    out = dict(nbytes=G.nbytes, two_m=G.two_m, labels=lab.cpu().numpy(), stats=st, map=mp.cpu().numpy(), cut=cut,
               cn=C.n, same_ro=same_ro)
    G.free()
    x, a, w, v = lp.lp_decompress(C)
    out.update(cx=x.cpu().numpy().view(np.uint64), ca=a.cpu().numpy(), cw=w.cpu().numpy(), cv=v.cpu().numpy())
    del x, a, w, v
    C.free()
    progress(f"rmat-s26: GPU compress, cluster, cut, contract and copy-back in {time.time() - t:.0f}s "
             f"({out['nbytes']} code bytes, coarse n {out['cn']})")
    return out


def test_offsets_beyond_32_bits(gpu_run):
    assert gpu_run["two_m"] > 2**31 and gpu_run["nbytes"] > 2**32


def test_labels_and_counts_match_oracle(oracle_mod, rmat26, gpu_run, progress):
    exp, props, moves = oracle_rounds(oracle_mod, rmat26, CAP, ROUNDS, SEED, progress, "rmat-s26")
    assert np.array_equal(gpu_run["labels"], exp)
    st = gpu_run["stats"]
    assert st.rounds_run == len(props)
    assert st.proposals == props and st.moves == moves
    assert gpu_run["same_ro"]  # the degree-ordered copy gives the same labels and counts


def test_cut_matches_oracle(oracle_mod, rmat26, gpu_run):
    assert gpu_run["cut"] == oracle_mod.edge_cut(rmat26, gpu_run["labels"])


def test_coarse_graph(rmat26, gpu_run, progress):
    g, r = rmat26, gpu_run
    cmap, cn = coarse_map(r["labels"])
    assert r["cn"] == cn and np.array_equal(r["map"], cmap)
    assert np.array_equal(r["cv"], np.bincount(cmap, minlength=cn).astype(np.int32))
    cx = r["cx"]
    assert cx[0] == 0 and int(cx[-1]) == len(r["ca"]) and np.all(np.diff(cx.astype(np.int64)) >= 0)
    assert int(r["cw"].astype(np.int64).sum()) == 2 * r["cut"]
    t = time.time()
    k = check_coarse_rows(g, cmap, cn, cx, r["ca"], r["cw"], sample=1500, seed=11)
    progress(f"rmat-s26: {k} coarse rows checked in {time.time() - t:.0f}s")
