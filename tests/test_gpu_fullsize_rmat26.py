"""Full-size parity on the large coarsening workload: R-MAT scale 26, edge
factor 32, level 0 of the coarsening to 2^14 vertices (cap 12288, 5 rounds,
seed 1), in the launch configuration bench.py times. The graph has
4,157,283,128 adjacency entries (past any signed 32-bit edge index) and
9.2 GB of code bytes (past any 32-bit byte offset), so the 64-bit edge and
byte offset paths of compression, rating, contraction and the cut run. Every label and the per-round proposal / move counts against the
oracle, rated on the graph as given and on its degree-ordered copy; the cut against the oracle; the coarse graph: the fine-to-coarse map
and every coarse vertex weight, the total coarse edge weight (twice the
cut), and sampled coarse rows plus the 20 heaviest clusters recomputed from
the definition of the quotient graph; the coarsening loop: its stop rule and
cap, and the second level's labels against the oracle on that level's
graph."""
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
    # the coarsening loop (R-20) as the library runs it: every level's labels,
    # the coarse sizes, and the second level's graph for the oracle
    levels, final, n_target, cap = lp.coarsen(G, SEED)
    out.update(n_target=n_target, cap=cap, level_n=[L.n for L, _, _ in levels], final_n=final.n,
               level0_labels_equal=bool((levels[0][1] == lab).all().item()))
    if len(levels) > 1:
        L1, lab1, _ = levels[1]
        x1, a1, w1, v1 = lp.lp_decompress(L1)
        out.update(g1=dict(xadj=x1.cpu().numpy().view(np.uint64), adjncy=a1.cpu().numpy(), adjwgt=w1.cpu().numpy(),
                           vwgt=v1.cpu().numpy()), labels1=lab1.cpu().numpy())
        del x1, a1, w1, v1
    for L, _, _ in levels[1:]:
        L.free()
    final.free()
    del levels
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


def test_coarsening_loop(oracle_mod, synth_mod, gpu_run, progress):
    # the stop rule and the level-constant cap of R-20 for n = 2^26 unit
    # vertices: n_target = min(2^14, max(256, n / 64)) = 16384, cap = 3n / n_target
    r = gpu_run
    assert (r["n_target"], r["cap"]) == (16384, CAP)
    assert r["level0_labels_equal"] and r["level_n"][0] == 1 << 26
    assert len(r["level_n"]) >= 2 and r["level_n"][1] == r["cn"]
    # the loop stops at the first level that shrinks by less than 5 % (or
    # reaches n_target), and not before
    sizes = r["level_n"] + [r["final_n"]]
    for k in range(1, len(sizes) - 1):
        assert 100 * sizes[k] <= 95 * sizes[k - 1] and sizes[k] > 16384
    assert 100 * sizes[-1] > 95 * sizes[-2] or sizes[-1] <= 16384
    # level 1 clusters the coarse graph with seed + 1: labels and counts equal
    # the oracle's on that graph (which test_coarse_graph checks on samples)
    g1 = synth_mod.Graph(r["level_n"][1], **r["g1"], name="rmat26-level1")
    t = time.time()
    exp1, props, moves = oracle_rounds(oracle_mod, g1, CAP, ROUNDS, SEED + 1, progress, "rmat-s26 level 1")
    progress(f"rmat-s26 level 1: oracle in {time.time() - t:.0f}s")
    assert np.array_equal(r["labels1"], exp1)
    assert coarse_map(exp1)[1] == r["final_n"]

