"""Benchmark: LP-round edges/s of size-constrained label propagation on a
compressed R-MAT graph, one MI355X.

One step = one pass of the whole hot path over the resident compressed graph:
lp_cluster (degree buckets + 5 synchronous rounds of rating, acceptance and
apply), lp_contract (coarse graph) and lp_edge_cut. The graph is generated,
compressed and made resident before the timed region.

Workload (default): R-MAT scale 26, edge factor 32 (2^31 samples),
(a, b, c, d) = (0.57, 0.19, 0.19, 0.05), symmetrised, self-loops and
duplicates removed, no ID permutation, unit weights; level 0 of the
coarsening to 2^14 vertices: max cluster weight 12288, 5 rounds, seed 1.

value = 2m / t_round, t_round = median over every round of the timed steps
of one LP round (rating + acceptance + apply), timed with HIP events on the
call's stream. The JSON line also carries the step rate (contraction and cut
included), a per-phase breakdown, the roofline of the dominant rating kernel
(algorithmic bytes / event-timed duration against 8 TB/s HBM), the round's
algorithmic-byte model, the CPU oracle timed on a bounded sample, the
R-MAT scale 24 rate, and the batched and served forms.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PHASE_KERNEL = {
    "lane": "k_rate_lane",
    "tile": "k_rate_tile (small tiles)",
    "block": "k_rate_tile (large tiles)",
    "hub": "k_hub_piece+k_hub_reduce+k_hub_combine",
    "accept": "acceptance (compaction, radix sort, segmented scan, admit, apply)",
}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def workload(name: str):
    import synth
    if name == "rmat26":
        os.environ["SYNTH_PROGRESS"] = "1"  # the generator reports its phases on stderr
        return (synth.rmat_scale(26, 32, seed=1), 12288,
                "rmat-s26-ef32 (0.57,0.19,0.19,0.05), unit weights, level 0 of the coarsening to 2^14")
    if name == "rmat24":
        return synth.rmat_scale(24, 16, seed=1), 256, "rmat-s24-ef16 (0.57,0.19,0.19,0.05), unit weights"
    if name == "rmat20":
        return synth.rmat_scale(20, 16, seed=1), 256, "rmat-s20-ef16 (0.57,0.19,0.19,0.05), unit weights"
    if name == "rgg2d16k":
        return synth.rgg2d_16k(seed=1), 32, "rgg2d n=16384 avg-deg~8, unit weights"
    raise SystemExit(f"unknown workload {name}")


TRAFFIC_SOURCES = ("paper_2410_19119_amd/csrc/cluster.hip", "paper_2410_19119_amd/csrc/decode.h",
                   "paper_2410_19119_amd/csrc/lp_device.h", "paper_2410_19119_amd/csrc/lp_common.h")
TRAFFIC_FILE = "profiles/rmat26_rating_hbm_traffic.md"
ROUND_TRAFFIC_FILE = "profiles/rmat26_round_hbm_traffic.md"


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(path: str = TRAFFIC_FILE, key: str = "hbm_bytes_per_launch"):
    """HBM bytes from a committed PMC summary (per launch of the dominant
    kernel, or per LP round), or None when it is missing or the kernel
    sources changed since the counters were taken."""
    path = os.path.join(ROOT, path)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_hash") != kernel_source_hash():
        return None
    try:
        return int(vals[key])
    except (KeyError, ValueError):
        return None


def phase_bytes(st, phase: str, n_per_bucket, proposals) -> float:
    """Algorithmic bytes of one launch of a phase (one round)."""
    idx = {"lane": 0, "tile": 1, "block": 2, "hub": 3}
    if phase in idx:
        b = idx[phase]
        nv = n_per_bucket[b]
        # compressed records + per-edge label gather + per-vertex offset,
        # degree, list entry, own label, one cluster weight, proposal writes
        return st.bucket_bytes[b] + 4.0 * st.bucket_edges[b] + 40.0 * nv
    if phase == "accept":
        return 4.0 * sum(n_per_bucket) + 20.0 * proposals
    return 0.0


def bench_batch(args) -> dict:
    """Many uneven graphs: one batched launch sequence vs sequential plain calls."""
    import math

    import torch

    import paper_2410_19119_amd as lp
    import synth
    from paper_2410_19119_amd import autotune

    count = args.batch_graphs
    t0 = time.time()
    recipe = synth.batch_recipe(count, 1000)
    gs = [synth.batch_graph(*r) for r in recipe]
    tot_n = sum(g.n for g in gs)
    tot_m = sum(g.two_m for g in gs)
    log(f"[batch] generated {count} graphs: n={tot_n} 2m={tot_m} in {time.time() - t0:.1f}s")
    hs = [lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy) for g in gs]
    caps = [3 * max(1, math.ceil(g.two_m / max(g.n, 1))) for g in gs]
    seeds = [r[3] for r in recipe]
    rounds = args.rounds
    out_plain = [torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda") for g in gs]
    out_batch = [torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda") for g in gs]
    union_lab = torch.empty(max(tot_n, 1), dtype=torch.int32, device="cuda")

    def plain():
        for i, h in enumerate(hs):
            lp.lp_cluster(h, caps[i], rounds, seeds[i], labels=out_plain[i])

    def batched():
        lp.lp_batch_cluster(hs, caps, rounds, seeds, labels=out_batch)

    b = lp.lp_batch_create(hs)
    cfg = {}

    def resident():
        lp.lp_batch_cluster_ex(b, caps, rounds, seeds, labels=union_lab, config=cfg or None)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return sum(ts) / len(ts)

    t_plain = timed(plain, args.batch_reps)
    log(f"[batch] plain: {t_plain * 1e3:.1f} ms for {count} graphs")
    t_batch = timed(batched, args.batch_reps)
    log(f"[batch] batched (union built per call): {t_batch * 1e3:.1f} ms")
    t_res = timed(resident, args.batch_reps)
    log(f"[batch] batched (resident union, default knobs): {t_res * 1e3:.1f} ms")
    best, table = autotune.tune_batch(lp, b, caps, seeds, rounds=1)
    cfg.update(best)
    t_tuned = timed(resident, args.batch_reps)
    log(f"[batch] batched (resident union, autotuned {best}): {t_tuned * 1e3:.1f} ms")
    same = all(torch.equal(out_plain[i][: g.n], out_batch[i][: g.n]) for i, g in enumerate(gs))
    parts = b.split(union_lab)
    same = same and all(torch.equal(out_plain[i][: g.n], parts[i]) for i, g in enumerate(gs))
    log(f"[batch] identical labels batched vs plain: {same}")
    return {
        "graphs": count, "n": tot_n, "two_m": tot_m, "rounds": rounds,
        "plain_graphs_per_s": count / t_plain,
        "batched_graphs_per_s": count / t_batch,
        "resident_graphs_per_s": count / t_res,
        "autotuned_graphs_per_s": count / t_tuned,
        "autotuned_knobs": best,
        "speedup_vs_plain": t_plain / t_batch,
        "identical_labels": bool(same),
        "plain_ms": t_plain * 1e3, "batched_ms": t_batch * 1e3, "resident_ms": t_res * 1e3,
        "autotuned_ms": t_tuned * 1e3,
    }


def bench_serve(args) -> dict:
    """Poisson request stream of coarsening jobs on resident compressed graphs:
    continuous batching vs sequential plain calls, same arrival trace."""
    import torch

    import paper_2410_19119_amd as lp
    import synth
    from paper_2410_19119_amd import serve

    t0 = time.time()
    recipe = synth.serve_pool(args.serve_pool, 5000)
    gs = [synth.batch_graph(*r) for r in recipe]
    pool = [lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy) for g in gs]
    torch.cuda.synchronize()
    log(f"[serve] pool of {len(pool)} graphs, 2m from {min(g.two_m for g in gs)} to "
        f"{max(g.two_m for g in gs)} (total {sum(g.two_m for g in gs)}) in {time.time() - t0:.1f}s")
    del gs
    # warm-up: one job of each graph
    for h in pool:
        lp.coarsen(h, seed=1)
    torch.cuda.synchronize()
    rates = [float(r) for r in (args.serve_rates or "10,30,100,300,1000").split(",")]
    out = {"pool": len(pool), "pool_two_m": [int(h.two_m) for h in pool], "budget_bytes": 200 * 10**9,
           "split_edges": args.serve_split, "rates": {}}
    for rate in rates:
        # requests per rate: fixed, or (0) those arriving in --serve-window seconds, 100 to 2000
        count = args.serve_requests or min(2000, max(100, int(rate * args.serve_window)))
        reqs = serve.requests(synth.serve_trace(rate, count, len(pool), seed=7))
        seq = serve.summarize(serve.run_sequential(pool, reqs))
        srv_obj = serve.Server(pool, budget_bytes=200 * 10**9, max_active=args.serve_slots,
                               split_edges=args.serve_split)
        res = srv_obj.run(reqs)
        srv = serve.summarize(res)
        srv["peak_active"] = srv_obj.peak_active
        srv["steps"] = srv_obj.steps
        out["rates"][str(rate)] = {"requests": count, "sequential": seq, "served": srv}
        log(f"[serve] rate {rate}/s: sequential {seq['throughput_per_s']:.1f} jobs/s p50 {seq['p50_ms']:.1f} ms "
            f"p99 {seq['p99_ms']:.1f} ms | served {srv['throughput_per_s']:.1f} jobs/s p50 {srv['p50_ms']:.1f} ms "
            f"p99 {srv['p99_ms']:.1f} ms (peak {srv_obj.peak_active} active)")
    return out


def level_checks(lp, cur, labels, nxt, cap, total_vwgt, sample: int = 256) -> dict:
    """Properties of one coarsening level that hold at any size (no oracle):
    labels in range, no multi-member cluster above the cap, vertex weight
    conserved, coarse edge weight = 2 * cut, coarse adjacency symmetric on a
    sample of coarse vertices."""
    import torch

    n = cur.n
    lab = labels[:n].to(torch.int64)
    ok_range = bool(((lab >= 0) & (lab < n)).all())
    _, _, _, vw = lp.lp_decompress(cur) if not cur.compressed else (None, None, None, None)
    w = vw.to(torch.int64) if vw is not None else torch.ones(n, dtype=torch.int64, device="cuda")
    cw = torch.zeros(n, dtype=torch.int64, device="cuda").index_add_(0, lab, w)
    members = torch.bincount(lab, minlength=n)
    ok_cap = bool(((members < 2) | (cw <= cap)).all())
    xa, ad, aw, cvw = lp.lp_decompress(nxt)
    ok_w = int(cvw.to(torch.int64).sum()) == int(total_vwgt)
    cut = lp.lp_edge_cut(cur, labels)
    ok_cut = int(aw.to(torch.int64).sum()) == 2 * cut
    # symmetry on sampled coarse vertices: every (a, b, w) has (b, a, w)
    g = torch.Generator(device="cpu").manual_seed(5)
    pick = torch.randint(0, max(nxt.n, 1), (min(sample, nxt.n),), generator=g)
    xh = xa.cpu()
    ok_sym = True
    for a in pick.tolist():
        b0, b1 = int(xh[a]), int(xh[a + 1])
        for j in range(b0, min(b1, b0 + 8)):
            b = int(ad[j])
            c0, c1 = int(xh[b]), int(xh[b + 1])
            row = ad[c0:c1]
            k = int(torch.searchsorted(row, torch.tensor([a], device="cuda", dtype=row.dtype)))
            if k >= c1 - c0 or int(row[k]) != a or int(aw[c0 + k]) != int(aw[j]):
                ok_sym = False
                break
        if not ok_sym:
            break
    return {"labels_in_range": ok_range, "cap_respected": ok_cap, "vertex_weight_conserved": ok_w,
            "edge_weight_is_2cut": ok_cut, "symmetric_sample": ok_sym, "cut": cut}


def bench_subrounds(args, G=None) -> dict:
    """Sub-round LP (S sub-rounds per round) against plain synchronous rounds on
    the R-MAT scale 24 graph: one clustering level (round time, moves, cut) and
    the whole coarsening (levels, final size, and the cut of the composed
    clustering, i.e. half the edge weight left in the coarsest graph)."""
    import torch

    import paper_2410_19119_amd as lp
    import synth

    if G is None:
        g = synth.rmat_scale(24, 16, seed=1)
        G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
        del g
    out = {}
    for S in [int(x) for x in args.subrounds.split(",")]:
        cfg = dict(timing=1, subrounds=S)
        lp.lp_cluster(G, 256, args.rounds, 1, config=cfg)  # builds and caches the sub-round plans
        torch.cuda.synchronize()
        lab, st = lp.lp_cluster(G, 256, args.rounds, 1, config=cfg, stats=True)
        cut = lp.lp_edge_cut(G, lab)
        C, _ = lp.lp_contract(G, lab, want_map=False)
        level = {"round_ms": round(st.phase_ms["round"] / max(1, st.phase_launches["round"]), 3),
                 "moves": int(sum(st.moves)), "cut": int(cut), "coarse_n": C.n}
        C.free()
        torch.cuda.synchronize()
        t = time.perf_counter()
        levels, final, n_target, _ = lp.coarsen(G, seed=1, rounds=args.rounds, subrounds=S)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        _, _, w, _ = lp.lp_decompress(final) if not final.compressed else (None, None, None, None)
        left = int(w.to(torch.int64).sum()) // 2 if w is not None else None
        out[str(S)] = {"one_level": level, "coarsening": {"levels": len(levels), "final_n": final.n,
                                                            "cut_of_hierarchy": left, "ms": round(1e3 * dt, 1)}}
        for lv in levels[1:]:
            lv[0].free()
        if final is not G:
            final.free()
        log(f"[subrounds] S={S}: round {level['round_ms']} ms, cut {cut}, coarse n {level['coarse_n']} | "
            f"coarsening {len(levels)} levels to n={out[str(S)]['coarsening']['final_n']}, cut {left}, "
            f"{1e3 * dt:.0f} ms")
    return out


def bench_partition(args, G=None) -> dict:
    """Multilevel k-way partition of the R-MAT scale 24 graph, of RGG-2D with
    2^24 vertices and average degree 8, or of RGG-3D with 2^26 vertices and
    average degree 27 (k from --partition-k, eps 3 %):
    coarsening under the partition cap, contiguous initial partition and
    refinement of the coarsest graph, then projection and refinement on every
    finer level, all on the device. Reports the end-to-end time (after one
    untimed run), the cut per level, the balance, and the refinement round
    rate on the input graph."""
    import torch

    import paper_2410_19119_amd as lp
    import synth

    if G is None:
        if args.partition_graph == "rgg2d":
            g = synth.rgg(2, 1 << 24, synth.rgg_radius(2, 1 << 24, 8.0), seed=1)
        elif args.partition_graph == "rgg3d":
            g = synth.rgg3d(1 << 26, 27.0, seed=1)
        else:
            g = synth.rmat_scale(24, 16, seed=1)
        G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
        del g
    out = {}
    for k in [int(x) for x in args.partition_k.split(",")]:
        lmax = lp.max_block_weight(G.total_vwgt, k)
        S = args.partition_subrounds
        _, trace = lp.partition(G, k, seed=1, rounds=args.rounds, subrounds=S, refine_subrounds=S, trace=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        blocks = lp.partition(G, k, seed=1, rounds=args.rounds, subrounds=S, refine_subrounds=S)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        cut = lp.lp_edge_cut(G, blocks)
        bw = torch.bincount(blocks.to(torch.int64), minlength=k)
        # the same partition with every refinement rated from a sparse gain table
        blocks_gt = lp.partition(G, k, seed=1, rounds=args.rounds, subrounds=S, refine_subrounds=S, gain_table=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        blocks_gt = lp.partition(G, k, seed=1, rounds=args.rounds, subrounds=S, refine_subrounds=S, gain_table=True)
        torch.cuda.synchronize()
        dt_gt = time.perf_counter() - t
        same = bool(torch.equal(blocks_gt, blocks))
        # refinement of the input graph from its contiguous split, rated from
        # the graph and from the gain table (built in the call's setup)
        ip = lp.lp_initial_partition(G, k)
        ref = {}
        for name, cfg in (("graph", dict(timing=1)), ("gain_table", dict(timing=1, gain_table=1))):
            lp.lp_refine(G, ip, k, lmax, args.rounds, 1, config=cfg)
            torch.cuda.synchronize()
            _, st = lp.lp_refine(G, ip, k, lmax, args.rounds, 1, config=cfg, stats=True)
            nr = max(1, st.phase_launches["round"])
            rms = st.phase_ms["round"] / nr
            acc = st.phase_ms["accept"] / nr  # acceptance and moves (and the table update)
            ref[name] = {"round_ms": round(rms, 3), "rate_ms": round(rms - acc, 3), "accept_ms": round(acc, 3),
                         "setup_ms": round(st.phase_ms["setup"], 3), "moves": [int(x) for x in st.moves]}
        T = lp.GainTable(G, ip, k)
        slots, tbytes, _, _ = T.info()
        T.free()
        ref["gain_table"].update({"slots": int(slots), "bytes": int(tbytes), "graph_bytes": int(G.nbytes)})
        out[str(k)] = {"subrounds": S, "ms": round(1e3 * dt, 1), "ms_gain_table": round(1e3 * dt_gt, 1),
                       "identical_blocks": same,
                       "levels": len(trace) - 1, "coarsest_n": trace[0][0],
                       "cut": int(cut), "cut_per_level": [int(c) for _, c in trace],
                       "max_block_weight": int(bw.max()), "bound": lmax,
                       "imbalance": round(float(bw.max()) * k / G.total_vwgt - 1.0, 5),
                       "refine_input_from_ip": ref}
        log(f"[partition] k={k}: {1e3 * dt:.0f} ms ({1e3 * dt_gt:.0f} ms with gain tables, identical {same}), "
            f"{len(trace) - 1} levels (coarsest n={trace[0][0]}), cut {cut} ({cut / (G.two_m // 2):.3f} of m), "
            f"max block {int(bw.max())} / bound {lmax}, refinement round {ref['graph']['round_ms']:.2f} ms "
            f"(rating {ref['graph']['rate_ms']:.2f}) | gain table {ref['gain_table']['round_ms']:.2f} ms "
            f"(selection {ref['gain_table']['rate_ms']:.2f}, accept + update {ref['gain_table']['accept_ms']:.2f}) "
            f"after {ref['gain_table']['setup_ms']:.1f} ms setup; "
            f"{slots} slots, {tbytes / 1e9:.2f} GB vs {G.nbytes / 1e9:.2f} GB compressed graph)")
    return out


def bench_quality(args) -> dict:
    """Coarsening quality of plain synchronous rounds (S = 1) and of S
    sub-rounds per round, on geometric graphs where synchronous moves stall:
    the 16k-vertex RGG-2D graph and RGG-3D with 2^20 vertices. Per setting:
    levels, final size and the cut of the composed clustering (half the edge
    weight left in the coarsest graph)."""
    import torch

    import paper_2410_19119_amd as lp
    import synth

    out = {}
    for name, g in (("rgg2d-16k", synth.rgg2d_16k()), ("rgg3d-2^20", synth.rgg3d(1 << 20, 27.0, seed=1))):
        G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
        two_m = g.two_m
        del g
        res = {}
        for S in (1, 2, 4):
            torch.cuda.synchronize()
            t = time.perf_counter()
            levels, final, n_target, _ = lp.coarsen(G, seed=1, rounds=args.rounds, subrounds=S)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            w = lp.lp_decompress(final)[2] if not final.compressed else None
            cut = int(w.to(torch.int64).sum()) // 2 if w is not None else two_m // 2
            res[str(S)] = {"levels": len(levels), "final_n": final.n, "n_target": n_target, "cut_of_hierarchy": cut,
                           "ms": round(1e3 * dt, 1)}
            for lv in levels[1:]:
                lv[0].free()
            if final is not G:
                final.free()
        out[name] = res
        G.free()
        log(f"[quality] {name}: " + "; ".join(f"S={k}: {v['levels']} levels, n={v['final_n']} "
                                              f"(target {v['n_target']}), cut {v['cut_of_hierarchy']}, {v['ms']} ms"
                                              for k, v in res.items()))
    return out


def bench_coarsen(args) -> dict:
    """Full coarsening of one large graph (cluster + contract until 2^14)."""
    import torch

    import paper_2410_19119_amd as lp
    import synth

    os.environ["SYNTH_PROGRESS"] = "1"  # the generator reports its phases on stderr
    t0 = time.time()
    sc = args.coarsen_scale
    if args.coarsen_graph == "rmat":
        g = synth.rmat_scale(sc, 32, seed=1)
        desc = f"rmat-s{sc}-ef32 (0.57,0.19,0.19,0.05), unit weights"
    else:
        g = synth.rgg3d(1 << sc, 27.0, seed=1)
        desc = f"rgg3d n=2^{sc} avg-deg~27, cell-ordered, unit weights"
    log(f"[coarsen] generated {desc}: n={g.n} 2m={g.two_m} in {time.time() - t0:.1f}s")
    t0 = time.time()
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
    torch.cuda.synchronize()
    n0, m0 = g.n, g.two_m
    del g
    log(f"[coarsen] compressed: {G.nbytes} bytes ({G.nbytes / max(m0, 1):.3f} B/edge) in {time.time() - t0:.1f}s")
    n_target, cap = lp.coarsen_params(G.n, G.total_vwgt)
    levels = []
    cur = G
    total_ms = 0.0
    lvl = 0
    checks = []
    while lvl < 32 and cur.n > n_target:
        torch.cuda.synchronize()
        t = time.perf_counter()
        lab, st = lp.lp_cluster(cur, cap, args.rounds, 1 + lvl, config=dict(timing=1, subrounds=args.coarsen_subrounds),
                                stats=True)
        torch.cuda.synchronize()
        t_lp = time.perf_counter() - t
        t = time.perf_counter()
        nxt, _ = lp.lp_contract(cur, lab, want_map=False)
        torch.cuda.synchronize()
        t_ct = time.perf_counter() - t
        total_ms += 1e3 * (t_lp + t_ct)
        rec = {"level": lvl, "n": cur.n, "two_m": cur.two_m, "compressed": cur.compressed,
               "rounds_run": st.rounds_run, "lp_ms": round(1e3 * t_lp, 2), "contract_ms": round(1e3 * t_ct, 2),
               "lp_round_edges_per_s": cur.two_m * st.rounds_run / (st.phase_ms["round"] / 1e3)
               if st.phase_ms["round"] > 0 else None, "coarse_n": nxt.n}
        levels.append(rec)
        log(f"[coarsen] level {lvl}: n={cur.n} 2m={cur.two_m} lp {rec['lp_ms']} ms "
            f"({rec['lp_round_edges_per_s'] or 0:.3e} edges/s/round) contract {rec['contract_ms']} ms -> n'={nxt.n}")
        if not args.no_checks:
            c = level_checks(lp, cur, lab, nxt, cap, G.total_vwgt)
            checks.append(c)
            log(f"[coarsen] level {lvl} checks: {c}")
        prev_n = cur.n
        if cur is not G:
            cur.free()
        cur = nxt
        lvl += 1
        if 100 * cur.n > 95 * prev_n:
            break
    return {"workload": desc, "subrounds": args.coarsen_subrounds, "n": n0, "two_m": m0, "compressed_bytes": G.nbytes,
            "n_target": n_target, "cap": cap,
            "levels": levels, "end_to_end_ms": total_ms, "final_n": cur.n, "checks": checks,
            "all_checks_pass": all(all(v for k, v in c.items() if k != "cut") for c in checks)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat26")
    ap.add_argument("--rounds", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-forms", action="store_true", help="skip the batched and served comparisons")
    ap.add_argument("--cpu-rounds", type=int, default=1, help="oracle rounds timed for the baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the R-MAT scale 24 round rate")
    ap.add_argument("--no-as-given", action="store_true",
                    help="skip the rounds rated on the graph as given (profiled runs keep one configuration)")
    ap.add_argument("--batch-graphs", type=int, default=512)
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--serve-pool", type=int, default=24)
    ap.add_argument("--serve-requests", type=int, default=0,
                    help="requests per rate (0: those arriving within --serve-window seconds, 100..2000)")
    ap.add_argument("--serve-window", type=float, default=3.0)
    ap.add_argument("--serve-rates", default=None,
                    help="comma-separated request rates (default: 10..1000 for --workload serve, "
                         "100,1000 inside the default run)")
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--subrounds", default="1,2,4", help="sub-round counts compared by the subrounds form")
    ap.add_argument("--serve-split", type=int, default=0,
                    help="directed edges from which a job runs in the big-job lane (0: one lane)")
    ap.add_argument("--partition-k", default="64", help="block counts of the partition form")
    ap.add_argument("--partition-graph", default="rmat", choices=["rmat", "rgg2d", "rgg3d"])
    ap.add_argument("--partition-subrounds", type=int, default=1,
                    help="sub-rounds per LP round in the partition's coarsening and refinement")
    ap.add_argument("--coarsen-graph", default="rmat", choices=["rmat", "rgg3d"])
    ap.add_argument("--coarsen-subrounds", type=int, default=1, help="sub-rounds per LP round in the coarsening")
    ap.add_argument("--coarsen-scale", type=int, default=26)
    ap.add_argument("--no-checks", action="store_true")
    ap.add_argument("--knobs", default=";hub_part=1024;hub_part=512;hub_part=4096;overlap=1",
                    help="semicolon-separated knob settings of the knobs form (k=v,k=v)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path exists as a "
              f"design only", file=sys.stderr)
        return 2

    import torch
    import paper_2410_19119_amd as lp

    torch.cuda.set_device(0)
    if args.workload == "batch512":
        res = bench_batch(args)
        print(json.dumps({"metric": "graphs/s batched vs plain", "value": res["batched_graphs_per_s"],
                          "unit": "graphs/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
                          "dtype": "int32", "config": {"workload": "batch of uneven RGG-2D / R-MAT graphs"},
                          "batched": res}))
        return 0
    if args.workload == "copy":
        # calibration for the HBM byte counters: a plain device copy of known size
        nbytes = 1 << 30
        a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "copy", "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                          "copies": 3}))
        return 0
    if args.workload == "knobs":
        # result-invariant knobs on the headline workload: phase times per setting
        import torch
        g, cap, desc = workload("rmat26")
        G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
        del g
        lab0 = None
        res = {}
        for spec in args.knobs.split(";"):
            cfg = dict(timing=1)
            for kv in filter(None, spec.split(",")):
                k, v = kv.split("=")
                cfg[k] = int(v)
            lab, _ = lp.lp_cluster(G, cap, args.rounds, 1, config=cfg, stats=True)
            rms, ph = [], {}
            for _ in range(2):
                lab, st = lp.lp_cluster(G, cap, args.rounds, 1, config=cfg, stats=True)
                rms += st.round_ms
                for p_ in ("lane", "tile", "block", "hub", "accept"):
                    ph[p_] = ph.get(p_, 0.0) + st.phase_ms[p_] / max(1, st.phase_launches[p_]) / 2
            same = True if lab0 is None else bool(torch.equal(lab, lab0))
            if lab0 is None:
                lab0 = lab.clone()
            res[spec or "default"] = {"round_ms_median": round(float(np.median(rms)), 3),
                                      "phases_ms": {k: round(v, 3) for k, v in ph.items()}, "identical_labels": same}
            log(f"[knobs] {spec or 'default'}: {res[spec or 'default']}")
        print(json.dumps({"workload": desc, "knobs": res}))
        return 0
    if args.workload == "intervals":
        print(json.dumps({"metric": "LP-round time and bytes per edge with interval encoding", "unit": "ms",
                          "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "int32",
                          "intervals": bench_intervals(args, args.coarsen_scale)}))
        return 0
    if args.workload == "gather":
        # calibration for the HBM byte counters on random 4-byte gathers:
        # 2^26 gathers at uniform random positions of an int32 array of 2^24
        # (64 MiB) and of 2^28 (1 GiB) elements; each launch also streams the
        # 8-byte indices in and the 4-byte results out
        cnt = 1 << 26
        gen = torch.Generator(device="cuda").manual_seed(3)
        res = {"workload": "gather", "gathers_per_launch": cnt, "index_bytes_read": 8 * cnt,
               "result_bytes_written": 4 * cnt, "sources": {}}
        for lg in (24, 28):
            src = torch.arange(1 << lg, dtype=torch.int32, device="cuda")
            idx = torch.randint(0, 1 << lg, (cnt,), device="cuda", dtype=torch.int64, generator=gen)
            out = torch.empty(cnt, dtype=torch.int32, device="cuda")
            ts = []
            for _ in range(3):
                a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a_.record()
                torch.take(src, idx, out=out)
                b_.record()
                torch.cuda.synchronize()
                ts.append(a_.elapsed_time(b_))
            assert torch.equal(out, idx.to(torch.int32))
            res["sources"][f"2^{lg}"] = {"source_bytes": 4 << lg, "ms": [round(t, 4) for t in ts]}
            del src, idx, out
        print(json.dumps(res))
        return 0
    if args.workload == "coarsen26":
        res = bench_coarsen(args)
        lv0 = res["levels"][0] if res["levels"] else {}
        print(json.dumps({"metric": "LP-round edges/s (level 0) and end-to-end coarsening time",
                          "value": lv0.get("lp_round_edges_per_s"), "unit": "edges/s", "n_gpus": 1,
                          "higher_is_better": True, "data": "synthetic", "dtype": "int32",
                          "config": {"workload": res["workload"]}, "coarsening": res}))
        return 0
    if args.workload == "quality":
        res = bench_quality(args)
        print(json.dumps({"metric": "cut of the coarsening hierarchy by sub-rounds per round",
                          "value": res["rgg3d-2^20"]["4"]["cut_of_hierarchy"], "unit": "edges",
                          "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "int32",
                          "config": {"workload": "rgg2d-16k and rgg3d n=2^20, 5 rounds per level"},
                          "quality": res}))
        return 0
    if args.workload == "subrounds":
        res = bench_subrounds(args)
        print(json.dumps({"metric": "cut of the coarsening hierarchy and LP round time, by sub-rounds per round",
                          "value": res[max(res, key=int)]["coarsening"]["cut_of_hierarchy"], "unit": "edges",
                          "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "int32",
                          "config": {"workload": "rmat-s24-ef16, cap 256, 5 rounds"}, "subrounds": res}))
        return 0
    if args.workload == "partition":
        res = bench_partition(args)
        top = res[max(res, key=int)]
        print(json.dumps({"metric": "multilevel k-way partition time and cut", "value": top["ms"], "unit": "ms",
                          "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "int32",
                          "config": {"workload": {"rgg2d": "rgg2d n=2^24 avg-deg~8, cell-ordered",
                                                  "rgg3d": "rgg3d n=2^26 avg-deg~27, cell-ordered"}.get(
                                                      args.partition_graph, "rmat-s24-ef16")
                                                 + ", eps 3 %, 5 rounds per level"},
                          "partition": res}))
        return 0
    if args.workload == "serve":
        res = bench_serve(args)
        top = res["rates"][max(res["rates"], key=float)]
        print(json.dumps({"metric": "coarsening jobs/s and p99 latency, served vs sequential",
                          "value": top["served"]["throughput_per_s"], "unit": "jobs/s", "n_gpus": 1,
                          "higher_is_better": True, "data": "synthetic", "dtype": "int32",
                          "config": {"workload": "Poisson stream of coarsening jobs on resident RGG-2D / R-MAT"},
                          "served": res}))
        return 0
    out = bench_headline(args)
    print(json.dumps(out))
    return 0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def median(xs):
    return float(np.median(xs)) if len(xs) else None


def round_model(g_n: int, two_m: int, nbytes: int, proposals: float, kappa: float = 2.0) -> int:
    """Algorithmic bytes of one LP round: compressed neighbourhoods, offsets,
    the 4-byte label gather per adjacency entry, 16 bytes per vertex (own
    label, vertex weight, label write, cluster weight write) and 20 bytes per
    proposal and pass through acceptance."""
    return int(nbytes + 8 * (g_n + 1) + 4 * two_m + 16 * g_n + 20 * proposals * kappa)


def dominant_phase(phase_ms: dict, hub_kernels: dict):
    """The rating phase whose single kernel takes the most time per round:
    lanes, small tiles or large tiles by their kernel's time, the hub path by
    the longest of its kernels (whole hubs, pieces, reduction), timed one by
    one. The hub path's algorithmic bytes are counted for the path as a whole,
    so when one of its kernels dominates, the phase reported is "hub".
    Acceptance is several small kernels and never the dominant one."""
    kernel_ms = {p: phase_ms[p] for p in ("lane", "tile", "block") if p in phase_ms}
    if "hub" in phase_ms:
        kernel_ms.update(hub_kernels)
    if not kernel_ms:
        return None
    dom = max(kernel_ms, key=kernel_ms.get)
    return "hub" if dom in hub_kernels else dom


def lp_rate(lp, G, cap: int, rounds: int, steps: int, warmup: int, labels=None) -> dict:
    """Median LP round time of `steps` clustering calls (after `warmup`)."""
    import torch
    cfg = dict(timing=1)
    for _ in range(warmup):
        lp.lp_cluster(G, cap, rounds, 1, labels=labels, config=cfg)
    torch.cuda.synchronize()
    rms = []
    ph, nl = {}, {}
    for _ in range(steps):
        _, st = lp.lp_cluster(G, cap, rounds, 1, labels=labels, config=cfg, stats=True)
        rms += st.round_ms
        for p in ("lane", "tile", "block", "hub", "accept"):
            ph[p] = ph.get(p, 0.0) + st.phase_ms[p]
            nl[p] = nl.get(p, 0) + st.phase_launches[p]
    med = median(rms)
    return {"round_ms_median": round(med, 4), "lp_round_edges_per_s": G.two_m / (med / 1e3),
            "rounds_timed": len(rms),
            "phase_ms_per_round": {p: round(ph[p] / nl[p], 4) for p in ph if nl[p]}}


def bench_intervals(args, scale: int = 26) -> dict:
    """Interval encoding on the geometric graph of the large coarsening
    workload (RGG-3D, 2^26 vertices, average degree 27, cell-ordered IDs):
    compressed bytes per edge with gap encoding alone and with intervals, and
    the median LP round time of level 0 (cap 12288, 5 rounds, seed 1) on
    each; the two must give the same labels."""
    import torch

    import paper_2410_19119_amd as lp
    import synth

    t0 = time.time()
    g = synth.rgg3d(1 << scale, 27.0, seed=1)
    log(f"[intervals] generated rgg3d n=2^{scale}: 2m={g.two_m} in {time.time() - t0:.1f}s")
    out = {"workload": f"rgg3d n=2^{scale} avg-deg~27, cell-ordered, cap 12288, 5 rounds, seed 1", "two_m": g.two_m}
    labs = {}
    for name, itv in (("gap", False), ("intervals", True)):
        G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy, intervals=itv)
        lab = torch.empty(G.n, dtype=torch.int32, device="cuda")
        r = lp_rate(lp, G, 12288, args.rounds, 3, 1, labels=lab)
        labs[name] = lab
        r.update({"bytes": G.nbytes, "bytes_per_edge": round(G.nbytes / g.two_m, 4)})
        out[name] = r
        log(f"[intervals] {name}: {G.nbytes} bytes ({G.nbytes / g.two_m:.3f} B/edge), round {r['round_ms_median']} ms")
        G.free()
    out["identical_labels"] = bool(torch.equal(labs["gap"], labs["intervals"]))
    out["bytes_ratio"] = round(out["intervals"]["bytes"] / out["gap"]["bytes"], 4)
    return out


def bench_headline(args) -> dict:
    import torch
    import paper_2410_19119_amd as lp

    t0 = time.time()
    g, cap, desc = workload(args.workload)
    log(f"[bench] generated {desc}: n={g.n} 2m={g.two_m} in {time.time() - t0:.1f}s")
    t0 = time.time()
    G = lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy)
    torch.cuda.synchronize()
    log(f"[bench] compressed on GPU: {G.nbytes} bytes ({G.nbytes / max(g.two_m, 1):.3f} B/edge) "
        f"in {time.time() - t0:.1f}s")
    n, two_m = g.n, g.two_m
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    cfg = dict(timing=1)

    split = {"cluster": 0.0, "contract": 0.0, "cut": 0.0}

    def step():
        # each call synchronises its stream before returning (statistics,
        # coarse size, cut), so host clocks split the step between them
        t = time.perf_counter()
        lab, st = lp.lp_cluster(G, cap, args.rounds, 1, labels=labels, config=cfg, stats=True)
        t1 = time.perf_counter()
        C, _ = lp.lp_contract(G, lab, want_map=False)
        t2 = time.perf_counter()
        cut = lp.lp_edge_cut(G, lab)
        t3 = time.perf_counter()
        split["cluster"] += t1 - t
        split["contract"] += t2 - t1
        split["cut"] += t3 - t2
        n_coarse = C.n
        C.free()
        return st, cut, n_coarse

    # the first call on the handle builds the plans; a call with the copy
    # forced (zero rounds) builds the degree-ordered copy, which later calls
    # use automatically on a skewed graph of at least 2^20 vertices
    torch.cuda.synchronize()
    t = time.perf_counter()
    lp.lp_cluster(G, cap, 0, 1, labels=labels)
    torch.cuda.synchronize()
    first_call_ms = 1e3 * (time.perf_counter() - t)
    t = time.perf_counter()
    lp.lp_cluster(G, cap, 0, 1, labels=labels, config=dict(reorder=1))
    torch.cuda.synchronize()
    copy_build_ms = 1e3 * (time.perf_counter() - t)
    log(f"[bench] first call (plans) {first_call_ms:.1f} ms, degree-ordered copy {copy_build_ms:.1f} ms")
    for i in range(args.warmup):
        step()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    for k in split:
        split[k] = 0.0
    times, stats = [], []
    for i in range(args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, cut, n_coarse = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        stats.append(st)
        log(f"[bench] step {i + 1}/{args.steps}: {times[-1] * 1e3:.2f} ms, rounds {st.rounds_run}, "
            f"round ms {[round(v, 2) for v in st.round_ms]}, coarse n {n_coarse}, cut {cut}")
    total = sum(times)
    ms_per_step = 1e3 * total / args.steps
    st = stats[-1]
    rounds_run = st.rounds_run
    all_rounds = [v for s_ in stats for v in s_.round_ms]
    t_round = median(all_rounds)
    value = two_m / (t_round / 1e3)
    step_rate = two_m * rounds_run * args.steps / total

    # per-phase times: the rating paths run one after another on the call's
    # stream, so each phase's events time exactly its own kernels
    round_phases = ("lane", "tile", "block", "hub", "accept")
    nb = st.buckets
    props = float(np.mean([np.mean(s_.proposals) for s_ in stats if s_.proposals])) if st.proposals else 0.0
    phases = {}
    for p in round_phases:
        launches = sum(s_.phase_launches[p] for s_ in stats)
        if not launches:
            continue
        avg_ms = sum(s_.phase_ms[p] for s_ in stats) / launches
        b = phase_bytes(st, p, nb, props)
        phases[p] = {"kernel": PHASE_KERNEL[p], "launches_per_step": launches // args.steps,
                     "avg_ms": round(avg_ms, 4), "alg_bytes": int(b),
                     "alg_GBs": round(b / (avg_ms / 1e3) / 1e9, 1) if avg_ms > 0 else None,
                     "frac_hbm": round(b / (avg_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if avg_ms > 0 else None}
    hub_kernels = {}
    for p in ("hub_whole", "hub_pieces", "hub_reduce"):
        launches = sum(s_.phase_launches[p] for s_ in stats)
        if launches:
            hub_kernels[p] = round(sum(s_.phase_ms[p] for s_ in stats) / launches, 4)
    if "hub" in phases:
        phases["hub"]["kernels_avg_ms"] = hub_kernels
    dom = dominant_phase({p: phases[p]["avg_ms"] for p in phases}, hub_kernels)
    roofline = None
    if dom:
        ach = phases[dom]["alg_GBs"]
        tr = measured_traffic(TRAFFIC_FILE, f"{dom}_bytes_per_launch") if args.workload == "rmat26" else None
        roofline = {"bound": "hbm", "kernel": phases[dom]["kernel"], "achieved": ach, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": tr,
                    "alg_bytes_per_launch": phases[dom]["alg_bytes"], "avg_launch_ms": phases[dom]["avg_ms"]}
    a_round = round_model(n, two_m, G.nbytes, props)
    round_traffic = measured_traffic(ROUND_TRAFFIC_FILE, "round_bytes") if args.workload == "rmat26" else None

    # the same rounds rated on the graph as given (no degree-ordered copy)
    t_round_asis = None
    if not args.no_as_given:
        asis = []
        for _ in range(2):
            _, st_a = lp.lp_cluster(G, cap, args.rounds, 1, labels=labels, config=dict(timing=1, reorder=2),
                                    stats=True)
            asis += st_a.round_ms
        t_round_asis = median(asis)
        log(f"[bench] rounds on the graph as given: median {t_round_asis:.2f} ms")

    # a1 uncached: the same call with a plan built for it (non-default
    # thresholds that bucket every vertex as the defaults do, except tiles
    # of 4095 instead of 4096 edges), zero rounds
    _, st0 = lp.lp_cluster(G, cap, 0, 1, labels=labels, config=dict(timing=1, t_block=4095), stats=True)
    _, st0 = lp.lp_cluster(G, cap, 0, 1, labels=labels, config=dict(timing=1, t_block=4095), stats=True)
    setup_uncached = st0.phase_ms["setup"]

    cpu = None
    if not args.no_cpu:
        import oracle
        threads = os.cpu_count() or 1
        oracle.set_threads(threads)
        t = time.perf_counter()
        _, ost = oracle.lp_cluster(g, cap, args.cpu_rounds, 1)
        dt = time.perf_counter() - t
        done = ost.rounds_run
        cpu = {"value": two_m * done / dt, "unit": "edges/s", "cores": threads, "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"oracle lp_cluster on the full graph, first {done} round(s) ({dt:.1f} s wall, "
                         f"rating + acceptance + apply, no contraction), {threads} threads"}
        log(f"[bench] cpu oracle: {done} round(s) in {dt:.1f}s with {threads} threads")
        # the small workload (RGG-2D, n = 16384, cap 32, 5 rounds) on one thread and on all
        import synth
        g0 = synth.rgg2d_16k(seed=1)
        small = {}
        for th in (1, threads):
            oracle.set_threads(th)
            reps, t = 0, time.perf_counter()
            while reps < 3 or time.perf_counter() - t < 1.0:
                _, o0 = oracle.lp_cluster(g0, 32, 5, 1)
                reps += 1
            dt0 = (time.perf_counter() - t) / reps
            small[str(th)] = g0.two_m * o0.rounds_run / dt0
        oracle.set_threads(threads)
        cpu["small_workload_edges_per_s_by_threads"] = small
    del g

    extra = {}
    if not args.no_extra and args.workload == "rmat26":
        import synth
        t0 = time.time()
        g1 = synth.rmat_scale(24, 16, seed=1)
        G1 = lp.lp_compress(g1.n, g1.xadj.view(np.int64), g1.adjncy)
        del g1
        lab1 = torch.empty(G1.n, dtype=torch.int32, device="cuda")
        r1 = lp_rate(lp, G1, 256, args.rounds, 3, 1, labels=lab1)
        r1.update({"workload": "rmat-s24-ef16, cap 256, 5 rounds, seed 1", "two_m": G1.two_m})
        extra["rmat24"] = r1
        G1.free()
        log(f"[bench] rmat24: round {r1['round_ms_median']} ms ({r1['lp_round_edges_per_s']:.3e} edges/s) "
            f"in {time.time() - t0:.1f}s")

    if not args.no_extra and args.workload == "rmat26":
        extra["rgg3d26_intervals"] = bench_intervals(args)

    forms = {}
    if not args.no_forms:
        b = bench_batch(args)
        forms["batched"] = {k: b[k] for k in ("graphs", "two_m", "plain_graphs_per_s", "batched_graphs_per_s",
                                              "autotuned_graphs_per_s", "speedup_vs_plain", "identical_labels")}
        forms["served"] = bench_serve(args)

    out = {
        "metric": "LP-round edges/s",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "two_m": two_m, "compressed_bytes": G.nbytes,
                   "max_cluster_weight": cap, "rounds": args.rounds, "rounds_run": rounds_run, "seed": 1,
                   "step": "lp_cluster + lp_contract + lp_edge_cut"},
        "t_round_ms_median": round(t_round, 4),
        "round_ms_all": [round(v, 3) for v in all_rounds],
        "step_edges_per_s": step_rate,
        "round_model": {"alg_bytes": a_round, "ms": round(t_round, 4),
                        "frac_hbm": round(a_round / (t_round / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                        "proposals_per_round": props, "kappa": 2,
                        "traffic": round_traffic,
                        "traffic_over_alg": round(round_traffic / a_round, 2) if round_traffic else None},
        "phases": phases,
        "setup_ms_cached": round(st.phase_ms["setup"], 3),
        "setup_ms_uncached": round(setup_uncached, 3),
        "first_call_ms": round(first_call_ms, 1),
        "copy_build_ms": round(copy_build_ms, 1),
        "t_round_ms_median_graph_as_given": round(t_round_asis, 4) if t_round_asis else None,
        "step_split_ms": {k: round(1e3 * v / args.steps, 2) for k, v in split.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    out.update(forms)
    G.free()
    return out


if __name__ == "__main__":
    sys.exit(main())
