"""Serving form: every job's levels must be the same alone (coarsen) and in the
continuous-batching mix, whatever the admission order, slots and budget."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _pool(lp, synth_mod):
    recipe = [("rgg2d", 3000, 8, 11), ("rmat", 2000, 12, 12), ("rmat", 9000, 9, 13), ("rgg2d", 20000, 8, 14),
              ("rmat", 600, 16, 15), ("rgg2d", 700, 8, 16)]
    gs = [synth_mod.batch_graph(*r) for r in recipe]
    return gs, [lp.lp_compress(g.n, g.xadj.view(np.int64), g.adjncy) for g in gs]


@pytest.mark.parametrize("slots,budget,split", [(64, 200 * 10**9, 1 << 22), (3, 200 * 10**9, 1 << 22),
                                                (64, 1, 1 << 22), (64, 200 * 10**9, 60000),
                                                (2, 200 * 10**9, 60000), (64, 1, 60000), (64, 200 * 10**9, 0)])
def test_served_results_equal_alone(lp, synth_mod, slots, budget, split):
    from paper_2410_19119_amd import serve

    gs, pool = _pool(lp, synth_mod)
    if 0 < split < 1 << 22:  # both lanes get jobs
        assert min(g.two_m for g in pool) < split <= max(g.two_m for g in pool)
    reqs = serve.requests(synth_mod.serve_trace(2000.0, 25, len(pool), seed=3))
    srv = serve.Server(pool, budget_bytes=budget, max_active=slots, keep_labels=True, split_edges=split)
    res = srv.run(reqs)
    assert [r.rid for r in res] == list(range(len(reqs)))
    if slots > 3 and budget > 1:
        assert srv.peak_active > 1  # jobs really shared steps
    if budget == 1:
        assert srv.peak_active == 1  # the budget holds across lanes: one job at a time
    # admitted estimates stay within the budget, except a job admitted alone
    assert srv.peak_used <= max(srv.budget, max(serve.job_bytes(g) for g in pool))
    for r, q in zip(res, reqs):
        levels, final, _, _ = lp.coarsen(pool[q.graph], seed=q.seed)
        assert len(r.labels) == len(levels) and r.final_n == final.n, q.rid
        for lab, lv in zip(r.labels, levels):
            assert np.array_equal(lab.cpu().numpy(), lv[1].cpu().numpy()), q.rid
        assert r.done >= r.arrival


def test_sequential_baseline_and_summary(lp, synth_mod):
    from paper_2410_19119_amd import serve

    _, pool = _pool(lp, synth_mod)
    reqs = serve.requests(synth_mod.serve_trace(500.0, 8, len(pool), seed=4))
    seq = serve.run_sequential(pool, reqs)
    srv = serve.Server(pool).run(reqs)
    assert [r.final_n for r in seq] == [r.final_n for r in srv]
    assert [r.levels for r in seq] == [r.levels for r in srv]
    s = serve.summarize(seq)
    assert s["requests"] == len(reqs) and s["p99_ms"] >= s["p50_ms"] > 0
