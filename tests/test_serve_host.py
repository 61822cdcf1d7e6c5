"""Host-side pieces of the serving form (no GPU): arrival traces and the
latency summary."""
import math

import pytest


def test_trace_is_poisson_like_and_seeded(synth_mod):
    tr = synth_mod.serve_trace(100.0, 4000, 24, seed=7)
    assert tr == synth_mod.serve_trace(100.0, 4000, 24, seed=7)
    t = [a for a, _, _ in tr]
    assert all(b > a for a, b in zip(t, t[1:]))
    gaps = [b - a for a, b in zip([0.0] + t, t)]
    mean = sum(gaps) / len(gaps)
    assert abs(mean - 0.01) < 0.001  # rate 100 / s
    # exponential gaps: P(gap > mean) = 1/e
    frac = sum(g > mean for g in gaps) / len(gaps)
    assert abs(frac - math.exp(-1)) < 0.03
    assert {gi for _, gi, _ in tr} == set(range(24))


def test_pool_sizes_span_the_range(synth_mod):
    pool = synth_mod.serve_pool(200)
    m2 = [n * (8 if k == "rgg2d" else 2 * p) for k, n, p, _ in pool]
    assert min(m2) < 3e4 and max(m2) > 3e7
    assert all(5e3 < x < 1.2e8 for x in m2)


def test_summary_percentiles():
    pytest.importorskip("torch")
    from paper_2410_19119_amd.serve import Result, summarize

    rs = [Result(i, 0.0, 0.0, (i + 1) / 1000.0) for i in range(100)]
    s = summarize(rs)
    assert s["requests"] == 100
    assert s["p50_ms"] == pytest.approx(50.0)
    assert s["p99_ms"] == pytest.approx(99.0)
    assert s["throughput_per_s"] == pytest.approx(1000.0)
