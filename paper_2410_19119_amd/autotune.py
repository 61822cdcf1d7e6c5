"""Autotuner for the result-invariant knobs of lp_cluster / lp_batch_cluster_ex
(degree-bucket thresholds t_lane, t_tile, t_block and the hub partition size).

Every valid setting gives identical labels, so the tuner only measures: it runs
the first `rounds` rounds of the clustering with per-phase event timing for
each candidate setting and keeps the fastest. Candidates are a small grid
around the defaults; the measured times come from HIP events on the call's
stream (phase_ms of the statistics)."""
from __future__ import annotations

import itertools

DEFAULT = dict(t_lane=16, t_tile=2048, t_block=4096, hub_part=2048)

GRID = dict(
    t_lane=(8, 16),
    t_tile=(512, 2048),
    t_block=(2048, 4096),
    hub_part=(1024, 2048, 4096),
)


def candidates(grid: dict = GRID):
    keys = list(grid)
    for vals in itertools.product(*(grid[k] for k in keys)):
        c = dict(zip(keys, vals))
        if c["t_lane"] <= c["t_tile"] <= c["t_block"]:
            yield c


def _round_ms(stats) -> float:
    return stats.phase_ms.get("round", 0.0) + stats.phase_ms.get("setup", 0.0)


def tune(run, grid: dict = GRID, repeats: int = 2):
    """run(config) -> ClusterStats (with timing). Returns (best config, table of
    (config, ms)) where ms is the best of `repeats` timed runs."""
    table = []
    for c in candidates(grid):
        cfg = dict(c, timing=1)
        best = min(_round_ms(run(cfg)) for _ in range(repeats))
        table.append((c, best))
    table.sort(key=lambda t: t[1])
    return table[0][0], table


def tune_cluster(lp, g, cap: int, seed: int = 1, rounds: int = 1, grid: dict = GRID):
    """Tune lp_cluster on one graph."""
    def run(cfg):
        _, st = lp.lp_cluster(g, cap, rounds, seed, config=cfg, stats=True)
        return st
    return tune(run, grid)


def tune_batch(lp, b, caps, seeds, rounds: int = 1, grid: dict = GRID):
    """Tune lp_batch_cluster_ex on a batch handle."""
    def run(cfg):
        _, st = lp.lp_batch_cluster_ex(b, caps, rounds, seeds, config=cfg, stats=True)
        return st
    return tune(run, grid)
