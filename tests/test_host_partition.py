"""Host arithmetic of the device partition driver (no GPU): the balance
bound, the coarsening cap before a k-way partition and the coarsening
parameters must equal the oracle's, or the same partition cannot come out."""
import numpy as np


def test_partition_bounds_match_the_oracle(oracle_mod):
    import paper_2410_19119_amd as lp
    rng = np.random.default_rng(3)
    for _ in range(500):
        total = int(rng.integers(1, 1 << 40))
        n0 = int(rng.integers(1, 1 << 31))
        k = int(rng.integers(1, 1 << 16))
        eps = int(rng.integers(0, 200))
        assert lp.max_block_weight(total, k, eps) == oracle_mod.max_block_weight(total, k, eps)
        assert lp.partition_cap(n0, total, k, eps) == oracle_mod.partition_cap(n0, total, k, eps)
        assert lp.coarsen_params(n0, total) == oracle_mod.coarsen_params(n0, total)
