"""The multicore CPU baseline (cpu_baseline/, OpenMP, GVE-Louvain style):
a timing baseline, checked here for validity and quality, never equality.

Its membership must be a partition of the vertices whose exact modularity is
at least the lowest the sequential oracle reaches over visiting orders minus
0.002 (the concurrent order changes the local optimum reached, as for the GPU
runs); on a ring of cliques below the resolution limit it must return exactly
the cliques, as the oracle does; any thread count works.
"""
import numpy as np
import pytest

import cpu_baseline
import graphgen as gg
import oracle
from oracle.orders import async_floor


def q_of(g, memb):
    g.weights = np.asarray(g.weights, dtype=np.int64)
    return oracle.modularity(g, memb)


@pytest.mark.parametrize("threads", [1, 4])
@pytest.mark.parametrize("make", [lambda: gg.planted_partition(seed=1), lambda: gg.rmat(14, 16, seed=3),
                                  lambda: gg.sbm_degree(5000, 8, 24.0, seed=5, wmin=1, wmax=4),
                                  lambda: gg.grid(64, 64, seed=7)], ids=["planted", "rmat14", "sbm", "grid"])
def test_valid_partition_near_oracle_quality(make, threads):
    g = make()
    memb, st = cpu_baseline.louvain(g, threads=threads)
    assert memb.shape == (g.n,) and memb.min() >= 0 and memb.max() < g.n
    assert st["passes"] >= 1 and st["iterations"] >= st["passes"]
    assert q_of(g, memb) >= async_floor(g)


def test_ring_of_cliques_recovered():
    r, k = 12, 5
    g = gg.ring_of_cliques(r, k)
    memb, _ = cpu_baseline.louvain(g, threads=4)
    blocks = [set(memb[c * k:(c + 1) * k].tolist()) for c in range(r)]
    assert all(len(b) == 1 for b in blocks)
    assert len(set.union(*blocks)) == r


def test_later_start_tolerance_is_used():
    """A run continued after p passes starts at tau = 0.01 / 10^p: with a far
    smaller tolerance the local-moving phase cannot stop earlier."""
    g = gg.sbm_degree(4000, 16, 10.0, seed=9, wmin=1, wmax=4)
    _, st0 = cpu_baseline.louvain(g, threads=1, max_passes=1)
    _, st3 = cpu_baseline.louvain(g, threads=1, max_passes=1, tol_den=100 * 10 ** 3)
    assert st3["iterations"] >= st0["iterations"]
