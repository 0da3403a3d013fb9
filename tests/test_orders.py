"""CPU checks of the visiting-order reading of the ASYNC bound (oracle/orders.py).

relabel() must be a pure renaming: modularity of a partition, the total
weight and the degree multiset are unchanged, and renaming back restores the
graph.  The sequential oracle's result does depend on the order: on the SBM
graphs below (drawn as the batched workload draws them) its modularity moves
by far more than 0.002 between relabellings, which is why the per-graph ASYNC
bound is taken against the lowest modularity over the orders.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle.orders import oracle_q_orders, relabel


@pytest.mark.parametrize("make", [lambda: gg.rmat(9, 8, seed=2), lambda: gg.random_small(40, 0.2, 5, self_loops=True),
                                  lambda: gg.sbm_degree(500, 8, 12.0, seed=3, wmin=1, wmax=4)])
def test_relabel_is_a_renaming(make):
    g = make()
    g.weights = g.weights.astype(np.int64)
    perm = np.random.default_rng(1).permutation(g.n)
    gp = relabel(g, perm)
    assert gp.total_weight == g.total_weight
    assert np.array_equal(np.sort(gp.degrees()), np.sort(g.degrees()))
    memb = oracle.louvain(g).membership
    # the same partition, renamed, has the same exact modularity
    memb_p = np.empty_like(memb)
    memb_p[perm] = memb
    assert oracle.modularity_parts(gp, memb_p) == oracle.modularity_parts(g, memb)
    back = relabel(gp, np.argsort(perm))
    assert np.array_equal(back.offsets, g.offsets) and np.array_equal(back.indices, g.indices)
    assert np.array_equal(back.weights, g.weights)


def test_identity_order_is_the_oracle():
    g = gg.planted_partition(seed=1)
    qs = oracle_q_orders(g, orders=2)
    g.weights = g.weights.astype(np.int64)
    assert qs[0] == oracle.modularity(g, oracle.louvain(g).membership)


# Graphs 16 and 23 of the batched SBM workload (vertex counts log-uniform in
# [200, 20000], default_rng(4) draws, graph k seeded 4000 + k).
@pytest.mark.parametrize("n,k,deg,seed", [(4854, 14, 12.6, 4016), (17616, 26, 18.3, 4023)])
def test_oracle_order_spread_exceeds_the_bound_on_weak_sbm(n, k, deg, seed):
    rng = np.random.default_rng(4)
    params = []
    for _ in range(seed - 4000 + 1):
        nn = int(np.exp(rng.uniform(np.log(200), np.log(20000))))
        params.append((nn, int(rng.integers(4, 65)), float(rng.uniform(8, 32))))
    nn, kk, dd = params[-1]
    assert (nn, kk, round(dd, 1)) == (n, k, deg)
    g = gg.sbm_degree(nn, kk, dd, seed=seed, wmin=1, wmax=4)
    qs = oracle_q_orders(g)
    assert max(qs) - min(qs) > 0.02
