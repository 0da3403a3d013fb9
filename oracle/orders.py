"""Visiting-order spread of the sequential oracle (test infrastructure, like
the rest of this package: used by the tests and by the benchmark's quality
report, never by the GPU library).

The paper leaves the order in which the asynchronous local-moving phase
visits vertices open: the multicore and GPU designs process vertices
concurrently, in no fixed order.  The sequential oracle visits them in
ascending id, so every relabelling of a graph's vertices is an equally valid
sequential run of the method.  On graphs with weak community structure these
runs end in local optima whose modularity differs by more than 0.002, so the
ASYNC bound is taken against the lowest modularity the oracle reaches over
the identity order and a fixed set of seeded relabellings.

relabel() only permutes vertex ids (no Louvain arithmetic); the runs
themselves are the oracle's.
"""
from __future__ import annotations

import numpy as np

import graphgen as gg

from . import louvain, modularity

ORDERS = 8      # seeded relabellings besides the identity order
ORDER_SEED = 100


def relabel(g, perm):
    """Graph with vertex v renamed perm[v] (rows sorted by neighbour id)."""
    perm = np.asarray(perm, dtype=np.int64)
    n = g.n
    deg = np.diff(np.asarray(g.offsets, dtype=np.int64))
    src = perm[np.repeat(np.arange(n, dtype=np.int64), deg)]
    dst = perm[np.asarray(g.indices, dtype=np.int64)]
    order = np.lexsort((dst, src))
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(np.bincount(src, minlength=n))
    return gg.CSRGraph(n, off, dst[order].astype(np.int32), np.asarray(g.weights, dtype=np.int64)[order],
                       g.name + "-relabelled")


def oracle_q_orders(g, orders: int = ORDERS, seed: int = ORDER_SEED, params=None):
    """Modularity the sequential oracle reaches on g in the identity order and
    in `orders` seeded relabellings (each evaluated on its own graph; Q is
    invariant under relabelling)."""
    g = gg.CSRGraph(g.n, g.offsets, g.indices, np.asarray(g.weights, dtype=np.int64), g.name)
    qs = [modularity(g, louvain(g, params).membership)]
    for r in range(orders):
        gp = relabel(g, np.random.default_rng(seed + r).permutation(g.n))
        qs.append(modularity(gp, louvain(gp, params).membership))
    return qs


def async_floor(g, bound: float = 0.002, **kw) -> float:
    """Lowest modularity an ASYNC run may reach: min over orders minus bound."""
    return min(oracle_q_orders(g, **kw)) - bound
