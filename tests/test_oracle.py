"""Pins for the CPU oracle: each test checks it against something other than
itself -- brute force over all partitions, a different formula for the same
quantity, closed forms, a library routine, invariants or a hand trace."""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import graphgen as gg
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ helpers (independent)

def dense_adjacency(g):
    """Dense arc-weight matrix A (A[i][i] = self-loop weight, stored once)."""
    A = np.zeros((g.n, g.n), dtype=object)
    for i in range(g.n):
        for e in range(g.offsets[i], g.offsets[i + 1]):
            A[i, g.indices[e]] += int(g.weights[e])
    return A


def q_pairwise(A, memb):
    """Modularity as the pairwise double sum (1/W) sum_ij [A_ij - K_i K_j / W] delta(c_i, c_j)."""
    n = A.shape[0]
    K = [sum(int(A[i, j]) for j in range(n)) for i in range(n)]
    W = sum(K)
    if W == 0:
        return Fraction(0)
    s = Fraction(0)
    for i in range(n):
        for j in range(n):
            if memb[i] == memb[j]:
                s += Fraction(int(A[i, j])) - Fraction(K[i] * K[j], W)
    return s / W


def set_partitions(n):
    """All set partitions of range(n) as restricted-growth label arrays."""
    out = []

    def rec(prefix, mx):
        if len(prefix) == n:
            out.append(list(prefix))
            return
        for c in range(mx + 2):
            prefix.append(c)
            rec(prefix, max(mx, c))
            prefix.pop()

    if n == 0:
        return [[]]
    rec([0], 0)
    return out


def max_q_bruteforce(g):
    """max over every set partition of Q * W^2 (vectorised integer arithmetic)."""
    A = dense_adjacency(g).astype(np.int64)
    K = A.sum(axis=1)
    W = int(K.sum())
    L = np.array(set_partitions(g.n), dtype=np.int8)
    same = L[:, :, None] == L[:, None, :]
    intra = (same * A[None]).sum(axis=(1, 2))
    kk = (same * np.outer(K, K)[None]).sum(axis=(1, 2))
    vals = W * intra - kk
    best = int(vals.max())
    return Fraction(best, W * W), L[int(vals.argmax())]


def loose_params(**kw):
    """Run to a fixed point: no tolerance, unbounded passes, no shrink test."""
    base = dict(max_iterations=1000, max_passes=0, tol_num=0, tol_den=1, agg_num=1, agg_den=1)
    base.update(kw)
    return oracle.Params(**base)


SMALL = [gg.random_small(n, p, seed, wmax=4, self_loops=sl)
         for n, p, seed, sl in [(6, 0.5, 1, False), (7, 0.4, 2, True), (8, 0.35, 3, True), (9, 0.3, 4, False),
                                (10, 0.3, 5, True), (8, 0.6, 6, False)]]


# ------------------------------------------------------------------- Eq. (1)

@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_modularity_matches_pairwise_definition(g):
    A = dense_adjacency(g)
    rng = np.random.default_rng(11)
    for _ in range(5):
        memb = rng.integers(0, max(1, g.n // 2), size=g.n).astype(np.int32)
        assert oracle.modularity_exact(g, memb) == q_pairwise(A, memb)


def test_modularity_matches_networkx():
    nx = pytest.importorskip("networkx")
    g = gg.planted_partition(seed=3)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    for i in range(g.n):
        for e in range(g.offsets[i], g.offsets[i + 1]):
            j = int(g.indices[e])
            if i < j:
                G.add_edge(i, j, weight=int(g.weights[e]))
    for memb in (g.labels, np.arange(g.n) % 7, np.zeros(g.n, dtype=np.int32)):
        comms = [set(np.flatnonzero(memb == c).tolist()) for c in np.unique(memb)]
        ref = nx.community.modularity(G, comms, weight="weight")
        assert abs(oracle.modularity(g, memb) - ref) < 1e-12


@pytest.mark.parametrize("c,k", [(2, 3), (3, 4), (5, 5), (8, 3)])
def test_modularity_disjoint_cliques_closed_form(c, k):
    edges = [(t * k + x, t * k + y, 1) for t in range(c) for x in range(k) for y in range(x + 1, k)]
    g = gg.from_edges(c * k, edges)
    memb = np.repeat(np.arange(c), k)
    assert oracle.modularity_exact(g, memb) == 1 - Fraction(1, c)
    assert oracle.modularity_exact(g, np.zeros(c * k, dtype=np.int32)) == 0


def test_modularity_empty_graph_is_zero():
    g = gg.from_edges(4, [])
    assert oracle.modularity_exact(g, np.arange(4)) == 0


# ------------------------------------------------------------------- Eq. (2)

@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_integer_gain_equals_modularity_difference(g):
    """gain * 2 / W^2 == Q(after) - Q(before) for every vertex and every target."""
    A = dense_adjacency(g)
    W = g.total_weight
    rng = np.random.default_rng(5)
    memb = rng.integers(0, 4, size=g.n).astype(np.int32)
    q0 = q_pairwise(A, memb)
    for i in range(g.n):
        for d in range(4):
            if d == memb[i]:
                continue
            after = memb.copy()
            after[i] = d
            assert Fraction(2 * oracle.gain(g, memb, i, d), W * W) == q_pairwise(A, after) - q0


# ------------------------------------------------------------ local moving

@pytest.mark.parametrize("g", SMALL + [gg.ring_of_cliques(3, 3)], ids=lambda g: g.name)
@pytest.mark.parametrize("mode", [oracle.ASYNC, oracle.SYNC])
def test_louvain_bounded_by_bruteforce_max(g, mode):
    r = oracle.louvain(g, loose_params(mode=mode))
    best, _ = max_q_bruteforce(g)
    assert oracle.modularity_exact(g, r.membership) <= best


@pytest.mark.parametrize("edges,n", [
    # two triangles joined by one bridge
    ([(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (2, 3)], 6),
    # two K4 joined by one bridge
    ([(a, b) for a in range(4) for b in range(a + 1, 4)] + [(a + 4, b + 4) for a in range(4) for b in range(a + 1, 4)]
     + [(0, 4)], 8),
    # three triangles in a ring
    ([(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (6, 7), (7, 8), (6, 8), (2, 3), (5, 6), (8, 0)], 9),
])
def test_louvain_reaches_bruteforce_optimum_on_bridged_cliques(edges, n):
    g = gg.from_edges(n, [(a, b, 1) for a, b in edges])
    best, _ = max_q_bruteforce(g)
    r = oracle.louvain(g, loose_params(mode=oracle.ASYNC))
    assert oracle.modularity_exact(g, r.membership) == best


def _final_level(g, r):
    """Graph and C' of the last local-moving phase from a trace."""
    level = g if not r.graphs else gg.CSRGraph(r.graphs[-1]["n"], r.graphs[-1]["offsets"],
                                               r.graphs[-1]["indices"], r.graphs[-1]["weights"])
    last_pass = r.iters[-1]["pass_"]
    return level, r.iters[-1]["cprime"], last_pass


@pytest.mark.parametrize("g", SMALL + [gg.planted_partition(seed=2), gg.erdos(60, 0.1, seed=3)],
                         ids=lambda g: g.name)
def test_async_without_pruning_ends_locally_optimal(g):
    """With tau = 0 and no pruning the last local-moving phase ends only when a
    full sweep finds no move: no single vertex move may gain (brute force on
    the final level via Q differences)."""
    r = oracle.louvain(g, loose_params(mode=oracle.ASYNC, prune=0), trace=True)
    level, cp, _ = _final_level(g, r)
    assert r.iters[-1]["moves"] == 0
    q0 = oracle.modularity_exact(level, cp)
    comms = np.unique(cp)
    for i in range(level.n):
        nbr = {int(cp[level.indices[e]]) for e in range(level.offsets[i], level.offsets[i + 1])
               if level.indices[e] != i}
        for d in nbr | set(comms[:3].tolist()):
            if d == cp[i]:
                continue
            after = cp.copy()
            after[i] = d
            assert oracle.modularity_exact(level, after) <= q0


@pytest.mark.parametrize("r_,k", [(10, 5), (21, 5), (6, 4), (7, 3)])
def test_ring_of_cliques_closed_form(r_, k):
    """Ring of r cliques K_k: the cliques are optimal among merges when
    r < k(k-1)+2, and Q = (K-2)/K - 1/r with K = k(k-1)+2."""
    K = k * (k - 1) + 2
    assert r_ < K
    g = gg.ring_of_cliques(r_, k)
    res = oracle.louvain(g, oracle.Params(max_passes=0, agg_num=1, agg_den=1))
    assert res.communities == r_
    # the communities are exactly the cliques
    for t in range(r_):
        assert len(set(res.membership[t * k:(t + 1) * k].tolist())) == 1
    assert oracle.modularity_exact(g, res.membership) == Fraction(K - 2, K) - Fraction(1, r_)


def test_ring_of_cliques_merges_beyond_resolution_limit():
    """r > K: merging two adjacent cliques gains, so Louvain returns fewer communities than cliques."""
    k = 3
    K = k * (k - 1) + 2  # 8
    g = gg.ring_of_cliques(20, k)
    res = oracle.louvain(g, loose_params(mode=oracle.ASYNC))
    assert 20 > K and res.communities < 20
    assert oracle.modularity_exact(g, res.membership) > Fraction(K - 2, K) - Fraction(1, 20)


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.mark.parametrize("mode", ["sync", "async"])
def test_k2_hand_trace(mode):
    gold = _golden("k2_traces.json")[mode]
    g = gg.from_edges(2, [(0, 1, 1)])
    r = oracle.louvain(g, oracle.Params(mode=oracle.SYNC if mode == "sync" else oracle.ASYNC), trace=True)
    got = [[x["pass_"], x["iter"], x["cprime"].tolist(), x["moves"], x["gain"]] for x in r.iters]
    assert got == gold["iters"]
    graphs = [[x["offsets"].tolist(), x["indices"].tolist(), x["weights"].tolist()] for x in r.graphs]
    assert graphs == gold["graphs"]
    assert r.membership.tolist() == gold["membership"]


def test_tolerance_boundary_is_inclusive():
    """K2 async: S = 1 after t = 0, W = 2 -> Delta Q = 2S/W^2 = 1/2.  tau = 1/2 converges
    at t = 0 (test is <=) and stops the run; tau = 1/3 does not."""
    g = gg.from_edges(2, [(0, 1, 1)])
    r = oracle.louvain(g, oracle.Params(tol_num=1, tol_den=2))
    assert (r.passes, r.iterations) == (1, 1)
    r = oracle.louvain(g, oracle.Params(tol_num=1, tol_den=3))
    assert (r.passes, r.iterations) == (2, 3)


def test_tolerance_drops_per_pass():
    """The same gain that passes tau_0 fails tau_1 = tau_0/drop: ring of cliques,
    pass 1 sees no move either way, so only the drop decides nothing here; instead
    check the exact threshold on K2 with a huge drop in pass 0 only (drop^0 = 1)."""
    g = gg.from_edges(2, [(0, 1, 1)])
    a = oracle.louvain(g, oracle.Params(tol_num=1, tol_den=2, tol_drop=10**6))
    b = oracle.louvain(g, oracle.Params(tol_num=1, tol_den=2, tol_drop=1))
    assert (a.passes, a.iterations) == (b.passes, b.iterations) == (1, 1)


# ------------------------------------------------------------- invariants

@pytest.mark.parametrize("mode", [oracle.ASYNC, oracle.SYNC])
@pytest.mark.parametrize("g", [gg.planted_partition(seed=4), gg.random_small(40, 0.15, 9, self_loops=True),
                               gg.grid(12, 12, seed=3), gg.rmat(9, 8, seed=5)], ids=lambda g: g.name)
def test_trace_invariants(g, mode):
    """Every iteration: sum of Sigma' = W and Sigma'_c = sum of K' over c's
    members; every pass: W preserved and row sums equal the communities' Sigma."""
    r = oracle.louvain(g, oracle.Params(mode=mode), trace=True)
    W = g.total_weight
    levels = [g] + [gg.CSRGraph(x["n"], x["offsets"], x["indices"], x["weights"]) for x in r.graphs]
    for rec in r.iters:
        lvl = levels[rec["pass_"]]
        K = np.zeros(lvl.n, dtype=np.int64)
        np.add.at(K, np.repeat(np.arange(lvl.n), np.diff(lvl.offsets)), lvl.weights.astype(np.int64))
        assert int(rec["sigma"].sum()) == W
        expect = np.zeros(lvl.n, dtype=np.int64)
        np.add.at(expect, rec["cprime"], K.astype(np.int64))
        assert np.array_equal(expect, rec["sigma"])
    for lvl in levels[1:]:
        assert lvl.total_weight == W


# ------------------------------------------------------------- aggregation

def _dict_aggregate(g, cp):
    acc = {}
    for i in range(g.n):
        for e in range(g.offsets[i], g.offsets[i + 1]):
            key = (int(cp[i]), int(cp[g.indices[e]]))
            acc[key] = acc.get(key, 0) + int(g.weights[e])
    return acc


@pytest.mark.parametrize("g", [gg.random_small(30, 0.2, 3, self_loops=True), gg.planted_partition(seed=5),
                               gg.grid(10, 10, seed=1)], ids=lambda g: g.name)
def test_aggregation_against_dict_and_modularity(g):
    rng = np.random.default_rng(2)
    k = max(2, g.n // 6)
    cp = rng.integers(0, k, size=g.n).astype(np.int32)
    _, cp = np.unique(cp, return_inverse=True)
    cp = cp.astype(np.int32)
    nc = int(cp.max()) + 1
    off, idx, w = oracle.aggregate(g, cp, nc)
    # against an independent dict construction
    ref = _dict_aggregate(g, cp)
    got = {}
    for c in range(nc):
        row = idx[off[c]:off[c + 1]]
        assert np.all(np.diff(row) > 0), "rows sorted, no duplicates"
        for e in range(off[c], off[c + 1]):
            got[(c, int(idx[e]))] = int(w[e])
    assert got == ref
    sup = gg.CSRGraph(nc, off, idx, w)
    assert sup.total_weight == g.total_weight
    # symmetric
    assert all(got.get((d, c)) == x for (c, d), x in got.items())
    # modularity preserved: Q(G'', singletons) == Q(G', C')
    assert oracle.modularity_exact(sup, np.arange(nc)) == oracle.modularity_exact(g, cp)


# ----------------------------------------------------------- planted partition

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_planted_partition_recovered(seed):
    g = gg.planted_partition(seed=seed)
    r = oracle.louvain(g, oracle.Params(max_passes=0, agg_num=1, agg_den=1))
    q_planted = oracle.modularity(g, g.labels)
    q = oracle.modularity(g, r.membership)
    assert q >= q_planted - 0.01
    # each planted block is (almost) one community
    agree = 0
    for b in range(10):
        vals, counts = np.unique(r.membership[g.labels == b], return_counts=True)
        agree += counts.max()
    assert agree >= 0.95 * g.n


def test_isolated_vertices_stay_singletons():
    g = gg.from_edges(7, [(0, 1, 1), (1, 2, 1), (0, 2, 1), (4, 5, 2)])
    r = oracle.louvain(g)
    assert len({r.membership[3], r.membership[6]}) == 2
    assert r.membership[3] not in set(r.membership[[0, 1, 2, 4, 5]].tolist())
    assert sorted(set(r.membership.tolist())) == list(range(r.communities))


def test_bruteforce_partition_enumeration_counts():
    # Bell numbers, to pin the enumerator the max-Q checks rely on
    assert [len(set_partitions(n)) for n in range(1, 8)] == [1, 2, 5, 15, 52, 203, 877]


# ------------------------------------------------------- hand-derived traces

def _case_graph(case):
    if case["edges"] == "cycle":
        return gg.from_edges(case["n"], [(i, (i + 1) % case["n"], 1) for i in range(case["n"])])
    return gg.from_edges(case["n"], [tuple(e) for e in case["edges"]])


@pytest.mark.parametrize("case", _golden("small_traces.json")["cases"], ids=lambda c: c["name"][:40])
def test_small_hand_traces(case):
    g = _case_graph(case)
    r = oracle.louvain(g, oracle.Params(**case["params"]), trace=True)
    if "iters" in case:
        got = [[x["pass_"], x["iter"], x["cprime"].tolist(), x["moves"], x["gain"]] for x in r.iters]
        assert got == case["iters"]
    assert r.membership.tolist() == case["membership"]
    assert (r.passes, r.iterations) == (case["passes"], case["iterations"])


# ------------------------------------------------------- trace properties

@pytest.mark.parametrize("g", [gg.planted_partition(seed=6), gg.random_small(30, 0.2, 4, self_loops=True),
                               gg.grid(9, 9, seed=2), gg.rmat(8, 8, seed=1, wmax=5)], ids=lambda g: g.name)
def test_async_gain_sum_is_exact_modularity_change(g):
    """Sequential in-place moves: each gain is taken against the current state,
    so an iteration's gain sum equals the exact change of Q times W^2/2."""
    r = oracle.louvain(g, oracle.Params(mode=oracle.ASYNC), trace=True)
    W = g.total_weight
    levels = [g] + [gg.CSRGraph(x["n"], x["offsets"], x["indices"], x["weights"]) for x in r.graphs]
    prev = None
    for rec in r.iters:
        lvl = levels[rec["pass_"]]
        before = np.arange(lvl.n) if (prev is None or prev["pass_"] != rec["pass_"]) else prev["cprime"]
        dq = oracle.modularity_exact(lvl, rec["cprime"]) - oracle.modularity_exact(lvl, before)
        assert dq * W * W == 2 * rec["gain"]
        assert rec["moves"] <= rec["gain"]  # every applied gain is a positive integer
        prev = rec


@pytest.mark.parametrize("g", [gg.random_small(n, 0.5, s, wmax=3) for n, s in [(5, 1), (6, 2), (8, 3), (12, 4)]]
                         + [gg.planted_partition(seed=7), gg.grid(8, 8, seed=5)], ids=lambda g: g.name)
def test_sync_movers_are_neighbours_of_previous_movers(g):
    """SYNC pruning: after iteration t only neighbours (other than itself) of
    t's movers are evaluated, so every mover of t+1 is such a neighbour."""
    r = oracle.louvain(g, oracle.Params(mode=oracle.SYNC), trace=True)
    levels = [g] + [gg.CSRGraph(x["n"], x["offsets"], x["indices"], x["weights"]) for x in r.graphs]
    prev_c, prev_movers, prev_pass = None, None, -1
    for rec in r.iters:
        lvl = levels[rec["pass_"]]
        start = np.arange(lvl.n) if rec["pass_"] != prev_pass else prev_c
        movers = np.flatnonzero(rec["cprime"] != start)
        assert len(movers) == rec["moves"]
        if rec["pass_"] == prev_pass:
            allowed = set()
            for i in prev_movers:
                allowed |= {int(j) for j in lvl.indices[lvl.offsets[i]:lvl.offsets[i + 1]] if j != i}
            assert set(movers.tolist()) <= allowed
        prev_c, prev_movers, prev_pass = rec["cprime"], movers, rec["pass_"]


@pytest.mark.parametrize("g", [gg.random_small(12, 0.35, 511, wmax=3), gg.random_small(20, 0.3, 8, wmax=3),
                               gg.planted_partition(seed=8), gg.grid(10, 10, seed=4)], ids=lambda g: g.name)
def test_async_pruning_order(g):
    """ASYNC visits flagged vertices in ascending id order and flags the
    neighbours of each mover.  So a vertex v can move in iteration t+1 only if
    a neighbour j > v moved in iteration t (flag set after v's turn) or a
    neighbour j < v moved earlier in iteration t+1."""
    r = oracle.louvain(g, oracle.Params(mode=oracle.ASYNC), trace=True)
    levels = [g] + [gg.CSRGraph(x["n"], x["offsets"], x["indices"], x["weights"]) for x in r.graphs]
    prev_c, prev_movers, prev_pass = None, None, -1
    for rec in r.iters:
        lvl = levels[rec["pass_"]]
        start = np.arange(lvl.n) if rec["pass_"] != prev_pass else prev_c
        movers = set(np.flatnonzero(rec["cprime"] != start).tolist())
        if rec["pass_"] == prev_pass:
            for v in movers:
                nbrs = {int(j) for j in lvl.indices[lvl.offsets[v]:lvl.offsets[v + 1]] if j != v}
                assert any((j in prev_movers and j > v) or (j in movers and j < v) for j in nbrs), v
        prev_c, prev_movers, prev_pass = rec["cprime"], movers, rec["pass_"]


@pytest.mark.parametrize("g", [gg.planted_partition(seed=1), gg.random_small(30, 0.2, 6, wmax=4, self_loops=True)],
                         ids=lambda g: g.name)
def test_sync_without_pruning_matches_single_vertex_sweeps(g):
    """SYNC without pruning: every vertex decides against the iteration's
    start state.  Rebuild each iteration from the single-vertex decision
    routine (a separate sparse implementation) and compare."""
    W = g.total_weight
    w = g.weights.astype(np.int64)
    K = np.zeros(g.n, dtype=np.int64)
    np.add.at(K, np.repeat(np.arange(g.n), np.diff(g.offsets)), w)
    C = np.arange(g.n, dtype=np.int32)
    S = K.copy()
    r = oracle.louvain(g, oracle.Params(mode=oracle.SYNC, prune=0), trace=True)
    for rec in [x for x in r.iters if x["pass_"] == 0][:8]:
        t = rec["iter"]
        pl = (t + 2) % 4 == 0
        dec = C.copy()
        for i in range(g.n):
            d, gain = oracle.best_move(g, W, C, S, i)
            if d is None or gain <= 0 or (pl and d > C[i]):
                continue
            dec[i] = d
        for i in np.flatnonzero(dec != C):
            S[C[i]] -= K[i]
            S[dec[i]] += K[i]
        C = dec
        assert np.array_equal(C, rec["cprime"]) and np.array_equal(S, rec["sigma"])
