"""Device-driven iterations (device_loop = 1).

The tests between two local-moving iterations -- the tolerance test of
Alg. 1 (per graph in a batch), the next queue's sizes and the end of the
pass -- run on the GPU, and the host reads a pass's state back once per
chunk of 2, 4, 8, ... iterations.  SYNC runs must equal the oracle exactly,
as the host-driven loop does: membership, passes, iterations, communities and
exact modularity, for single graphs (every bucket path, pruning on and off,
parameters that end passes by every rule) and for batches graph by graph;
the moves match the host-driven run.  ASYNC runs keep the quality bound of
the host-driven ones (the oracle's lowest modularity over visiting orders,
minus 0.002).  The host waits a bounded number of times per pass instead of
once per iteration.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle.orders import async_floor

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lv = pytest.importorskip("paper_2501_19004_amd")

ALL_HUB = dict(bucket_max_degree=[-1] * 5, agg_bucket_max=[-1] * 4)
SMALL_B = dict(bucket_max_degree=[2, 8, 16, 64, 128], agg_bucket_max=[4, 16, 64, 256])
CONFIGS = {"default": {}, "all_hub": ALL_HUB, "small_buckets": SMALL_B, "no_pruning": dict(pruner=lv.PRUNE_NONE)}


def star_plus_cliques(leaves=9000, cliques=30, k=6):
    edges = [(0, 1 + i, 1) for i in range(leaves)]
    base = leaves + 1
    for c in range(cliques):
        for x in range(k):
            for y in range(x + 1, k):
                edges.append((base + c * k + x, base + c * k + y, 2))
        edges.append((base + c * k, 1 + c, 1))
    return gg.from_edges(base + cliques * k, edges, "star+cliques")


GRAPHS = {
    "planted": lambda: gg.planted_partition(seed=1),
    "small_loops": lambda: gg.random_small(60, 0.12, 3, wmax=5, self_loops=True),
    "rmat12w": lambda: gg.rmat(12, 16, seed=4, wmax=7),
    "grid48": lambda: gg.grid(48, 48, seed=5),
    "sbm": lambda: gg.sbm_degree(6000, 24, 14.0, seed=6, wmin=1, wmax=4),
    "star": star_plus_cliques,
    "k2": lambda: gg.from_edges(2, [(0, 1, 1)]),
}


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return "cuda:0"


def run(g, mode, **kw):
    off, idx, w = lv.graph_tensors(g, dev())
    L = lv.Louvain(off, idx, w, mode=mode, **kw)
    L.run()
    memb = L.membership().cpu().numpy()
    q = L.modularity()
    st = L.stats()
    L.close()
    return memb, q, st


def oracle_params(kw, mode):
    p = oracle.Params(mode=mode)
    for k, v in kw.items():
        if k == "pruner":
            p.prune = v
        elif k not in ("bucket_max_degree", "agg_bucket_max") and hasattr(p, k):
            setattr(p, k, v)
    return p


def chunk_count(max_iterations):
    """Readbacks of one pass that runs all its iterations: chunks end after
    2, 6, 14, ... iterations (and at max_iterations)."""
    k, end, step = 0, 0, 2
    while end < max_iterations:
        end = min(max_iterations, end + step)
        step *= 2
        k += 1
    return k


def assert_sync_equal(g, kw):
    print(f"[case] device loop SYNC {g.name} {kw}", flush=True)
    memb, (q, num, den), st = run(g, lv.SYNC, device_loop=1, **kw)
    ref = oracle.louvain(g, oracle_params(kw, oracle.SYNC))
    assert np.array_equal(memb, ref.membership)
    assert (st.passes, st.iterations, st.communities) == (ref.passes, ref.iterations, ref.communities)
    assert (num, den) == oracle.modularity_parts(g, memb)
    _, _, host = run(g, lv.SYNC, **kw)
    assert st.moves == host.moves
    assert list(st.iterations_per_pass) == list(host.iterations_per_pass)
    return st, host


@pytest.mark.parametrize("cfg", list(CONFIGS))
@pytest.mark.parametrize("name", list(GRAPHS))
def test_sync_equals_oracle(name, cfg):
    assert_sync_equal(GRAPHS[name](), CONFIGS[cfg])


@pytest.mark.parametrize("kw", [dict(max_passes=0, agg_num=1, agg_den=1), dict(tol_num=0, tol_den=1),
                                dict(pick_less=0, max_iterations=7), dict(pick_less=2, tol_drop=1),
                                dict(max_iterations=1), dict(max_iterations=3, tol_num=0, tol_den=1)],
                         ids=["to_convergence", "zero_tol", "no_pl", "pl2", "one_iteration", "iteration_cap"])
def test_sync_parameters(kw):
    assert_sync_equal(gg.planted_partition(seed=2), kw)


@pytest.mark.parametrize("g", [gg.from_edges(1, []), gg.from_edges(6, []), gg.from_edges(4, [(1, 1, 3), (2, 2, 1)])],
                         ids=["one_vertex", "no_edges", "self_loops_only"])
@pytest.mark.parametrize("mode", [lv.SYNC, lv.ASYNC])
def test_degenerate_graphs(g, mode):
    memb, (q, num, den), st = run(g, mode, device_loop=1)
    ref = oracle.louvain(g, oracle.Params(mode=mode))
    if mode == lv.SYNC:
        assert np.array_equal(memb, ref.membership)
    assert sorted(set(memb.tolist())) == list(range(st.communities))
    assert (num, den) == oracle.modularity_parts(g, memb)


def test_host_waits_bounded_per_pass():
    """A zero tolerance keeps passes going until no move is left (many
    iterations per pass): the host-driven loop waits at least once per
    iteration, the device-driven one a bounded number of times per pass."""
    g = gg.rmat(12, 16, seed=9)
    kw = dict(tol_num=0, tol_den=1, max_iterations=60)
    st, host = assert_sync_equal(g, kw)
    print(f"iterations {st.iterations} passes {st.passes}: host waits {host.host_syncs} host-driven, "
          f"{st.host_syncs} device-driven", flush=True)
    assert host.host_syncs >= host.iterations
    # per pass: pass set-up and aggregation readbacks (at most 20) and one per chunk
    assert st.host_syncs <= st.passes * (20 + chunk_count(60)) + 4
    assert st.host_syncs < host.host_syncs


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_async_quality_planted(seed):
    g = gg.planted_partition(seed=seed)
    memb, (q, num, den), st = run(g, lv.ASYNC, device_loop=1)
    assert (num, den) == oracle.modularity_parts(g, memb)
    assert q >= async_floor(g), (q, async_floor(g))


@pytest.mark.parametrize("make", [lambda: gg.rmat(14, 16, seed=5), lambda: gg.grid(128, 128, seed=6),
                                  lambda: gg.sbm_degree(20000, 32, 16.0, seed=7, wmin=1, wmax=4),
                                  lambda: gg.rmat(12, 8, seed=8, wmax=9), star_plus_cliques],
                         ids=["rmat14", "grid128", "sbm20k", "rmat12w", "star"])
def test_async_quality(make):
    g = make()
    print(f"[case] device loop ASYNC {g.name}", flush=True)
    memb, (q, num, den), st = run(g, lv.ASYNC, device_loop=1)
    assert (num, den) == oracle.modularity_parts(g, memb)
    assert sorted(set(memb.tolist())) == list(range(st.communities))
    floor = async_floor(g)
    print(f"Q_gpu - floor = {q - floor:+.5f}")
    assert q >= floor, (q, floor)


# ------------------------------------------------------------------ batches

def mixed_batch():
    return [gg.planted_partition(seed=1), gg.rmat(10, 8, seed=3), gg.ring_of_cliques(10, 5),
            gg.from_edges(3, []), gg.sbm_degree(3000, 12, 14.0, seed=6, wmin=1, wmax=4), gg.grid(20, 20, seed=5),
            gg.from_edges(2, [(0, 1, 1)]), gg.from_edges(1, []),
            gg.random_small(60, 0.12, 3, wmax=5, self_loops=True), star_plus_cliques(6000, 20, 5),
            gg.rmat(12, 16, seed=4, wmax=7), gg.from_edges(4, [(1, 1, 3), (2, 2, 1)])]


def sbm_batch(count, seed, nmax=5000):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(np.exp(rng.uniform(np.log(200), np.log(nmax))))
        out.append(gg.sbm_degree(n, int(rng.integers(4, 65)), float(rng.uniform(8, 32)), seed=seed * 1000 + k,
                                 wmin=1, wmax=4))
    return out


def run_batch(graphs, mode, **kw):
    off, idx, w, vbase = lv.batch_tensors(graphs, dev())
    L = lv.Louvain(off, idx, w, vbase=vbase, mode=mode, **kw)
    L.run()
    memb = L.membership().cpu().numpy()
    q, num, den = L.modularity_batch()
    passes, iters, comms = L.batch_results()
    st = L.stats()
    L.close()
    parts = [memb[vbase[k]:vbase[k + 1]] for k in range(len(graphs))]
    return parts, q, num, den, passes, iters, comms, st


BATCH_CONFIGS = {"default": {}, "all_hub": ALL_HUB, "no_pruning": dict(pruner=lv.PRUNE_NONE),
                 "max_passes2": dict(max_passes=2), "zero_tol": dict(tol_num=0, tol_den=1, max_iterations=40)}


@pytest.mark.parametrize("cfg", list(BATCH_CONFIGS))
def test_batch_sync_equals_oracle_per_graph(cfg):
    kw = BATCH_CONFIGS[cfg]
    graphs = mixed_batch() + sbm_batch(16, 7)
    print(f"[case] device loop batched SYNC {cfg}", flush=True)
    parts, q, num, den, passes, iters, comms, st = run_batch(graphs, lv.SYNC, device_loop=1, **kw)
    P = oracle_params(kw, oracle.SYNC)
    for k, g in enumerate(graphs):
        ref = oracle.louvain(g, P)
        assert np.array_equal(parts[k], ref.membership), k
        assert (passes[k], iters[k], comms[k]) == (ref.passes, ref.iterations, ref.communities), k
        assert (num[k], den[k]) == oracle.modularity_parts(g, parts[k]), k
    host = run_batch(graphs, lv.SYNC, **kw)[-1]
    print(f"host waits: {host.host_syncs} host-driven, {st.host_syncs} device-driven", flush=True)
    assert st.moves == host.moves and st.iterations == host.iterations
    assert st.host_syncs <= host.host_syncs


@pytest.mark.parametrize("make", [mixed_batch, lambda: sbm_batch(48, 5)], ids=["mixed", "sbm48"])
def test_batch_async_quality(make):
    graphs = make()
    print(f"[case] device loop batched ASYNC {len(graphs)} graphs", flush=True)
    parts, q, num, den, passes, iters, comms, st = run_batch(graphs, lv.ASYNC, device_loop=1)
    d = []
    for k, g in enumerate(graphs):
        assert (num[k], den[k]) == oracle.modularity_parts(g, parts[k]), k
        assert sorted(set(parts[k].tolist())) == list(range(comms[k])), k
        d.append(q[k] - async_floor(g))
    print(f"Q_gpu - (floor over orders) per graph: min {min(d):+.5f} mean {np.mean(d):+.5f}")
    bad = [(k, graphs[k].name, round(d[k], 5)) for k in range(len(graphs)) if d[k] < 0]
    assert not bad, bad


def test_refused_with_learned_pruner_or_iteration_trace():
    g = gg.planted_partition(seed=1)
    off, idx, w = lv.graph_tensors(g, dev())
    wts = torch.zeros(lv.MLP_PARAMS, dtype=torch.float32, device=dev())
    with pytest.raises(lv.LouvainError) as e:
        lv.Louvain(off, idx, w, device_loop=1, pruner=lv.PRUNE_LEARNED, pruner_weights=wts)
    assert e.value.status == lv.LOUVAIN_ERR_INVALID
    L = lv.Louvain(off, idx, w, device_loop=1)
    L.trace(lambda *a: None, None)
    with pytest.raises(lv.LouvainError) as e:
        L.run()
    assert e.value.status == lv.LOUVAIN_ERR_INVALID
    L.trace(None, lambda *a: None)  # a pass trace alone is served
    L.run()
    assert L.stats().passes >= 1
    L.close()
