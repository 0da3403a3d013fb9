"""Full-size parity against stored oracle results.

The sequential oracle needs minutes on these graphs, so its results were
computed once by tests/golden/make_full_size.py (oracle and seeded generators
only) and stored as SHA-256 digests of little-endian arrays.  The GPU run
must reproduce them exactly:

* R-MAT scale 22, edge factor 16 (hubs, the workgroup bucket, big-community
  aggregation at scale): per iteration the moves, the exact gain sum, C' and
  Sigma'; per pass the super-graph CSR; the final membership, pass and
  iteration counts and the exact modularity.
* A sample of the batched SBM recipe over its whole vertex range [200,
  200000] (its four largest graphs and every 128th one), batched with 64-bit
  offsets: each graph's membership, passes, iterations, communities and
  exact modularity equal its lone oracle run.
* The same sample batched in ASYNC mode, 3 runs: every run's membership is
  valid with the exact modularity the oracle computes for it, and graph by
  graph Q is compared with the lowest modularity the sequential oracle
  reaches over the identity order and 8 seeded relabellings (stored per
  graph).  Where those sequential runs agree within 0.002 (25 of the 36
  graphs), every run must reach that lowest order less 0.002.  On the 11
  weak-structure graphs the sequential orders themselves end up to 0.074
  apart and concurrent runs vary as much from run to run (one graph moved
  by 0.019 over five runs), so no single run is a meaningful sample: there
  the median of the 3 runs must reach the lowest order less the orders'
  own spread.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lv = pytest.importorskip("paper_2501_19004_amd")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
RUNS = 3  # concurrent (ASYNC) runs of the full-range batch


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return "cuda:0"


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).astype(a.dtype.newbyteorder("<"), copy=False).tobytes())
    return h.hexdigest()


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_full_size_sync_rmat22_every_iteration():
    ref = load("rmat22_sync.json")
    g = gg.rmat(22, 16, seed=22)
    assert (g.n, g.nnz) == (ref["n"], ref["nnz"])
    assert sha(np.asarray(g.offsets, np.int64), np.asarray(g.indices, np.int32)) == ref["graph_sha256"]
    print("[case] R-MAT 22 SYNC full run with per-iteration digests", flush=True)
    off, idx, w = lv.graph_tensors(g, dev())
    L = lv.Louvain(off, idx, w, mode=lv.SYNC)
    iters, graphs = [], []
    L.trace(lambda p, t, cp, sig, m, gain: iters.append((p, t, m, gain, sha(cp.astype(np.int32)),
                                                         sha(sig.astype(np.int64)))),
            lambda p, n, o, i, ww, it: graphs.append((n, int(o[-1]), sha(o.astype(np.int64), i.astype(np.int32),
                                                                          ww.astype(np.int64)))))
    L.run()
    memb = L.membership().cpu().numpy()
    q, num, den = L.modularity()
    st = L.stats()
    L.close()
    assert len(iters) == len(ref["iters"])
    for a, b in zip(iters, ref["iters"]):
        where = f"pass {b['pass']} iter {b['iter']}"
        assert (a[0], a[1]) == (b["pass"], b["iter"]), where
        assert (a[2], a[3]) == (b["moves"], int(b["gain"])), where
        assert a[4] == b["cprime_sha256"], where
        assert a[5] == b["sigma_sha256"], where
    assert [(x[0], x[1], x[2]) for x in graphs] == [(b["n"], b["nnz"], b["csr_sha256"]) for b in ref["graphs"]]
    assert (st.passes, st.iterations, st.communities) == (ref["passes"], ref["iterations"], ref["communities"])
    assert sha(memb.astype(np.int32)) == ref["membership_sha256"]
    assert (num, den) == (int(ref["q_num"]), int(ref["q_den"]))


def test_full_range_sbm_batch_sync_per_graph():
    ref = load("sbm_fullrange_sync.json")["graphs"]
    specs = gg.sbm_batch_specs(4096, 200_000)
    graphs = [gg.sbm_batch_graph(specs[r["index"]]) for r in ref]
    for g, r in zip(graphs, ref):
        assert sha(np.asarray(g.offsets, np.int64), np.asarray(g.indices, np.int32),
                   np.asarray(g.weights, np.int32)) == r["graph_sha256"], r["index"]
    print(f"[case] batched SYNC over {len(graphs)} graphs of the full-range SBM recipe, 64-bit offsets", flush=True)
    off, idx, w, vbase = lv.batch_tensors(graphs, dev(), offset_bits=64)
    assert off.dtype == torch.int64
    L = lv.Louvain(off, idx, w, vbase=vbase, mode=lv.SYNC)
    L.run()
    memb = L.membership().cpu().numpy()
    q, num, den = L.modularity_batch()
    passes, iters, comms = L.batch_results()
    L.close()
    for k, r in enumerate(ref):
        part = memb[vbase[k]:vbase[k + 1]]
        where = (k, r["index"], r["n"])
        assert sha(part.astype(np.int32)) == r["membership_sha256"], where
        assert (passes[k], iters[k], comms[k]) == (r["passes"], r["iterations"], r["communities"]), where
        assert (num[k], den[k]) == (int(r["q_num"]), int(r["q_den"])), where


def test_full_range_sbm_batch_async_per_graph():
    ref = load("sbm_fullrange_async.json")["graphs"]
    specs = gg.sbm_batch_specs(4096, 200_000)
    graphs = [gg.sbm_batch_graph(specs[r["index"]]) for r in ref]
    assert [(g.n, g.nnz) for g in graphs] == [(r["n"], r["nnz"]) for r in ref]
    print(f"[case] batched ASYNC over {len(graphs)} graphs of the full-range SBM recipe, 64-bit offsets, 3 runs",
          flush=True)
    off, idx, w, vbase = lv.batch_tensors(graphs, dev(), offset_bits=64)
    L = lv.Louvain(off, idx, w, vbase=vbase, mode=lv.ASYNC)
    runs = []
    for _ in range(RUNS):
        L.run()
        memb = L.membership().cpu().numpy()
        q, num, den = L.modularity_batch()
        passes, iters, comms = L.batch_results()
        for k, g in enumerate(graphs):
            part = memb[vbase[k]:vbase[k + 1]]
            assert (num[k], den[k]) == oracle.modularity_parts(g, part), k
            assert sorted(set(part.tolist())) == list(range(comms[k])), k
        runs.append(np.array(q))
    L.close()
    runs = np.array(runs)
    bad = []
    for k, r in enumerate(ref):
        qs = r["q_orders"]
        spread = max(qs) - min(qs)
        if spread <= 0.002:  # a well-defined sequential optimum: every run within 0.002 of the lowest order
            got, floor = runs[:, k].min(), min(qs) - 0.002
        else:  # weak structure: the median run within the sequential runs' own spread of the lowest order
            got, floor = float(np.median(runs[:, k])), min(qs) - spread
        if got < floor:
            bad.append((r["index"], r["n"], round(spread, 5), round(got - floor, 5)))
    print(f"per-run Q_gpu - lowest order: min {float((runs - np.array([min(r['q_orders']) for r in ref])).min()):+.5f}")
    assert not bad, bad
