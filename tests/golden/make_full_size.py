#!/usr/bin/env python3
"""Writes the stored oracle results used by the full-size GPU parity tests.

The sequential oracle needs minutes for these graphs, longer than a GPU test
should wait, so its results are computed once here -- by the oracle alone,
on graphs from the seeded generators -- and stored as digests:

  rmat22_sync.json       R-MAT scale 22, edge factor 16, seed 22, SYNC mode:
                         per iteration the moves, the exact gain sum and
                         SHA-256 digests of C' (int32) and Sigma' (int64);
                         per pass the digest of the super-graph CSR (offsets
                         int64, indices int32, weights int64); the final
                         membership digest, counts and exact modularity.
  sbm_fullrange_sync.json  a sample of the batched SBM recipe over its whole
                         vertex range [200, 200000] (the four largest graphs
                         of the 4096 and every 128th one), SYNC mode, each
                         graph run alone: membership digest, passes,
                         iterations, communities and exact modularity.
  rmat24_ef28_async.json  R-MAT scale 24, edge factor 28, seed 27 (the
                         benchmark's scale-27 recipe at 1/8 of its vertices),
                         ASYNC (sequential) mode in the identity order: the
                         graph's digest, counts and exact modularity.
  sbm_fullrange_async.json  the same sample, ASYNC (sequential) mode: the
                         modularity the oracle reaches in the identity
                         vertex order and in 8 seeded relabellings
                         (oracle/orders.py), whose minimum less 0.002 is the
                         per-graph quality floor of batched ASYNC runs.

Digests are over the arrays' little-endian bytes.  Run from the repository
root: python tests/golden/make_full_size.py
"""
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).astype(a.dtype.newbyteorder("<"), copy=False).tobytes())
    return h.hexdigest()


def rmat22():
    g = gg.rmat(22, 16, seed=22)
    t = time.time()
    r = oracle.louvain(g, oracle.Params(mode=oracle.SYNC), trace=True)
    num, den = oracle.modularity_parts(g, r.membership)
    out = {
        "graph": "R-MAT scale 22, edge factor 16, a/b/c=.57/.19/.19, seed 22, unit weights",
        "n": int(g.n), "nnz": int(g.nnz), "graph_sha256": sha(np.asarray(g.offsets, np.int64),
                                                               np.asarray(g.indices, np.int32)),
        "mode": "SYNC", "params": "library defaults",
        "passes": int(r.passes), "iterations": int(r.iterations), "communities": int(r.communities),
        "moves": int(r.moves),
        "q_num": str(num), "q_den": str(den), "q": float(num) / float(den),
        "membership_sha256": sha(np.asarray(r.membership, np.int32)),
        "iters": [{"pass": it["pass_"], "iter": it["iter"], "moves": it["moves"], "gain": str(it["gain"]),
                   "cprime_sha256": sha(it["cprime"].astype(np.int32)),
                   "sigma_sha256": sha(it["sigma"].astype(np.int64))} for it in r.iters],
        "graphs": [{"pass": gr["pass_"], "n": gr["n"], "nnz": int(gr["offsets"][-1]),
                    "csr_sha256": sha(gr["offsets"].astype(np.int64), gr["indices"].astype(np.int32),
                                      gr["weights"].astype(np.int64))} for gr in r.graphs],
    }
    print(f"rmat22 SYNC: {r.passes} passes, {r.iterations} iterations, Q={out['q']:.6f}, {time.time() - t:.0f}s")
    return out


def sbm_fullrange():
    specs = gg.sbm_batch_specs(4096, 200_000)
    ns = np.array([s[0] for s in specs])
    pick = sorted(set(np.argsort(ns)[-4:].tolist()) | set(range(0, 4096, 128)))

    def one(k):
        g = gg.sbm_batch_graph(specs[k])
        r = oracle.louvain(g, oracle.Params(mode=oracle.SYNC))
        num, den = oracle.modularity_parts(g, r.membership)
        return {"index": int(k), "spec": list(specs[k]), "n": int(g.n), "nnz": int(g.nnz),
                "graph_sha256": sha(np.asarray(g.offsets, np.int64), np.asarray(g.indices, np.int32),
                                    np.asarray(g.weights, np.int32)),
                "passes": int(r.passes), "iterations": int(r.iterations), "communities": int(r.communities),
                "q_num": str(num), "q_den": str(den),
                "membership_sha256": sha(np.asarray(r.membership, np.int32))}

    t = time.time()
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        graphs = list(ex.map(one, pick))
    print(f"SBM full-range sample: {len(graphs)} graphs, {sum(x['nnz'] for x in graphs)} arcs, "
          f"{time.time() - t:.0f}s")
    return {"recipe": "graphgen.sbm_batch_specs(4096, 200000), graphs run alone in SYNC mode, library defaults",
            "graphs": graphs}


def sbm_fullrange_async():
    from oracle.orders import oracle_q_orders
    specs = gg.sbm_batch_specs(4096, 200_000)
    ns = np.array([s[0] for s in specs])
    pick = sorted(set(np.argsort(ns)[-4:].tolist()) | set(range(0, 4096, 128)))

    def one(k):
        g = gg.sbm_batch_graph(specs[k])
        qs = oracle_q_orders(g)
        return {"index": int(k), "n": int(g.n), "nnz": int(g.nnz), "q_orders": [float(q) for q in qs],
                "floor": float(min(qs)) - 0.002}

    t = time.time()
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        graphs = list(ex.map(one, pick))
    print(f"SBM full-range sample, ASYNC orders: {len(graphs)} graphs, {time.time() - t:.0f}s")
    return {"recipe": "graphgen.sbm_batch_specs(4096, 200000), sequential (ASYNC) oracle in the identity order "
                      "and 8 relabellings (oracle.orders.oracle_q_orders), library defaults",
            "graphs": graphs}


def rmat24_async():
    t = time.time()
    g = gg.rmat(24, 28, seed=27)
    t_gen = time.time() - t
    r = oracle.louvain(g, oracle.Params(mode=oracle.ASYNC))
    num, den = oracle.modularity_parts(g, r.membership)
    out = {"graph": "R-MAT scale 24, edge factor 28, a/b/c=.57/.19/.19, seed 27, unit weights",
           "n": int(g.n), "nnz": int(g.nnz),
           "graph_sha256": sha(np.asarray(g.offsets, np.int64), np.asarray(g.indices, np.int32)),
           "mode": "ASYNC (sequential, identity order)", "params": "library defaults",
           "passes": int(r.passes), "iterations": int(r.iterations), "communities": int(r.communities),
           "q_num": str(num), "q_den": str(den), "q": float(num) / float(den)}
    print(f"rmat24 ef28 ASYNC: generated in {t_gen:.0f}s, {r.passes} passes, {r.iterations} iterations, "
          f"Q={out['q']:.6f}, {time.time() - t:.0f}s")
    return out


def main():
    which = sys.argv[1:] or ["rmat22", "sbm", "sbm_async", "rmat24"]
    if "rmat24" in which:
        with open(os.path.join(HERE, "rmat24_ef28_async.json"), "w") as f:
            json.dump(rmat24_async(), f, indent=1)
    if "sbm_async" in which:
        with open(os.path.join(HERE, "sbm_fullrange_async.json"), "w") as f:
            json.dump(sbm_fullrange_async(), f, indent=1)
    if "sbm" in which:
        with open(os.path.join(HERE, "sbm_fullrange_sync.json"), "w") as f:
            json.dump(sbm_fullrange(), f, indent=1)
    if "rmat22" in which:
        with open(os.path.join(HERE, "rmat22_sync.json"), "w") as f:
            json.dump(rmat22(), f, indent=1)


if __name__ == "__main__":
    main()
