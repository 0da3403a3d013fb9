#!/usr/bin/env python3
"""Benchmark: plain Louvain (local moving + aggregation, all passes) on one MI355X.

Workload (default): R-MAT scale 22, edge factor 16 (a/b/c/d = .57/.19/.19/.05,
seed 22, duplicates and self-loops removed, unit weights, int32 CSR), paper
defaults (20 iterations, 10 passes, tau 0.01 dropped 10x, tau_agg 0.8,
Pick-Less every 4, vertex pruning), ASYNC local moving.

One step = one complete louvain_run on the device-resident graph.  The
metric counts stored arcs (each undirected edge twice), as the paper does.
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E


def make_graph(name):
    import graphgen as gg
    if name == "rmat22":
        return gg.rmat(22, 16, seed=22), "R-MAT scale 22, edge factor 16, a/b/c=.57/.19/.19, seed 22, unit weights"
    if name == "grid4096":
        return gg.grid(4096, 4096, seed=4096), "4096x4096 grid, 10% deleted, 1% diagonals, weights U[1,16], seed 4096"
    if name == "planted":
        return gg.planted_partition(seed=1), "planted partition 10x100, p_in .1, p_out .002, seed 1"
    if name.startswith("rmat"):
        s = int(name[4:])
        return gg.rmat(s, 16, seed=22), f"R-MAT scale {s}, edge factor 16, seed 22, unit weights"
    raise SystemExit(f"unknown workload {name}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--mode", default="async", choices=["async", "sync"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="do not record per-kernel HIP events")
    ap.add_argument("--kernels", action="store_true", help="also print the per-kernel table to stderr")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2501_19004_amd as lv

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    t0 = time.time()
    g, desc = make_graph(args.workload)
    print(f"[bench] generated {desc}: n={g.n} arcs={g.nnz} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    off, idx, w = lv.graph_tensors(g, "cuda:0")
    mode = lv.ASYNC if args.mode == "async" else lv.SYNC
    L = lv.Louvain(off, idx, w, mode=mode)
    for _ in range(args.warmup):
        L.run()
    if not args.no_profile:
        L.set_profiling(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        L.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / max(args.steps, 1)
    st = L.stats()
    q, num, den = L.modularity()
    print(f"[bench] {args.steps} runs, {dt * 1e3:.2f} ms/run, Q={q:.5f}, passes={st.passes} "
          f"iterations={st.iterations} communities={st.communities}", file=sys.stderr, flush=True)

    roofline = None
    kstats = L.kernel_stats() if not args.no_profile else []
    if kstats:
        if args.kernels:
            for k in kstats:
                gbs = k["alg_bytes"] / (k["ms"] * 1e-3) / 1e9 if k["ms"] > 0 and k["alg_bytes"] else 0.0
                print(f"[kernel] {k['name']:16s} launches={k['launches']:6d} ms={k['ms']:9.3f} "
                      f"alg_GB={k['alg_bytes'] / 1e9:8.3f} GB/s={gbs:8.1f}", file=sys.stderr)
        moves = [k for k in kstats if k["name"].startswith("move_")]
        if moves:
            dom = max(moves, key=lambda k: k["ms"])
            ms_launch = dom["ms"] / dom["launches"]
            bytes_launch = dom["alg_bytes"] / dom["launches"]
            ach = bytes_launch / (ms_launch * 1e-3) / 1e9
            tot_ms = sum(k["ms"] for k in moves)
            tot_b = sum(k["alg_bytes"] for k in moves)
            roofline = {"bound": "hbm", "kernel": dom["name"], "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
                        "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": None,
                        "avg_launch_us": round(ms_launch * 1e3, 2),
                        "alg_bytes_per_launch": int(bytes_launch),
                        "local_move_phase_GBs": round(tot_b / (tot_ms * 1e-3) / 1e9, 1) if tot_ms else None,
                        "local_move_ms_per_run": round(tot_ms / args.steps, 3)}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        g.weights = g.weights.astype(np.int64)
        cores = 1
        t = time.perf_counter()
        ref = oracle.louvain(g, oracle.Params())
        tc = time.perf_counter() - t
        q_or = oracle.modularity(g, ref.membership)
        cpu = {"value": round(g.nnz / tc / 1e6, 2), "unit": "M edges/s", "cores": cores, "kind": "oracle",
               "sample": f"whole workload, sequential ASYNC oracle, one run ({tc:.1f} s)",
               "q_oracle": round(q_or, 6), "q_gpu_minus_oracle": round(q - q_or, 6)}
        print(f"[bench] oracle {tc:.1f}s Q={q_or:.5f} (gpu-oracle {q - q_or:+.5f})", file=sys.stderr, flush=True)

    out = {
        "metric": "Louvain M edges/s (plain, ASYNC, paper defaults)",
        "value": round(g.nnz / dt / 1e6, 2),
        "unit": "M edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": desc, "vertices": g.n, "arcs": g.nnz, "undirected_edges": g.nnz // 2,
                   "mode": args.mode, "pruner": "flags", "modularity": round(q, 6), "passes": st.passes,
                   "iterations": st.iterations, "communities": st.communities,
                   "undirected_Medges_per_s": round(g.nnz / 2 / dt / 1e6, 2)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    L.close()


if __name__ == "__main__":
    main()
