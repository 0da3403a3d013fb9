"""Seeded synthetic graphs in symmetric CSR form.

This module is the one source of inputs shared by the CPU oracle and the GPU
path.  It contains no community-detection arithmetic: only random draws,
edge deduplication and CSR layout.  Heavy generators (R-MAT, grid, SBM) run in
``libgraphgen.so`` (plain C, built from ``graphgen.c``); small hand-made graphs
are assembled in numpy.

Every graph is undirected: an edge {u, v} with u != v is stored as the two arcs
(u, v) and (v, u); a self-loop (only hand-built graphs have them) is stored
once.  Rows are sorted by neighbour id.  Weights are positive integers.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libgraphgen.so with gcc (OpenMP for the R-MAT draws)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.gg_rand.restype = ctypes.c_uint64
        lib.gg_rand.argtypes = [ctypes.c_uint64] * 3
        lib.gg_rmat_keys.restype = ctypes.c_int64
        lib.gg_rmat_keys.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_uint64, ctypes.c_int, u64p]
        lib.gg_grid_keys.restype = ctypes.c_int64
        lib.gg_grid_keys.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_uint64, u64p]
        lib.gg_sbm_keys.restype = ctypes.c_int64
        lib.gg_sbm_keys.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_uint64, ctypes.c_int, u64p, ctypes.c_int64, i32p]
        lib.gg_erdos_keys.restype = ctypes.c_int64
        lib.gg_erdos_keys.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, u64p, ctypes.c_int64]
        lib.gg_csr_from_keys.restype = None
        lib.gg_csr_from_keys.argtypes = [ctypes.c_int64, ctypes.c_int64, u64p, ctypes.c_uint64,
                                         ctypes.c_int32, ctypes.c_int32, i64p, i32p, i32p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


@dataclasses.dataclass
class CSRGraph:
    """Undirected graph in symmetric CSR form.

    offsets: int64[n+1]; indices: int32[nnz]; weights: int32 or int64 [nnz].
    ``labels`` holds planted block labels when the generator has them.
    """
    n: int
    offsets: np.ndarray
    indices: np.ndarray
    weights: np.ndarray
    name: str = ""
    labels: np.ndarray | None = None

    @property
    def nnz(self) -> int:
        return int(self.offsets[-1])

    @property
    def total_weight(self) -> int:
        return int(self.weights.sum(dtype=np.int64))

    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets)

    def edges_undirected(self) -> int:
        """Undirected edge count (a self-loop counts once)."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees())
        loops = int((src == self.indices).sum())
        return (self.nnz - loops) // 2 + loops


def _from_keys(n: int, keys: np.ndarray, m: int, seed: int, wmin: int, wmax: int, name: str,
               labels=None) -> CSRGraph:
    lib = _load()
    off = np.empty(n + 1, dtype=np.int64)
    idx = np.empty(2 * m, dtype=np.int32)
    w = np.empty(2 * m, dtype=np.int32)
    lib.gg_csr_from_keys(n, m, _ptr(keys, ctypes.c_uint64), seed, wmin, wmax,
                         _ptr(off, ctypes.c_int64), _ptr(idx, ctypes.c_int32), _ptr(w, ctypes.c_int32))
    return CSRGraph(n, off, idx, w, name, labels)


def rmat(scale: int, edge_factor: int, a=0.57, b=0.19, c=0.19, seed: int = 22, permute: bool = True,
         wmin: int = 1, wmax: int = 1) -> CSRGraph:
    """R-MAT graph: edge_factor * 2**scale tuples before deduplication."""
    n = 1 << scale
    nt = edge_factor * n
    keys = np.empty(nt, dtype=np.uint64)
    m = _load().gg_rmat_keys(scale, nt, a, b, c, seed, int(permute), _ptr(keys, ctypes.c_uint64))
    if m < 0:
        raise MemoryError("R-MAT generation failed")
    return _from_keys(n, keys, m, seed, wmin, wmax, f"rmat-s{scale}-ef{edge_factor}-seed{seed}")


def grid(rows: int, cols: int, p_del: float = 0.1, p_diag: float = 0.01, wmin: int = 1, wmax: int = 16,
         seed: int = 4096) -> CSRGraph:
    """Road-like lattice with deleted edges, random diagonals and weights in [wmin, wmax]."""
    n = rows * cols
    keys = np.empty(max(1, 3 * n), dtype=np.uint64)
    m = _load().gg_grid_keys(rows, cols, p_del, p_diag, seed, _ptr(keys, ctypes.c_uint64))
    if m < 0:
        raise MemoryError("grid generation failed")
    return _from_keys(n, keys, m, seed, wmin, wmax, f"grid-{rows}x{cols}-seed{seed}")


def sbm(n: int, k: int, p_in: float, p_out: float, seed: int = 1, permute: bool = True, wmin: int = 1,
        wmax: int = 1) -> CSRGraph:
    """Stochastic block model with k near-equal blocks; ``labels`` holds the planted blocks."""
    exp_m = p_in * n * max(n // max(k, 1), 1) / 2 + p_out * n * n / 2
    cap = int(exp_m + 10 * math.sqrt(exp_m + 1) + 1024)
    keys = np.empty(cap, dtype=np.uint64)
    labels = np.empty(n, dtype=np.int32)
    m = _load().gg_sbm_keys(n, k, p_in, p_out, seed, int(permute), _ptr(keys, ctypes.c_uint64), cap,
                            _ptr(labels, ctypes.c_int32))
    if m < 0:
        raise MemoryError("SBM generation overflowed its key buffer")
    return _from_keys(n, keys, m, seed, wmin, wmax, f"sbm-n{n}-k{k}-seed{seed}", labels)


def planted_partition(n_comm: int = 10, comm_size: int = 100, p_in: float = 0.1, p_out: float = 0.002,
                      seed: int = 1) -> CSRGraph:
    """Planted partition: n_comm equal blocks, unit weights, no self-loops."""
    g = sbm(n_comm * comm_size, n_comm, p_in, p_out, seed=seed, permute=True)
    g.name = f"planted-{n_comm}x{comm_size}-seed{seed}"
    return g


def sbm_degree(n: int, k: int, avg_degree: float, ratio: float = 4.0, seed: int = 1, wmin: int = 1,
               wmax: int = 4) -> CSRGraph:
    """SBM parametrised by mean degree and intra:inter degree ratio.

    Intra-block degree d_in = avg*ratio/(1+ratio), inter d_out = avg/(1+ratio);
    p_in = d_in/(s-1) with block size s, p_out = d_out/(n-s); k is reduced until p_in <= 1.
    """
    while k > 1:
        s = n / k
        if avg_degree * ratio / (1 + ratio) / max(s - 1, 1) <= 1.0:
            break
        k -= 1
    s = n / k
    d_in = avg_degree * ratio / (1 + ratio)
    d_out = avg_degree / (1 + ratio)
    p_in = min(1.0, d_in / max(s - 1, 1))
    p_out = min(1.0, d_out / max(n - s, 1)) if k > 1 else 0.0
    g = sbm(n, k, p_in, p_out, seed=seed, permute=True, wmin=wmin, wmax=wmax)
    g.name = f"sbm-n{n}-k{k}-d{avg_degree:.1f}-seed{seed}"
    return g


def erdos(n: int, p: float, seed: int = 7, wmin: int = 1, wmax: int = 1) -> CSRGraph:
    cap = n * (n - 1) // 2 + 1
    keys = np.empty(cap, dtype=np.uint64)
    m = _load().gg_erdos_keys(n, p, seed, _ptr(keys, ctypes.c_uint64), cap)
    return _from_keys(n, keys, m, seed, wmin, wmax, f"erdos-n{n}-p{p}-seed{seed}")


def from_edges(n: int, edges, name: str = "") -> CSRGraph:
    """Build a CSR from (u, v, w) triples; {u,v} becomes two arcs, (u,u,w) one arc.

    Repeated edges are merged by summing their weights.
    """
    acc: dict[tuple[int, int], int] = {}
    for e in edges:
        u, v = int(e[0]), int(e[1])
        w = int(e[2]) if len(e) > 2 else 1
        if w <= 0:
            raise ValueError("weights must be positive")
        a, b = min(u, v), max(u, v)
        acc[(a, b)] = acc.get((a, b), 0) + w
    arcs = []
    for (a, b), w in acc.items():
        arcs.append((a, b, w))
        if a != b:
            arcs.append((b, a, w))
    arcs.sort()
    off = np.zeros(n + 1, dtype=np.int64)
    for a, _, _ in arcs:
        off[a + 1] += 1
    off = np.cumsum(off).astype(np.int64)
    idx = np.array([b for _, b, _ in arcs], dtype=np.int32)
    w = np.array([x for _, _, x in arcs], dtype=np.int64)
    wdt = np.int32 if (w.size == 0 or w.max() < 2**31) else np.int64
    return CSRGraph(n, off, idx, w.astype(wdt), name)


def ring_of_cliques(r: int, k: int) -> CSRGraph:
    """r cliques K_k; clique t's vertex 0 joins clique t+1's vertex 1 by one edge."""
    edges = []
    for t in range(r):
        base = t * k
        for x in range(k):
            for y in range(x + 1, k):
                edges.append((base + x, base + y, 1))
        nxt = ((t + 1) % r) * k
        edges.append((base, nxt + 1, 1))
    g = from_edges(r * k, edges, f"ring-{r}x{k}")
    g.labels = np.repeat(np.arange(r, dtype=np.int32), k)
    return g


def random_small(n: int, p: float, seed: int, wmax: int = 5, self_loops: bool = False) -> CSRGraph:
    """Tiny random weighted graph (numpy RNG seeded by `seed`), optionally with self-loops."""
    rng = np.random.default_rng(seed)
    edges = []
    for u in range(n):
        for v in range(u + 1, n):
            if rng.random() < p:
                edges.append((u, v, int(rng.integers(1, wmax + 1))))
        if self_loops and rng.random() < 0.3:
            edges.append((u, u, int(rng.integers(1, wmax + 1))))
    return from_edges(n, edges, f"small-n{n}-p{p}-seed{seed}")


def to_int32_offsets(g: CSRGraph) -> np.ndarray:
    if g.nnz >= 2**31:
        raise ValueError("graph too large for int32 offsets")
    return g.offsets.astype(np.int32)
