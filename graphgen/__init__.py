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
_DEV_SRC = os.path.join(_HERE, "rmat_device.hip")
_DEV_LIB = os.path.join(_HERE, "libgraphgen_hip.so")
_lib = None
_dev_lib = None


def build(force: bool = True) -> str:
    """Compile libgraphgen.so with gcc (OpenMP for the R-MAT draws)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_device(force: bool = True) -> str:
    """Compile libgraphgen_hip.so (the device R-MAT tuple generator) for gfx950."""
    if force or not os.path.exists(_DEV_LIB):
        tmp = _DEV_LIB + ".tmp"
        hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
        subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-o", tmp, "-x", "hip", _DEV_SRC],
                              stderr=subprocess.DEVNULL if os.environ.get("GG_QUIET") else None)
        os.replace(tmp, _DEV_LIB)
    return _DEV_LIB


def _load_device():
    global _dev_lib
    if _dev_lib is None:
        if not os.path.exists(_DEV_LIB):
            raise RuntimeError(f"{_DEV_LIB} is not built (graphgen.build_device())")
        lib = ctypes.CDLL(_DEV_LIB)
        vp = ctypes.c_void_p
        lib.gg_dev_rmat_hist.restype = ctypes.c_int
        lib.gg_dev_rmat_hist.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_uint64, vp, ctypes.c_int, vp, vp]
        lib.gg_dev_rmat_select.restype = ctypes.c_int
        lib.gg_dev_rmat_select.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_uint64, vp, ctypes.c_int, ctypes.c_int64,
                                           ctypes.c_int64, vp, ctypes.c_int64, vp, vp]
        _dev_lib = lib
    return _dev_lib


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
        lib.gg_perm.restype = None
        lib.gg_perm.argtypes = [ctypes.c_int64, ctypes.c_uint64, i32p]
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


_M64 = (1 << 64) - 1
_ST_RMAT = 1


def _mix64(z: int) -> int:
    z = (z + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


class _TupleKernels:
    """The two tuple kernels of libgraphgen_hip.so on the current stream of
    `device`, called with torch tensors."""

    def __init__(self, device):
        import torch
        self.lib = _load_device()
        self.stream = ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)

    @staticmethod
    def _p(t):
        return ctypes.c_void_p(t.data_ptr() if t is not None else 0)

    def hist(self, scale, nt, a, ab, abc, base, perm, shift, hist):
        if self.lib.gg_dev_rmat_hist(scale, nt, a, ab, abc, base, self._p(perm), shift, self._p(hist), self.stream):
            raise RuntimeError("device R-MAT histogram failed")

    def select(self, scale, nt, a, ab, abc, base, perm, shift, blo, bhi, out, cnt):
        if self.lib.gg_dev_rmat_select(scale, nt, a, ab, abc, base, self._p(perm), shift, blo, bhi, self._p(out),
                                       out.numel(), self._p(cnt), self.stream):
            raise RuntimeError("device R-MAT selection failed")


def rmat_device(scale: int, edge_factor: int, a=0.57, b=0.19, c=0.19, seed: int = 22, permute: bool = True,
                device="cuda", round_cap: int = 1 << 28, kernels=None):
    """R-MAT graph built on the GPU: the same graph as ``rmat`` (unit weights).

    Returns (offsets int64 [n+1], indices int32 [nnz]) as device tensors.  The
    tuples are drawn on the device from the same counter-based stream as the
    host generator; keys are collected in rounds of at most ``round_cap``
    (by ranges of the smaller endpoint), sorted and deduplicated per round,
    then laid out as a symmetric CSR with ascending rows, again in rounds of
    at most ``round_cap`` arcs.  Peak device memory is about
    8 B x unique edges + 4 B x arcs + a few x 8 B x round_cap.
    ``kernels`` replaces the two tuple kernels (hist, select), for tests.
    """
    import torch

    n = 1 << scale
    nt = edge_factor * n
    dev = torch.device(device)
    kern = kernels if kernels is not None else _TupleKernels(dev)
    perm_d = None
    if permute:
        perm = np.empty(n, dtype=np.int32)
        _load().gg_perm(n, seed, _ptr(perm, ctypes.c_int32))
        perm_d = torch.from_numpy(perm).to(dev)
        del perm
    base = _mix64(seed ^ _mix64(_ST_RMAT))
    ab = a + b
    abc = a + b + c
    shift = max(0, scale - 12)
    nbins = 1 << (scale - shift)
    hist = torch.zeros(nbins, dtype=torch.int64, device=dev)
    kern.hist(scale, nt, a, ab, abc, base, perm_d, shift, hist)
    h = hist.cpu().numpy()
    if h.max(initial=0) > round_cap:
        raise RuntimeError("one R-MAT key bin exceeds round_cap; raise round_cap")
    rounds, lo, acc = [], 0, 0
    for bi in range(nbins):
        if acc + h[bi] > round_cap:
            rounds.append((lo, bi))
            lo, acc = bi, 0
        acc += int(h[bi])
    rounds.append((lo, nbins))
    buf = torch.empty(min(round_cap, max(1, int(h.sum()))), dtype=torch.int64, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    uniq = []
    for blo, bhi in rounds:
        expect = int(h[blo:bhi].sum())
        if expect == 0:
            continue
        cnt.zero_()
        kern.select(scale, nt, a, ab, abc, base, perm_d, shift, blo, bhi, buf, cnt)
        k = int(cnt.item())
        if k != expect:
            raise RuntimeError(f"device R-MAT round found {k} keys, histogram said {expect}")
        keys = torch.sort(buf[:k]).values
        uniq.append(torch.unique_consecutive(keys))
        del keys
    del buf, perm_d
    mask = n - 1
    deg = torch.zeros(n, dtype=torch.int64, device=dev)
    for u in uniq:
        deg += torch.bincount(u >> scale, minlength=n)
        deg += torch.bincount(u & mask, minlength=n)
    off = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    off[1:] = torch.cumsum(deg, 0)
    del deg
    nnz = int(off[-1].item())
    idx = torch.empty(nnz, dtype=torch.int32, device=dev)
    offh = off.cpu().numpy()
    r0 = 0
    while r0 < n:
        # rows [r0, r1) with at most round_cap arcs (at least one row)
        r1 = int(np.searchsorted(offh, offh[r0] + round_cap, side="right")) - 1
        r1 = min(n, max(r1, r0 + 1))
        parts = []
        for u in uniq:
            src = u >> scale
            dst = u & mask
            up = u[(src >= r0) & (src < r1)]
            if up.numel():
                parts.append(up)
            sel = (dst >= r0) & (dst < r1)
            low = u[sel]
            if low.numel():
                parts.append(((low & mask) << scale) | (low >> scale))
            del src, dst, sel, up, low
        e0, e1 = int(offh[r0]), int(offh[r1])
        if parts:
            arcs = torch.sort(torch.cat(parts)).values
            if arcs.numel() != e1 - e0:
                raise RuntimeError("device R-MAT CSR round size mismatch")
            idx[e0:e1] = (arcs & mask).to(torch.int32)
            del arcs
        elif e1 != e0:
            raise RuntimeError("device R-MAT CSR round size mismatch")
        del parts
        r0 = r1
    del uniq
    return off, idx


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


def sbm_batch_specs(count: int, nmax: int = 200_000, nmin: int = 200, seed: int = 4):
    """Recipe of the batched SBM workload: for graph k, (n, communities,
    average degree, seed) with n log-uniform in [nmin, nmax], 4 to 64
    communities, average degree uniform in [8, 32] and seed 4000 + k (drawn in
    order from numpy's default generator seeded with `seed`)."""
    rng = np.random.default_rng(seed)
    specs = []
    for k in range(count):
        n = int(np.exp(rng.uniform(np.log(nmin), np.log(nmax))))
        specs.append((n, int(rng.integers(4, 65)), float(rng.uniform(8, 32)), 4000 + k))
    return specs


def sbm_batch_graph(spec) -> CSRGraph:
    """One graph of sbm_batch_specs: intra/inter degree ratio 4, weights in [1, 4]."""
    n, k, d, s = spec
    return sbm_degree(n, k, d, seed=s, wmin=1, wmax=4)


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
