"""Generator checks: symmetric CSR, sorted rows, no self-loops or duplicates,
weights in range, seeded determinism, and the expected sizes of each workload."""
import numpy as np
import pytest

import graphgen as gg


def check_csr(g, allow_loops=False):
    off, idx, w = g.offsets, g.indices, g.weights
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == idx.size == w.size
    assert idx.size == 0 or (idx.min() >= 0 and idx.max() < g.n)
    assert w.size == 0 or w.min() > 0
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(off))
    if not allow_loops:
        assert not np.any(src == idx)
    for i in range(min(g.n, 2000)):
        row = idx[off[i]:off[i + 1]]
        assert np.all(np.diff(row) > 0)
    fwd = src * g.n + idx
    rev = idx.astype(np.int64) * g.n + src
    o1, o2 = np.argsort(fwd), np.argsort(rev)
    assert np.array_equal(fwd[o1], rev[o2]), "symmetric"
    assert np.array_equal(w[o1], w[o2]), "symmetric weights"


@pytest.mark.parametrize("make", [
    lambda: gg.planted_partition(seed=1),
    lambda: gg.rmat(12, 16, seed=3),
    lambda: gg.grid(40, 50, seed=2),
    lambda: gg.sbm_degree(3000, 16, 12.0, seed=4),
    lambda: gg.erdos(80, 0.1, seed=1, wmax=7),
])
def test_generators_make_valid_symmetric_csr(make):
    check_csr(make())


def test_generators_are_seeded():
    a, b, c = gg.rmat(11, 8, seed=5), gg.rmat(11, 8, seed=5), gg.rmat(11, 8, seed=6)
    assert np.array_equal(a.indices, b.indices) and np.array_equal(a.offsets, b.offsets)
    assert not (a.nnz == c.nnz and np.array_equal(a.indices, c.indices))


def test_planted_partition_size():
    g = gg.planted_partition(seed=1)
    # expected undirected edges: 10*C(100,2)*0.1 + C(10,2)*100^2*0.002 = 4950 + 900
    assert abs(g.edges_undirected() - 5850) < 5 * np.sqrt(5850)
    assert np.bincount(g.labels).tolist() == [100] * 10
    assert g.weights.max() == 1


def test_grid_shape_and_weights():
    g = gg.grid(64, 64, seed=9)
    full = 2 * 64 * 63
    e = g.edges_undirected()
    expect = 0.9 * full + 0.01 * 63 * 63
    assert abs(e - expect) < 5 * np.sqrt(expect)
    assert g.weights.min() >= 1 and g.weights.max() <= 16
    assert np.diff(g.offsets).max() <= 6


def test_rmat_skew():
    g = gg.rmat(14, 16, seed=1)
    d = np.diff(g.offsets)
    assert g.n == 1 << 14
    assert d.max() > 20 * d.mean()           # heavy tail
    assert (d == 0).sum() > 0.1 * g.n        # many isolated vertices


def test_sbm_degree_parameters():
    g = gg.sbm_degree(20000, 32, 16.0, ratio=4.0, seed=3, wmin=1, wmax=4)
    assert abs(g.nnz / g.n - 16.0) < 0.5
    same = g.labels[np.repeat(np.arange(g.n), np.diff(g.offsets))] == g.labels[g.indices]
    assert abs(same.mean() - 0.8) < 0.02      # intra:inter = 4:1
    assert g.weights.min() >= 1 and g.weights.max() <= 4


class _NumpyTupleKernels:
    """The device generator's two tuple kernels redone in numpy on the host:
    the R-MAT draw of every tuple from the published SplitMix64 stream."""

    @staticmethod
    def _keys(scale, nt, a, ab, abc, base, perm):
        def mix(z):
            z = z + np.uint64(0x9E3779B97F4A7C15)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            return z ^ (z >> np.uint64(31))
        k = np.arange(nt, dtype=np.uint64)
        u = np.zeros(nt, np.int64)
        v = np.zeros(nt, np.int64)
        with np.errstate(over="ignore"):
            for lvl in range(scale):
                r = (mix(np.uint64(base) + k * np.uint64(scale) + np.uint64(lvl)) >> np.uint64(11)).astype(np.float64)
                r *= 1.0 / 9007199254740992.0
                u = (u << 1) | (r >= ab)
                v = (v << 1) | (((r >= a) & (r < ab)) | (r >= abc))
        if perm is not None:
            p = perm.cpu().numpy().astype(np.int64)
            u, v = p[u], p[v]
        keep = u != v
        lo, hi = np.minimum(u, v)[keep], np.maximum(u, v)[keep]
        return lo, (lo << scale) | hi

    def hist(self, scale, nt, a, ab, abc, base, perm, shift, hist):
        import torch
        lo, _ = self._keys(scale, nt, a, ab, abc, base, perm)
        hist.copy_(torch.from_numpy(np.bincount(lo >> shift, minlength=hist.numel())))

    def select(self, scale, nt, a, ab, abc, base, perm, shift, blo, bhi, out, cnt):
        import torch
        lo, keys = self._keys(scale, nt, a, ab, abc, base, perm)
        b = lo >> shift
        sel = keys[(b >= blo) & (b < bhi)]
        np.random.default_rng(0).shuffle(sel)  # the device appends in no fixed order
        k = min(out.numel(), sel.size)
        out[:k] = torch.from_numpy(sel[:k])
        cnt[0] = sel.size


@pytest.mark.parametrize("scale,ef,seed,permute,cap", [(10, 8, 3, True, 1 << 20), (12, 16, 22, True, 1 << 11),
                                                       (11, 4, 9, False, 1 << 10)])
def test_device_rmat_rounds_and_layout_on_host(scale, ef, seed, permute, cap):
    """The device generator's host-side logic (key rounds, deduplication,
    symmetric CSR rounds) with its two kernels replaced by a numpy draw of
    the same tuples equals the host generator; small rounds force several."""
    torch = pytest.importorskip("torch")
    off, idx = gg.rmat_device(scale, ef, seed=seed, permute=permute, device="cpu", round_cap=cap,
                              kernels=_NumpyTupleKernels())
    g = gg.rmat(scale, ef, seed=seed, permute=permute)
    assert np.array_equal(off.numpy(), g.offsets)
    assert np.array_equal(idx.numpy(), g.indices)
