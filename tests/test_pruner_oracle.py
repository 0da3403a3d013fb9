"""Pins of the oracle's learned move-pruner (features, MLP, sweep guard,
training samples) and of the float64 training reference.

Every expected value here is derived independently of the oracle's C code:
features are recomputed from the per-iteration membership traces with
Python integers, gains by the definition of Eq. (2), the MLP in float64
numpy, gradients by central finite differences.
"""
import math

import numpy as np
import pytest

import graphgen as gg
import oracle
import oracle.mlp as mlp

f32 = np.float32


def mitchell(x: int) -> np.float32:
    e = x.bit_length() - 1
    p = 1 << e
    return f32(e) + f32(x - p) / f32(p)


def py_features(deg, K, own, adv, nm, moved_last, p, t):
    return np.array([mitchell(1 + deg) / f32(16), f32(own) / f32(K) if K else f32(0),
                     mitchell(1 + nm) / f32(16), f32(nm) / f32(deg) if deg else f32(0),
                     f32(1.0 if moved_last else 0.0), f32(p) / f32(10), f32(t) / f32(20),
                     f32(adv) / f32(K) if K else f32(0)], dtype=np.float32)


def rand_weights(seed, scale=0.4):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(mlp.N_PARAMS) * scale).astype(np.float32)


# --------------------------------------------------------------- features

def test_mitchell_log2_error_bound():
    """Mitchell's approximation never exceeds log2 and errs by < 0.0861."""
    for x in list(range(1, 5000)) + [2 ** k + r for k in range(13, 40) for r in (-1, 0, 1, 12345)]:
        f = oracle.features(x - 1, 1, 0, 0, 0, False, 0, 1)[0] * 16.0
        err = math.log2(x) - float(f)
        assert -1e-5 <= err < 0.0861, (x, err)
        if x & (x - 1) == 0:
            assert float(f) == x.bit_length() - 1


def test_features_closed_form():
    f = oracle.features(7, 10, 4, -2, 3, True, 2, 5)
    expect = [3 / 16, 0.4, 2 / 16, 3 / 7, 1.0, 0.2, 0.25, -0.2]
    assert np.array_equal(f, np.array(expect, dtype=np.float32))
    f = oracle.features(2, 0, 0, 0, 0, False, 0, 1)
    assert np.array_equal(f, np.array([1.5 / 16, 0, 0, 0, 0, 0, 0.05, 0], dtype=np.float32))
    big = oracle.features(3, 3 << 40, 1 << 40, 1 << 41, 2, False, 9, 19)
    assert np.array_equal(big, py_features(3, 3 << 40, 1 << 40, 1 << 41, 2, False, 9, 19))


# --------------------------------------------------------------------- MLP

def test_mlp_logit_matches_float64():
    rng = np.random.default_rng(1)
    for s in range(4):
        w = rand_weights(s)
        X = rng.random((64, 8)).astype(np.float32) * 2 - 0.5
        z32 = oracle.mlp_logit(w, X)
        z64, _ = mlp.forward(w.astype(np.float64), X.astype(np.float64))
        assert np.allclose(z32, z64, rtol=1e-5, atol=1e-5)


def test_mlp_special_cases():
    w = np.zeros(mlp.N_PARAMS, dtype=np.float32)
    w[-1] = -1.25  # b3 only
    assert oracle.mlp_logit(w, np.ones((1, 8)))[0] == f32(-1.25)
    # single path x3 -> h1[0] -> h2[0] -> z, ReLU passes positives only
    w = np.zeros(mlp.N_PARAMS, dtype=np.float32)
    w[0 * 8 + 3] = 1.0                 # W1[0][3]
    w[256 + 32 + 0 * 32 + 0] = 2.0     # W2[0][0]
    w[256 + 32 + 1024 + 32 + 0] = 3.0  # w3[0]
    x = np.zeros((2, 8), dtype=np.float32)
    x[0, 3], x[1, 3] = 0.5, -0.5
    assert list(oracle.mlp_logit(w, x)) == [3.0, 0.0]
    assert list(mlp.forward(w, x)[0]) == [3.0, 0.0]


def test_loss_grad_finite_differences():
    rng = np.random.default_rng(2)
    w = rand_weights(7).astype(np.float64)
    X = rng.random((40, 8))
    y = (rng.random(40) < 0.4).astype(np.float64)
    L, g = mlp.loss_grad(w, X, y, 2.5)
    assert L == pytest.approx(mlp.loss(w, X, y, 2.5), rel=1e-12)
    for k in list(range(0, mlp.N_PARAMS, 37)) + [mlp.N_PARAMS - 1]:
        e = 1e-6
        wp, wm = w.copy(), w.copy()
        wp[k] += e
        wm[k] -= e
        fd = (mlp.loss(wp, X, y, 2.5) - mlp.loss(wm, X, y, 2.5)) / (2 * e)
        assert fd == pytest.approx(g[k], abs=1e-7, rel=1e-5), k


def test_loss_zero_weights_closed_form():
    y = np.array([1, 0, 0, 1, 0], dtype=np.float64)
    L, g = mlp.loss_grad(np.zeros(mlp.N_PARAMS), np.ones((5, 8)), y, 3.0)
    assert L == pytest.approx(math.log(2) * (2 * 3.0 + 3) / 5)
    # only b3 has a gradient: mean of c * (1/2 - y)
    assert g[-1] == pytest.approx((2 * 3.0 * -0.5 + 3 * 0.5) / 5)
    assert np.count_nonzero(g[:-1]) == 0


def test_adam_first_step_is_signed_lr():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(w[:3], -0.01 * np.sign(g[:3]), rtol=1e-4)
    assert w[3] == 0.0


@pytest.mark.parametrize("steps", [2, 3, 10, 100])
def test_adam_constant_gradient_closed_form(steps):
    """With the same gradient g at every step, both bias-corrected moments
    equal g and g^2 exactly (m_k = (1 - beta1^k) g, v_k = (1 - beta2^k) g^2),
    so every step moves w by lr * g / (|g| + eps): w_k = w_0 - k lr g / (|g| + eps).
    A wrong bias-correction exponent or moment recurrence breaks this from
    step 2 on."""
    g = np.array([0.3, -2.0, 1e-3, 5e-7, 0.0])
    lr = 0.01
    w, m, v = np.full(5, 0.25), np.zeros(5), np.zeros(5)
    for k in range(1, steps + 1):
        w, m, v = mlp.adam_step(w, g, m, v, k, lr)
    expect = 0.25 - steps * lr * g / (np.abs(g) + mlp.EPS)
    assert np.allclose(w, expect, rtol=1e-12, atol=1e-14)


def test_adam_two_steps_varying_gradient_closed_form():
    """Two steps with gradients a then b: m_hat = (beta1 a + b) / (1 + beta1)
    and v_hat = (beta2 a^2 + b^2) / (1 + beta2) (the moment recurrences
    unrolled by hand), after a first step of -lr * sign(a)."""
    a = np.array([0.5, -1.0, 2.0, 1e-2])
    b = np.array([-0.25, -3.0, 0.5, 1e-2])
    lr, b1, b2 = 0.03, 0.9, 0.999
    w, m, v = mlp.adam_step(np.zeros(4), a, np.zeros(4), np.zeros(4), 1, lr)
    w, m, v = mlp.adam_step(w, b, m, v, 2, lr)
    w1 = -lr * a / (np.abs(a) + mlp.EPS)
    mh = (b1 * a + b) / (1 + b1)
    vh = (b2 * a * a + b * b) / (1 + b2)
    assert np.allclose(w, w1 - lr * mh / (np.sqrt(vh) + mlp.EPS), rtol=1e-12, atol=1e-15)


def test_glorot_init_bounds():
    w = mlp.glorot_init(11)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(w)
    for arr, fi, fo in ((W1, 8, 32), (W2, 32, 32), (w3, 32, 1)):
        lim = math.sqrt(6 / (fi + fo))
        assert np.abs(arr).max() <= lim
        assert abs(arr.std() - lim / math.sqrt(3)) < 0.2 * lim
    assert not b1.any() and not b2.any() and b3 == 0
    assert np.array_equal(w, mlp.glorot_init(11)) and not np.array_equal(w, mlp.glorot_init(12))


def test_splitmix64_published_values():
    # first outputs of SplitMix64 seeded with 0 (reference sequence of the generator)
    assert mlp.splitmix64(0) == 0xE220A8397B1DCDAF
    assert mlp.splitmix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4


# ------------------------------------------------- replay of the features

def _level_graphs(g, res):
    levels = [(g.offsets.astype(np.int64), g.indices.astype(np.int64), g.weights.astype(np.int64))]
    for gr in res.graphs:
        levels.append((gr["offsets"], gr["indices"].astype(np.int64), gr["weights"]))
    return levels


def _scan(off, idx, w, C, v):
    acc = {}
    for e in range(off[v], off[v + 1]):
        j = int(idx[e])
        if j == v:
            continue
        acc[int(C[j])] = acc.get(int(C[j]), 0) + int(w[e])
    return acc


def _best(off, idx, w, C, S, K, W, v):
    acc = _scan(off, idx, w, C, v)
    c = int(C[v])
    kic = acc.get(c, 0)
    best = None
    for d, kd in acc.items():
        if d == c:
            continue
        gain = W * (kd - kic) - int(K[v]) * (int(S[d]) - int(S[c]) + int(K[v]))
        if best is None or gain > best[0] or (gain == best[0] and d < best[1]):
            best = (gain, d, kd)
    return kic, best


@pytest.mark.parametrize("make", [lambda: gg.planted_partition(seed=3),
                                  lambda: gg.random_small(80, 0.08, 5, wmax=4, self_loops=True)],
                         ids=["planted", "small_loops"])
def test_sync_samples_replay(make):
    """SYNC, flag pruning, every sample recorded: each sample's features and
    label equal a recomputation from the iteration traces."""
    g = make()
    res = oracle.louvain(g, oracle.Params(mode=oracle.SYNC, sample_per_mille=1000), trace=True, samples=True)
    levels = _level_graphs(g, res)
    W = int(g.weights.astype(np.int64).sum())
    got = {(p, t, v): (f, lab) for p, t, v, f, lab in res.samples}
    expected = 0
    for p in range(res.passes):
        off, idx, w = levels[p]
        n = len(off) - 1
        K = np.array([int(w[off[v]:off[v + 1]].sum()) for v in range(n)], dtype=object)
        recs = [r for r in res.iters if r["pass_"] == p]
        own = [0] * n
        adv = [0] * n
        prevC, prevS = np.arange(n), K.copy()
        moved_prev = np.zeros(n, dtype=bool)
        queue = list(range(n))
        for t, r in enumerate(recs):
            nm = [sum(1 for e in range(off[v], off[v + 1]) if idx[e] != v and moved_prev[idx[e]]) for v in range(n)]
            newC = r["cprime"]
            for v in queue:
                if t > 0:
                    deg = int(off[v + 1] - off[v])
                    f = py_features(deg, int(K[v]), own[v], adv[v], nm[v], bool(moved_prev[v]), p, t)
                    key = (p, t, v)
                    assert key in got, key
                    assert np.array_equal(got[key][0], f), (key, got[key][0], f)
                    assert got[key][1] == int(newC[v] != prevC[v]), key
                    expected += 1
                kic, best = _best(off, idx, w, prevC, prevS, K, W, v)
                own[v] = kic
                adv[v] = (best[2] if best else 0) - kic
            moved = newC != prevC
            queue = sorted({int(idx[e]) for v in np.flatnonzero(moved) for e in range(off[v], off[v + 1])
                            if idx[e] != v})
            moved_prev = moved
            prevC, prevS = newC, r["sigma"]
    assert expected == len(res.samples) and expected > 100


def test_async_sample_labels_match_trace():
    g = gg.planted_partition(seed=4)
    res = oracle.louvain(g, oracle.Params(mode=oracle.ASYNC, sample_per_mille=1000), trace=True, samples=True)
    by = {(r["pass_"], r["iter"]): r["cprime"] for r in res.iters}
    assert res.samples
    for p, t, v, f, lab in res.samples:
        assert lab == int(by[(p, t)][v] != by[(p, t - 1)][v])
        assert 0 <= f[1] <= 1 and -1 <= f[7] <= 1 and 0 <= f[3] <= 1 and f[4] in (0, 1)


def test_sample_rate():
    g = gg.planted_partition(seed=5)
    full = oracle.louvain(g, oracle.Params(mode=oracle.SYNC, sample_per_mille=1000), samples=True)
    part = oracle.louvain(g, oracle.Params(mode=oracle.SYNC, sample_per_mille=250), samples=True)
    keys = {(p, t, v) for p, t, v, _, _ in full.samples}
    pk = {(p, t, v) for p, t, v, _, _ in part.samples}
    assert pk <= keys
    assert 0.18 < len(pk) / len(keys) < 0.32


# ----------------------------------------------------------- sweep guard

def _no_positive_gain(off, idx, w, C, S, K, W):
    for v in range(len(off) - 1):
        _, best = _best(off, idx, w, C, S, K, W, v)
        if best is not None and best[0] > 0:
            return v
    return None


@pytest.mark.parametrize("mode", [oracle.SYNC, oracle.ASYNC])
@pytest.mark.parametrize("theta", [0.0, 0.35, 0.5, 0.65, 1.0])
def test_strict_guard_leaves_no_positive_move(mode, theta):
    """guard_tolerance = 0: a pass that ends before max_iterations ends in a
    state where no vertex has a move of positive gain."""
    g = gg.planted_partition(seed=6)
    w8 = rand_weights(3)
    res = oracle.louvain(g, oracle.Params(mode=mode, prune=oracle.PRUNE_LEARNED, mlp=w8, threshold=theta,
                                          guard_tolerance=0, max_iterations=50), trace=True)
    levels = _level_graphs(g, res)
    W = int(g.weights.astype(np.int64).sum())
    checked = 0
    for p in range(res.passes):
        recs = [r for r in res.iters if r["pass_"] == p]
        if len(recs) >= 50:
            continue
        off, idx, w = levels[p]
        n = len(off) - 1
        K = [int(w[off[v]:off[v + 1]].sum()) for v in range(n)]
        assert recs[-1]["moves"] == 0
        assert _no_positive_gain(off, idx, w, recs[-1]["cprime"], recs[-1]["sigma"], K, W) is None
        checked += 1
    assert checked >= 1 and res.sweeps >= res.passes


@pytest.mark.parametrize("mode", [oracle.SYNC, oracle.ASYNC])
def test_drop_all_equals_no_pruning(mode):
    """threshold 1 skips every flagged vertex, so every iteration is a sweep:
    with the tolerance exit this is exactly the unpruned method."""
    g = gg.rmat(9, 8, seed=2, wmax=3)
    w8 = rand_weights(4)
    a = oracle.louvain(g, oracle.Params(mode=mode, prune=oracle.PRUNE_LEARNED, mlp=w8, threshold=1.0,
                                        guard_tolerance=1), trace=True)
    b = oracle.louvain(g, oracle.Params(mode=mode, prune=oracle.PRUNE_NONE), trace=True)
    assert np.array_equal(a.membership, b.membership)
    assert len(a.iters) == len(b.iters) and a.sweeps == len(a.iters)
    for x, y in zip(a.iters, b.iters):
        assert np.array_equal(x["cprime"], y["cprime"]) and x["gain"] == y["gain"]


@pytest.mark.parametrize("mode", [oracle.SYNC, oracle.ASYNC])
def test_keep_all_follows_flag_pruning_then_sweeps(mode):
    """threshold 0 keeps every flagged vertex: the first pass repeats flag
    pruning up to its convergence, then runs the guard sweep."""
    g = gg.planted_partition(seed=7)
    w8 = rand_weights(5)
    a = oracle.louvain(g, oracle.Params(mode=mode, prune=oracle.PRUNE_LEARNED, mlp=w8, threshold=0.0,
                                        max_passes=1), trace=True)
    b = oracle.louvain(g, oracle.Params(mode=mode, prune=oracle.PRUNE_FLAGS, max_passes=1), trace=True)
    nb = len(b.iters)
    assert a.pruned == 0 and len(a.iters) > nb
    for x, y in zip(a.iters[:nb], b.iters):
        assert np.array_equal(x["cprime"], y["cprime"]) and x["gain"] == y["gain"]


def test_learned_needs_weights():
    with pytest.raises(RuntimeError):
        oracle.louvain(gg.planted_partition(seed=1), oracle.Params(prune=oracle.PRUNE_LEARNED))


def test_sample_selection_hash():
    """Recorded samples are exactly the keys whose SplitMix64 value mod 1000
    falls below the rate."""
    g = gg.planted_partition(seed=5)
    full = oracle.louvain(g, oracle.Params(mode=oracle.SYNC, sample_per_mille=1000), samples=True)
    part = oracle.louvain(g, oracle.Params(mode=oracle.SYNC, sample_per_mille=250), samples=True)
    sel = {(p, t, v) for p, t, v, _, _ in full.samples
           if mlp.splitmix64(v + ((p * 65536 + t) << 32)) % 1000 < 250}
    assert sel == {(p, t, v) for p, t, v, _, _ in part.samples}


def _converged(S, W, p, tol_num=1, tol_den=100, drop=10):
    return 2 * S * tol_den * drop ** p <= tol_num * W * W


def replay_sync_learned(g, w8, theta, guard, **kw):
    """Replays a SYNC learned-pruner run from its traces in Python and checks
    the queue of every iteration (sweep, or flagged and kept by the float64
    MLP), the recorded samples, the pruned and sweep counts and the end of
    every pass.  Returns (result, number of sweeps whose evaluated vertices
    had positive gains that Pick-Less blocked entirely)."""
    P = oracle.Params(mode=oracle.SYNC, prune=oracle.PRUNE_LEARNED, mlp=w8, threshold=theta,
                      guard_tolerance=guard, sample_per_mille=1000, **kw)
    res = oracle.louvain(g, P, trace=True, samples=True)
    levels = _level_graphs(g, res)
    W = int(g.weights.astype(np.int64).sum())
    zt = math.log(theta / (1 - theta)) if 0 < theta < 1 else (-math.inf if theta <= 0 else math.inf)
    got = {(p, t, v): (f, lab) for p, t, v, f, lab in res.samples}
    seen, pruned, sweeps, ambiguous, blocked = 0, 0, 0, 0, 0
    for p in range(res.passes):
        off, idx, w = levels[p]
        n = len(off) - 1
        K = [int(w[off[v]:off[v + 1]].sum()) for v in range(n)]
        recs = [r for r in res.iters if r["pass_"] == p]
        own, adv = [0] * n, [0] * n
        prevC, prevS = np.arange(n), list(K)
        moved_prev = np.zeros(n, dtype=bool)
        flagged = list(range(n))
        sweep_next = True
        ended = False
        for t, r in enumerate(recs):
            assert not ended
            nm = [sum(1 for e in range(off[v], off[v + 1]) if idx[e] != v and moved_prev[idx[e]]) for v in range(n)]
            feats = {}
            sweep = sweep_next
            if not sweep:
                kept = []
                for v in flagged:
                    f = py_features(int(off[v + 1] - off[v]), K[v], own[v], adv[v], nm[v], bool(moved_prev[v]), p, t)
                    z = float(mlp.forward(w8.astype(np.float64), f.astype(np.float64))[0][0])
                    ambiguous += abs(z - zt) < 1e-4
                    if z >= zt:
                        kept.append(v)
                        feats[v] = f
                if kept:
                    pruned += len(flagged) - len(kept)
                else:
                    sweep = True
            sweeps += sweep
            queue = list(range(n)) if sweep else kept
            newC = r["cprime"]
            moved = newC != prevC
            assert set(np.flatnonzero(moved)) <= set(queue)
            positive = 0
            for v in queue:
                if not sweep:
                    key = (p, t, v)
                    assert np.array_equal(got[key][0], feats[v]) and got[key][1] == int(moved[v]), key
                    seen += 1
                kic, best = _best(off, idx, w, prevC, prevS, K, W, v)
                own[v] = kic
                adv[v] = (best[2] if best else 0) - kic
                positive += best is not None and best[0] > 0
            conv = _converged(r["gain"], W, p)
            blocked += sweep and positive > 0 and r["moves"] == 0
            if sweep and (conv if guard else positive == 0):
                ended = True
            sweep_next = (not sweep) and conv
            flagged = sorted({int(idx[e]) for v in np.flatnonzero(moved) for e in range(off[v], off[v + 1])
                              if idx[e] != v})
            moved_prev = moved
            prevC, prevS = newC, r["sigma"]
        assert ended or len(recs) == P.max_iterations
    assert ambiguous == 0
    assert seen == len(res.samples) and pruned == res.pruned and sweeps == res.sweeps
    return res, blocked


@pytest.mark.parametrize("guard", [0, 1])
@pytest.mark.parametrize("theta", [0.35, 0.5, 0.65])
def test_sync_learned_replay(theta, guard):
    res, _ = replay_sync_learned(gg.planted_partition(seed=6), rand_weights(3), theta, guard)
    assert (res.pruned > 0) == (theta >= 0.5)  # these weights score every flagged vertex near 0.4-0.5


def test_strict_guard_counts_pick_less_blocked_gains():
    """A sweep in a Pick-Less iteration can move nothing although some vertex
    has a positive gain; the strict guard must not end the pass there."""
    g = gg.random_small(12, 0.3, 32, wmax=3)
    res, blocked = replay_sync_learned(g, rand_weights(3), 1.0, 0, max_passes=1)
    assert blocked >= 1
