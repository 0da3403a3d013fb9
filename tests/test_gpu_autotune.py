"""Degree-bucket autotuner: it keeps one of the candidate threshold sets when
it beats the handle's own thresholds by more than their run-to-run spread
without losing modularity, and later runs use it.  SYNC results do not depend on the
thresholds, so a tuned SYNC handle must still equal the oracle; a tuned
ASYNC handle must still meet the modularity bound."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lv = pytest.importorskip("paper_2501_19004_amd")

CANDIDATES = [[0] * 5, [4, 16, 64, 256, 2048], [-1, -1, -1, -1, 4096], [2, 8, 16, 64, 128]]


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return "cuda:0"


def test_autotune_sync_keeps_oracle_result():
    g = gg.rmat(12, 16, seed=4, wmax=7)
    off, idx, w = lv.graph_tensors(g, dev())
    L = lv.Louvain(off, idx, w, mode=lv.SYNC)
    best, ms = L.autotune(CANDIDATES, reps=3)
    assert -1 <= best < len(CANDIDATES) and all(x > 0 for x in ms)
    # SYNC: every candidate has the same modularity, so the kept one is the fastest
    assert best == -1 or ms[best] == min(ms)
    L.run()
    memb = L.membership().cpu().numpy()
    q, num, den = L.modularity()
    L.close()
    g.weights = g.weights.astype(np.int64)
    ref = oracle.louvain(g, oracle.Params(mode=oracle.SYNC))
    assert np.array_equal(memb, ref.membership)
    assert (num, den) == oracle.modularity_parts(g, memb)


def test_autotune_async_quality():
    g = gg.rmat(14, 16, seed=5)
    off, idx, w = lv.graph_tensors(g, dev())
    L = lv.Louvain(off, idx, w, mode=lv.ASYNC)
    best, ms = L.autotune(CANDIDATES, reps=3)
    L.run()
    memb = L.membership().cpu().numpy()
    q, num, den = L.modularity()
    L.close()
    g.weights = g.weights.astype(np.int64)
    assert (num, den) == oracle.modularity_parts(g, memb)
    qo = oracle.modularity(g, oracle.louvain(g).membership)
    print(f"autotune picked {best} ({ms}); Q_gpu - Q_oracle = {q - qo:+.5f}")
    assert q >= qo - 0.002
