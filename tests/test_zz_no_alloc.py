"""louvain_pruner_train_noalloc (static device scratch, no allocation)
against louvain_pruner_train (caller scratch), through the C ABI.

Mini-batches of at most 64 samples are summed by a single wave, so both
entry points add every gradient and loss term in the same order and their
weights and losses must agree bit for bit.  Two calls run back to back, the
second on a smaller sample set and batch, so the second call starts from the
scratch contents the first one left behind.
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lv = pytest.importorskip("paper_2501_19004_amd")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return "cuda:0"


def samples(count, seed):
    rng = np.random.default_rng(seed)
    s = np.empty((count, lv.SAMPLE_FLOATS), dtype=np.float32)
    s[:, :8] = rng.uniform(0.0, 1.0, size=(count, 8))
    s[:, 8] = (rng.uniform(size=count) < 0.4).astype(np.float32)
    return torch.from_numpy(s).to(dev())


def train_both(count, batch, steps, seed):
    S = samples(count, seed)
    w0 = lv.pruner_init(seed, dev())
    wa, wb = w0.clone(), w0.clone()
    stream = torch.cuda.current_stream().cuda_stream
    scratch = torch.empty(lv.louvain_pruner_scratch_floats(batch), dtype=torch.float32, device=dev())
    la = lv.louvain_pruner_train(wa.data_ptr(), S.data_ptr(), count, steps, batch, 3e-3, 1.5, seed,
                                 scratch.data_ptr(), stream)
    lb = lv.louvain_pruner_train_noalloc(wb.data_ptr(), S.data_ptr(), count, steps, batch, 3e-3, 1.5, seed, stream)
    torch.cuda.synchronize()
    return wa, wb, la, lb, w0


def test_noalloc_train_equals_train_twice():
    print("[case] noalloc train: 5000 samples, batch 64, 40 steps; then 700 samples, batch 32, 12 steps", flush=True)
    for count, batch, steps, seed in ((5000, 64, 40, 11), (700, 32, 12, 12)):
        wa, wb, la, lb, w0 = train_both(count, batch, steps, seed)
        assert not torch.equal(wa, w0)  # training did move the weights
        assert torch.equal(wa, wb), (count, (wa - wb).abs().max().item())
        assert la == lb, (count, la, lb)


def test_noalloc_rejects_bad_arguments():
    lib = lv.load_library()
    loss = ctypes.c_double()
    assert lib.louvain_pruner_train_noalloc(None, None, 0, 1, 1, 1e-3, 1.0, 0, ctypes.byref(loss),
                                            None) == lv.LOUVAIN_ERR_INVALID
    w = lv.pruner_init(1, dev())
    S = samples(100, 1)
    assert lib.louvain_pruner_train_noalloc(w.data_ptr(), S.data_ptr(), 100, 1, 0, 1e-3, 1.0, 0, ctypes.byref(loss),
                                            None) == lv.LOUVAIN_ERR_INVALID
