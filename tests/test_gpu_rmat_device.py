"""The device R-MAT generator builds the same graph as the host generator.

The full-size R-MAT workload (scale 27, edge factor 28) is generated on the
GPU; it must be the graph the host generator defines.  Here both build
smaller instances (several key rounds and CSR rounds forced by a small round
size) and the CSR arrays must be identical.
"""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return "cuda:0"


@pytest.mark.parametrize("scale,ef,seed,permute,cap", [
    (10, 8, 3, True, 1 << 20),
    (14, 16, 22, True, 1 << 14),
    (13, 4, 9, False, 1 << 12),
    (16, 28, 27, True, 1 << 18),
])
def test_device_rmat_equals_host(scale, ef, seed, permute, cap):
    d = dev()
    print(f"[case] device R-MAT scale {scale} ef {ef} seed {seed} permute {permute} cap {cap}", flush=True)
    off, idx = gg.rmat_device(scale, ef, seed=seed, permute=permute, device=d, round_cap=cap)
    g = gg.rmat(scale, ef, seed=seed, permute=permute)
    assert np.array_equal(off.cpu().numpy(), g.offsets)
    assert np.array_equal(idx.cpu().numpy(), g.indices)
