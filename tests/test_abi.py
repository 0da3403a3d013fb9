"""Host-side checks of the C ABI: the library loads, exports every entry point
that include/louvain.h declares, and rejects bad arguments before touching a
GPU.  No compute call is made here."""
import ctypes
import os
import re

import pytest

import paper_2501_19004_amd as lv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "louvain.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(louvain_[a-z_]+)\s*\(", text)) - {"louvain_iter_fn", "louvain_pass_fn"})


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lv.LIB_PATH):
        pytest.skip("library not built")
    return lv.load_library()


def test_library_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(lv.EXPORTED) == syms


def test_params_default_are_the_papers(lib):
    p = lv.louvain_params_default()
    assert (p.max_iterations, p.max_passes, p.tol_num, p.tol_den, p.tol_drop) == (20, 10, 1, 100, 10)
    assert (p.agg_num, p.agg_den, p.pick_less, p.mode, p.pruner) == (4, 5, 4, lv.ASYNC, lv.PRUNE_FLAGS)


STRUCTS = {"louvain_graph": "LouvainGraph", "louvain_params": "LouvainParams", "louvain_stats": "LouvainStats",
           "louvain_kernel_stat": "LouvainKernelStat"}


def test_struct_layouts_match_header(lib, tmp_path):
    """Every ctypes field sits at the offset the C compiler gives it in
    include/louvain.h, and every struct has the header's size."""
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "louvain.h"', "int main(void) {"]
    for cname, pname in STRUCTS.items():
        cls = getattr(lv, pname)
        lines.append(f'printf("{pname} size %zu\\n", sizeof({cname}));')
        for f in cls._fields_:
            lines.append(f'printf("{pname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, pname in STRUCTS.items():
        cls = getattr(lv, pname)
        assert got[(pname, "size")] == ctypes.sizeof(cls), pname
        for f in cls._fields_:
            assert got[(pname, f[0])] == getattr(cls, f[0]).offset, (pname, f[0])


def test_learned_entry_points_reject_bad_arguments(lib):
    assert lib.louvain_collect_samples(None, None, 0, 0) == lv.LOUVAIN_ERR_INVALID
    assert lib.louvain_sample_count(None, None) == lv.LOUVAIN_ERR_INVALID
    assert lib.louvain_pruner_init(None, 1, None) == lv.LOUVAIN_ERR_INVALID
    assert lib.louvain_pruner_predict(None, None, -1, None, None) == lv.LOUVAIN_ERR_INVALID
    assert lib.louvain_pruner_loss_grad(None, None, 5, 1.0, None, None, None) == lv.LOUVAIN_ERR_INVALID
    assert lib.louvain_pruner_train(None, None, 0, 1, 1, 1e-3, 1.0, 0, None, None, None) == lv.LOUVAIN_ERR_INVALID
    assert lib.louvain_pruner_scratch_floats(4096) >= 3 * lv.MLP_PARAMS + 2
    fake = 4096
    g = lv.LouvainGraph(10, 20, 32, fake, fake, None)
    p = lv.louvain_params_default()
    p.pruner = lv.PRUNE_LEARNED
    assert _create_status(g, p)[0] == lv.LOUVAIN_ERR_INVALID            # learned pruner without weights
    assert "pruner_weights" in lv.louvain_last_error(None)
    p = lv.louvain_params_default()
    p.guard_tolerance = 2
    assert _create_status(g, p)[0] == lv.LOUVAIN_ERR_INVALID
    p = lv.louvain_params_default()
    assert (p.guard_tolerance, p.pruner_weights, p.pruner_threshold) == (0, None, 0.5)
    assert (p.async_coherent, p.async_slices, p.async_slice_min, p.async_hub_groups, p.async_min_label) == \
        (0, 64, 256, 32, 1)


def test_workspace_size_is_host_only_and_monotone(lib):
    p = lv.louvain_params_default()
    sizes = []
    for n, m in [(0, 0), (10, 20), (1000, 20000), (1 << 20, 1 << 24)]:
        g = lv.LouvainGraph(n, m, 32, None, None, None)
        sizes.append(lv.louvain_workspace_size(g, p))
    assert sizes == sorted(sizes) and sizes[0] > 0


@pytest.mark.parametrize("field,value", [("n", -1), ("nnz", -5), ("n", 1 << 31)])
def test_workspace_size_rejects_bad_sizes(lib, field, value):
    g = lv.LouvainGraph(10, 20, 32, None, None, None)
    setattr(g, field, value)
    with pytest.raises(lv.LouvainError) as e:
        lv.louvain_workspace_size(g, lv.louvain_params_default())
    assert e.value.status == lv.LOUVAIN_ERR_INVALID


def _create_status(g, p, ws=None, ws_bytes=0):
    h = ctypes.c_void_p()
    st = lib_handle().louvain_create(ctypes.byref(g), ctypes.byref(p), None, ws, ws_bytes, ctypes.byref(h))
    return st, h


def lib_handle():
    return lv.load_library()


def test_create_rejects_bad_arguments_before_device_access(lib):
    p = lv.louvain_params_default()
    fake = 4096  # never dereferenced: every case fails argument checks first
    g = lv.LouvainGraph(10, 20, 16, fake, fake, None)
    assert _create_status(g, p)[0] == lv.LOUVAIN_ERR_INVALID           # offset_bits
    g = lv.LouvainGraph(10, 1 << 31, 32, fake, fake, None)
    assert _create_status(g, p)[0] == lv.LOUVAIN_ERR_INVALID           # nnz too big for 32-bit offsets
    g = lv.LouvainGraph(10, 20, 32, None, fake, None)
    assert _create_status(g, p)[0] == lv.LOUVAIN_ERR_INVALID           # missing offsets
    g = lv.LouvainGraph(10, 20, 32, fake, fake, None)
    bad = lv.louvain_params_default()
    bad.tol_den = 0
    assert _create_status(g, bad)[0] == lv.LOUVAIN_ERR_INVALID         # tolerance denominator
    bad = lv.louvain_params_default()
    bad.mode = 7
    assert _create_status(g, bad)[0] == lv.LOUVAIN_ERR_INVALID
    bad = lv.louvain_params_default()
    bad.device_loop = 2
    assert _create_status(g, bad)[0] == lv.LOUVAIN_ERR_INVALID         # device_loop is 0 or 1
    bad.device_loop = 1
    bad.pruner = lv.PRUNE_LEARNED
    bad.pruner_weights = fake
    assert _create_status(g, bad)[0] == lv.LOUVAIN_ERR_INVALID         # not with the learned pruner
    assert "device_loop" in lv.louvain_last_error(None)
    ok = lv.louvain_params_default()
    ok.device_loop = 1
    assert _create_status(g, ok, None, 0)[0] == lv.LOUVAIN_ERR_WORKSPACE  # accepted; no workspace
    assert _create_status(g, p, None, 0)[0] == lv.LOUVAIN_ERR_WORKSPACE  # no workspace
    assert _create_status(g, p, fake + 8, 1 << 40)[0] == lv.LOUVAIN_ERR_WORKSPACE  # misaligned
    assert "256-byte" in lv.louvain_last_error(None)


def test_null_handle_calls_fail_cleanly(lib):
    assert lib.louvain_run(None) == lv.LOUVAIN_ERR_INVALID
    assert lib.louvain_get_membership(None, None) == lv.LOUVAIN_ERR_INVALID
    lib.louvain_destroy(None)


def test_batch_create_rejects_bad_arguments(lib):
    fake = 4096
    g = lv.LouvainGraph(10, 20, 32, fake, fake, None)
    p = lv.louvain_params_default()
    h = ctypes.c_void_p()

    def create(vb, count, params=p):
        arr = (ctypes.c_int64 * len(vb))(*vb)
        return lib.louvain_create_batch(ctypes.byref(g), arr, count, ctypes.byref(params), None, None, 0,
                                        ctypes.byref(h))
    assert create([0, 5, 10], 0) == lv.LOUVAIN_ERR_INVALID      # count must be >= 1
    assert create([0, 5, 9], 2) == lv.LOUVAIN_ERR_INVALID       # must end at n
    assert create([0, 7, 5, 10], 3) == lv.LOUVAIN_ERR_INVALID   # non-decreasing
    assert create([1, 5, 10], 2) == lv.LOUVAIN_ERR_INVALID      # must start at 0
    learned = lv.louvain_params_default()
    learned.pruner = lv.PRUNE_LEARNED
    learned.pruner_weights = fake
    for mode in (lv.SYNC, lv.ASYNC):
        learned.mode = mode
        assert create([0, 5, 10], 2, learned) == lv.LOUVAIN_ERR_WORKSPACE  # accepted; no workspace
    assert create([0, 5, 10], 2) == lv.LOUVAIN_ERR_WORKSPACE    # arguments fine, no workspace
    single = lv.louvain_workspace_size(g, p)
    assert lv.louvain_workspace_size_batch(g, 2, p) > single == lv.louvain_workspace_size_batch(g, 0, p)


def test_autotune_rejects_bad_arguments(lib):
    arr = (ctypes.c_int32 * 8)()
    best = ctypes.c_int32()
    assert lib.louvain_autotune(None, arr, 1, 1, ctypes.byref(best), None) == lv.LOUVAIN_ERR_INVALID
