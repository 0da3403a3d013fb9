"""Python binding of the gfx950 Louvain library (``lib/liblouvain_hip.so``).

Every function mirrors an ``extern "C"`` entry point of ``include/louvain.h``
under the same name and only marshals arguments; all computation runs in the
HIP kernels.  PyTorch is used for device memory (tensors, the workspace) and
for the current HIP stream.  There is no CPU fallback: when the library is not
built, or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "liblouvain_hip.so")

LOUVAIN_OK = 0
LOUVAIN_ERR_INVALID = -1
LOUVAIN_ERR_NOMEM = -2
LOUVAIN_ERR_WORKSPACE = -3
LOUVAIN_ERR_HIP = -4
LOUVAIN_ERR_OVERFLOW = -5
LOUVAIN_ERR_STATE = -6
ASYNC = 0
SYNC = 1
PRUNE_NONE = 0
PRUNE_FLAGS = 1
PRUNE_LEARNED = 2
MLP_PARAMS = 32 * 8 + 32 + 32 * 32 + 32 + 32 + 1
SAMPLE_FLOATS = 9

EXPORTED = ["louvain_params_default", "louvain_workspace_size", "louvain_create", "louvain_run",
            "louvain_get_membership", "louvain_modularity", "louvain_get_stats", "louvain_set_profiling",
            "louvain_get_kernel_stats", "louvain_set_trace", "louvain_last_error", "louvain_destroy",
            "louvain_collect_samples", "louvain_sample_count", "louvain_pruner_init", "louvain_pruner_predict",
            "louvain_pruner_loss_grad", "louvain_pruner_scratch_floats", "louvain_pruner_train",
            "louvain_workspace_size_batch", "louvain_create_batch", "louvain_modularity_batch",
            "louvain_batch_results", "louvain_autotune", "louvain_pruner_train_noalloc"]
NOALLOC_SCRATCH_FLOATS = 8192


class LouvainGraph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("offset_bits", ctypes.c_int32),
                ("offsets", ctypes.c_void_p), ("indices", ctypes.c_void_p), ("weights", ctypes.c_void_p)]


class LouvainParams(ctypes.Structure):
    _fields_ = [("max_iterations", ctypes.c_int32), ("max_passes", ctypes.c_int32),
                ("tol_num", ctypes.c_int64), ("tol_den", ctypes.c_int64), ("tol_drop", ctypes.c_int64),
                ("agg_num", ctypes.c_int64), ("agg_den", ctypes.c_int64), ("pick_less", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("pruner", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("bucket_max_degree", ctypes.c_int32 * 8), ("agg_bucket_max", ctypes.c_int32 * 8),
                ("async_coherent", ctypes.c_int32), ("bucket_order", ctypes.c_int32),
                ("async_slices", ctypes.c_int32), ("async_slice_iters", ctypes.c_int32),
                ("guard_tolerance", ctypes.c_int32), ("async_slice_min", ctypes.c_int32),
                ("async_hub_groups", ctypes.c_int32), ("async_min_label", ctypes.c_int32),
                ("pruner_weights", ctypes.c_void_p), ("pruner_threshold", ctypes.c_double),
                ("async_interleave", ctypes.c_int32), ("table_values_64", ctypes.c_int32),
                ("device_loop", ctypes.c_int32)]


class LouvainStats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int32), ("iterations", ctypes.c_int32), ("moves", ctypes.c_int64),
                ("communities", ctypes.c_int64), ("vertices_evaluated", ctypes.c_int64),
                ("arcs_scanned", ctypes.c_int64), ("distinct_scanned", ctypes.c_int64),
                ("ms_total", ctypes.c_double), ("ms_move", ctypes.c_double), ("ms_aggregate", ctypes.c_double),
                ("iterations_per_pass", ctypes.c_int32 * 32), ("communities_per_pass", ctypes.c_int64 * 32),
                ("sweeps", ctypes.c_int64), ("pruned", ctypes.c_int64), ("host_syncs", ctypes.c_int64)]


class LouvainKernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_int64)]


_I32P = ctypes.POINTER(ctypes.c_int32)
_I64P = ctypes.POINTER(ctypes.c_int64)
ITER_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _I32P, _I64P,
                           ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64)
PASS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, _I64P, _I32P, _I64P,
                           ctypes.c_int32)

_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblouvain_hip.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    lib.louvain_params_default.restype = None
    lib.louvain_params_default.argtypes = [ctypes.POINTER(LouvainParams)]
    lib.louvain_workspace_size.restype = ctypes.c_int
    lib.louvain_workspace_size.argtypes = [ctypes.POINTER(LouvainGraph), ctypes.POINTER(LouvainParams),
                                           ctypes.POINTER(sz)]
    lib.louvain_create.restype = ctypes.c_int
    lib.louvain_create.argtypes = [ctypes.POINTER(LouvainGraph), ctypes.POINTER(LouvainParams), vp, vp, sz,
                                   ctypes.POINTER(vp)]
    lib.louvain_run.restype = ctypes.c_int
    lib.louvain_run.argtypes = [vp]
    lib.louvain_get_membership.restype = ctypes.c_int
    lib.louvain_get_membership.argtypes = [vp, vp]
    lib.louvain_modularity.restype = ctypes.c_int
    lib.louvain_modularity.argtypes = [vp, ctypes.POINTER(ctypes.c_double), _I64P, _I64P]
    lib.louvain_get_stats.restype = ctypes.c_int
    lib.louvain_get_stats.argtypes = [vp, ctypes.POINTER(LouvainStats)]
    lib.louvain_set_profiling.restype = ctypes.c_int
    lib.louvain_set_profiling.argtypes = [vp, ctypes.c_int32]
    lib.louvain_get_kernel_stats.restype = ctypes.c_int
    lib.louvain_get_kernel_stats.argtypes = [vp, ctypes.POINTER(LouvainKernelStat), ctypes.c_int32, _I32P]
    lib.louvain_set_trace.restype = ctypes.c_int
    lib.louvain_set_trace.argtypes = [vp, ITER_FN, PASS_FN, vp]
    lib.louvain_last_error.restype = ctypes.c_char_p
    lib.louvain_last_error.argtypes = [vp]
    lib.louvain_destroy.restype = None
    lib.louvain_destroy.argtypes = [vp]
    lib.louvain_workspace_size_batch.restype = ctypes.c_int
    lib.louvain_workspace_size_batch.argtypes = [ctypes.POINTER(LouvainGraph), ctypes.c_int64,
                                                 ctypes.POINTER(LouvainParams), ctypes.POINTER(ctypes.c_size_t)]
    lib.louvain_create_batch.restype = ctypes.c_int
    lib.louvain_create_batch.argtypes = [ctypes.POINTER(LouvainGraph), _I64P, ctypes.c_int64,
                                         ctypes.POINTER(LouvainParams), vp, vp, sz, ctypes.POINTER(vp)]
    lib.louvain_modularity_batch.restype = ctypes.c_int
    lib.louvain_modularity_batch.argtypes = [vp, ctypes.POINTER(ctypes.c_double), _I64P, _I64P]
    lib.louvain_batch_results.restype = ctypes.c_int
    lib.louvain_batch_results.argtypes = [vp, _I32P, _I32P, _I64P]
    lib.louvain_autotune.restype = ctypes.c_int
    lib.louvain_autotune.argtypes = [vp, _I32P, ctypes.c_int32, ctypes.c_int32, _I32P,
                                     ctypes.POINTER(ctypes.c_double)]
    lib.louvain_collect_samples.restype = ctypes.c_int
    lib.louvain_collect_samples.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32]
    lib.louvain_sample_count.restype = ctypes.c_int
    lib.louvain_sample_count.argtypes = [vp, _I64P]
    lib.louvain_pruner_init.restype = ctypes.c_int
    lib.louvain_pruner_init.argtypes = [vp, ctypes.c_uint64, vp]
    lib.louvain_pruner_predict.restype = ctypes.c_int
    lib.louvain_pruner_predict.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
    lib.louvain_pruner_loss_grad.restype = ctypes.c_int
    lib.louvain_pruner_loss_grad.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_float, vp,
                                             ctypes.POINTER(ctypes.c_double), vp]
    lib.louvain_pruner_scratch_floats.restype = ctypes.c_int64
    lib.louvain_pruner_scratch_floats.argtypes = [ctypes.c_int32]
    lib.louvain_pruner_train.restype = ctypes.c_int
    lib.louvain_pruner_train.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_uint64, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.louvain_pruner_train_noalloc.restype = ctypes.c_int
    lib.louvain_pruner_train_noalloc.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                                 ctypes.c_float, ctypes.c_float, ctypes.c_uint64,
                                                 ctypes.POINTER(ctypes.c_double), vp]
    _lib = lib
    return lib


class LouvainError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"louvain status {status}: {msg}")
        self.status = status


def _check(status: int, handle=None):
    if status != LOUVAIN_OK:
        msg = load_library().louvain_last_error(handle)
        raise LouvainError(status, msg.decode() if msg else "")


# ------------------------------------------------------------ thin wrappers

def louvain_params_default() -> LouvainParams:
    p = LouvainParams()
    load_library().louvain_params_default(ctypes.byref(p))
    return p


def louvain_workspace_size(g: LouvainGraph, p: LouvainParams) -> int:
    n = ctypes.c_size_t()
    _check(load_library().louvain_workspace_size(ctypes.byref(g), ctypes.byref(p), ctypes.byref(n)))
    return n.value


def louvain_create(g: LouvainGraph, p: LouvainParams, stream: int, workspace: int, workspace_bytes: int):
    h = ctypes.c_void_p()
    _check(load_library().louvain_create(ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(stream),
                                         ctypes.c_void_p(workspace), workspace_bytes, ctypes.byref(h)))
    return h


def louvain_run(h) -> None:
    _check(load_library().louvain_run(h), h)


def louvain_get_membership(h, out_ptr: int) -> None:
    _check(load_library().louvain_get_membership(h, ctypes.c_void_p(out_ptr)), h)


def louvain_modularity(h):
    """Returns (q, numerator, denominator) with exact Python ints."""
    q = ctypes.c_double()
    num = (ctypes.c_int64 * 2)()
    den = (ctypes.c_int64 * 2)()
    _check(load_library().louvain_modularity(h, ctypes.byref(q), num, den), h)

    def i128(x):
        return (int(x[0]) << 64) + (int(x[1]) & ((1 << 64) - 1))
    return q.value, i128(num), i128(den)


def louvain_get_stats(h) -> LouvainStats:
    s = LouvainStats()
    _check(load_library().louvain_get_stats(h, ctypes.byref(s)), h)
    return s


def louvain_set_profiling(h, enable: bool) -> None:
    _check(load_library().louvain_set_profiling(h, int(enable)), h)


def louvain_get_kernel_stats(h) -> list[dict]:
    arr = (LouvainKernelStat * 64)()
    cnt = ctypes.c_int32()
    _check(load_library().louvain_get_kernel_stats(h, arr, 64, ctypes.byref(cnt)), h)
    return [dict(name=arr[i].name.decode(), launches=arr[i].launches, ms=arr[i].ms, alg_bytes=arr[i].alg_bytes)
            for i in range(min(cnt.value, 64))]


def louvain_set_trace(h, iter_fn, pass_fn, user=None) -> None:
    _check(load_library().louvain_set_trace(h, iter_fn or ITER_FN(), pass_fn or PASS_FN(), user), h)


def louvain_last_error(h=None) -> str:
    msg = load_library().louvain_last_error(h)
    return msg.decode() if msg else ""


def louvain_workspace_size_batch(g: LouvainGraph, count: int, p: LouvainParams) -> int:
    n = ctypes.c_size_t()
    _check(load_library().louvain_workspace_size_batch(ctypes.byref(g), count, ctypes.byref(p), ctypes.byref(n)))
    return int(n.value)


def louvain_create_batch(g: LouvainGraph, vbase, p: LouvainParams, stream: int, workspace: int,
                         workspace_bytes: int):
    vb = (ctypes.c_int64 * len(vbase))(*[int(x) for x in vbase])
    h = ctypes.c_void_p()
    _check(load_library().louvain_create_batch(ctypes.byref(g), vb, len(vbase) - 1, ctypes.byref(p), stream,
                                               workspace, workspace_bytes, ctypes.byref(h)))
    return h


def louvain_modularity_batch(h, count: int):
    """Per-graph (q, numerator, denominator) lists; exact values as Python ints."""
    q = (ctypes.c_double * count)()
    num = (ctypes.c_int64 * (2 * count))()
    den = (ctypes.c_int64 * (2 * count))()
    _check(load_library().louvain_modularity_batch(h, q, num, den), h)

    def i128(a, k):
        return (int(a[2 * k]) << 64) + (int(a[2 * k + 1]) & ((1 << 64) - 1))
    return list(q), [i128(num, k) for k in range(count)], [i128(den, k) for k in range(count)]


def louvain_batch_results(h, count: int):
    """Per-graph (passes, iterations, communities) lists."""
    pa = (ctypes.c_int32 * count)()
    it = (ctypes.c_int32 * count)()
    co = (ctypes.c_int64 * count)()
    _check(load_library().louvain_batch_results(h, pa, it, co), h)
    return list(pa), list(it), list(co)


def louvain_collect_samples(h, buffer_ptr: int, capacity: int, sample_per_mille: int) -> None:
    _check(load_library().louvain_collect_samples(h, buffer_ptr or None, capacity, sample_per_mille), h)


def louvain_sample_count(h) -> int:
    c = ctypes.c_int64()
    _check(load_library().louvain_sample_count(h, ctypes.byref(c)), h)
    return int(c.value)


def louvain_pruner_init(weights_ptr: int, seed: int, stream: int) -> None:
    _check(load_library().louvain_pruner_init(weights_ptr, seed, stream))


def louvain_pruner_predict(weights_ptr: int, features_ptr: int, count: int, logit_ptr: int, stream: int) -> None:
    _check(load_library().louvain_pruner_predict(weights_ptr, features_ptr, count, logit_ptr, stream))


def louvain_pruner_loss_grad(weights_ptr: int, samples_ptr: int, count: int, pos_weight: float, grad_ptr: int,
                             stream: int) -> float:
    loss = ctypes.c_double()
    _check(load_library().louvain_pruner_loss_grad(weights_ptr, samples_ptr, count, pos_weight, grad_ptr,
                                                   ctypes.byref(loss), stream))
    return float(loss.value)


def louvain_pruner_scratch_floats(batch: int) -> int:
    return int(load_library().louvain_pruner_scratch_floats(batch))


def louvain_pruner_train(weights_ptr: int, samples_ptr: int, count: int, steps: int, batch: int, lr: float,
                         pos_weight: float, seed: int, scratch_ptr: int, stream: int) -> float:
    loss = ctypes.c_double()
    _check(load_library().louvain_pruner_train(weights_ptr, samples_ptr, count, steps, batch, lr, pos_weight, seed,
                                               scratch_ptr, ctypes.byref(loss), stream))
    return float(loss.value)


def louvain_pruner_train_noalloc(weights_ptr: int, samples_ptr: int, count: int, steps: int, batch: int, lr: float,
                                 pos_weight: float, seed: int, stream: int) -> float:
    loss = ctypes.c_double()
    _check(load_library().louvain_pruner_train_noalloc(weights_ptr, samples_ptr, count, steps, batch, lr, pos_weight,
                                                       seed, ctypes.byref(loss), stream))
    return float(loss.value)


def louvain_autotune(h, candidates, reps: int = 1):
    """candidates: list of bucket_max_degree lists (up to 8 entries each).
    Returns (index of the kept candidate or -1 when the handle's thresholds
    stay, mean ms per candidate)."""
    nc = len(candidates)
    arr = (ctypes.c_int32 * (8 * nc))()
    for c, cand in enumerate(candidates):
        for k, x in enumerate(cand):
            arr[8 * c + k] = int(x)
    best = ctypes.c_int32(-1)
    ms = (ctypes.c_double * nc)()
    _check(load_library().louvain_autotune(h, arr, nc, reps, ctypes.byref(best), ms), h)
    return int(best.value), [float(x) for x in ms]


def louvain_destroy(h) -> None:
    if h:
        load_library().louvain_destroy(h)


# --------------------------------------------------------- torch plumbing

def _check_graph_tensors(offsets, indices, weights):
    """The C ABI reads raw device pointers: reject tensors whose dtype,
    layout or device would make it read a different graph than the caller's."""
    import torch
    dev = offsets.device
    for name, t, dtypes in (("offsets", offsets, (torch.int32, torch.int64)), ("indices", indices, (torch.int32,)),
                            ("weights", weights, (torch.int32,))):
        if t is None:
            if name == "weights":
                continue
            raise ValueError(f"{name} is required")
        if t.dtype not in dtypes:
            raise ValueError(f"{name} must have dtype {' or '.join(str(d) for d in dtypes)}, got {t.dtype}")
        if not t.is_cuda or t.device != dev:
            raise ValueError(f"{name} must be a CUDA tensor on {dev}, got {t.device}")
        if not t.is_contiguous() or t.dim() != 1:
            raise ValueError(f"{name} must be a contiguous 1-D tensor")
    if offsets.numel() < 1:
        raise ValueError("offsets must hold n + 1 >= 1 entries")
    if weights is not None and weights.numel() != indices.numel():
        raise ValueError("weights and indices must have the same length")


class Louvain:
    """A handle on one device-resident graph.

    offsets/indices/weights are torch tensors on the current GPU (offsets
    int32 or int64, indices int32, weights int32 or None for unit weights).
    The workspace is a torch uint8 tensor; kernels run on the current stream.
    """

    def __init__(self, offsets, indices, weights=None, params: LouvainParams | None = None, vbase=None,
                 **overrides):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU available: the Louvain library runs only on the GPU")
        load_library()
        _check_graph_tensors(offsets, indices, weights)
        self._keep = (offsets, indices, weights, overrides.get("pruner_weights"))
        self.params = params or louvain_params_default()
        for k, v in overrides.items():
            if k == "pruner_weights":
                if v is not None and (v.dtype != torch.float32 or v.numel() != MLP_PARAMS or not v.is_cuda
                                      or not v.is_contiguous()):
                    raise ValueError(f"pruner_weights must be a contiguous float32 GPU tensor of {MLP_PARAMS}")
                self.params.pruner_weights = v.data_ptr() if v is not None else None
            elif k in ("bucket_max_degree", "agg_bucket_max"):
                arr = getattr(self.params, k)
                for i, x in enumerate(v):
                    arr[i] = x
            else:
                setattr(self.params, k, v)
        n = offsets.numel() - 1
        g = LouvainGraph()
        g.n = n
        g.nnz = indices.numel()
        g.offset_bits = 64 if offsets.dtype == torch.int64 else 32
        g.offsets = offsets.data_ptr()
        g.indices = indices.data_ptr() if indices.numel() else 0
        g.weights = weights.data_ptr() if weights is not None else None
        self.graph = g
        self.n = n
        self.count = 0 if vbase is None else len(vbase) - 1
        nbytes = louvain_workspace_size_batch(g, self.count, self.params)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=offsets.device)
        self.stream = torch.cuda.current_stream(offsets.device)
        if vbase is None:
            self.h = louvain_create(g, self.params, self.stream.cuda_stream, self.workspace.data_ptr(), nbytes)
        else:
            self.h = louvain_create_batch(g, vbase, self.params, self.stream.cuda_stream, self.workspace.data_ptr(),
                                          nbytes)
        self._cb = None

    def run(self):
        louvain_run(self.h)
        return self

    def membership(self):
        import torch
        out = torch.empty(self.n, dtype=torch.int32, device=self.workspace.device)
        if self.n:
            louvain_get_membership(self.h, out.data_ptr())
        return out

    def modularity(self):
        return louvain_modularity(self.h)

    def modularity_batch(self):
        """Per-graph (q, numerator, denominator) lists of a batched handle."""
        return louvain_modularity_batch(self.h, self.count)

    def batch_results(self):
        """Per-graph (passes, iterations, communities) lists of a batched handle."""
        return louvain_batch_results(self.h, self.count)

    def autotune(self, candidates, reps: int = 1):
        """Time the candidate bucket thresholds and keep the fastest (see
        louvain_autotune); returns (best index, mean ms per candidate)."""
        best, ms = louvain_autotune(self.h, candidates, reps)
        if best >= 0:
            for k, x in enumerate(candidates[best]):
                self.params.bucket_max_degree[k] = int(x)
        return best, ms

    def stats(self) -> LouvainStats:
        return louvain_get_stats(self.h)

    def set_profiling(self, enable: bool = True):
        louvain_set_profiling(self.h, enable)

    def kernel_stats(self):
        return louvain_get_kernel_stats(self.h)

    def trace(self, on_iter=None, on_pass=None):
        """Install Python callbacks receiving numpy copies of each iteration's
        (pass, iter, C', Sigma', moves, gain) and each pass's super-graph."""
        import numpy as np

        def it(_u, p, t, n, cp, sig, moves, ghi, glo):
            if on_iter:
                on_iter(int(p), int(t), np.ctypeslib.as_array(cp, shape=(n,)).copy() if n else np.zeros(0, np.int32),
                        np.ctypeslib.as_array(sig, shape=(n,)).copy() if n else np.zeros(0, np.int64), int(moves),
                        (int(ghi) << 64) + int(glo))

        def pa(_u, p, n, off, idx, w, iters):
            if on_pass:
                o = np.ctypeslib.as_array(off, shape=(n + 1,)).copy()
                m = int(o[-1])
                ii = np.ctypeslib.as_array(idx, shape=(m,)).copy() if m else np.zeros(0, np.int32)
                ww = np.ctypeslib.as_array(w, shape=(m,)).copy() if m else np.zeros(0, np.int64)
                on_pass(int(p), int(n), o, ii, ww, int(iters))

        self._cb = (ITER_FN(it) if on_iter else ITER_FN(), PASS_FN(pa) if on_pass else PASS_FN())
        louvain_set_trace(self.h, self._cb[0], self._cb[1])

    def collect_samples(self, capacity: int, sample_per_mille: int):
        """Record training samples during later runs into a new float32
        tensor [capacity, SAMPLE_FLOATS]; returns it (rows filled up to
        sample_count())."""
        import torch
        buf = torch.zeros((max(capacity, 1), SAMPLE_FLOATS), dtype=torch.float32, device=self.workspace.device)
        self._samples = buf
        louvain_collect_samples(self.h, buf.data_ptr(), capacity, sample_per_mille)
        return buf

    def sample_count(self) -> int:
        return louvain_sample_count(self.h)

    def close(self):
        """Destroy the handle and release the workspace (the graph tensors stay
        with the caller)."""
        if getattr(self, "h", None):
            louvain_destroy(self.h)
            self.h = None
        self.workspace = None
        self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_tensors(graphs, device="cuda", unit_weights: bool | None = None, offset_bits: int | None = None):
    """Lay graphgen.CSRGraphs end to end: returns (offsets, indices, weights-or-None,
    vbase) for Louvain(..., vbase=vbase).  Offsets are int64 when the union has
    2^31 or more arcs or offset_bits is 64."""
    import numpy as np
    import torch
    ns = [g.n for g in graphs]
    ms = [int(g.offsets[-1]) for g in graphs]
    vbase = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    ebase = np.concatenate([[0], np.cumsum(ms)]).astype(np.int64)
    big = ebase[-1] > 0x7fffffff or offset_bits == 64
    off = np.empty(vbase[-1] + 1, dtype=np.int64)
    off[-1] = ebase[-1]
    idx = np.empty(ebase[-1], dtype=np.int32)
    wts = np.empty(ebase[-1], dtype=np.int32)
    for k, g in enumerate(graphs):
        off[vbase[k]:vbase[k + 1]] = np.asarray(g.offsets[:-1], dtype=np.int64) + ebase[k]
        idx[ebase[k]:ebase[k + 1]] = np.asarray(g.indices, dtype=np.int64) + vbase[k]
        wts[ebase[k]:ebase[k + 1]] = g.weights
    unit = bool(unit_weights) if unit_weights is not None else bool(wts.size == 0 or wts.max() == 1)
    o = torch.from_numpy(off if big else off.astype(np.int32)).to(device)
    w = None if unit else torch.from_numpy(wts).to(device)
    return o, torch.from_numpy(idx).to(device), w, vbase.tolist()


def graph_tensors(g, device="cuda", offset_bits: int = 32, unit_weights: bool | None = None):
    """Upload a graphgen.CSRGraph: returns (offsets, indices, weights-or-None)."""
    import numpy as np
    import torch
    off = torch.from_numpy(np.ascontiguousarray(g.offsets, dtype=np.int64 if offset_bits == 64 else np.int32))
    idx = torch.from_numpy(np.ascontiguousarray(g.indices, dtype=np.int32))
    unit = bool(unit_weights) if unit_weights is not None else bool(g.weights.size == 0 or g.weights.max() == 1)
    w = None if unit else torch.from_numpy(np.ascontiguousarray(g.weights, dtype=np.int32)).to(device)
    return off.to(device), idx.to(device), w


# ------------------------------------------------------------ pruner MLP

def _stream_of(t):
    import torch
    return torch.cuda.current_stream(t.device).cuda_stream


def pruner_init(seed: int, device="cuda"):
    """Glorot-uniform pruner weights as a float32 tensor [MLP_PARAMS]."""
    import torch
    w = torch.empty(MLP_PARAMS, dtype=torch.float32, device=device)
    louvain_pruner_init(w.data_ptr(), seed, _stream_of(w))
    return w


def pruner_predict(weights, features):
    """Output logits of the pruner MLP for features [k, 8] (float32, GPU)."""
    import torch
    x = features.contiguous()
    out = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    louvain_pruner_predict(weights.data_ptr(), x.data_ptr(), x.shape[0], out.data_ptr(), _stream_of(x))
    return out


def pruner_loss_grad(weights, samples, pos_weight: float = 1.0):
    """(loss, gradient tensor) of the weighted cross-entropy over samples [k, 9]."""
    import torch
    s = samples.contiguous()
    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=s.device)
    loss = louvain_pruner_loss_grad(weights.data_ptr(), s.data_ptr(), s.shape[0], pos_weight, g.data_ptr(),
                                    _stream_of(s))
    return loss, g


def pruner_train(weights, samples, steps: int, batch: int = 4096, lr: float = 1e-3, pos_weight: float = 1.0,
                 seed: int = 0) -> float:
    """Adam training of weights (updated in place); returns the last loss."""
    import torch
    s = samples.contiguous()
    scratch = torch.empty(louvain_pruner_scratch_floats(batch), dtype=torch.float32, device=s.device)
    return louvain_pruner_train(weights.data_ptr(), s.data_ptr(), s.shape[0], steps, batch, lr, pos_weight, seed,
                                scratch.data_ptr(), _stream_of(s))
