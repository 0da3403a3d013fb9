"""CPU oracle for the Louvain method -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never loads it, and it shares no code
with the GPU library; the one common dependency is the seeded input generator
module ``graphgen`` (random draws and CSR layout only).

The arithmetic lives in ``louvain_oracle.c`` (sequential C, exact integers,
``__int128`` for products and sums of gains); this file only marshals numpy
arrays through ctypes.  See that file for the equations and algorithms each
function follows.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "louvain_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C11, no vectorisation tricks)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=gnu11", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("max_iterations", ctypes.c_int32), ("max_passes", ctypes.c_int32),
                ("tol_num", ctypes.c_int64), ("tol_den", ctypes.c_int64), ("tol_drop", ctypes.c_int64),
                ("agg_num", ctypes.c_int64), ("agg_den", ctypes.c_int64),
                ("mode", ctypes.c_int32), ("pick_less", ctypes.c_int32), ("prune", ctypes.c_int32),
                ("guard_tolerance", ctypes.c_int32), ("mlp", ctypes.POINTER(ctypes.c_float)),
                ("threshold", ctypes.c_double), ("sample_per_mille", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int32), ("iterations", ctypes.c_int32), ("moves", ctypes.c_int64),
                ("communities", ctypes.c_int64), ("sweeps", ctypes.c_int64), ("pruned", ctypes.c_int64)]


_I64P = ctypes.POINTER(ctypes.c_int64)
_U64P = ctypes.POINTER(ctypes.c_uint64)
_I32P = ctypes.POINTER(ctypes.c_int32)
_ITER_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _I32P, _I64P,
                            ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64)
_PASS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, _I64P, _I32P, _I64P,
                            ctypes.c_int32)
_F32P = ctypes.POINTER(ctypes.c_float)
_SAMPLE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _F32P,
                              ctypes.c_int32)

ASYNC, SYNC = 0, 1
PRUNE_NONE, PRUNE_FLAGS, PRUNE_LEARNED = 0, 1, 2
MLP_PARAMS = 32 * 8 + 32 + 32 * 32 + 32 + 32 + 1


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_modularity.restype = ctypes.c_int
        lib.oracle_modularity.argtypes = [ctypes.c_int64, _I64P, _I32P, _I64P, _I32P, _I64P, _U64P, _I64P, _U64P]
        lib.oracle_louvain.restype = ctypes.c_int
        lib.oracle_louvain.argtypes = [ctypes.c_int64, _I64P, _I32P, _I64P, ctypes.POINTER(_Params), _I32P,
                                       ctypes.POINTER(_Stats), _ITER_FN, _PASS_FN, ctypes.c_void_p]
        lib.oracle_louvain_samples.restype = ctypes.c_int
        lib.oracle_louvain_samples.argtypes = [ctypes.c_int64, _I64P, _I32P, _I64P, ctypes.POINTER(_Params), _I32P,
                                               ctypes.POINTER(_Stats), _ITER_FN, _PASS_FN, _SAMPLE_FN,
                                               ctypes.c_void_p]
        lib.oracle_mlp_logit.restype = ctypes.c_float
        lib.oracle_mlp_logit.argtypes = [_F32P, _F32P]
        lib.oracle_features.restype = None
        lib.oracle_features.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _F32P]
        lib.oracle_aggregate.restype = ctypes.c_int
        lib.oracle_aggregate.argtypes = [ctypes.c_int64, _I64P, _I32P, _I64P, _I32P, ctypes.c_int64, _I64P, _I32P,
                                         _I64P]
        lib.oracle_gain.restype = ctypes.c_int
        lib.oracle_gain.argtypes = [ctypes.c_int64, _I64P, _I32P, _I64P, _I32P, ctypes.c_int64, ctypes.c_int32,
                                    _I64P, _U64P]
        lib.oracle_best_move.restype = ctypes.c_int
        lib.oracle_best_move.argtypes = [ctypes.c_int64, _I64P, _I32P, _I64P, ctypes.c_int64, _I32P, _I64P,
                                         ctypes.c_int64, _I32P, _I64P, _U64P]
        _lib = lib
    return _lib


def _i128(hi: int, lo: int) -> int:
    return (int(hi) << 64) + int(lo)


def _arrays(g):
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    idx = np.ascontiguousarray(g.indices, dtype=np.int32)
    w = np.ascontiguousarray(g.weights, dtype=np.int64)
    if w.size and w.min() <= 0:
        raise ValueError("edge weights must be positive")
    return off, idx, w


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


@dataclasses.dataclass
class Params:
    """Louvain parameters; defaults are the paper's (20 iterations, 10 passes,
    tau = 1/100 dropped 10x per pass, tau_agg = 4/5, Pick-Less every 4)."""
    max_iterations: int = 20
    max_passes: int = 10
    tol_num: int = 1
    tol_den: int = 100
    tol_drop: int = 10
    agg_num: int = 4
    agg_den: int = 5
    mode: int = ASYNC
    pick_less: int = 4
    prune: int = 1
    guard_tolerance: int = 0          # PRUNE_LEARNED: sweep exit test (0 strict, 1 tolerance)
    mlp: np.ndarray | None = None     # PRUNE_LEARNED: MLP_PARAMS float32 weights
    threshold: float = 0.5            # PRUNE_LEARNED: evaluate iff sigmoid(logit) >= threshold
    sample_per_mille: int = 0         # training-sample selection rate

    def _c(self) -> _Params:
        mlp = None
        if self.mlp is not None:
            mlp = np.ascontiguousarray(self.mlp, dtype=np.float32)
            if mlp.size != MLP_PARAMS:
                raise ValueError(f"mlp must hold {MLP_PARAMS} floats")
        self._mlp_keep = mlp
        return _Params(self.max_iterations, self.max_passes, self.tol_num, self.tol_den, self.tol_drop,
                       self.agg_num, self.agg_den, self.mode, self.pick_less, self.prune, self.guard_tolerance,
                       _p(mlp, ctypes.c_float) if mlp is not None else None, float(self.threshold),
                       self.sample_per_mille)


@dataclasses.dataclass
class Result:
    membership: np.ndarray
    passes: int
    iterations: int
    moves: int
    communities: int
    iters: list = dataclasses.field(default_factory=list)   # per-iteration trace records
    graphs: list = dataclasses.field(default_factory=list)  # per-pass super-graphs
    sweeps: int = 0
    pruned: int = 0
    samples: list = dataclasses.field(default_factory=list)  # (pass, iter, v, features float32[8], label)


def modularity_exact(g, membership) -> Fraction:
    """Eq. (1) as an exact fraction (num / W^2)."""
    off, idx, w = _arrays(g)
    memb = np.ascontiguousarray(membership, dtype=np.int32)
    nh, nl, dh, dl = ctypes.c_int64(), ctypes.c_uint64(), ctypes.c_int64(), ctypes.c_uint64()
    rc = _load().oracle_modularity(g.n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32), _p(w, ctypes.c_int64),
                                   _p(memb, ctypes.c_int32), ctypes.byref(nh), ctypes.byref(nl), ctypes.byref(dh),
                                   ctypes.byref(dl))
    if rc != 0:
        raise ValueError(f"oracle_modularity failed ({rc})")
    return Fraction(_i128(nh.value, nl.value), _i128(dh.value, dl.value))


def modularity_parts(g, membership) -> tuple[int, int]:
    """(numerator, denominator) of Eq. (1) times W^2, unreduced."""
    off, idx, w = _arrays(g)
    memb = np.ascontiguousarray(membership, dtype=np.int32)
    nh, nl, dh, dl = ctypes.c_int64(), ctypes.c_uint64(), ctypes.c_int64(), ctypes.c_uint64()
    rc = _load().oracle_modularity(g.n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32), _p(w, ctypes.c_int64),
                                   _p(memb, ctypes.c_int32), ctypes.byref(nh), ctypes.byref(nl), ctypes.byref(dh),
                                   ctypes.byref(dl))
    if rc != 0:
        raise ValueError(f"oracle_modularity failed ({rc})")
    return _i128(nh.value, nl.value), _i128(dh.value, dl.value)


def modularity(g, membership) -> float:
    q = modularity_exact(g, membership)
    return float(q)


def louvain(g, params: Params | None = None, trace: bool = False, samples: bool = False) -> Result:
    """Run the oracle.  With trace=True, records (pass, iter, C', Sigma', moves,
    gain sum) after every local-moving iteration and every super-graph.  With
    samples=True, records the training samples selected by
    params.sample_per_mille."""
    params = params or Params()
    off, idx, w = _arrays(g)
    memb = np.empty(g.n, dtype=np.int32)
    st = _Stats()
    iters: list = []
    graphs: list = []

    def on_iter(_u, p, t, n, cp, sig, moves, ghi, glo):
        iters.append(dict(pass_=p, iter=t, cprime=np.ctypeslib.as_array(cp, shape=(n,)).copy(),
                          sigma=np.ctypeslib.as_array(sig, shape=(n,)).copy(), moves=int(moves),
                          gain=_i128(ghi, glo)))

    def on_pass(_u, p, n, o, i, ww, count):
        oo = np.ctypeslib.as_array(o, shape=(n + 1,)).copy()
        nnz = int(oo[-1])
        ii = np.ctypeslib.as_array(i, shape=(max(nnz, 1),))[:nnz].copy() if nnz else np.zeros(0, np.int32)
        www = np.ctypeslib.as_array(ww, shape=(max(nnz, 1),))[:nnz].copy() if nnz else np.zeros(0, np.int64)
        graphs.append(dict(pass_=p, n=int(n), offsets=oo, indices=ii, weights=www, iterations=int(count)))

    smp: list = []

    def on_sample(_u, p, t, v, f, label):
        smp.append((int(p), int(t), int(v), np.ctypeslib.as_array(f, shape=(8,)).copy(), int(label)))

    it_fn = _ITER_FN(on_iter) if trace else _ITER_FN()
    pa_fn = _PASS_FN(on_pass) if trace else _PASS_FN()
    sm_fn = _SAMPLE_FN(on_sample) if samples else _SAMPLE_FN()
    cp = params._c()
    rc = _load().oracle_louvain_samples(g.n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32),
                                        _p(w, ctypes.c_int64), ctypes.byref(cp), _p(memb, ctypes.c_int32),
                                        ctypes.byref(st), it_fn, pa_fn, sm_fn, None)
    if rc != 0:
        raise RuntimeError(f"oracle_louvain failed ({rc})")
    return Result(memb, st.passes, st.iterations, st.moves, st.communities, iters, graphs, st.sweeps, st.pruned,
                  smp)


def mlp_logit(weights, x) -> np.ndarray:
    """FP32 output logits of the pruner MLP for rows of x (float32 [k, 8]),
    with the oracle's fixed fused-multiply-add order."""
    wts = np.ascontiguousarray(weights, dtype=np.float32)
    xs = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 8)
    lib = _load()
    out = np.empty(xs.shape[0], dtype=np.float32)
    for k in range(xs.shape[0]):
        row = np.ascontiguousarray(xs[k])
        out[k] = lib.oracle_mlp_logit(_p(wts, ctypes.c_float), _p(row, ctypes.c_float))
    return out


def features(deg: int, K: int, own: int, adv: int, nm: int, moved_last: bool, pass_: int, t: int) -> np.ndarray:
    """The eight float32 pruner features of one vertex from its state."""
    f = np.zeros(8, dtype=np.float32)
    _load().oracle_features(deg, K, own, adv, nm, 1 if moved_last else 0, pass_, t, _p(f, ctypes.c_float))
    return f


def aggregate(g, cprime, ncom: int):
    """Super-vertex graph of g under the dense membership cprime (ids < ncom):
    returns (offsets int64[ncom+1], indices int32, weights int64), rows sorted."""
    off, idx, w = _arrays(g)
    c = np.ascontiguousarray(cprime, dtype=np.int32)
    o = np.empty(ncom + 1, dtype=np.int64)
    cap = max(int(off[-1]), 1)
    ii = np.empty(cap, dtype=np.int32)
    ww = np.empty(cap, dtype=np.int64)
    rc = _load().oracle_aggregate(g.n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32), _p(w, ctypes.c_int64),
                                  _p(c, ctypes.c_int32), ncom, _p(o, ctypes.c_int64), _p(ii, ctypes.c_int32),
                                  _p(ww, ctypes.c_int64))
    if rc != 0:
        raise ValueError(f"oracle_aggregate failed ({rc})")
    m = int(o[-1])
    return o, ii[:m].copy(), ww[:m].copy()


def gain(g, membership, i: int, d: int) -> int:
    """Integer gain of moving i to community d: Eq. (2) times W^2/2."""
    off, idx, w = _arrays(g)
    c = np.ascontiguousarray(membership, dtype=np.int32)
    hi, lo = ctypes.c_int64(), ctypes.c_uint64()
    _load().oracle_gain(g.n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32), _p(w, ctypes.c_int64),
                        _p(c, ctypes.c_int32), i, d, ctypes.byref(hi), ctypes.byref(lo))
    return _i128(hi.value, lo.value)


def best_move(g, W: int, cprime, sigma, i: int):
    """(best community, gain) of vertex i against the state (C', Sigma'), or (None, None)."""
    off, idx, w = _arrays(g)
    c = np.ascontiguousarray(cprime, dtype=np.int32)
    s = np.ascontiguousarray(sigma, dtype=np.int64)
    d, hi, lo = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_uint64()
    found = _load().oracle_best_move(g.n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32), _p(w, ctypes.c_int64),
                                     W, _p(c, ctypes.c_int32), _p(s, ctypes.c_int64), i, ctypes.byref(d),
                                     ctypes.byref(hi), ctypes.byref(lo))
    if not found:
        return None, None
    return int(d.value), _i128(hi.value, lo.value)
