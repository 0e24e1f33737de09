"""Python side of the graph builder in ``vamana.c`` (input preparation).

``build_graph`` returns (adjacency uint32 [n, R], entry id).  The shared
library is compiled with gcc on first use (or by the package build step).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vamana.c")
_LIB = os.path.join(_HERE, "_lib", "libvamana.so")
SENTINEL = 0xFFFFFFFF

_lib = None


def compile_lib(force: bool = False) -> str:
    """Compile ``vamana.c`` into ``synth/_lib/libvamana.so`` with gcc."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v4", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(compile_lib())
        lib.lvg_build.restype = ctypes.c_int64
        lib.lvg_build.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                                  ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p]
        lib.lvg_reachable.restype = ctypes.c_int64
        lib.lvg_reachable.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_uint32, ctypes.c_void_p]
        lib.lvg_medoid.restype = ctypes.c_uint32
        lib.lvg_medoid.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32]
        lib.lvg_repair.restype = ctypes.c_int64
        lib.lvg_repair.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_uint32, ctypes.c_void_p]
        _lib = lib
    return _lib


METRIC_L2, METRIC_IP = 0, 1


def build_graph(X: np.ndarray, R: int, L: int = 0, metric: int = METRIC_L2,
                alphas: Sequence[float] = (1.0, 1.0), maxc: int = 0,
                batch_frac: float = 0.02, seed: int = 7,
                threads: int = 0) -> Tuple[np.ndarray, int]:
    """Graph over the rows of X.

    Rows are rounded to float16 (as the secondary vectors are).  The
    default is the Euclidean rule (on unit-norm rows it ranks neighbours
    exactly as inner product does) with two passes at alpha = 1.0.  The
    paper's Euclidean setting is alpha = 1.2; on the synthetic cluster
    mixtures, whose members are nearly equidistant, alpha = 1.2 keeps the
    nearest R cluster members and the graph navigates poorly, while 1.0
    prunes them into diverse edges (recall@10 at window 100 on 300k vectors:
    0.88 vs 0.97).  L defaults to R (search window during construction):
    on the 1M x 768 mixture (R = 64), build windows of 64, 96, 128 and 200
    need search windows of 96, 112, 143 and 175 for 10-recall@10 = 0.90.  maxc caps the
    pruning pool (default 8R).  Deterministic for any thread count.
    """
    X = _as_f16(X)
    n, dim = X.shape
    L = L or R
    maxc = maxc or 8 * R
    al = np.ascontiguousarray(alphas, dtype=np.float32)
    adj = np.empty((n, R), dtype=np.uint32)
    entry = _load().lvg_build(X.ctypes.data, n, dim, metric, R, L, maxc, al.ctypes.data, len(al),
                              float(batch_frac), seed, threads, adj.ctypes.data)
    if entry < 0:
        raise ValueError("graph build rejected its arguments")
    # connect anything the entry cannot reach (deterministic, usually a few nodes)
    _load().lvg_repair(X.ctypes.data, n, dim, metric, R, L, entry, adj.ctypes.data)
    return adj, int(entry)


def reachable(adj: np.ndarray, entry: int) -> np.ndarray:
    adj = np.ascontiguousarray(adj, dtype=np.uint32)
    n, R = adj.shape
    mark = np.empty(n, dtype=np.uint8)
    _load().lvg_reachable(adj.ctypes.data, n, R, entry, mark.ctypes.data)
    return mark.astype(bool)


def medoid(X: np.ndarray) -> int:
    X = _as_f16(X)
    return int(_load().lvg_medoid(X.ctypes.data, X.shape[0], X.shape[1]))


def _as_f16(X: np.ndarray) -> np.ndarray:
    """The builder works on float16 copies (round to nearest even)."""
    if X.dtype == np.float16 and X.flags.c_contiguous:
        return X
    return np.ascontiguousarray(X, dtype=np.float16)
