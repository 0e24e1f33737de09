"""ctypes binding of ``liblv.so`` (the C ABI in include/leanvec.h).

Argument marshalling only: device arrays are torch tensors on the GPU (their
``data_ptr()`` is passed), host arrays are numpy arrays, streams default to
torch's current stream.  Every computation runs in the library.  A missing
library is an error: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "liblv.so")

LV_OK, LV_WNOTCONVERGED = 0, 1
LV_EINVAL, LV_ENOMEM, LV_EDEVICE, LV_EUNSUPPORTED = -1, -2, -3, -4
LV_F32, LV_F16, LV_LVQ8, LV_F16_RESID, LV_LVQ8_LEVEL2 = 0, 1, 2, 3, 4
LV_LAUNCH_PER_QUERY, LV_LAUNCH_PERSISTENT, LV_LAUNCH_TEAM = 0, 1, 2
LV_SENTINEL = 0xFFFFFFFF
LV_FW_INIT_ES, LV_FW_INIT_ZERO, LV_FW_INIT_GIVEN = 0, 1, 2

_c_i32, _c_i64, _c_u32, _c_dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
_vp = ctypes.c_void_p


class LVError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"leanvec error {code}: {msg}")
        self.code = code


class IndexDesc(ctypes.Structure):
    _fields_ = [("N", _c_i64), ("D", _c_i32), ("d", _c_i32), ("bits", _c_i32),
                ("record_stride", _c_i32), ("records", _vp), ("mu", _vp), ("sec_dtype", _c_i32),
                ("secondaries", _vp), ("R", _c_i32), ("adjacency", _vp), ("entry", _c_u32),
                ("A", _vp), ("sec_mu", _vp)]


class SearchParams(ctypes.Structure):
    _fields_ = [("hash_slots", _c_i32), ("probes", _c_i32), ("launch", _c_i32),
                ("expand", _c_i32)]


class Request(ctypes.Structure):
    _fields_ = [("sub", _c_i32), ("k", _c_i32), ("L", _c_i32), ("count", _c_i32)]


class BatchCaps(ctypes.Structure):
    _fields_ = [("max_requests", _c_i32), ("max_L", _c_i32), ("max_queries", _c_i64)]


LV_MAX_BUILD_PASSES = 8


class BuildParams(ctypes.Structure):
    _fields_ = [("R", _c_i32), ("L", _c_i32), ("passes", _c_i32), ("hash_slots", _c_i32),
                ("alphas", _c_dbl * LV_MAX_BUILD_PASSES), ("max_batch", _c_i64),
                ("stop_after", _c_i64), ("stats", _vp)]


LV_BUILD_STATS = 7
BUILD_STAT_NAMES = ("searches", "expansions", "scorings", "forward_candidates",
                    "reverse_targets", "reverse_prunes", "reverse_candidates")


class FWParams(ctypes.Structure):
    _fields_ = [("alpha", _c_dbl), ("tol", _c_dbl), ("max_iter", _c_i32), ("init", _c_i32)]


class FWReport(ctypes.Structure):
    _fields_ = [("iters", _c_i32), ("converged", _c_i32), ("f_first", _c_dbl),
                ("f_last", _c_dbl), ("f_hist", _vp), ("gap_hist", _vp)]


# name -> (restype, argtypes)
_SIGS = {
    "lv_version": (_c_i32, []),
    "lv_last_error": (ctypes.c_char_p, []),
    "lv_second_moment": (_c_i32, [_vp, _c_i64, _c_i32, _vp, _vp]),
    "lv_fit_id": (_c_i32, [_vp, _c_i32, _c_i32, _vp, _vp]),
    "lv_fit_ood": (_c_i32, [_vp, _c_i64, _vp, _c_i64, _c_i32, _c_i32, _vp, _vp, _vp, _vp]),
    "lv_fit_es": (_c_i32, [_vp, _c_i64, _vp, _c_i64, _c_i32, _c_i32, _c_dbl, _vp, _vp]),
    "lv_ood_loss": (_c_i32, [_vp, _c_i64, _vp, _c_i64, _c_i32, _c_i32, _vp, _vp, _vp]),
    "lv_mean_reduced": (_c_i32, [_vp, _c_i32, _c_i32, _vp, _c_i64, _vp]),
    "lv_to_bf16": (_c_i32, [_vp, _c_i64, _vp]),
    "lv_project": (_c_i32, [_vp, _c_i64, _c_i32, _vp, _c_i32, _vp, _vp]),
    "lv_record_stride": (_c_i32, [_c_i32, _c_i32]),
    "lv_secondary_row_bytes": (_c_i32, [_c_i32, _c_i32]),
    "lv_lvq_encode": (_c_i32, [_vp, _c_i64, _c_i32, _vp, _c_i32, _vp, _c_i32, _vp]),
    "lv_lvq_decode": (_c_i32, [_vp, _c_i64, _c_i32, _c_i32, _c_i32, _vp, _vp, _vp]),
    "lv_project_encode": (_c_i32, [_vp, _c_i64, _c_i32, _vp, _c_i32, _vp, _c_i32, _vp, _c_i32,
                                   _vp]),
    "lv_lvq_encode_level2": (_c_i32, [_vp, _c_i64, _c_i32, _vp, _c_i32, _vp, _c_i32, _vp,
                                      _c_i32, _vp]),
    "lv_to_f16": (_c_i32, [_vp, _c_i64, _vp, _vp]),
    "lv_index_create": (_c_i32, [ctypes.POINTER(IndexDesc), ctypes.POINTER(_vp)]),
    "lv_index_destroy": (_c_i32, [_vp]),
    "lv_search_workspace_size": (ctypes.c_size_t, [_vp, _c_i64]),
    "lv_search": (_c_i32, [_vp, _vp, _c_i64, _c_i32, _c_i32, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                           ctypes.POINTER(SearchParams), _vp]),
    "lv_search_projected": (_c_i32, [_vp, _vp, _vp, _c_i64, _c_i32, _c_i32, _vp, _vp, _vp,
                                     ctypes.POINTER(SearchParams), _vp]),
    "lv_search_noalloc": (_c_i32, [_vp, _vp, _c_i64, _c_i32, _c_i32, _vp, _vp, _vp,
                                   ctypes.POINTER(SearchParams), _vp]),
    "lv_multi_create": (_c_i32, [ctypes.POINTER(_vp), _c_i32, ctypes.POINTER(_vp)]),
    "lv_multi_destroy": (_c_i32, [_vp]),
    "lv_batch_create": (_c_i32, [_vp, ctypes.POINTER(BatchCaps), ctypes.POINTER(SearchParams),
                                 ctypes.POINTER(_vp)]),
    "lv_batch_destroy": (_c_i32, [_vp]),
    "lv_batch_step": (_c_i32, [_vp, ctypes.POINTER(Request), _c_i32, _vp, _vp, _vp, _vp, _vp]),
    "lv_batch_step_timed": (_c_i32, [_vp, ctypes.POINTER(Request), _c_i32, _vp, _vp, _vp, _vp,
                                     _vp, _vp, _vp]),
    "lv_autotune_window": (_c_i32, [_vp, _c_i32, _vp, _c_i64, _vp, _c_i32, _c_i32, _c_dbl,
                                    _c_i32, ctypes.POINTER(SearchParams),
                                    ctypes.POINTER(_c_i32), ctypes.POINTER(_c_dbl), _vp]),
    "lv_gemm": (_c_i32, [_vp, _c_i32, _c_i64, _vp, _c_i32, _c_i64, _vp, _c_i64, _c_i32, _c_i32,
                         _c_i32, ctypes.c_float, ctypes.c_float, _vp, ctypes.c_size_t, _vp]),
    "lv_gemm_split": (_c_i32, [_vp, _c_i32, _c_i64, _vp, _c_i32, _c_i64, _vp, _c_i64, _c_i32,
                               _c_i32, _c_i32, ctypes.c_float, ctypes.c_float, _vp,
                               ctypes.c_size_t, _vp]),
    "lv_gemm_bf16": (_c_i32, [_vp, _c_i64, _vp, _c_i64, _vp, _c_i64, _c_i32, _c_i32, _c_i32,
                              ctypes.c_float, ctypes.c_float, _vp]),
    "lv_gemm_workspace_size": (ctypes.c_size_t, [_c_i32, _c_i32]),
    "lv_projloss_workspace_size": (ctypes.c_size_t, [_c_i32, _c_i32, _c_i32, _c_i32]),
    "lv_projloss_fwd": (_c_i32, [_vp, _vp, _vp, _vp, _c_i32, _c_i32, _c_i32, _c_i32, _vp, _vp,
                                 _c_dbl, ctypes.c_float, _vp, _vp, ctypes.c_size_t, _vp]),
    "lv_projloss_bwd": (_c_i32, [_vp, _vp, _vp, _vp, _c_i32, _c_i32, _c_i32, _c_i32, _vp, _vp,
                                 ctypes.c_float, ctypes.c_float, _vp, _vp, _vp, ctypes.c_size_t,
                                 _vp]),
    "lv_adam_step": (_c_i32, [_vp, _vp, _vp, _vp, _c_i64, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, ctypes.c_float, _c_i32, _vp]),
    "lv_clip_spectral": (_c_i32, [_vp, _c_i32, _c_i32]),
    "lv_clip_spectral_device": (_c_i32, [_vp, _c_i32, _c_i32, _vp, ctypes.c_size_t, _vp]),
    "lv_clip_spectral_device_workspace_size": (ctypes.c_size_t, [_c_i32, _c_i32]),
    "lv_graph_build": (_c_i32, [_vp, _c_i32, _c_i64, _c_i32, _c_i32, _vp, _c_u32,
                                ctypes.POINTER(BuildParams), _vp, _vp]),
    "lv_autotune_knobs": (_c_i32, [_vp, ctypes.POINTER(BatchCaps), ctypes.POINTER(Request),
                                   _c_i32, _vp, _vp, _vp, _c_i32, ctypes.POINTER(SearchParams),
                                   ctypes.POINTER(_c_dbl), _vp]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load liblv.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2312_16335_amd/build.py "
                              "(or __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_names():
    return list(_SIGS)


def _check(rc: int, allow_warn: bool = False) -> int:
    if rc == LV_OK or (allow_warn and rc == LV_WNOTCONVERGED):
        return rc
    raise LVError(rc, load().lv_last_error().decode())


def _host(a: np.ndarray, dtype) -> np.ndarray:
    if not (isinstance(a, np.ndarray) and a.dtype == dtype and a.flags.c_contiguous):
        raise TypeError(f"expected a C-contiguous numpy {np.dtype(dtype)} array")
    return a


def _dev(t, dtype=None):
    """data_ptr of a contiguous CUDA tensor (or 0 for None)."""
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a GPU tensor")
    if not t.is_contiguous():
        raise TypeError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    return t.data_ptr()


def _need(t, n: int, what: str) -> None:
    """Raise ValueError unless tensor t holds at least n elements."""
    if t is not None and t.numel() < n:
        raise ValueError(f"{what} holds {t.numel()} elements, needs at least {n}")


def _rows_cols(t, what: str, cols: Optional[int] = None, min_rows: int = 0):
    """(rows, cols) of a 2-D tensor, checked against the expected columns and
    a minimum row count; raises ValueError otherwise."""
    if t.dim() != 2:
        raise ValueError(f"{what} must be 2-D, got shape {tuple(t.shape)}")
    r, c = int(t.shape[0]), int(t.shape[1])
    if cols is not None and c != cols:
        raise ValueError(f"{what} must have {cols} columns, got shape {tuple(t.shape)}")
    if r < min_rows:
        raise ValueError(f"{what} must have at least {min_rows} rows, got {r}")
    return r, c


def _stream(stream):
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


# ---------------------------------------------------------------- host fit

def lv_version() -> int:
    return load().lv_version()


def lv_second_moment(V: np.ndarray, K: np.ndarray, sum_: Optional[np.ndarray] = None) -> None:
    V = _host(V, np.float32)
    _host(K, np.float64)
    n, D = V.shape
    _check(load().lv_second_moment(V.ctypes.data, n, D, K.ctypes.data,
                                   None if sum_ is None else _host(sum_, np.float64).ctypes.data))


def lv_fit_id(KX: np.ndarray, d: int, with_evals: bool = False):
    KX = _host(KX, np.float64)
    D = KX.shape[0]
    P = np.empty((d, D), np.float64)
    ev = np.empty(D, np.float64) if with_evals else None
    _check(load().lv_fit_id(KX.ctypes.data, D, d, P.ctypes.data,
                            None if ev is None else ev.ctypes.data))
    return (P, ev) if with_evals else P


def lv_fit_ood(KQ, m, KX, n, d, alpha=0.9, tol=1e-3, max_iter=500, init=LV_FW_INIT_ES,
               A0=None, B0=None):
    KQ = _host(KQ, np.float64)
    KX = _host(KX, np.float64)
    D = KQ.shape[0]
    A = np.zeros((d, D)) if A0 is None else np.array(A0, np.float64, order="C")
    B = np.zeros((d, D)) if B0 is None else np.array(B0, np.float64, order="C")
    fh = np.zeros(max_iter + 1)
    gh = np.zeros(max_iter)
    rep = FWReport(0, 0, 0.0, 0.0, fh.ctypes.data, gh.ctypes.data)
    prm = FWParams(alpha, tol, max_iter, init)
    rc = _check(load().lv_fit_ood(KQ.ctypes.data, m, KX.ctypes.data, n, D, d, ctypes.byref(prm),
                                  A.ctypes.data, B.ctypes.data, ctypes.byref(rep)),
                allow_warn=True)
    info = {"iters": rep.iters, "converged": bool(rep.converged), "f_first": rep.f_first,
            "f_last": rep.f_last, "f": fh[:rep.iters + 1].copy(), "gap": gh[:rep.iters].copy(),
            "status": rc}
    return A, B, info


def lv_fit_es(KQ, m, KX, n, d, xtol=1e-4):
    KQ = _host(KQ, np.float64)
    KX = _host(KX, np.float64)
    D = KQ.shape[0]
    P = np.empty((d, D))
    beta = ctypes.c_double(0.0)
    _check(load().lv_fit_es(KQ.ctypes.data, m, KX.ctypes.data, n, D, d, xtol, P.ctypes.data,
                            ctypes.byref(beta)))
    return P, beta.value


def lv_ood_loss(KQ, m, KX, n, A, B) -> float:
    KQ, KX = _host(KQ, np.float64), _host(KX, np.float64)
    A = np.ascontiguousarray(A, np.float64)
    B = np.ascontiguousarray(B, np.float64)
    f = ctypes.c_double(0.0)
    _check(load().lv_ood_loss(KQ.ctypes.data, m, KX.ctypes.data, n, KQ.shape[0], A.shape[0],
                              A.ctypes.data, B.ctypes.data, ctypes.byref(f)))
    return f.value


def lv_mean_reduced(M: np.ndarray, sum_: np.ndarray, n: int) -> np.ndarray:
    M = _host(M, np.float64)
    mu = np.empty(M.shape[0], np.float32)
    _check(load().lv_mean_reduced(M.ctypes.data, M.shape[0], M.shape[1],
                                  _host(sum_, np.float64).ctypes.data, n, mu.ctypes.data))
    return mu


def lv_to_bf16(M: np.ndarray) -> np.ndarray:
    M = np.ascontiguousarray(M, np.float64)
    out = np.empty(M.shape, np.uint16)
    _check(load().lv_to_bf16(M.ctypes.data, M.size, out.ctypes.data))
    return out


# ------------------------------------------------------------ device calls

def lv_project(V, M_bf16, out, stream=None) -> None:
    """out[rows, d] = V[rows, D] @ M^T with M given as bfloat16 bits (int16 tensor)."""
    import torch

    rows, D = _rows_cols(V, "V")
    d, _ = _rows_cols(M_bf16, "M_bf16", cols=D)
    if M_bf16.element_size() != 2:
        raise ValueError("M_bf16 must hold 2-byte bfloat16 bits")
    _need(out, rows * d, "out")
    _check(load().lv_project(_dev(V, torch.float32), rows, D, _dev(M_bf16), d,
                             _dev(out, torch.float32), _stream(stream)))


def lv_record_stride(d: int, bits: int) -> int:
    return load().lv_record_stride(d, bits)


def lv_secondary_row_bytes(D: int, sec_dtype: int) -> int:
    return load().lv_secondary_row_bytes(D, sec_dtype)


def lv_lvq_encode(Y, mu, bits: int, records, stream=None) -> None:
    import torch

    n, d = _rows_cols(Y, "Y")
    _need(mu, d, "mu")
    _rows_cols(records, "records", min_rows=n)
    _check(load().lv_lvq_encode(_dev(Y, torch.float32), n, d, _dev(mu, torch.float32), bits,
                                _dev(records, torch.uint8), records.shape[1], _stream(stream)))


def lv_lvq_decode(records, d: int, bits: int, mu, out, stream=None) -> None:
    """out (device float32 [n][d], written) = the float32-rounded reconstruction
    of the LVQ records (device uint8 [n][stride])."""
    import torch

    n, stride = _rows_cols(records, "records")
    _need(mu, d, "mu")
    _rows_cols(out, "out", cols=d, min_rows=n)
    _check(load().lv_lvq_decode(_dev(records, torch.uint8), n, d, bits, stride,
                                _dev(mu, torch.float32), _dev(out, torch.float32),
                                _stream(stream)))


def lv_project_encode(V, M_bf16, mu, bits: int, records, stream=None) -> None:
    """LVQ records of V M^T (device uint8 [rows][stride], written) in one pass;
    the bytes lv_project followed by lv_lvq_encode would give."""
    import torch

    rows, D = _rows_cols(V, "V")
    d = _rows_cols(M_bf16, "M_bf16", cols=D)[0]
    if M_bf16.element_size() != 2:
        raise ValueError("M_bf16 must hold 2-byte bfloat16 bits")
    _need(mu, d, "mu")
    _rows_cols(records, "records", min_rows=rows)
    _check(load().lv_project_encode(_dev(V, torch.float32), rows, D, _dev(M_bf16), d,
                                    _dev(mu, torch.float32), bits, _dev(records, torch.uint8),
                                    records.shape[1], _stream(stream)))


def lv_lvq_encode_level2(Y, mu, bits: int, records, rows, stream=None) -> None:
    """Second level of a two-level LVQ: rows (device uint8 [n][row bytes]) from
    Y, mu and the primary records written by lv_lvq_encode with the same bits."""
    import torch

    n, d = _rows_cols(Y, "Y")
    _need(mu, d, "mu")
    _rows_cols(records, "records", min_rows=n)
    _rows_cols(rows, "rows", min_rows=n)
    _check(load().lv_lvq_encode_level2(_dev(Y, torch.float32), n, d, _dev(mu, torch.float32),
                                       bits, _dev(records, torch.uint8), records.shape[1],
                                       _dev(rows, torch.uint8), rows.shape[1], _stream(stream)))


def lv_to_f16(X, out, stream=None) -> None:
    import torch

    _need(out, X.numel(), "out")
    _check(load().lv_to_f16(_dev(X, torch.float32), X.numel(), _dev(out, torch.float16),
                            _stream(stream)))


def build_params(R: int, L: int, alphas=(1.0, 1.0), max_batch: int = 1, stop_after: int = 0,
                 hash_slots: int = 0) -> BuildParams:
    if not 1 <= len(alphas) <= LV_MAX_BUILD_PASSES:
        raise ValueError(f"1..{LV_MAX_BUILD_PASSES} passes")
    bp = BuildParams()
    bp.R, bp.L, bp.passes, bp.hash_slots = R, L, len(alphas), hash_slots
    for i, a in enumerate(alphas):
        bp.alphas[i] = float(a)
    bp.max_batch, bp.stop_after = max_batch, stop_after
    return bp


def lv_graph_build(records, N: int, d: int, bits: int, order: np.ndarray, entry: int,
                   params: BuildParams, adjacency, stream=None, stats: bool = False):
    """records: device uint8 [N][stride]; order: host uint32 [N]; adjacency:
    device int32 [N][R] (uint32 ids, LV_SENTINEL = -1), written.  With
    stats=True returns the work counters as a dict."""
    import torch

    order = _host(order, np.uint32)
    if order.shape != (N,) or records.shape[0] < N or tuple(adjacency.shape) != (N, params.R):
        raise ValueError("order must be [N], records [>= N][stride], adjacency [N][R]")
    st = np.zeros(LV_BUILD_STATS, dtype=np.int64)
    params.stats = st.ctypes.data if stats else None
    try:
        _check(load().lv_graph_build(_dev(records, torch.uint8), records.shape[1], N, d, bits,
                                     order.ctypes.data, entry, ctypes.byref(params),
                                     _dev(adjacency, torch.int32), _stream(stream)))
    finally:
        params.stats = None
    return dict(zip(BUILD_STAT_NAMES, st.tolist())) if stats else None


class Index:
    """Handle over device arrays (borrowed: keep the tensors alive)."""

    def __init__(self, records, mu, secondaries, adjacency, entry: int, bits: int, d: int,
                 A_bf16=None, sec_mu=None, residual: bool = False, level2: bool = False,
                 D: int = 0):
        """secondaries: float16 or float32 [N][D], or (with sec_mu, float32 [D]) uint8
        LVQ-8 rows [N][D + 16] from lv_lvq_encode, or (residual=True) float16
        residual coordinates [N][D - d] with A_bf16 the [D][D] basis, or
        (level2=True) the primaries' second level, uint8 rows from
        lv_lvq_encode_level2; then D is the argument, else A_bf16's columns."""
        import torch

        N, sec_cols = _rows_cols(secondaries, "secondaries")
        if level2:
            if not D:
                if A_bf16 is None:
                    raise ValueError("level2 needs D or A_bf16")
                D = _rows_cols(A_bf16, "A_bf16")[1]
            sec_dtype = LV_LVQ8_LEVEL2
            if sec_cols != lv_secondary_row_bytes(d, LV_LVQ8_LEVEL2):
                raise ValueError(f"second-level rows need "
                                 f"{lv_secondary_row_bytes(d, LV_LVQ8_LEVEL2)} bytes for d = {d}")
        elif residual:
            sec_dtype, D = LV_F16_RESID, sec_cols + d
        elif sec_mu is not None:
            sec_dtype, D = LV_LVQ8, int(sec_mu.numel())
            if sec_cols != lv_secondary_row_bytes(D, LV_LVQ8):
                raise ValueError(f"LVQ-8 secondaries need rows of "
                                 f"{lv_secondary_row_bytes(D, LV_LVQ8)} bytes for D = {D}")
        else:
            sec_dtype = LV_F16 if secondaries.dtype == torch.float16 else LV_F32
            D = sec_cols
        # the library cannot see buffer sizes: check them here, before any launch
        _rows_cols(records, "records", min_rows=N)
        _need(mu, d, "mu")
        R = _rows_cols(adjacency, "adjacency", min_rows=N)[1]
        if not 0 <= entry < N:
            raise ValueError(f"entry {entry} outside [0, {N})")
        if A_bf16 is not None:
            _rows_cols(A_bf16, "A_bf16", cols=D, min_rows=D if residual else d)
        self._keep = (records, mu, secondaries, adjacency, A_bf16, sec_mu)
        self.desc = IndexDesc(N, D, d, bits, records.shape[1], _dev(records, torch.uint8),
                              _dev(mu, torch.float32), sec_dtype, _dev(secondaries),
                              adjacency.shape[1], _dev(adjacency, torch.int32), entry,
                              _dev(A_bf16) if A_bf16 is not None else None,
                              _dev(sec_mu, torch.float32) if sec_mu is not None else None)
        h = _vp()
        _check(load().lv_index_create(ctypes.byref(self.desc), ctypes.byref(h)))
        self.handle = h
        self.N, self.D, self.d, self.R = N, D, d, R
        # floats per projected query: P q, plus P_perp q with residual secondaries
        self.qp_width = D if residual else d

    def close(self):
        if self.handle:
            load().lv_index_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _params(hash_slots: int = 0, probes: int = 0, launch: int = 0, expand: int = 0):
    return ctypes.byref(SearchParams(hash_slots, probes, launch, expand))


def _search_outputs(m: int, k: int, ids, scores, counters) -> None:
    """ids and scores hold m * k results, counters two per query."""
    if k >= 1:
        _need(ids, m * k, "ids")
        _need(scores, m * k, "scores")
    _need(counters, 2 * m, "counters")


def lv_search_workspace_size(index: Index, m: int) -> int:
    return load().lv_search_workspace_size(index.handle, m)


def lv_search(index: Index, Q, k: int, L: int, ids, scores, counters=None, ws=None,
              hash_slots: int = 0, stream=None, probes: int = 0, expand: int = 0,
              launch: int = LV_LAUNCH_PER_QUERY) -> None:
    import torch

    m = _rows_cols(Q, "Q", cols=index.D)[0]
    _search_outputs(m, k, ids, scores, counters)
    ws_bytes = ws.numel() * ws.element_size() if ws is not None else 0
    if ws_bytes < lv_search_workspace_size(index, m):
        raise ValueError(f"workspace of {ws_bytes} bytes, needs "
                         f"{lv_search_workspace_size(index, m)}")
    _check(load().lv_search(index.handle, _dev(Q, torch.float32), m, k, L,
                            _dev(ids, torch.int32), _dev(scores, torch.float32),
                            _dev(counters, torch.int32), _dev(ws), ws_bytes,
                            _params(hash_slots, probes, launch, expand), _stream(stream)))


LV_NOALLOC_SCRATCH_BYTES = 16 << 20


def lv_search_noalloc(index: Index, Q, k: int, L: int, ids, scores, counters=None,
                      hash_slots: int = 0, stream=None, probes: int = 0, expand: int = 0,
                      launch: int = LV_LAUNCH_PER_QUERY) -> None:
    """lv_search with the library's fixed scratch array instead of a workspace
    (allocates nothing; at most LV_NOALLOC_SCRATCH_BYTES of projected queries)."""
    import torch

    m = _rows_cols(Q, "Q", cols=index.D)[0]
    _search_outputs(m, k, ids, scores, counters)
    _check(load().lv_search_noalloc(index.handle, _dev(Q, torch.float32), m, k, L,
                                    _dev(ids, torch.int32), _dev(scores, torch.float32),
                                    _dev(counters, torch.int32),
                                    _params(hash_slots, probes, launch, expand),
                                    _stream(stream)))


def lv_search_projected(index: Index, Q, Qp, k: int, L: int, ids, scores, counters=None,
                        hash_slots: int = 0, stream=None, probes: int = 0,
                        expand: int = 0, launch: int = LV_LAUNCH_PER_QUERY) -> None:
    import torch

    m = _rows_cols(Q, "Q", cols=index.D)[0]
    _rows_cols(Qp, "Qp", cols=index.qp_width, min_rows=m)
    _search_outputs(m, k, ids, scores, counters)
    _check(load().lv_search_projected(index.handle, _dev(Q, torch.float32),
                                      _dev(Qp, torch.float32), m, k, L, _dev(ids, torch.int32),
                                      _dev(scores, torch.float32), _dev(counters, torch.int32),
                                      _params(hash_slots, probes, launch, expand),
                                      _stream(stream)))


# ------------------------------------------------------------ batched search

class Multi:
    """Several Index handles searched together (keeps them alive)."""

    def __init__(self, indexes):
        self._subs = list(indexes)
        self.D = self._subs[0].D if self._subs else 0
        arr = (_vp * len(self._subs))(*[ix.handle for ix in self._subs])
        h = _vp()
        _check(load().lv_multi_create(arr, len(self._subs), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            load().lv_multi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _step_buffers(multi: "Multi", reqs, Q, ids, scores, counters=None) -> None:
    """Q holds the requests' queries (rows packed in request order), ids and
    scores count * k results per request, counters two per query."""
    nq = sum(max(int(c), 0) for (_, _, _, c) in reqs)
    nres = sum(max(int(c), 0) * max(int(k), 0) for (_, k, _, c) in reqs)
    _rows_cols(Q, "Q", cols=multi.D, min_rows=nq)
    _need(ids, nres, "ids")
    _need(scores, nres, "scores")
    _need(counters, 2 * nq, "counters")


def _requests(reqs):
    arr = (Request * len(reqs))()
    for i, (sub, k, L, count) in enumerate(reqs):
        arr[i] = Request(sub, k, L, count)
    return arr


class Batch:
    """Captured batched step (lv_batch_create)."""

    def __init__(self, multi: Multi, max_requests: int, max_queries: int, max_L: int,
                 hash_slots: int = 0, probes: int = 0, launch: int = LV_LAUNCH_PER_QUERY,
                 expand: int = 0):
        self.multi = multi
        self.caps = BatchCaps(max_requests, max_L, max_queries)
        h = _vp()
        _check(load().lv_batch_create(multi.handle, ctypes.byref(self.caps),
                                      _params(hash_slots, probes, launch, expand),
                                      ctypes.byref(h)))
        self.handle = h

    def step(self, reqs, Q, ids, scores, counters=None, stream=None, events=None):
        """reqs: list of (sub, k, L, count); Q rows and outputs packed in request order.
        events: optional pair of timing torch.cuda.Event recorded around the traversal
        (lv_batch_step_timed)."""
        import torch

        _step_buffers(self.multi, reqs, Q, ids, scores, counters)
        arr = _requests(reqs)
        args = (self.handle, arr, len(reqs), _dev(Q, torch.float32), _dev(ids, torch.int32),
                _dev(scores, torch.float32), _dev(counters, torch.int32))
        if events is None:
            _check(load().lv_batch_step(*args, _stream(stream)))
            return
        raw = []
        for ev in events:
            if not ev.cuda_event:  # torch creates the event on its first record
                ev.record(None if isinstance(stream, int) else stream)
            raw.append(_vp(ev.cuda_event))
        _check(load().lv_batch_step_timed(*args, raw[0], raw[1], _stream(stream)))

    def close(self):
        if self.handle:
            load().lv_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lv_autotune_window(multi: Multi, sub: int, Q, truth: np.ndarray, k: int, target: float,
                       L_max: int, hash_slots: int = 0, stream=None, expand: int = 0):
    import torch

    truth = np.ascontiguousarray(truth, dtype=np.uint32)
    m = _rows_cols(Q, "Q", cols=multi.D)[0]
    if truth.ndim != 2 or truth.shape[0] < m or truth.shape[1] < k:
        raise ValueError(f"truth must be [{m}][>= {k}], got {truth.shape}")
    L = ctypes.c_int32(0)
    rec = ctypes.c_double(0.0)
    _check(load().lv_autotune_window(multi.handle, sub, _dev(Q, torch.float32), Q.shape[0],
                                      truth.ctypes.data, truth.shape[1], k, target, L_max,
                                      _params(hash_slots, 0, 0, expand), ctypes.byref(L),
                                      ctypes.byref(rec),
                                      _stream(stream)))
    return L.value, rec.value


def lv_autotune_knobs(multi: Multi, max_requests, max_queries, max_L, reqs, Q, ids, scores,
                      reps=3, stream=None, expand: int = 0):
    import torch

    _step_buffers(multi, reqs, Q, ids, scores)
    caps = BatchCaps(max_requests, max_L, max_queries)
    best = SearchParams(0, 0, 0, expand)
    ms = ctypes.c_double(0.0)
    _check(load().lv_autotune_knobs(multi.handle, ctypes.byref(caps), _requests(reqs), len(reqs),
                                    _dev(Q, torch.float32), _dev(ids, torch.int32),
                                    _dev(scores, torch.float32), reps, ctypes.byref(best),
                                    ctypes.byref(ms), _stream(stream)))
    return {"hash_slots": best.hash_slots, "probes": best.probes, "launch": best.launch,
            "expand": best.expand}, ms.value


# ------------------------------------------------- differentiable projection

def lv_gemm(A, B, C, M, N, K, a_kcont=True, b_kcont=True, lda=None, ldb=None, ldc=None,
            alpha=1.0, beta=0.0, workspace=None, stream=None, split=False):
    """C = alpha op(A) op(B)^T + beta C (lv_gemm; lv_gemm_split with split=True)."""
    import torch

    lda = lda if lda is not None else (K if a_kcont else M)
    ldb = ldb if ldb is not None else (K if b_kcont else N)
    ldc = ldc if ldc is not None else N
    # element extents of the strided operands (rows of ld elements)
    _need(A, (M - 1) * lda + K if a_kcont else (K - 1) * lda + M, "A")
    _need(B, (N - 1) * ldb + K if b_kcont else (K - 1) * ldb + N, "B")
    _need(C, (M - 1) * ldc + N, "C")
    ws, ws_bytes = None, 0
    if workspace is not None:
        ws, ws_bytes = _dev(workspace, workspace.dtype), workspace.numel() * workspace.element_size()
    fn = load().lv_gemm_split if split else load().lv_gemm
    _check(fn(_dev(A, torch.float32), int(a_kcont), lda, _dev(B, torch.float32), int(b_kcont),
              ldb, _dev(C, torch.float32), ldc, M, N, K, alpha, beta, ws, ws_bytes,
              _stream(stream)))


def lv_gemm_bf16(A, B, C, M, N, K, lda=None, ldb=None, ldc=None, alpha=1.0, beta=0.0,
                 stream=None):
    """C = alpha A B^T + beta C with A [M][lda], B [N][ldb] bfloat16 (k-contiguous
    rows; torch.bfloat16 or their int16 bits) and C float32 (lv_gemm_bf16)."""
    import torch

    lda = lda if lda is not None else K
    ldb = ldb if ldb is not None else K
    ldc = ldc if ldc is not None else N
    for t, what in ((A, "A"), (B, "B")):
        if t.dtype not in (torch.bfloat16, torch.int16):
            raise TypeError(f"{what} must hold bfloat16 (or its int16 bits), got {t.dtype}")
    _need(A, (M - 1) * lda + K if M > 0 else 0, "A")
    _need(B, (N - 1) * ldb + K if N > 0 else 0, "B")
    _need(C, (M - 1) * ldc + N if M > 0 else 0, "C")
    _check(load().lv_gemm_bf16(_dev(A), lda, _dev(B), ldb, _dev(C, torch.float32), ldc, M, N, K,
                               alpha, beta, _stream(stream)))


def lv_gemm_workspace_size(M, N) -> int:
    return load().lv_gemm_workspace_size(M, N)


def lv_projloss_workspace_size(bq, bx, D, d) -> int:
    return load().lv_projloss_workspace_size(bq, bx, D, d)


def _projloss_operands(A, B, Qb, Xb, ws, KQn, KXn):
    """Shapes of the refinement operands: A, B [d][D], Qb [bq][D], Xb [bx][D],
    KQn, KXn [D][D] (both or neither), workspace large enough."""
    d, D = _rows_cols(A, "A")
    _rows_cols(B, "B", cols=D, min_rows=d)
    bq = _rows_cols(Qb, "Qb", cols=D)[0]
    bx = _rows_cols(Xb, "Xb", cols=D)[0]
    if (KQn is None) != (KXn is None):
        raise ValueError("KQn and KXn are given together or not at all")
    if KQn is not None:
        _rows_cols(KQn, "KQn", cols=D, min_rows=D)
        _rows_cols(KXn, "KXn", cols=D, min_rows=D)
    need = lv_projloss_workspace_size(bq, bx, D, d)
    if ws.numel() * ws.element_size() < need:
        raise ValueError(f"workspace of {ws.numel() * ws.element_size()} bytes, needs {need}")
    return d, D


def lv_projloss_fwd(A, B, Qb, Xb, loss, ws, KQn=None, KXn=None, trace_const=0.0, lam=1.0,
                    stream=None):
    import torch

    d, D = _projloss_operands(A, B, Qb, Xb, ws, KQn, KXn)
    _need(loss, 3, "loss")
    _check(load().lv_projloss_fwd(_dev(A, torch.float32), _dev(B, torch.float32),
                                  _dev(Qb, torch.float32), _dev(Xb, torch.float32), Qb.shape[0],
                                  Xb.shape[0], D, d, _dev(KQn, torch.float32),
                                  _dev(KXn, torch.float32), trace_const, lam,
                                  _dev(loss, torch.float32), _dev(ws),
                                  ws.numel() * ws.element_size(), _stream(stream)))


def lv_projloss_bwd(A, B, Qb, Xb, dA, dB, ws, KQn=None, KXn=None, lam=1.0, grad_scale=1.0,
                    stream=None):
    import torch

    d, D = _projloss_operands(A, B, Qb, Xb, ws, KQn, KXn)
    _rows_cols(dA, "dA", cols=D, min_rows=d)
    _rows_cols(dB, "dB", cols=D, min_rows=d)
    _check(load().lv_projloss_bwd(_dev(A, torch.float32), _dev(B, torch.float32),
                                  _dev(Qb, torch.float32), _dev(Xb, torch.float32), Qb.shape[0],
                                  Xb.shape[0], D, d, _dev(KQn, torch.float32),
                                  _dev(KXn, torch.float32), lam, grad_scale,
                                  _dev(dA, torch.float32), _dev(dB, torch.float32), _dev(ws),
                                  ws.numel() * ws.element_size(), _stream(stream)))


def lv_adam_step(p, g, m, v, lr, t, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    import torch

    for buf, what in ((g, "g"), (m, "m"), (v, "v")):
        _need(buf, p.numel(), what)
    _check(load().lv_adam_step(_dev(p, torch.float32), _dev(g, torch.float32),
                               _dev(m, torch.float32), _dev(v, torch.float32), p.numel(), lr,
                               beta1, beta2, eps, t, _stream(stream)))


def lv_clip_spectral(M: np.ndarray) -> np.ndarray:
    M = np.array(M, dtype=np.float64, order="C")
    _check(load().lv_clip_spectral(M.ctypes.data, M.shape[0], M.shape[1]))
    return M


def lv_clip_spectral_device_workspace_size(d: int, D: int) -> int:
    return load().lv_clip_spectral_device_workspace_size(d, D)


def lv_clip_spectral_device(M, ws, stream=None) -> None:
    """In place on a device float32 [d][D] tensor; ws: device workspace tensor."""
    import torch

    d, D = _rows_cols(M, "M")
    need = lv_clip_spectral_device_workspace_size(d, D)
    if ws.numel() * ws.element_size() < need:
        raise ValueError(f"workspace of {ws.numel() * ws.element_size()} bytes, needs {need}")
    _check(load().lv_clip_spectral_device(_dev(M, torch.float32), d, D, _dev(ws),
                                          ws.numel() * ws.element_size(), _stream(stream)))
