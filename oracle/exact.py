"""Exact maximum-inner-product search (ground truth), float64.

Section 2 (notation) defines the task: for a query q, return the k database
vectors with the largest <q, x>.  Ties are broken towards the smaller id so
the answer is unique.  Recall follows Appendix D.3 ("Metrics"):
k-recall@k = |S intersect G| / k.

Pinned by: a full sort on tiny inputs (tests/test_oracle_exact.py).
"""
from __future__ import annotations

import numpy as np

SENTINEL = 0xFFFFFFFF


def topk_ids(scores: np.ndarray, k: int) -> np.ndarray:
    """Indices of the k largest entries of each row (ties: smaller index)."""
    scores = np.asarray(scores, dtype=np.float64)
    m, n = scores.shape
    k = min(k, n)
    out = np.empty((m, k), dtype=np.int64)
    for i in range(m):
        row = scores[i]
        if k < n:
            # everything strictly better than the k-th value, plus ties in id order
            kth = np.partition(row, n - k)[n - k]
            cand = np.flatnonzero(row >= kth)
        else:
            cand = np.arange(n)
        order = np.lexsort((cand, -row[cand]))
        out[i] = cand[order[:k]]
    return out


def ground_truth(Q: np.ndarray, X: np.ndarray, k: int, chunk: int = 1 << 16) -> np.ndarray:
    """Top-k ids of <q, x> over the original vectors, computed in float64."""
    Q64 = np.asarray(Q, dtype=np.float64)
    m = Q64.shape[0]
    n = X.shape[0]
    best_s = np.full((m, 0), -np.inf)
    best_i = np.zeros((m, 0), dtype=np.int64)
    for lo in range(0, n, chunk):
        Xc = np.asarray(X[lo:lo + chunk], dtype=np.float64)
        S = Q64 @ Xc.T
        kk = min(k, S.shape[1])
        idx = topk_ids(S, kk) + lo
        s = np.take_along_axis(S, idx - lo, axis=1)
        cs = np.concatenate([best_s, s], axis=1)
        ci = np.concatenate([best_i, idx], axis=1)
        order = np.lexsort((ci, -cs), axis=1)[:, :k]
        best_s = np.take_along_axis(cs, order, axis=1)
        best_i = np.take_along_axis(ci, order, axis=1)
    return best_i


def recall_at_k(found: np.ndarray, truth: np.ndarray, k: int) -> float:
    """Mean over queries of |found[:k] intersect truth[:k]| / k (sentinels never match)."""
    found = np.asarray(found)[:, :k]
    truth = np.asarray(truth)[:, :k]
    hits = 0
    for f, t in zip(found, truth):
        hits += len(set(int(x) for x in f if int(x) != SENTINEL) & set(int(x) for x in t))
    return hits / (k * len(truth))
