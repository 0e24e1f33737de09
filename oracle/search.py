"""Greedy graph search on primary vectors, then re-ranking with secondaries.

Follows Section 2 ("Search"): primary vectors quant(Bx) drive the graph
traversal with the approximation <q, x> ~ <Aq, quant(Bx)> (Eq. 1); more than
k candidates are kept and their inner products are recomputed with the
secondary vectors, whose top-k is returned.  Appendix D names the traversal
"greedy traversal with backtracking"; the reading used here is the
best-first beam with window L:

  list <- [(s(entry), entry)], visited <- {entry}
  repeat: p <- best not-yet-expanded entry of the list under the total
          order (score descending, id ascending); stop if there is none;
          mark p expanded; for each out-neighbour n of p not visited yet:
          mark visited, compute s(n), insert into the list and keep the
          best L entries.
  re-rank: s2(n) = <q, secondary(n)> for every entry of the final list;
           return the best k under (s2 descending, id ascending).

Scores are float64.  The primary score is the plain definition
<q~, y^_n> with y^_n the LVQ reconstruction (mu + lo + delta * c) and q~
the projected query on its grid (grid_query): every component rounded to
the nearest multiple of 2^-s, with s fixed by the largest component m so
that a step is at most 2^-22 m (a shared-exponent fixed point of 23 bits,
far finer than the bfloat16 products that compute the projection).  The
paper does not fix the arithmetic of the traversal's inner products; on
this grid <q~, c> is a sum of integers, exact in any order.  Re-ranking
reads the query as given.

Pinned by: brute force when L >= N on a connected graph, the exhaustive
"flat" variant, and the top-L-of-visited invariant (tests/test_oracle_search.py).
"""
from __future__ import annotations

import bisect
import os
import tempfile
from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np

SENTINEL = 0xFFFFFFFF


@dataclass
class Index:
    """Everything the search reads; arrays may be numpy memmaps."""

    adj: np.ndarray        # uint32 [N, R]
    entry: int
    codes: np.ndarray      # uint8 [N, d]   (one code per component)
    delta: np.ndarray      # float32 [N]
    lo: np.ndarray         # float32 [N]
    mu: np.ndarray         # float32 [d]
    sec: np.ndarray        # float16 or float32 [N, D]; uint8 LVQ-8 codes when sec_delta is set
    sec_delta: Optional[np.ndarray] = None   # float32 [N]  LVQ-8 secondaries (Section 3:
    sec_lo: Optional[np.ndarray] = None      # float32 [N]  secondary vectors compressed
    sec_mu: Optional[np.ndarray] = None      # float32 [D]  with LVQ-8)
    sec_resid: bool = False  # sec holds only the D - d residual coordinates (see below)
    sec_two_level: bool = False  # sec holds the 8-bit second level of the primaries
                                 # (uint8 [N, d] codes, sec_delta / sec_lo; see below)

    @property
    def N(self) -> int:
        return self.adj.shape[0]


def rowdot(M: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Row-wise inner products in float64 with one fixed summation tree.

    Every row is summed in the same order whatever the number of rows, so a
    vector scored twice gets the same bits (a BLAS matrix-vector product may
    round a row differently depending on the batch it sits in).
    """
    P = np.asarray(M, np.float64) * np.asarray(v, np.float64)[None, :]
    w = 1
    while w < P.shape[1]:
        w *= 2
    if w != P.shape[1]:
        P = np.concatenate([P, np.zeros((P.shape[0], w - P.shape[1]))], axis=1)
    while w > 1:
        w //= 2
        P = P[:, :w] + P[:, w:]
    return P[:, 0]


def grid_query(qp) -> np.ndarray:
    """The projected query on its grid, float64: with m the largest |q_j| and
    m = f 2^e, f in [0.5, 1) (e = 0 for m = 0), s = 22 - e and
    q~_j = rint(q_j 2^s) 2^-s (nearest, ties to even).  Every |rint(q_j 2^s)|
    is at most 2^22 and |q~_j - q_j| is at most half a step, 2^(e - 23) <=
    2^-22 m."""
    q = np.asarray(qp, dtype=np.float64)
    m = float(np.max(np.abs(q))) if q.size else 0.0
    e = int(np.frexp(m)[1])
    s = 22 - e
    return np.ldexp(np.rint(np.ldexp(q, s)), -s)


def primary_scores(index: Index, qp64: np.ndarray, ids) -> np.ndarray:
    """<q~, y^_n> in float64 for the given ids (Eq. 1 with LVQ reconstruction;
    q~ = grid_query(qp64))."""
    ids = np.asarray(ids, dtype=np.int64)
    qp64 = grid_query(qp64)
    yhat = (index.mu.astype(np.float64)[None, :]
            + index.lo[ids].astype(np.float64)[:, None]
            + index.delta[ids].astype(np.float64)[:, None]
            * index.codes[ids].astype(np.float64))
    return rowdot(yhat, qp64)


def secondary_scores(index: Index, q64: np.ndarray, ids, qp64=None) -> np.ndarray:
    """<q, secondary(n)> in float64 (Section 2, re-ranking); an LVQ-8 secondary
    is its reconstruction mu + lo + delta * c.

    Residual secondaries (sec_resid; the remark after Eq. pca: with an
    orthonormal M the error e = (I - M^T M) x needs only D - d coordinates):
    with R = [P; P_perp] orthonormal, <q, x> = <P q, P x> + <P_perp q, P_perp x>;
    sec holds P_perp x, q64 is P_perp q, and the first term is taken from the
    primary vector, so the score is the primary score <qp, y^> (qp64 = P q)
    plus <q64, sec(n)>."""
    ids = np.asarray(ids, dtype=np.int64)
    if index.sec_resid:
        return primary_scores(index, qp64, ids) + rowdot(index.sec[ids], q64)
    if index.sec_two_level:
        return two_level_scores(index, qp64, ids)
    if index.sec_delta is None:
        return rowdot(index.sec[ids], q64)
    xhat = (index.sec_mu.astype(np.float64)[None, :]
            + index.sec_lo[ids].astype(np.float64)[:, None]
            + index.sec_delta[ids].astype(np.float64)[:, None]
            * index.sec[ids].astype(np.float64))
    return rowdot(xhat, q64)


def two_level_scores(index: Index, qp64: np.ndarray, ids) -> np.ndarray:
    """Re-ranking with a two-level LVQ of the primaries (LVQ4x8 of the
    baseline setup, Appendix D and Fig. 1: the first level drives the search,
    the 8-bit second level refines the same reduced vector for the
    re-ranking): <q', y^_n + r^_n> with r^_n = lo2 + delta2 * c2 the second
    level's reconstruction, taken as the primary score (on the query's grid)
    plus <q', r^_n> (the query as given).  The
    query is the projected one; no full-dimension vector is read."""
    ids = np.asarray(ids, dtype=np.int64)
    r = (index.sec_lo[ids].astype(np.float64)[:, None]
         + index.sec_delta[ids].astype(np.float64)[:, None]
         * index.sec[ids].astype(np.float64))
    return primary_scores(index, qp64, ids) + rowdot(r, qp64)


@dataclass
class Trace:
    n_exp: int = 0          # expansions (adjacency rows read)
    n_dist: int = 0         # primary score evaluations
    n_rescored: int = 0     # evaluations of already-visited ids (bounded visited set)
    scored: Optional[dict] = None   # id -> score of every evaluation, when a dict is given


def beam(index: Index, qp, L: int, visited_cap: Optional[int] = None,
         trace: Optional[Trace] = None, scorer=None, expand: int = 1) -> List[Tuple[float, int]]:
    """Best-first traversal; returns the final list as (score, id), best first.

    visited_cap bounds the visited set (oldest entries forgotten first).  A
    forgotten node that is met again is scored again and merged only if it
    is not in the list already; the final list is the same as with an exact
    visited set (a node dropped earlier was worse than L others, and the
    L-th best score never decreases).  scorer(ids), when given, replaces
    the primary score (graph construction scores with a distance).

    expand > 1 is a throughput variant (not the paper's traversal): each
    iteration expands the `expand` best unexpanded entries together, scores
    the unvisited out-neighbours of all of them (row by row, in the order
    the entries are taken) and inserts them; it stops when every entry of
    the list is expanded.
    """
    tr = trace if trace is not None else Trace()
    if scorer is None:
        qp64 = np.asarray(qp, dtype=np.float32).astype(np.float64)

        def scorer(ids):
            return primary_scores(index, qp64, ids)
    adj = index.adj
    e = int(index.entry)
    s0 = float(scorer([e])[0])
    keys = [(-s0, e)]          # sorted ascending == score desc, id asc
    in_list = {e}
    expanded = set()
    visited = {e: None}        # dict keeps insertion order for the bounded variant
    tr.n_dist += 1
    if tr.scored is not None:
        tr.scored[e] = s0
    while True:
        ps = [i for _, i in keys if i not in expanded][:max(1, expand)]
        if not ps:
            break
        newly = []
        for p in ps:
            expanded.add(p)
            tr.n_exp += 1
            for n in adj[p]:
                n = int(n)
                if n == SENTINEL or n in visited:
                    continue
                # (an id met again after the bounded visited set forgot it is
                # scored again; the insertion below drops it if listed)
                visited[n] = None
                newly.append(n)
        rescored = [n for n in newly if n in in_list or n in expanded]
        if visited_cap is not None:
            while len(visited) > visited_cap:
                visited.pop(next(iter(visited)))
        if not newly:
            continue
        tr.n_dist += len(newly)
        tr.n_rescored += len(rescored)
        sc = scorer(newly)
        for s, n in zip(sc.tolist(), newly):
            if tr.scored is not None:
                tr.scored[n] = s
            if n in in_list:
                continue
            key = (-s, n)
            if len(keys) >= L and key > keys[-1]:
                continue
            bisect.insort(keys, key)
            in_list.add(n)
            if len(keys) > L:
                _, gone = keys.pop()
                in_list.discard(gone)
    return [(-k, i) for k, i in keys]


def rerank(index: Index, q, cand_ids, k: int, qp=None) -> Tuple[np.ndarray, np.ndarray]:
    """Top-k of the candidates by secondary score (ties: smaller id).  With
    residual secondaries q is the residual query and qp the primary one; with
    two-level secondaries only qp is read."""
    q64 = np.asarray(q, dtype=np.float32).astype(np.float64)
    qp64 = None if qp is None else np.asarray(qp, dtype=np.float32).astype(np.float64)
    ids = np.asarray(cand_ids, dtype=np.int64)
    out_i = np.full(k, SENTINEL, dtype=np.int64)
    out_s = np.full(k, -np.inf)
    if ids.size:
        s2 = secondary_scores(index, q64, ids, qp64)
        order = np.lexsort((ids, -s2))[:k]
        out_i[:len(order)] = ids[order]
        out_s[:len(order)] = s2[order]
    return out_i, out_s


def search_one(index: Index, q, qp, k: int, L: int, visited_cap=None, trace=None, expand=1):
    """Full query: traversal with window L, then re-rank to k (requires L >= k)."""
    if L < k:
        raise ValueError("window L must be at least k")
    lst = beam(index, qp, L, visited_cap=visited_cap, trace=trace, expand=expand)
    return rerank(index, q, [i for _, i in lst], k, qp)


def flat_search(index: Index, q, qp, k: int, L: int):
    """Exhaustive variant: primary top-L over all vectors, then re-rank."""
    qp64 = np.asarray(qp, dtype=np.float32).astype(np.float64)
    s = primary_scores(index, qp64, np.arange(index.N))
    order = np.lexsort((np.arange(index.N), -s))[:L]
    return rerank(index, q, order, k, qp)


# ---------------------------------------------------------------------------
# Many queries, optionally over several processes (fresh interpreters that
# memory-map the index, so nothing but numpy runs in them).

_G = {}


def _init_worker(paths, entry, sec_resid=False, sec_two_level=False):
    arrs = {k: np.load(v, mmap_mode="r") for k, v in paths.items()}
    _G["index"] = Index(arrs["adj"], entry, arrs["codes"], arrs["delta"], arrs["lo"],
                        arrs["mu"], arrs["sec"], arrs.get("sec_delta"), arrs.get("sec_lo"),
                        arrs.get("sec_mu"), sec_resid, sec_two_level)


def _run_chunk(args):
    Q, Qp, k, L, lo, expand = args
    index = _G["index"]
    ids = np.empty((len(Q), k), dtype=np.int64)
    sc = np.empty((len(Q), k))
    cnt = np.zeros((len(Q), 2), dtype=np.int64)
    for i in range(len(Q)):
        tr = Trace()
        ids[i], sc[i] = search_one(index, Q[i], Qp[i], k, L, trace=tr, expand=expand)
        cnt[i] = (tr.n_exp, tr.n_dist)
    return lo, ids, sc, cnt


def search_many(index: Index, Q, Qp, k: int, L: int, procs: int = 1,
                chunk: int = 64, workdir: Optional[str] = None, expand: int = 1):
    """Search every query; returns (ids [m,k], scores [m,k], counts [m,2])."""
    Q = np.asarray(Q, dtype=np.float32)
    Qp = np.asarray(Qp, dtype=np.float32)
    m = len(Q)
    ids = np.empty((m, k), dtype=np.int64)
    sc = np.empty((m, k))
    cnt = np.zeros((m, 2), dtype=np.int64)
    if procs <= 1:
        _G["index"] = index
        for lo in range(0, m, chunk):
            _, a, b, c = _run_chunk((Q[lo:lo + chunk], Qp[lo:lo + chunk], k, L, lo, expand))
            ids[lo:lo + len(a)], sc[lo:lo + len(a)], cnt[lo:lo + len(a)] = a, b, c
        return ids, sc, cnt
    import multiprocessing as mp
    own = workdir is None
    wd = workdir or tempfile.mkdtemp(prefix="lv_oracle_")
    paths = {}
    names = ["adj", "codes", "delta", "lo", "mu", "sec"]
    names += [n for n in ("sec_delta", "sec_lo", "sec_mu") if getattr(index, n) is not None]
    for name in names:
        arr = getattr(index, name)
        p = os.path.join(wd, name + ".npy")
        if not os.path.exists(p):
            np.save(p, np.ascontiguousarray(arr))
        paths[name] = p
    from concurrent.futures import ProcessPoolExecutor

    try:
        # a worker that dies raises BrokenProcessPool here instead of hanging
        with ProcessPoolExecutor(procs, mp_context=mp.get_context("spawn"),
                                 initializer=_init_worker,
                                 initargs=(paths, int(index.entry), bool(index.sec_resid),
                                           bool(index.sec_two_level))) as pool:
            jobs = [(Q[lo:lo + chunk], Qp[lo:lo + chunk], k, L, lo, expand)
                    for lo in range(0, m, chunk)]
            for lo, a, b, c in pool.map(_run_chunk, jobs):
                ids[lo:lo + len(a)], sc[lo:lo + len(a)], cnt[lo:lo + len(a)] = a, b, c
    finally:
        if own:
            for p in paths.values():
                os.unlink(p)
            os.rmdir(wd)
    return ids, sc, cnt
