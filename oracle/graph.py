"""Graph construction on the primary vectors (test infrastructure: only the
tests, the smoke check and the benchmark's CPU baseline may use this module).

Appendix A describes graph construction as an update run for every node x:
search the current graph with x as the query for a candidate set larger
than R, prune that set to at most R diverse out-neighbours, and make them
x's out-edges.  Section 2 ("Graph construction") fixes the data: only the
primary vectors quant(Bx) take part.  Appendix D names Vamana with its
pruning factor alpha.  Reading used here (Vamana with batch-synchronous
insertion, so that a parallel build has one defined result):

  distance  f(a, b) = ||y^_a - y^_b||^2 of the LVQ reconstructions
            y^ = mu + lo + delta * c, by its definition: both vectors
            decoded in float64 (mu cancels in the difference and is left
            out), subtracted, squared and summed (see `l2`);
  order     a permutation of the nodes (an input); pass 0 inserts batches
            of 1, 2, 4, ... nodes up to max_batch, later passes use
            max_batch throughout; pass t prunes with alphas[t];
  batch     every node p of the batch, against the graph as it was when
            the batch started: best-first search from the entry with window
            L and similarity -f(p, .) (`oracle.search.beam`), pool = final
            window followed by p's current out-neighbours, new row of p =
            prune(p, pool);
            then the rows of the batch are replaced, and every target j of
            a new edge p -> j gets its reverse edge: union = row(j)
            followed by the new sources not in row(j), in ascending id; if
            the union holds at most R ids it becomes row(j), otherwise
            row(j) = prune(j, union);
  prune     candidates sorted by (f(p, c) ascending, id ascending), p
            itself and repeats skipped; c is kept unless an already kept k
            has alpha^2 * f(k, c) <= f(p, c); at most R are kept, in that
            order.
Rows hold their valid ids first, then 0xFFFFFFFF.

Every decision of the build compares two distances (the search's order of
its scored candidates, the pruning order, the pruning test).  `build`
reports each of them to an optional monitor (`Monitor`), so that a caller
can tell which decisions are too close to call for an implementation whose
distance carries a different rounding error.

Pinned by: the distance against exact rational arithmetic on the decoded
vectors, a hand-worked pruning example (tests/golden/prune_hand.json), the
path graph that points on a line must produce, brute force for the search
when L >= N, hand-traced states after the first batches, and the row
invariants (tests/test_oracle_graph.py).
"""
from __future__ import annotations

from typing import Callable, List, Optional, Sequence

import numpy as np

from . import search as _search

SENTINEL = 0xFFFFFFFF


class Primaries:
    """Codes and LVQ constants of the database's primary vectors."""

    def __init__(self, codes: np.ndarray, delta: np.ndarray, lo: np.ndarray):
        self.codes = np.asarray(codes, dtype=np.int64)
        self.delta = np.asarray(delta, dtype=np.float32).astype(np.float64)
        self.lo = np.asarray(lo, dtype=np.float32).astype(np.float64)
        self.n, self.d = self.codes.shape

    def decode(self, ids) -> np.ndarray:
        """y^ - mu = lo + delta * c for each id, float64 (delta * c is exact)."""
        ids = np.asarray(ids, dtype=np.int64)
        return self.lo[ids][..., None] + self.delta[ids][..., None] * self.codes[ids]

    def l2(self, a, b) -> np.ndarray:
        """f(a, b) = sum_j (y^_a,j - y^_b,j)^2 elementwise over broadcast id
        arrays a, b, in float64."""
        a = np.asarray(a, dtype=np.int64)
        b = np.asarray(b, dtype=np.int64)
        a, b = np.broadcast_arrays(a, b)
        diff = self.decode(a) - self.decode(b)
        return np.sum(diff * diff, axis=-1)


class Monitor:
    """Receives every comparison of distances the build decides on.

    scored(p, ids, f): the distances from node p of every candidate its
        construction search scored (the search orders them, keeps the best
        L and expands them in that order);
    ordered(p, ids, f): the pruning pool of p, ranked by (f, id);
    tested(p, c, kept, f_kc, f_pc, alpha2): the pruning test of candidate c
        against the kept nodes (c goes when alpha2 * f(k, c) <= f(p, c)).
    `batch` holds the index of the batch being built (over all passes).
    """

    batch = 0

    def scored(self, p, ids, f):
        pass

    def ordered(self, p, ids, f):
        pass

    def tested(self, p, c, kept, f_kc, f_pc, alpha2):
        pass


def prune(p: int, pool: Sequence[int], dist: Callable, alpha: float, R: int,
          monitor: Optional[Monitor] = None) -> List[int]:
    """Diverse subset of the pool (Appendix A "Pruning"; Vamana's rule).

    dist(a, b) returns the distances of id array b to id(s) a.
    """
    ids = np.array([int(c) for c in pool if int(c) != SENTINEL and int(c) != p], dtype=np.int64)
    if ids.size == 0:
        return []
    fp = np.asarray(dist(np.full(ids.shape, p), ids), dtype=np.float64)
    order = np.lexsort((ids, fp))
    if monitor is not None:
        monitor.ordered(p, ids[order], fp[order])
    alpha2 = float(alpha) * float(alpha)
    kept: List[int] = []
    last = None
    for o in order:
        c = int(ids[o])
        if c == last:
            continue
        last = c
        if len(kept) == R:
            break
        if kept:
            fk = np.asarray(dist(np.array(kept, dtype=np.int64), np.full(len(kept), c)),
                            dtype=np.float64)
            if monitor is not None:
                monitor.tested(p, c, list(kept), fk, float(fp[o]), alpha2)
            if np.any(alpha2 * fk <= fp[o]):
                continue
        kept.append(c)
    return kept


def reverse_row(j: int, cur: Sequence[int], sources: Sequence[int], dist: Callable,
                alpha: float, R: int, monitor: Optional[Monitor] = None) -> List[int]:
    """Row of j after the reverse edges of one batch: the current row, then
    the new sources not in it (ascending); pruned when longer than R."""
    have = set(int(x) for x in cur)
    union = [int(x) for x in cur] + [int(p) for p in sorted(sources)
                                     if int(p) not in have and int(p) != j]
    if len(union) <= R:
        return union
    return prune(j, union, dist, alpha, R, monitor)


def _pad(row: Sequence[int], R: int) -> np.ndarray:
    out = np.full(R, SENTINEL, dtype=np.uint32)
    out[:len(row)] = np.asarray(row, dtype=np.uint32)
    return out


def window(prim: Primaries, adj: np.ndarray, entry: int, p: int, L: int,
           monitor: Optional[Monitor] = None) -> List[int]:
    """Ids of the final search window for node p (best first)."""
    ix = _search.Index(adj=adj, entry=int(entry), codes=prim.codes, delta=prim.delta,
                       lo=prim.lo, mu=np.zeros(prim.d), sec=None)
    tr = _search.Trace(scored={} if monitor is not None else None)
    lst = _search.beam(ix, None, L, trace=tr,
                       scorer=lambda ids: -prim.l2(np.full(len(ids), p), ids))
    if monitor is not None:
        ids = np.fromiter(tr.scored.keys(), dtype=np.int64, count=len(tr.scored))
        monitor.scored(p, ids, -np.fromiter(tr.scored.values(), dtype=np.float64,
                                            count=len(ids)))
    return [i for _, i in lst]


def build(prim: Primaries, order: Sequence[int], entry: int, R: int, L: int,
          alphas: Sequence[float], max_batch: int, stop_after: int = 0,
          monitor: Optional[Monitor] = None) -> np.ndarray:
    """Adjacency uint32 [N, R] built as described in the module text.

    stop_after > 0 stops after that many batches (counted over all passes).
    monitor, when given, receives every comparison of distances (`Monitor`).
    """
    n = prim.n
    order = np.asarray(order, dtype=np.int64)
    if sorted(order.tolist()) != list(range(n)):
        raise ValueError("order must be a permutation of the node ids")
    adj = np.full((n, R), SENTINEL, dtype=np.uint32)
    batches = 0
    for t, alpha in enumerate(alphas):
        bs = 1 if t == 0 else max_batch
        start = 0
        while start < n:
            if stop_after and batches == stop_after:
                return adj
            batch = order[start:start + bs]
            if monitor is not None:
                monitor.batch = batches
            frozen = adj.copy()
            rows = []
            for p in batch.tolist():
                pool = window(prim, frozen, entry, p, L, monitor)
                pool += [int(x) for x in frozen[p] if x != SENTINEL]
                rows.append(prune(p, pool, prim.l2, alpha, R, monitor))
            sources = {}
            for p, row in zip(batch.tolist(), rows):
                adj[p] = _pad(row, R)
                for j in row:
                    sources.setdefault(j, []).append(p)
            for j in sorted(sources):
                cur = [int(x) for x in adj[j] if x != SENTINEL]
                adj[j] = _pad(reverse_row(j, cur, sources[j], prim.l2, alpha, R, monitor), R)
            batches += 1
            start += len(batch)
            bs = min(2 * bs, max_batch)
    return adj


def check_rows(adj: np.ndarray, n: Optional[int] = None) -> None:
    """Raise if a row has a self loop, a repeated id, an id out of range, or
    a valid id after padding."""
    n = adj.shape[0] if n is None else n
    for i, row in enumerate(adj):
        valid = row[row != SENTINEL]
        k = valid.size
        if np.any(row[k:] != SENTINEL):
            raise AssertionError("row %d: id after padding" % i)
        if np.any(valid >= n):
            raise AssertionError("row %d: id out of range" % i)
        if np.any(valid == i):
            raise AssertionError("row %d: self loop" % i)
        if np.unique(valid).size != k:
            raise AssertionError("row %d: repeated id" % i)


def reachable(adj: np.ndarray, entry: int) -> np.ndarray:
    """Nodes reachable from the entry (breadth-first)."""
    n = adj.shape[0]
    seen = np.zeros(n, dtype=bool)
    seen[entry] = True
    frontier = [int(entry)]
    while frontier:
        nxt = []
        for u in frontier:
            for v in adj[u]:
                v = int(v)
                if v != SENTINEL and not seen[v]:
                    seen[v] = True
                    nxt.append(v)
        frontier = nxt
    return seen
