"""Which decisions of a graph build are too close to call.

The oracle (oracle/graph.py) computes f(a, b) = ||y^_a - y^_b||^2 of the
LVQ reconstructions by its definition: decode, subtract, square, sum.  The
GPU evaluates the same distance from exact integer code sums as
  f = d e^2 + da^2 S_aa + db^2 S_bb - 2 da db S_ab + 2 e (da S_a - db S_b),
e = lo_a - lo_b, a fixed sequence of float64 operations.  Both differ from
the exact value by rounding only, so the two builds take the same decision
whenever the distances compared differ by more than both error bounds:

  GPU:    every term is rounded at most four times and the five terms are
          summed left to right, so |f_gpu - f| <= 8 u T with T the sum of
          the terms' magnitudes (T >= f); 16 u T is used;
  oracle: decoding, subtracting and squaring cost at most
          3 u sum_j |y^_a - y^_b|_j (|y^_a|_j + |y^_b|_j + |y^_a - y^_b|_j)
          <= 3 u sqrt(f) (|y^_a| + |y^_b|) + 3 u f, summing d u f;

u = 2^-53, and the sum of both bounds is doubled.  A comparison of x and y
is fragile when |x - y| (with the pruning factor alpha^2 on one side) is
within the two distances' bounds, unless both distances come from identical
operands (the same node against two candidates whose records are equal):
then each side computes equal values and both break the tie by id.
"""
from __future__ import annotations

import numpy as np

from oracle import graph as og

U = 2.0 ** -53


class TieMonitor(og.Monitor):
    """Counts the fragile decisions of an oracle build and the first batch
    holding one."""

    def __init__(self, prim: og.Primaries):
        self.prim = prim
        c = prim.codes.astype(np.float64)
        self.S = c.sum(axis=1)
        self.SS = (c * c).sum(axis=1)
        y = prim.decode(np.arange(prim.n))
        self.norm = np.sqrt((y * y).sum(axis=1))
        # equal records (codes and constants) give equal distances on both sides
        keys = {}
        self.rec_class = np.empty(prim.n, dtype=np.int64)
        for i in range(prim.n):
            k = (prim.codes[i].tobytes(), prim.delta[i], prim.lo[i])
            self.rec_class[i] = keys.setdefault(k, len(keys))
        self.fragile = 0
        self.decisions = 0
        self.first_batch = None

    def tau(self, a, b, f) -> np.ndarray:
        """Bound on |f_gpu - f_oracle| for pairs (a, b) with oracle value f."""
        p = self.prim
        a = np.asarray(a, dtype=np.int64)
        b = np.asarray(b, dtype=np.int64)
        sab = (p.codes[a].astype(np.float64) * p.codes[b]).sum(axis=-1)
        e = p.lo[a] - p.lo[b]
        da, db = p.delta[a], p.delta[b]
        T = (p.d * e * e + da * da * self.SS[a] + db * db * self.SS[b] + 2 * da * db * sab
             + 2 * np.abs(e) * (da * self.S[a] + db * self.S[b]))
        f = np.abs(np.asarray(f, dtype=np.float64))
        orc = 3 * U * np.sqrt(f) * (self.norm[a] + self.norm[b]) + (p.d + 3) * U * f
        return 2 * (16 * U * T + orc)

    def _flag(self, n):
        if n:
            self.fragile += int(n)
            if self.first_batch is None:
                self.first_batch = self.batch

    def _ranked(self, p, ids, f):
        """Candidates ranked by (f, id): adjacent values must be separable
        (then every pair is); equal records are exempt."""
        if len(ids) < 2:
            return
        order = np.lexsort((ids, f))
        ids, f = np.asarray(ids)[order], np.asarray(f)[order]
        t = self.tau(np.full(len(ids), p), ids, f)
        gap = np.diff(f)
        same = self.rec_class[ids[1:]] == self.rec_class[ids[:-1]]
        self.decisions += len(gap)
        self._flag(np.count_nonzero((gap <= t[1:] + t[:-1]) & ~same))

    def scored(self, p, ids, f):
        self._ranked(p, ids, f)

    def ordered(self, p, ids, f):
        self._ranked(p, ids, f)

    def tested(self, p, c, kept, f_kc, f_pc, alpha2):
        kept = np.asarray(kept, dtype=np.int64)
        t_kc = self.tau(kept, np.full(len(kept), c), f_kc)
        t_pc = self.tau(np.array([p]), np.array([c]), np.array([f_pc]))[0]
        margin = alpha2 * t_kc + t_pc + 4 * U * max(abs(f_pc), 1e-300)
        self.decisions += len(kept)
        self._flag(np.count_nonzero(np.abs(alpha2 * np.asarray(f_kc) - f_pc) <= margin))
