"""Shared set-up for the GPU parity tests (inputs from synth, expectations from oracle)."""
from __future__ import annotations

import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

from oracle import fit as ofit
from oracle import lvq as olvq
from oracle import search as osearch
from synth import gen, graph

CACHE = os.environ.get("LV_CACHE", "/tmp/lv_cache")


@dataclass
class Case:
    wl: gen.Workload
    X: np.ndarray          # float32 [N, D]
    Q: np.ndarray          # float32 [m, D] test queries
    P: np.ndarray          # float64 [d, D] projection (A = B = P)
    Y: np.ndarray          # float32 [N, d] reduced database (oracle float64 projection)
    Qp: np.ndarray         # float32 [m, d] reduced queries (oracle float64 projection)
    mu: np.ndarray         # float32 [d]
    adj: np.ndarray        # uint32 [N, R]
    entry: int
    sec: np.ndarray        # secondaries (float16 or float32) [N, D]
    stride: int

    def oracle_index(self) -> osearch.Index:
        codes, delta, lo = olvq.encode(self.Y, self.mu, self.wl.bits)
        return osearch.Index(self.adj, self.entry, codes, delta, lo, self.mu, self.sec)


def stride_for(d: int, bits: int) -> int:
    need = d * bits // 8 + 8
    for s in (64, 96, 128, 192, 256, 512, 768, 1024):
        if need <= s:
            return s
    raise ValueError("no stride")


def graph_cached(wl: gen.Workload, X: np.ndarray):
    os.makedirs(CACHE, exist_ok=True)
    key = f"{wl.name}_s{wl.seed_data}_n{wl.N}_R{wl.R}_a{'-'.join(map(str, wl.graph_alphas))}_v6"
    p = os.path.join(CACHE, key + ".npz")
    if os.path.exists(p):
        z = np.load(p)
        return z["adj"], int(z["entry"])
    adj, entry = graph.build_graph(X, wl.R, alphas=wl.graph_alphas)
    np.savez(p + ".tmp.npz", adj=adj, entry=np.int64(entry))
    os.replace(p + ".tmp.npz", p)
    return adj, entry


def make_case(wl: gen.Workload, fit: str = "id", m: Optional[int] = None) -> Case:
    mix = gen.mixture(wl)
    X = gen.database(wl, mix)
    Q = gen.queries(wl, "test", m=m, mix=mix)
    if fit == "id":
        P = ofit.fit_id(ofit.second_moment(X), wl.d)
    else:
        Ql = gen.queries(wl, "learn", mix=mix)
        A, B, _ = ofit.frank_wolfe(ofit.second_moment(Ql), len(Ql), ofit.second_moment(X),
                                   len(X), wl.d)
        P = A  # only used where A = B is not needed
    Y = ofit.project(X, P).astype(np.float32)
    Qp = ofit.project(Q, P).astype(np.float32)
    mu = ofit.mean_reduced(X, P).astype(np.float32)
    adj, entry = graph_cached(wl, X)
    sec = X.astype(np.float16) if wl.sec_dtype == "f16" else X
    return Case(wl, X, Q, P, Y, Qp, mu, adj, entry, sec, stride_for(wl.d, wl.bits))
