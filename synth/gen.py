"""Seeded synthetic workloads standing in for the paper's datasets.

The paper evaluates on real embedding collections (Table 1: rqa-768-1M, the
512-dimensional cross-modal sets, ...) that are not available here.  This
module draws data with the same shapes, similarity (inner product on
L2-normalised vectors) and the two regimes the paper studies: queries drawn
from the database distribution (in-distribution, Section 2.1) and queries
from a different distribution (out-of-distribution, Section 2.2).

This module holds no arithmetic of the search method: it only draws numbers.
Both the oracle and the GPU path consume its arrays.

Recipe (all draws in float64 from ``numpy.random.PCG64``, L2-normalisation in
float64, cast to float32 at the very end):

* ``iso`` spectrum: centres c_k ~ N(0, I_D); sample x = c_z + sigma * eps.
* ``inv`` spectrum: eigenvalues lambda_i = 1/i; U is a Haar rotation (QR of a
  Gaussian matrix with the signs of diag(R) folded in); centres
  c_k = U diag(sqrt(lambda)) z_k; sample x = c_z + sigma U diag(sqrt(lambda)) eps.
  The global spectrum then decays like 1/i, so that a d-dimensional linear
  projection keeps most of the energy, as it does for real embeddings.
* OOD queries: g is a raw (unnormalised) mixture sample; the query is
  normalise(sqrt(1/2) g + sqrt(1/2) O g + shift * rho * m), with O a Haar
  rotation (moving half the energy into random directions), m a fixed random
  unit vector and rho = sqrt(E||g||^2) (closed form), so a shift of 0.5 is half
  a typical norm.
* Labels z are uniform over the K clusters.  Large sets are drawn in chunks of
  65,536 rows, chunk c from ``SeedSequence([seed, c])``, so the result does not
  depend on the number of threads.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np
from threadpoolctl import threadpool_limits

CHUNK = 65536


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: data distribution plus index/search settings."""

    name: str
    D: int                 # full dimension
    d: int                 # reduced dimension
    N: int                 # database size
    K: int                 # mixture clusters
    spectrum: str          # "iso" or "inv"
    sigma: float           # within-cluster noise scale
    seed_basis: int        # centres (and U for "inv")
    seed_data: int         # database rows
    seed_test: int         # test queries
    seed_learn: int        # learning (calibration / fit) queries
    m_test: int
    m_learn: int
    bits: int              # LVQ bits of the primary vectors
    sec_dtype: str         # "f32" or "f16" secondary vectors
    R: int                 # graph out-degree
    L_list: Tuple[int, ...]
    k: int
    fit: str = "id"        # "id" (PCA) or "ood" (Frank-Wolfe)
    ood: bool = False
    seed_rot: int = 0
    seed_shift: int = 0
    shift: float = 0.5
    graph_alphas: Tuple[float, ...] = (1.0, 1.0)   # pruning factor per build pass

    def scaled(self, N: Optional[int] = None, m_test: Optional[int] = None,
               m_learn: Optional[int] = None) -> "Workload":
        """Same distribution, fewer rows (for oracle-sized parity cases)."""
        return replace(self, N=self.N if N is None else N,
                       m_test=self.m_test if m_test is None else m_test,
                       m_learn=self.m_learn if m_learn is None else m_learn)


WORKLOADS = {
    # Small plain LeanVec-ID case: 10k x 128 mixture of 50 isotropic Gaussians.
    "id-small": Workload("id-small", D=128, d=32, N=10_000, K=50, spectrum="iso",
                         sigma=0.3, seed_basis=100, seed_data=101, seed_test=102,
                         seed_learn=103, m_test=100, m_learn=1000, bits=8,
                         sec_dtype="f32", R=32, L_list=(50,), k=10, graph_alphas=(1.0,)),
    # LeanVec-ID at scale: 1M x 768, 1000 anisotropic clusters, d=160.
    "id-1m-768": Workload("id-1m-768", D=768, d=160, N=1_000_000, K=1000,
                          spectrum="inv", sigma=0.3, seed_basis=200, seed_data=201,
                          seed_test=202, seed_learn=203, m_test=10_000,
                          m_learn=10_000, bits=8, sec_dtype="f16", R=64,
                          L_list=(20, 40, 60, 100, 150, 200), k=10),
    # LeanVec-OOD cross-modal analogue: 1M x 512 database, rotated+shifted queries.
    "ood-1m-512": Workload("ood-1m-512", D=512, d=128, N=1_000_000, K=1000,
                           spectrum="inv", sigma=0.3, seed_basis=300, seed_data=301,
                           seed_test=302, seed_learn=303, m_test=10_000,
                           m_learn=10_000, bits=4, sec_dtype="f16", R=64,
                           L_list=(20, 40, 60, 100, 150, 200), k=10, fit="ood",
                           ood=True, seed_rot=304, seed_shift=305),
    # Differentiable refinement data: OOD generator at D=768, 100k queries.
    "ood-1m-768": Workload("ood-1m-768", D=768, d=128, N=1_000_000, K=1000,
                           spectrum="inv", sigma=0.3, seed_basis=500, seed_data=501,
                           seed_test=502, seed_learn=503, m_test=10_000,
                           m_learn=100_000, bits=8, sec_dtype="f16", R=64,
                           L_list=(20, 40, 60, 100), k=10, fit="ood", ood=True,
                           seed_rot=504, seed_shift=505),
}


def _threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def haar(D: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed rotation: QR of a Gaussian with sign(diag R) folded in."""
    G = rng.standard_normal((D, D))
    Q, Rm = np.linalg.qr(G)
    return Q * np.sign(np.diag(Rm))[None, :]


@dataclass
class Mixture:
    """Cluster centres (latent coordinates) and the map latent -> ambient."""

    wl: Workload
    Z: np.ndarray                  # [K, D] latent centre coordinates
    scale: np.ndarray              # [D] per-axis std of the latent (sqrt lambda)
    U: Optional[np.ndarray]        # [D, D] rotation (None for "iso")
    O: Optional[np.ndarray] = None
    shift_dir: Optional[np.ndarray] = None
    rho: float = 1.0

    def raw(self, labels: np.ndarray, eps: np.ndarray) -> np.ndarray:
        """Unnormalised samples c_z + sigma * (scaled noise), float64 [n, D]."""
        W = (self.Z[labels] + self.wl.sigma * eps) * self.scale[None, :]
        if self.U is None:
            return W
        return W @ self.U.T


def mixture(wl: Workload) -> Mixture:
    rng = np.random.Generator(np.random.PCG64(wl.seed_basis))
    if wl.spectrum == "iso":
        scale = np.ones(wl.D)
        U = None
        Z = rng.standard_normal((wl.K, wl.D))
        energy = (1.0 + wl.sigma ** 2) * wl.D
    elif wl.spectrum == "inv":
        lam = 1.0 / np.arange(1, wl.D + 1, dtype=np.float64)
        scale = np.sqrt(lam)
        U = haar(wl.D, rng)
        Z = rng.standard_normal((wl.K, wl.D))
        energy = (1.0 + wl.sigma ** 2) * float(lam.sum())
    else:
        raise ValueError(f"unknown spectrum {wl.spectrum!r}")
    mix = Mixture(wl, Z, scale, U, rho=math.sqrt(energy))
    if wl.ood:
        mix.O = haar(wl.D, np.random.Generator(np.random.PCG64(wl.seed_rot)))
        v = np.random.Generator(np.random.PCG64(wl.seed_shift)).standard_normal(wl.D)
        mix.shift_dir = v / np.linalg.norm(v)
    return mix


def _normalise_rows(V: np.ndarray) -> np.ndarray:
    return V / np.linalg.norm(V, axis=1, keepdims=True)


def _chunk(mix: Mixture, seed: int, c: int, rows: int, ood: bool) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, c])))
    # a full chunk of labels is always drawn, so a row's values do not depend
    # on how many rows were requested
    labels = rng.integers(0, mix.wl.K, size=CHUNK)[:rows]
    eps = rng.standard_normal((rows, mix.wl.D))
    g = mix.raw(labels, eps)
    if ood:
        h = math.sqrt(0.5)
        g = h * g + h * (g @ mix.O.T) + mix.wl.shift * mix.rho * mix.shift_dir[None, :]
    return _normalise_rows(g).astype(np.float32)


def _draw(mix: Mixture, seed: int, n: int, ood: bool,
          out: Optional[np.ndarray] = None) -> np.ndarray:
    if out is None:
        out = np.empty((n, mix.wl.D), dtype=np.float32)
    nchunks = (n + CHUNK - 1) // CHUNK

    def one(c: int) -> None:
        lo = c * CHUNK
        hi = min(n, lo + CHUNK)
        out[lo:hi] = _chunk(mix, seed, c, hi - lo, ood)

    if nchunks == 1:
        one(0)
    else:
        # chunks run in parallel threads, each with single-threaded BLAS
        with threadpool_limits(1), ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(one, range(nchunks)))
    return out


def database(wl: Workload, mix: Optional[Mixture] = None,
             out: Optional[np.ndarray] = None) -> np.ndarray:
    """Database vectors X, float32 [N, D], unit L2 norm."""
    mix = mix or mixture(wl)
    return _draw(mix, wl.seed_data, wl.N, ood=False, out=out)


def queries(wl: Workload, which: str = "test", m: Optional[int] = None,
            mix: Optional[Mixture] = None) -> np.ndarray:
    """Query vectors, float32 [m, D], unit L2 norm (test or learning set)."""
    mix = mix or mixture(wl)
    if which == "test":
        seed, m = wl.seed_test, (wl.m_test if m is None else m)
    elif which == "learn":
        seed, m = wl.seed_learn, (wl.m_learn if m is None else m)
    else:
        raise ValueError(which)
    return _draw(mix, seed, m, ood=wl.ood)


def subindex_sizes(n_sub: int = 64, lo: int = 10_000, hi: int = 500_000,
                   seed: int = 400) -> np.ndarray:
    """Sizes of the multi-index workload: log-uniform in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(math.log(lo), math.log(hi), size=n_sub)
    return np.rint(np.exp(u)).astype(np.int64)


def request_stream(n_req: int, n_sub: int, pool: int, seed: int = 401,
                   max_batch: int = 4096, ks: Tuple[int, ...] = (1, 10, 100)):
    """Request stream for batched search: (sub-index, batch size, k) triples.

    Batch sizes are uniform in [1, max_batch]; k uniform over ``ks``; queries
    of a request are taken cyclically from its sub-index's pool of ``pool``.
    Returns int64 arrays (sub, count, k, pool_offset).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sub = rng.integers(0, n_sub, size=n_req)
    cnt = rng.integers(1, max_batch + 1, size=n_req)
    kk = np.asarray(ks, dtype=np.int64)[rng.integers(0, len(ks), size=n_req)]
    cursor = np.zeros(n_sub, dtype=np.int64)
    off = np.empty(n_req, dtype=np.int64)
    for i in range(n_req):
        off[i] = cursor[sub[i]] % pool
        cursor[sub[i]] += cnt[i]
    return sub.astype(np.int64), cnt.astype(np.int64), kk, off
