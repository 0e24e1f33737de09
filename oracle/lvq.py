"""LVQ: per-vector scale-and-bias scalar quantisation of the reduced vectors.

The paper quantises the reduced database vectors with LVQ (Eq. 1 uses
quant(Bx); Section 2 names LVQ and cites it without restating it).  Reading
used here (a per-vector min/max quantiser after removing a global mean):

  r_j   = y_j - mu_j                         (float64 from float32 inputs)
  l, u  = min_j r_j, max_j r_j
  delta = float32((u - l) / (2^b - 1)),  lo = float32(l)   (round to nearest even)
  c_j   = clamp(floor((r_j - lo) / delta + 0.5), 0, 2^b - 1)   (float64 arithmetic;
          all codes 0 when delta == 0)
  decode: y^_j = mu_j + lo + delta * c_j

Record layout shared with the device library (the boundary's format): code
bytes first (b = 8: one byte per component; b = 4: component 2i in the low
nibble and 2i+1 in the high nibble of byte i), then delta and lo as
little-endian float32, then zero padding up to the record stride.

Two-level LVQ (LVQ4x8 in the paper's experimental setup, where the cited
LVQ's 4-bit first level serves the search and an 8-bit second level the
re-ranking; the paper names the scheme without restating it).  Reading used
here: the second level quantises the first level's residual with the same
per-vector min/max quantiser at 8 bits and no centring,

  r2_j   = (y_j - mu_j) - (lo + delta * c_j)          (float64, in this order;
                                                       delta * c_j is exact)
  delta2 = float32((max r2 - min r2) / 255),  lo2 = float32(min r2)
  c2_j   = clamp(floor((r2_j - lo2) / delta2 + 0.5), 0, 255)
  decode: y^_j = mu_j + lo + delta * c_j + lo2 + delta2 * c2_j

so the two-level reconstruction is within half a second-level step of y
(delta2 <= delta / 255 because |r2_j| <= delta / 2).

Pinned by: the half-step error bound, the code range and endpoints, and the
encode(decode(x)) fixed point; for the second level, a hand-worked example
(tests/golden/lvq_hand.json), its half-step bound and the bound relative to
the first level's step (tests/test_oracle_lvq.py).

Test infrastructure only: the search library never imports this module.
"""
from __future__ import annotations

import numpy as np


def encode(Y: np.ndarray, mu: np.ndarray, bits: int):
    """Codes (uint8, one per component), delta (float32), lo (float32)."""
    if bits not in (4, 8):
        raise ValueError("bits must be 4 or 8")
    levels = (1 << bits) - 1
    r = np.asarray(Y, dtype=np.float32).astype(np.float64) - \
        np.asarray(mu, dtype=np.float32).astype(np.float64)[None, :]
    l = r.min(axis=1)
    u = r.max(axis=1)
    delta = ((u - l) / levels).astype(np.float32)
    lo = l.astype(np.float32)
    d64 = delta.astype(np.float64)
    safe = np.where(d64 > 0, d64, 1.0)
    t = (r - lo.astype(np.float64)[:, None]) / safe[:, None]
    c = np.clip(np.floor(t + 0.5), 0, levels)
    c[d64 == 0] = 0
    return c.astype(np.uint8), delta, lo


def decode(codes: np.ndarray, delta: np.ndarray, lo: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """Reconstructed reduced vectors, float64."""
    return (np.asarray(mu, np.float32).astype(np.float64)[None, :]
            + np.asarray(lo, np.float32).astype(np.float64)[:, None]
            + np.asarray(delta, np.float32).astype(np.float64)[:, None]
            * np.asarray(codes, np.float64))


def residual(Y: np.ndarray, mu: np.ndarray, codes: np.ndarray, delta: np.ndarray,
             lo: np.ndarray) -> np.ndarray:
    """First-level residual r2 = (y - mu) - (lo + delta * c), float64."""
    r = np.asarray(Y, dtype=np.float32).astype(np.float64) - \
        np.asarray(mu, dtype=np.float32).astype(np.float64)[None, :]
    rec = (np.asarray(lo, np.float32).astype(np.float64)[:, None]
           + np.asarray(delta, np.float32).astype(np.float64)[:, None]
           * np.asarray(codes, np.float64))
    return r - rec


def encode_residual(Y: np.ndarray, mu: np.ndarray, codes: np.ndarray, delta: np.ndarray,
                    lo: np.ndarray):
    """Second level: 8-bit codes (uint8), delta2 and lo2 (float32) of the residual."""
    r = residual(Y, mu, codes, delta, lo)
    l = r.min(axis=1)
    u = r.max(axis=1)
    delta2 = ((u - l) / 255.0).astype(np.float32)
    lo2 = l.astype(np.float32)
    d64 = delta2.astype(np.float64)
    safe = np.where(d64 > 0, d64, 1.0)
    t = (r - lo2.astype(np.float64)[:, None]) / safe[:, None]
    c = np.clip(np.floor(t + 0.5), 0, 255)
    c[d64 == 0] = 0
    return c.astype(np.uint8), delta2, lo2


def decode_two_level(codes, delta, lo, codes2, delta2, lo2, mu) -> np.ndarray:
    """y^ = mu + lo + delta c + lo2 + delta2 c2, float64."""
    return (decode(codes, delta, lo, mu)
            + np.asarray(lo2, np.float32).astype(np.float64)[:, None]
            + np.asarray(delta2, np.float32).astype(np.float64)[:, None]
            * np.asarray(codes2, np.float64))


def code_bytes(d: int, bits: int) -> int:
    return d * bits // 8


def pack_records(codes: np.ndarray, delta: np.ndarray, lo: np.ndarray, bits: int,
                 stride: int) -> np.ndarray:
    """Byte records [n, stride] in the layout described in the module text."""
    n, d = codes.shape
    cb = code_bytes(d, bits)
    if stride < cb + 8:
        raise ValueError("stride too small")
    out = np.zeros((n, stride), dtype=np.uint8)
    if bits == 8:
        out[:, :cb] = codes
    else:
        out[:, :cb] = (codes[:, 0::2] & 0xF) | ((codes[:, 1::2] & 0xF) << 4)
    out[:, cb:cb + 4] = np.asarray(delta, np.float32).reshape(n, 1).view(np.uint8)
    out[:, cb + 4:cb + 8] = np.asarray(lo, np.float32).reshape(n, 1).view(np.uint8)
    return out


def pack_level2_rows(codes2: np.ndarray, delta2: np.ndarray, lo2: np.ndarray) -> np.ndarray:
    """Second-level rows in the device library's layout: d code bytes, zero
    padding to a multiple of 16, float32 delta2, float32 lo2, 8 zero bytes."""
    n, d = codes2.shape
    pad = (d + 15) // 16 * 16
    out = np.zeros((n, pad + 16), dtype=np.uint8)
    out[:, :d] = codes2
    out[:, pad:pad + 4] = np.asarray(delta2, np.float32).reshape(n, 1).view(np.uint8)
    out[:, pad + 4:pad + 8] = np.asarray(lo2, np.float32).reshape(n, 1).view(np.uint8)
    return out


def unpack_records(rec: np.ndarray, d: int, bits: int):
    """Inverse of pack_records: (codes, delta, lo)."""
    rec = np.ascontiguousarray(rec, dtype=np.uint8)
    n = rec.shape[0]
    cb = code_bytes(d, bits)
    if bits == 8:
        codes = rec[:, :cb].copy()
    else:
        codes = np.empty((n, d), dtype=np.uint8)
        codes[:, 0::2] = rec[:, :cb] & 0xF
        codes[:, 1::2] = rec[:, :cb] >> 4
    delta = rec[:, cb:cb + 4].copy().view(np.float32).reshape(n)
    lo = rec[:, cb + 4:cb + 8].copy().view(np.float32).reshape(n)
    return codes, delta, lo
