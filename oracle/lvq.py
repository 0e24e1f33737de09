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

Pinned by: the half-step error bound, the code range and endpoints, and the
encode(decode(x)) fixed point (tests/test_oracle_lvq.py).
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
