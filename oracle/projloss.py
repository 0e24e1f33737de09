"""Sampled-pair refinement loss for the projections, float64.

Built from the LeanVec-OOD objective (Problem leanvec_orthonormal): the
error of the approximation <q, x> ~ <Aq, Bx> over query/database pairs.  For
a block of b_q queries (rows of Qb) and b_x database vectors (rows of Xb),
with P = b_q * b_x pairs:

  G = A Qb^T (d x b_q),  H = B Xb^T (d x b_x)
  Rm = Qb Xb^T - G^T H                   (b_q x b_x residuals)
  pair(A, B) = ||Rm||_F^2 / P
  loss = pair + lam * f(A, B; K_Q / m, K_X / n)   (trace form, Problem
         leanvec_efficient, on normalised second moments)

Gradients of the pair part (direct differentiation of the squared residual):
  d pair / dA = -(2/P) H Rm^T Qb,   d pair / dB = -(2/P) G Rm Xb
and of the trace part, Eq. leanvec_gradients on the normalised moments.

When the block holds every (query, database) pair, pair(A, B) equals
f(A, B)/(n m) exactly; the tests use that identity and central finite
differences as pins (tests/test_oracle_projloss.py).
"""
from __future__ import annotations

import numpy as np

from . import fit


def pair_loss(A, B, Qb, Xb) -> float:
    A, B = np.asarray(A, np.float64), np.asarray(B, np.float64)
    Qb, Xb = np.asarray(Qb, np.float64), np.asarray(Xb, np.float64)
    Rm = Qb @ Xb.T - (A @ Qb.T).T @ (B @ Xb.T)
    return float(np.sum(Rm * Rm) / Rm.size)


def pair_grads(A, B, Qb, Xb):
    A, B = np.asarray(A, np.float64), np.asarray(B, np.float64)
    Qb, Xb = np.asarray(Qb, np.float64), np.asarray(Xb, np.float64)
    G = A @ Qb.T
    H = B @ Xb.T
    Rm = Qb @ Xb.T - G.T @ H
    P = Rm.size
    dA = -(2.0 / P) * (H @ Rm.T) @ Qb
    dB = -(2.0 / P) * (G @ Rm) @ Xb
    return dA, dB


def loss(A, B, Qb, Xb, KQn, KXn, lam: float = 1.0) -> float:
    """Pair part plus lam times the trace loss on normalised moments."""
    return pair_loss(A, B, Qb, Xb) + lam * fit.loss_trace(A, B, KQn, KXn)


def grads(A, B, Qb, Xb, KQn, KXn, lam: float = 1.0):
    dA, dB = pair_grads(A, B, Qb, Xb)
    return (dA + lam * fit.grad_A(A, B, KQn, KXn), dB + lam * fit.grad_B(A, B, KQn, KXn))
