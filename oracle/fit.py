"""Projection learning in float64: LeanVec-ID and LeanVec-OOD.

Notation follows Section 2: vectors are the columns of X (D x n) and Q
(D x m); this module stores them as rows, so X_paper = X.T.  Projections
A, B are d x D.

* LeanVec-ID (Section 2.1, Problem pca): A = B = M, the d leading left
  singular vectors of X, i.e. the d leading eigenvectors of K_X = X X^T.
* LeanVec-OOD loss (Problem leanvec_orthonormal and Eq. leanvec_loss):
  f(A, B) = || Q^T A^T B X - Q^T X ||_F^2.
* Trace form (Problem leanvec_efficient): with K_Q = Q Q^T, K_X = X X^T,
  f = tr(A K_Q A^T B K_X B^T + K_Q K_X - 2 K_Q A^T B K_X).
* Partial gradients (Eq. leanvec_gradients).
* Frank-Wolfe block coordinate descent (Algorithm 1) over the spectral-norm
  ball C (Eq. stiefel_convex_hull), with the linear minimisation step
  S = U V^T from the SVD of the negative gradient (Section 2.3) and the stop
  rule |f_{t+1} - f_t| / f_t <= tol.
* Eigenvector search (Section 2.4, Algorithm 2): P = the d leading
  eigenvectors of K_beta = (1-beta)/m K_Q + beta/n K_X, beta chosen by a
  bounded Brent minimisation of the equalised loss (Problem
  leanvec_loss_same_proj_equalized).

Readings where the paper leaves a choice open: K_Q and K_X are used
normalised by m and n (this scales f and both gradients by 1/(nm) and leaves
every Frank-Wolfe iterate unchanged); the default Frank-Wolfe start is the
eigenvector-search projection at beta = 1/2 because the zero start suggested
in Algorithm 1 makes the first A-gradient vanish; alpha = 0.9 (the paper
leaves alpha in (0, 1) open; 0.9 reaches the stop rule in about the 50
iterations the paper reports, smaller values wander longer) and at most 500
iterations.  Eigenvector rows are ordered by decreasing eigenvalue and signed
so that the largest-magnitude entry is positive.

Pinned by: Eckart-Young and an independent SVD of the data, trace form vs
the direct Frobenius form, central finite differences of the gradients, the
LMO optimality, the FW gap sign, Proposition 1's first inequality, the
eigenvector-search endpoints, a trace of Algorithm 1 worked by hand on
D = 2, d = 1 (iterates, losses, gaps, B-step at the new A, the step
schedule and the stop rule's denominator; tests/golden/fw_hand.json), and
a hand example of the centring vector (tests/test_oracle_fit.py).

Test infrastructure only: the search library never imports this module.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np


def second_moment(V: np.ndarray) -> np.ndarray:
    """K = sum_i v_i v_i^T in float64 (Problem leanvec_efficient)."""
    V64 = np.asarray(V, dtype=np.float64)
    return V64.T @ V64


def sign_rows(P: np.ndarray) -> np.ndarray:
    """Flip each row so its largest-magnitude entry is positive."""
    P = np.array(P, dtype=np.float64, copy=True)
    idx = np.argmax(np.abs(P), axis=1)
    s = np.sign(P[np.arange(P.shape[0]), idx])
    s[s == 0] = 1.0
    return P * s[:, None]


def top_eigvecs(K: np.ndarray, d: int) -> Tuple[np.ndarray, np.ndarray]:
    """d leading eigenvectors (rows) and all eigenvalues, descending."""
    w, V = np.linalg.eigh(np.asarray(K, dtype=np.float64))
    order = np.argsort(-w, kind="stable")
    w = w[order]
    P = V[:, order[:d]].T
    return sign_rows(P), w


def fit_id(KX: np.ndarray, d: int) -> np.ndarray:
    """LeanVec-ID: A = B = M = d leading eigenvectors of K_X (Section 2.1)."""
    P, _ = top_eigvecs(KX, d)
    return P


def loss_frobenius(A, B, Q, X) -> float:
    """f(A,B) = ||Q^T A^T B X - Q^T X||_F^2 with rows as vectors (Eq. leanvec_loss)."""
    Q = np.asarray(Q, np.float64)
    X = np.asarray(X, np.float64)
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    approx = (Q @ A.T) @ (B @ X.T)
    exact = Q @ X.T
    return float(np.sum((approx - exact) ** 2))


def loss_trace(A, B, KQ, KX) -> float:
    """Trace form of f (Problem leanvec_efficient)."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    t1 = np.trace(A @ KQ @ A.T @ B @ KX @ B.T)
    t2 = np.trace(KQ @ KX)
    t3 = np.trace(KQ @ A.T @ B @ KX)
    return float(t1 + t2 - 2.0 * t3)


def grad_A(A, B, KQ, KX) -> np.ndarray:
    """d f / d A = 2 B K_X B^T A K_Q - 2 B K_X K_Q (Eq. leanvec_gradients)."""
    return 2.0 * B @ KX @ B.T @ A @ KQ - 2.0 * B @ KX @ KQ


def grad_B(A, B, KQ, KX) -> np.ndarray:
    """d f / d B = 2 A K_Q A^T B K_X - 2 A K_Q K_X (Eq. leanvec_gradients)."""
    return 2.0 * A @ KQ @ A.T @ B @ KX - 2.0 * A @ KQ @ KX


def lmo(C: np.ndarray) -> np.ndarray:
    """argmax over ||S||_op <= 1 of <S, C>: S = U V^T from the thin SVD of C (Section 2.3)."""
    U, _, Vt = np.linalg.svd(np.asarray(C, np.float64), full_matrices=False)
    return U @ Vt


@dataclass
class FWReport:
    iters: int = 0
    f: List[float] = field(default_factory=list)        # f(A_t, B_t), t = 0..iters
    gap_A: List[float] = field(default_factory=list)    # <S_A - A, -grad_A> per iteration
    gap_B: List[float] = field(default_factory=list)
    converged: bool = False


def eigsearch_projection(KQ, m, KX, n, d, beta: float) -> np.ndarray:
    """projection(beta) of Algorithm 2: leading eigenvectors of K_beta."""
    Kb = (1.0 - beta) / m * np.asarray(KQ, np.float64) + beta / n * np.asarray(KX, np.float64)
    P, _ = top_eigvecs(Kb, d)
    return P


def frank_wolfe(KQ, m, KX, n, d, alpha: float = 0.9, tol: float = 1e-3, T: int = 500,
                init: str = "es", A0=None, B0=None) -> Tuple[np.ndarray, np.ndarray, FWReport]:
    """Algorithm 1 (Frank-Wolfe BCD) on the normalised second moments."""
    KQn = np.asarray(KQ, np.float64) / m
    KXn = np.asarray(KX, np.float64) / n
    D = KQn.shape[0]
    if A0 is not None:
        A = np.asarray(A0, np.float64).copy()
        B = np.asarray(B0 if B0 is not None else A0, np.float64).copy()
    elif init == "es":
        A = eigsearch_projection(KQ, m, KX, n, d, 0.5)
        B = A.copy()
    elif init == "zero":
        A = np.zeros((d, D))
        B = np.zeros((d, D))
    else:
        raise ValueError(init)
    rep = FWReport()
    f_prev = loss_trace(A, B, KQn, KXn)
    rep.f.append(f_prev)
    for t in range(T + 1):
        gamma = 1.0 / (t + 1) ** alpha
        CA = -grad_A(A, B, KQn, KXn)
        SA = _lmo_or_fallback(CA, KQn, d)
        rep.gap_A.append(float(np.sum((SA - A) * CA)))
        A = (1.0 - gamma) * A + gamma * SA
        CB = -grad_B(A, B, KQn, KXn)
        SB = _lmo_or_fallback(CB, KQn, d)
        rep.gap_B.append(float(np.sum((SB - B) * CB)))
        B = (1.0 - gamma) * B + gamma * SB
        f = loss_trace(A, B, KQn, KXn)
        rep.f.append(f)
        rep.iters = t + 1
        if f_prev != 0 and abs(f - f_prev) / abs(f_prev) <= tol:
            rep.converged = True
            break
        f_prev = f
    return A, B, rep


def _lmo_or_fallback(C, KQn, d):
    # With a zero gradient every point of the ball is a minimiser; take the
    # leading eigenvectors of K_Q so the zero start is well defined.
    if not np.any(C):
        P, _ = top_eigvecs(KQn, d)
        return P
    return lmo(C)


def equalised_loss(P, KQ, m, KX, n) -> float:
    """Loss of Problem leanvec_loss_same_proj_equalized for P = A = B."""
    KQn = np.asarray(KQ, np.float64) / m
    KXn = np.asarray(KX, np.float64) / n
    return float(np.trace(P @ KQn @ P.T @ P @ KXn @ P.T) - 2.0 * np.trace(KQn @ P.T @ P @ KXn))


def eigsearch(KQ, m, KX, n, d, xtol: float = 1e-4):
    """Algorithm 2: beta in [0, 1] minimising the equalised loss (Brent, bounded)."""
    from scipy.optimize import minimize_scalar

    res = minimize_scalar(lambda b: equalised_loss(eigsearch_projection(KQ, m, KX, n, d, b),
                                                   KQ, m, KX, n),
                          bounds=(0.0, 1.0), method="bounded", options={"xatol": xtol})
    beta = float(res.x)
    return eigsearch_projection(KQ, m, KX, n, d, beta), beta


def project(V, M) -> np.ndarray:
    """Reduced vectors M v for every row v, float64 (Eq. 1: Aq and Bx)."""
    return np.asarray(V, np.float64) @ np.asarray(M, np.float64).T


def mean_reduced(X, B) -> np.ndarray:
    """Global LVQ centring vector mu = B * mean(x), float64."""
    return np.asarray(B, np.float64) @ np.asarray(X, np.float64).mean(axis=0)
