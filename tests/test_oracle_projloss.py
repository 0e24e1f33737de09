"""Pins for the sampled-pair refinement loss: finite differences and the all-pairs identity."""
import numpy as np
import pytest

from oracle import fit, projloss


def _tiny(D=12, d=3, bq=5, bx=7, seed=0):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((d, D)) * 0.4, rng.standard_normal((d, D)) * 0.4,
            rng.standard_normal((bq, D)), rng.standard_normal((bx, D)))


def test_pair_gradients_central_differences():
    A, B, Qb, Xb = _tiny()
    KQn = fit.second_moment(Qb) / len(Qb)
    KXn = fit.second_moment(Xb) / len(Xb)
    h = 1e-6
    gA, gB = projloss.grads(A, B, Qb, Xb, KQn, KXn, lam=0.7)
    for M, g in ((A, gA), (B, gB)):
        fd = np.zeros_like(M)
        for i in range(M.shape[0]):
            for j in range(M.shape[1]):
                M[i, j] += h
                fp = projloss.loss(A, B, Qb, Xb, KQn, KXn, lam=0.7)
                M[i, j] -= 2 * h
                fm = projloss.loss(A, B, Qb, Xb, KQn, KXn, lam=0.7)
                M[i, j] += h
                fd[i, j] = (fp - fm) / (2 * h)
        assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g)


def test_all_pairs_block_equals_normalised_trace_loss():
    A, B, Qb, Xb = _tiny(D=10, d=4, bq=9, bx=13, seed=1)
    KQn = fit.second_moment(Qb) / len(Qb)
    KXn = fit.second_moment(Xb) / len(Xb)
    assert projloss.pair_loss(A, B, Qb, Xb) == pytest.approx(fit.loss_trace(A, B, KQn, KXn),
                                                            rel=1e-10)
    gA, gB = projloss.pair_grads(A, B, Qb, Xb)
    assert np.allclose(gA, fit.grad_A(A, B, KQn, KXn), rtol=1e-10, atol=1e-12)
    assert np.allclose(gB, fit.grad_B(A, B, KQn, KXn), rtol=1e-10, atol=1e-12)
