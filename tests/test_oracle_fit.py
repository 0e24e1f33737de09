"""Pins for the projection-learning oracle (LeanVec-ID, LeanVec-OOD)."""
import numpy as np
import pytest

from oracle import fit


def _data(D=16, n=300, m=200, seed=0, ood=True):
    rng = np.random.default_rng(seed)
    scale = 1.0 / np.sqrt(np.arange(1, D + 1))
    X = rng.standard_normal((n, D)) * scale
    if ood:
        Rot, _ = np.linalg.qr(rng.standard_normal((D, D)))
        Q = (rng.standard_normal((m, D)) * scale) @ Rot.T + 0.3
    else:
        Q = rng.standard_normal((m, D)) * scale
    return X, Q


def _subspace_gap(P1, P2):
    return np.linalg.norm(P1.T @ P1 - P2.T @ P2)


def test_fit_id_equals_svd_of_data_and_eckart_young():
    X, _ = _data(ood=False)
    d = 5
    P = fit.fit_id(fit.second_moment(X), d)
    # the d leading left singular vectors of the column-stacked data (Problem pca)
    U, s, _ = np.linalg.svd(X.T, full_matrices=False)
    assert _subspace_gap(P, U[:, :d].T) < 1e-10
    resid = np.sum((X.T - P.T @ (P @ X.T)) ** 2)
    assert resid == pytest.approx(np.sum(s[d:] ** 2), rel=1e-10)
    # orthonormal rows, descending energy, sign convention
    assert np.allclose(P @ P.T, np.eye(d), atol=1e-12)
    energy = np.sum((P @ X.T) ** 2, axis=1)
    assert np.all(np.diff(energy) <= 1e-9 * energy[0])
    assert np.all(P[np.arange(d), np.abs(P).argmax(1)] > 0)


def test_fit_id_beats_random_projections():
    X, _ = _data(ood=False, seed=3)
    d = 4
    P = fit.fit_id(fit.second_moment(X), d)
    best = np.sum((X.T - P.T @ (P @ X.T)) ** 2)
    rng = np.random.default_rng(9)
    for _ in range(200):
        M, _ = np.linalg.qr(rng.standard_normal((X.shape[1], d)))
        M = M.T
        assert best <= np.sum((X.T - M.T @ (M @ X.T)) ** 2) + 1e-9


def test_trace_form_equals_frobenius_form():
    X, Q = _data()
    rng = np.random.default_rng(4)
    A = rng.standard_normal((4, 16))
    B = rng.standard_normal((4, 16))
    f1 = fit.loss_frobenius(A, B, Q, X)
    f2 = fit.loss_trace(A, B, fit.second_moment(Q), fit.second_moment(X))
    assert f2 == pytest.approx(f1, rel=1e-10)


def test_gradients_match_central_differences():
    X, Q = _data(D=10, n=60, m=40)
    KQ, KX = fit.second_moment(Q), fit.second_moment(X)
    rng = np.random.default_rng(5)
    A = rng.standard_normal((3, 10)) * 0.3
    B = rng.standard_normal((3, 10)) * 0.3
    h = 1e-6
    for which, g in (("A", fit.grad_A(A, B, KQ, KX)), ("B", fit.grad_B(A, B, KQ, KX))):
        fd = np.zeros_like(g)
        for i in range(g.shape[0]):
            for j in range(g.shape[1]):
                Ap, Am, Bp, Bm = A.copy(), A.copy(), B.copy(), B.copy()
                if which == "A":
                    Ap[i, j] += h
                    Am[i, j] -= h
                else:
                    Bp[i, j] += h
                    Bm[i, j] -= h
                fd[i, j] = (fit.loss_trace(Ap, Bp, KQ, KX) - fit.loss_trace(Am, Bm, KQ, KX)) / (2 * h)
        assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g)


def test_lmo_is_optimal_over_the_spectral_ball():
    rng = np.random.default_rng(6)
    C = rng.standard_normal((4, 11))
    S = fit.lmo(C)
    assert np.linalg.norm(S, 2) <= 1 + 1e-12
    val = np.sum(S * C)
    # nuclear norm through the square roots of the eigenvalues of C C^T
    nuc = np.sum(np.sqrt(np.clip(np.linalg.eigvalsh(C @ C.T), 0, None)))
    assert val == pytest.approx(nuc, rel=1e-12)
    for _ in range(300):
        T = rng.standard_normal((4, 11))
        T /= np.linalg.norm(T, 2)
        assert np.sum(T * C) <= val + 1e-12


def test_proposition1_first_inequality_any_AB():
    X, Q = _data()
    rng = np.random.default_rng(7)
    for _ in range(20):
        A = rng.standard_normal((4, 16))
        B = rng.standard_normal((4, 16))
        lhs = fit.loss_frobenius(A, B, Q, X)
        rhs = np.sum(Q ** 2) * np.sum((A.T @ (B @ X.T) - X.T) ** 2)
        assert lhs <= rhs * (1 + 1e-12)


def test_frank_wolfe_gap_descent_and_stop_rule():
    X, Q = _data(D=24, n=500, m=400)
    KQ, KX = fit.second_moment(Q), fit.second_moment(X)
    m, n, d = len(Q), len(X), 6
    A, B, rep = fit.frank_wolfe(KQ, m, KX, n, d, tol=1e-3, T=500)
    assert all(g >= -1e-10 for g in rep.gap_A + rep.gap_B)
    assert rep.converged
    assert abs(rep.f[-1] - rep.f[-2]) / rep.f[-2] <= 1e-3
    # iterates stay in the spectral-norm ball
    assert np.linalg.norm(A, 2) <= 1 + 1e-9 and np.linalg.norm(B, 2) <= 1 + 1e-9
    # on out-of-distribution queries it improves on PCA of the database
    P = fit.fit_id(KX, d)
    assert fit.loss_trace(A, B, KQ / m, KX / n) < fit.loss_trace(P, P, KQ / m, KX / n)


def test_frank_wolfe_zero_start_is_defined():
    X, Q = _data(D=12, n=200, m=150, seed=11)
    KQ, KX = fit.second_moment(Q), fit.second_moment(X)
    A, B, rep = fit.frank_wolfe(KQ, len(Q), KX, len(X), 3, init="zero", T=200)
    assert np.isfinite(rep.f[-1]) and rep.f[-1] < rep.f[0]
    # the FW gap shrinks towards stationarity
    assert rep.gap_A[-1] + rep.gap_B[-1] < 0.2 * (rep.gap_A[0] + rep.gap_B[0])


def test_eigsearch_endpoints_and_id_fallback():
    X, Q = _data(D=14, n=400, m=300, seed=12)
    KQ, KX = fit.second_moment(Q), fit.second_moment(X)
    m, n, d = len(Q), len(X), 4
    P0 = fit.eigsearch_projection(KQ, m, KX, n, d, 0.0)
    P1 = fit.eigsearch_projection(KQ, m, KX, n, d, 1.0)
    Uq = np.linalg.svd(Q.T, full_matrices=False)[0][:, :d].T
    Ux = np.linalg.svd(X.T, full_matrices=False)[0][:, :d].T
    assert _subspace_gap(P0, Uq) < 1e-10
    assert _subspace_gap(P1, Ux) < 1e-10
    # identical query and database sets: the projection does not depend on beta
    Pa = fit.eigsearch_projection(KX, n, KX, n, d, 0.2)
    Pb = fit.eigsearch_projection(KX, n, KX, n, d, 0.9)
    assert _subspace_gap(Pa, Pb) < 1e-10
    P, beta = fit.eigsearch(KQ, m, KX, n, d)
    assert 0.0 <= beta <= 1.0
    f_best = fit.equalised_loss(P, KQ, m, KX, n)
    for b in np.linspace(0, 1, 11):
        assert f_best <= fit.equalised_loss(fit.eigsearch_projection(KQ, m, KX, n, d, b),
                                            KQ, m, KX, n) + 1e-9 * abs(f_best)


def _fw_hand():
    import json
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fw_hand.json")
    return json.load(open(path))


def test_frank_wolfe_hand_worked_trace():
    """Algorithm 1 on D = 2, d = 1 against the trace worked by hand
    (tests/golden/fw_hand.json): the iterates A^(t), B^(t), the losses, the
    linear steps' gaps after each of the first six iterations, and the early
    stop with the loss at (A^(t), B^(t)) as denominator.  A B-step taken from
    the gradient at A^(t) instead of A^(t+1), or a step that ignores alpha,
    misses the second iterate by far more than the tolerance."""
    g = _fw_hand()
    KQ, KX = np.array(g["KQ"]), np.array(g["KX"])
    A0, B0 = np.array([g["A0"]]), np.array([g["B0"]])
    its = g["iterations"]
    for T in range(len(its) - 1):   # the loop runs t = 0, ..., T
        A, B, rep = fit.frank_wolfe(KQ, g["m"], KX, g["n"], g["d"], alpha=g["alpha"], tol=0.0,
                                    T=T, A0=A0, B0=B0)
        want = its[T + 1]
        assert rep.iters == T + 1
        np.testing.assert_allclose(A[0], want["A"], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(B[0], want["B"], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(rep.f, g["f"][:T + 2], rtol=1e-12)
        np.testing.assert_allclose(rep.gap_A[T], want["gap_A"], rtol=1e-11)
        np.testing.assert_allclose(rep.gap_B[T], want["gap_B"], rtol=1e-11)
    for s in g["stops"]:
        _, _, rep = fit.frank_wolfe(KQ, 1, KX, 1, 1, alpha=g["alpha"], tol=s["tol"], T=50,
                                    A0=A0, B0=B0)
        assert rep.converged and rep.iters == s["iters"], (s, rep.iters)


def test_hand_trace_separates_plausible_mistakes():
    """The golden second iterate is far (>> the tolerance above) from what a
    B-step at A^(t) or a step 1/(t+1) would give, so the trace test above
    catches both (evaluated here with the oracle's own gradient and linear
    step, reordered)."""
    g = _fw_hand()
    KQ, KX = np.array(g["KQ"]), np.array(g["KX"])
    A, B = np.array([g["A0"]]), np.array([g["B0"]])
    for t in range(2):  # B-step at the old A
        gam = 1.0 / (t + 1) ** g["alpha"]
        SA = fit.lmo(-fit.grad_A(A, B, KQ, KX))
        SB = fit.lmo(-fit.grad_B(A, B, KQ, KX))
        A, B = (1 - gam) * A + gam * SA, (1 - gam) * B + gam * SB
    assert np.abs(B[0] - g["iterations"][2]["B"]).max() > 1e-2
    A, B = np.array([g["A0"]]), np.array([g["B0"]])
    for t in range(2):  # step ignoring alpha
        gam = 1.0 / (t + 1)
        A = (1 - gam) * A + gam * fit.lmo(-fit.grad_A(A, B, KQ, KX))
        B = (1 - gam) * B + gam * fit.lmo(-fit.grad_B(A, B, KQ, KX))
    assert np.abs(A[0] - g["iterations"][2]["A"]).max() > 1e-2


def test_mean_reduced_hand_example():
    """mu = B mean(x) (the LVQ centring vector): rows (1, 2), (3, 4), (5, 9)
    have mean (3, 5); B = [[1, 0], [1, 1], [2, -1]] maps it to (3, 8, 1)."""
    X = np.array([[1.0, 2.0], [3.0, 4.0], [5.0, 9.0]], np.float32)
    B = np.array([[1.0, 0.0], [1.0, 1.0], [2.0, -1.0]])
    np.testing.assert_array_equal(fit.mean_reduced(X, B), [3.0, 8.0, 1.0])
