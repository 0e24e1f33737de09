"""Pins for the exact-search oracle against a full sort."""
import numpy as np

from oracle import exact


def test_topk_matches_full_sort_with_ties():
    rng = np.random.default_rng(0)
    S = rng.integers(0, 5, size=(20, 50)).astype(np.float64)  # many ties
    got = exact.topk_ids(S, 7)
    for i in range(20):
        order = sorted(range(50), key=lambda j: (-S[i, j], j))[:7]
        assert got[i].tolist() == order


def test_ground_truth_chunked_equals_brute_force():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((300, 8)).astype(np.float32)
    Q = rng.standard_normal((5, 8)).astype(np.float32)
    got = exact.ground_truth(Q, X, 10, chunk=37)
    S = Q.astype(np.float64) @ X.astype(np.float64).T
    for i in range(5):
        order = sorted(range(300), key=lambda j: (-S[i, j], j))[:10]
        assert got[i].tolist() == order


def test_recall_definition():
    truth = np.array([[1, 2, 3, 4]])
    found = np.array([[4, 9, 1, exact.SENTINEL]])
    assert exact.recall_at_k(found, truth, 4) == 0.5
