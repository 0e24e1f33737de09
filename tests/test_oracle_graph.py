"""Pins for the graph-construction oracle: the distance against decoded
vectors, a hand-worked pruning example, the path graph of points on a line,
brute force for the construction search, and the row invariants."""
import json
import os

import numpy as np
import pytest

from oracle import graph as og
from oracle import lvq, search

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "prune_hand.json")
SENT = og.SENTINEL


def _random_primaries(n, d, bits, seed):
    rng = np.random.default_rng(seed)
    Y = rng.standard_normal((n, d)).astype(np.float32)
    mu = Y.mean(axis=0).astype(np.float32)
    codes, delta, lo = lvq.encode(Y, mu, bits)
    return og.Primaries(codes, delta, lo), lvq.decode(codes, delta, lo, mu)


@pytest.mark.parametrize("bits", [8, 4])
def test_l2_equals_decoded_distance(bits):
    prim, Yh = _random_primaries(200, 24, bits, 3)
    rng = np.random.default_rng(4)
    a = rng.integers(0, 200, 500)
    b = rng.integers(0, 200, 500)
    direct = ((Yh[a] - Yh[b]) ** 2).sum(axis=1)
    got = prim.l2(a, b)
    assert np.allclose(got, direct, rtol=1e-12, atol=1e-12 * direct.max())
    # a node's distance to itself cancels exactly: x + x - 2 x with one rounding each
    assert np.all(prim.l2(a, a) == 0.0)


def test_prune_hand_worked():
    g = json.load(open(GOLDEN))
    P = np.array(g["points"], dtype=np.float64)

    def dist(a, b):
        return ((P[np.asarray(a)] - P[np.asarray(b)]) ** 2).sum(axis=-1)

    for case in g["cases"]:
        got = og.prune(0, g["pool"], dist, case["alpha"], case["R"])
        assert got == case["kept"], case["why"]


def test_prune_ties_by_id():
    # two candidates at the same distance: the smaller id comes first
    P = np.array([[0, 0], [1, 0], [-1, 0], [0, 3]], dtype=np.float64)

    def dist(a, b):
        return ((P[np.asarray(a)] - P[np.asarray(b)]) ** 2).sum(axis=-1)

    assert og.prune(0, [2, 1, 3], dist, 1.0, 1) == [1]
    assert og.prune(0, [2, 1, 3], dist, 1.0, 3) == [1, 2, 3]


def test_reverse_row_rule():
    P = np.array([[0.0], [1.0], [2.0], [3.0], [-1.0], [-2.5], [0.5]])

    def dist(a, b):
        return ((P[np.asarray(a)] - P[np.asarray(b)]) ** 2).sum(axis=-1)

    # union fits: current row, then new sources ascending, repeats and j skipped
    assert og.reverse_row(0, [3, 1], [6, 1, 0, 4], dist, 1.0, 4) == [3, 1, 4, 6]
    # union too long: pruned around node 0 (nearest on each side of 0.0)
    assert og.reverse_row(0, [3, 1], [6, 5, 4], dist, 1.0, 3) == [6, 4]


def _line_primaries(t, d=8):
    # points t_i * (1, ..., 1): every LVQ record has delta = 0 and lo = t_i,
    # so f(a, b) = d (t_a - t_b)^2 exactly
    Y = (np.asarray(t, np.float32)[:, None] * np.ones((1, d), np.float32))
    codes, delta, lo = lvq.encode(Y, np.zeros(d, np.float32), 8)
    assert np.all(delta == 0)
    return og.Primaries(codes, delta, lo)


def _path_rows(t):
    order = np.argsort(t)
    left = {int(order[i]): int(order[i - 1]) for i in range(1, len(t))}
    right = {int(order[i]): int(order[i + 1]) for i in range(len(t) - 1)}
    return {i: {x for x in (left.get(i), right.get(i)) if x is not None} for i in range(len(t))}


@pytest.mark.parametrize("max_batch,passes", [(1, 1), (1, 2), (4, 2)])
def test_points_on_a_line_give_the_path(max_batch, passes):
    # alpha = 1, R = 2, a window holding every node: each node keeps its
    # nearest neighbour on each side and drops everything behind them
    rng = np.random.default_rng(11)
    n = 40
    t = rng.permutation(n).astype(np.float64) * 0.25 + rng.uniform(0, 0.1, n)
    prim = _line_primaries(t)
    order = rng.permutation(n)
    adj = og.build(prim, order, entry=int(order[0]), R=2, L=n, alphas=[1.0] * passes,
                   max_batch=max_batch)
    want = _path_rows(t)
    for i in range(n):
        assert set(int(x) for x in adj[i] if x != SENT) == want[i], i


def test_construction_search_is_brute_force_when_window_holds_all():
    prim, _ = _random_primaries(60, 16, 8, 5)
    rng = np.random.default_rng(6)
    adj = np.full((60, 6), SENT, dtype=np.uint32)
    for i in range(60):  # connected: a ring plus random edges
        adj[i, 0] = (i + 1) % 60
        adj[i, 1:4] = rng.choice([j for j in range(60) if j != i], 3, replace=False)
    for p in (0, 17, 59):
        got = og.window(prim, adj, 3, p, 60)
        f = prim.l2(np.full(60, p), np.arange(60))
        want = np.lexsort((np.arange(60), f)).tolist()
        assert got == want


def test_built_graph_rows_and_reachability():
    rng = np.random.default_rng(8)
    centers = rng.standard_normal((6, 16)) * 3
    Y = (centers[rng.integers(0, 6, 300)] + rng.standard_normal((300, 16))).astype(np.float32)
    codes, delta, lo = lvq.encode(Y, Y.mean(axis=0).astype(np.float32), 8)
    prim = og.Primaries(codes, delta, lo)
    order = rng.permutation(300)
    adj = og.build(prim, order, entry=0, R=8, L=16, alphas=[1.0, 1.0], max_batch=16)
    og.check_rows(adj)
    deg = (adj != SENT).sum(axis=1)
    assert deg.min() >= 1 and deg.max() <= 8
    assert og.reachable(adj, 0).mean() >= 0.95
    # a node's out-neighbours are mostly among its 8 nearest (by the same f)
    near = 0
    for p in range(0, 300, 10):
        f = prim.l2(np.full(300, p), np.arange(300))
        f[p] = np.inf
        nn = set(np.argsort(f)[:8].tolist())
        near += len(nn & set(int(x) for x in adj[p] if x != SENT)) > 0
    assert near >= 28


def test_stop_after_and_bad_order():
    prim, _ = _random_primaries(50, 8, 8, 9)
    order = np.arange(50)
    a1 = og.build(prim, order, 0, 4, 8, [1.0], 4, stop_after=1)
    assert (a1 != SENT).sum() == 0  # the first batch is node 0 alone: nothing to link to
    # batches {0}, {1, 2}: both new nodes see only node 0 and link to it,
    # node 0 gets both reverse edges, and 1 and 2 do not see each other
    a2 = og.build(prim, order, 0, 4, 8, [1.0], 4, stop_after=2)
    assert [set(a2[i].tolist()) - {SENT} for i in range(3)] == [{1, 2}, {0}, {0}]
    assert (a2[3:] == SENT).all()
    with pytest.raises(ValueError):
        og.build(prim, np.r_[order[:-1], 0], 0, 4, 8, [1.0], 4)
