"""Pins for the graph-search oracle: hand-traced example, brute force, invariants."""
import json
import os
from dataclasses import replace

import numpy as np
import pytest

from oracle import exact, lvq, search
from oracle import fit as ofit
from synth import gen, graph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "beam_hand.json")
SENT = search.SENTINEL


def _hand_index():
    g = json.load(open(GOLDEN))
    n = len(g["v"])
    codes = np.zeros((n, 4), dtype=np.uint8)
    codes[:, 0] = g["v"]
    adj = np.array([[SENT if a < 0 else a for a in row] for row in g["adj"]], dtype=np.uint32)
    sec = np.zeros((n, 2), dtype=np.float32)
    sec[:, 0] = g["w"]
    idx = search.Index(adj, g["entry"], codes, np.ones(n, np.float32), np.zeros(n, np.float32),
                       np.zeros(4, np.float32), sec)
    return g, idx


def test_hand_traced_traversal():
    g, idx = _hand_index()
    qp = np.array([1, 0, 0, 0], np.float32)
    q = np.array([1, 0], np.float32)
    for case in g["cases"]:
        tr = search.Trace()
        lst = search.beam(idx, qp, case["L"], trace=tr)
        assert [i for _, i in lst] == case["list_ids"], case["why"]
        assert (tr.n_exp, tr.n_dist) == (case["n_exp"], case["n_dist"]), case["why"]
        ids, sc = search.search_one(idx, q, qp, case["k"], case["L"])
        assert ids.tolist() == case["topk_ids"] and sc.tolist() == case["topk_scores"]


def test_window_smaller_than_k_rejected():
    _, idx = _hand_index()
    with pytest.raises(ValueError):
        search.search_one(idx, np.zeros(2, np.float32), np.zeros(4, np.float32), 5, 3)


TINY = gen.Workload("tiny", D=48, d=12, N=1200, K=20, spectrum="inv", sigma=0.3, seed_basis=11,
                    seed_data=12, seed_test=13, seed_learn=14, m_test=6, m_learn=200, bits=8,
                    sec_dtype="f16", R=16, L_list=(24,), k=5)


@pytest.fixture(scope="module")
def tiny():
    wl = TINY
    mix = gen.mixture(wl)
    X = gen.database(wl, mix)
    Q = gen.queries(wl, "test", mix=mix)
    P = ofit.fit_id(ofit.second_moment(X), wl.d)
    Y = ofit.project(X, P).astype(np.float32)
    Qp = ofit.project(Q, P).astype(np.float32)
    mu = ofit.mean_reduced(X, P).astype(np.float32)
    codes, delta, lo = lvq.encode(Y, mu, wl.bits)
    adj, entry = graph.build_graph(X, wl.R)
    assert graph.reachable(adj, entry).all()
    idx = search.Index(adj, entry, codes, delta, lo, mu, X.astype(np.float16))
    return wl, idx, Q, Qp


def test_full_window_equals_brute_force(tiny):
    wl, idx, Q, Qp = tiny
    k = wl.k
    S = idx.sec.astype(np.float64) @ Q.astype(np.float64).T
    for i in range(3):
        ids, sc = search.search_one(idx, Q[i], Qp[i], k, idx.N)
        truth = sorted(range(idx.N), key=lambda j: (-S[j, i], j))[:k]
        assert ids.tolist() == truth
        fids, fsc = search.flat_search(idx, Q[i], Qp[i], k, idx.N)
        assert fids.tolist() == truth and np.array_equal(fsc, sc)


def test_final_list_is_top_L_of_scored_set(tiny):
    wl, idx, Q, Qp = tiny
    for i in range(len(Q)):
        tr = search.Trace(scored={})
        lst = search.beam(idx, Qp[i], 24, trace=tr)
        best = sorted(tr.scored.items(), key=lambda t: (-t[1], t[0]))[:24]
        assert [i for _, i in lst] == [i for i, _ in best]
        assert tr.n_dist == len(tr.scored)


def test_bounded_visited_set_gives_identical_lists(tiny):
    wl, idx, Q, Qp = tiny
    for i in range(len(Q)):
        ref = search.beam(idx, Qp[i], 24)
        for cap in (4, 16, 64):
            tr = search.Trace()
            assert search.beam(idx, Qp[i], 24, visited_cap=cap, trace=tr) == ref


def test_primary_score_equals_factored_form(tiny):
    wl, idx, Q, Qp = tiny
    ids = np.arange(50)
    qp = Qp[0].astype(np.float64)
    qg = search.grid_query(qp)
    plain = search.primary_scores(idx, qp, ids)
    fact = (idx.delta[ids].astype(np.float64) * (idx.codes[ids].astype(np.float64) @ qg)
            + idx.lo[ids].astype(np.float64) * qg.sum() + idx.mu.astype(np.float64) @ qg)
    assert np.allclose(plain, fact, rtol=1e-12, atol=1e-12)
    # on the grid, <q~, c> is an integer sum times 2^-s: exact in int64
    s = 22 - int(np.frexp(np.abs(qp).max())[1])
    Qi = np.rint(np.ldexp(qp, s)).astype(np.int64)
    S = idx.codes[ids].astype(np.int64) @ Qi
    assert np.array_equal(np.ldexp(S.astype(np.float64), -s),
                          idx.codes[ids].astype(np.float64) @ qg)


def test_grid_query_hand_worked():
    """Largest component 3 = 0.75 * 2^2, so e = 2, s = 20: 3 stays; float32(0.1)
    = 13421773 * 2^-27 becomes rint(104857.6015625) = 104858 steps of 2^-20;
    -1e-9 is below half a step (rounds to zero).  Largest 1 = 0.5 * 2^1: s = 21,
    and 2.5 and 3.5 steps of 2^-21 round to the even 2 and 4 steps."""
    g = search.grid_query(np.array([3.0, np.float32(0.1), -1e-9, 0.0], np.float32))
    assert g.tolist() == [3.0, 104858 * 2.0 ** -20, 0.0, 0.0]
    g = search.grid_query(np.array([1.0, 2.5 * 2.0 ** -21, -3.5 * 2.0 ** -21], np.float32))
    assert g.tolist() == [1.0, 2 * 2.0 ** -21, -4 * 2.0 ** -21]
    assert search.grid_query(np.zeros(4, np.float32)).tolist() == [0.0] * 4


def test_grid_query_properties():
    """Multiples of 2^-s with at most 2^22 steps, within half a step (at most
    2^-22 of the largest component) of the query, unchanged by a second
    rounding, and scaled exactly with the query by powers of 2."""
    rng = np.random.default_rng(5)
    for t in range(200):
        q = (rng.standard_normal(160) * 10.0 ** rng.uniform(-30, 30)).astype(np.float32)
        q[rng.random(160) < 0.1] *= np.float32(1e-6)
        g = search.grid_query(q)
        q64 = q.astype(np.float64)
        s = 22 - int(np.frexp(np.abs(q64).max())[1])
        steps = np.ldexp(g, s)
        assert np.array_equal(steps, np.rint(steps)) and np.abs(steps).max() <= 2 ** 22
        assert np.all(np.abs(g - q64) <= np.ldexp(0.5, -s))
        assert np.all(np.abs(g - q64) <= 2.0 ** -22 * np.abs(q64).max())
        assert np.array_equal(search.grid_query(g), g)
        assert np.array_equal(search.grid_query(q * np.float32(2.0 ** 7)), g * 2.0 ** 7)


def test_parallel_search_matches_serial(tiny):
    wl, idx, Q, Qp = tiny
    a = search.search_many(idx, Q, Qp, wl.k, 24, procs=1)
    b = search.search_many(idx, Q, Qp, wl.k, 24, procs=2, chunk=2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_recall_reasonable_on_tiny(tiny):
    wl, idx, Q, Qp = tiny
    ids, _, _ = search.search_many(idx, Q, Qp, wl.k, 48)
    X64 = idx.sec.astype(np.float32)
    truth = exact.ground_truth(Q, X64, wl.k)
    assert exact.recall_at_k(ids, truth, wl.k) >= 0.8


def _lvq8_secondaries(idx, X):
    """The tiny index with LVQ-8 secondaries (centred on the database mean)."""
    smu = X.astype(np.float64).mean(axis=0).astype(np.float32)
    sc, sd, sl = lvq.encode(X, smu, 8)
    return replace(idx, sec=sc, sec_delta=sd, sec_lo=sl, sec_mu=smu), smu


def test_lvq8_secondaries_full_window_equals_brute_force(tiny):
    """With L >= N, the re-rank over LVQ-8 secondaries returns the exact top-k of
    <q, x^> over the reconstructed vectors (brute force with a full sort)."""
    wl, idx, Q, Qp = tiny
    X = idx.sec.astype(np.float32)
    idx8, smu = _lvq8_secondaries(idx, X)
    xhat = lvq.decode(idx8.sec, idx8.sec_delta, idx8.sec_lo, smu)
    S = xhat.astype(np.float64) @ Q.astype(np.float64).T
    for i in range(3):
        ids, sc = search.search_one(idx8, Q[i], Qp[i], wl.k, idx8.N)
        order = np.argsort(-S[:, i], kind="stable")[:wl.k]
        assert ids.tolist() == order.tolist()
        assert np.allclose(sc, S[order, i], rtol=0, atol=1e-12)


def test_lvq8_secondary_score_within_half_step_bound(tiny):
    """|<q, x^> - <q, x>| <= sum_j |q_j| (delta/2 + float32 rounding of lo), the
    per-component half-step bound of the quantiser."""
    wl, idx, Q, Qp = tiny
    X = idx.sec.astype(np.float32)
    idx8, smu = _lvq8_secondaries(idx, X)
    ids = np.arange(200)
    q64 = Q[0].astype(np.float64)
    got = search.secondary_scores(idx8, q64, ids)
    exact_s = X[ids].astype(np.float64) @ q64
    r = X[ids].astype(np.float64) - smu.astype(np.float64)
    slack = (idx8.sec_delta[ids].astype(np.float64) / 2
             + np.abs(idx8.sec_lo[ids].astype(np.float64) - r.min(axis=1))
             + 4 * np.finfo(np.float32).eps * np.abs(r).max(axis=1))
    assert (np.abs(got - exact_s) <= slack * np.abs(q64).sum() + 1e-12).all()


def test_lvq8_secondaries_parallel_matches_serial(tiny):
    wl, idx, Q, Qp = tiny
    idx8, _ = _lvq8_secondaries(idx, idx.sec.astype(np.float32))
    a = search.search_many(idx8, Q, Qp, wl.k, 24, procs=1)
    b = search.search_many(idx8, Q, Qp, wl.k, 24, procs=2, chunk=3)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_expand_variant_hand_traced():
    # several expansions per iteration (throughput variant), traced by hand on
    # the 6-node example of beam_hand.json (scores v = [10, 20, 5, 30, 25, 1])
    _, idx = _hand_index()
    qp = np.array([1, 0, 0, 0], np.float32)
    cases = [
        # L = 3, two per iteration: {0}, then {1, 2} (adds 3, 5, 4), then {3, 4}
        (3, 2, [3, 4, 1], 5, 6),
        # L = 2: {0} keeps 1 (2 falls off), {1} adds 3, {3} finds nothing new
        (2, 2, [3, 1], 3, 5),
        # expand = 1 is the traversal itself
        (3, 1, [i for _, i in search.beam(idx, qp, 3)], None, None),
    ]
    for L, e, want, n_exp, n_dist in cases:
        tr = search.Trace()
        got = [i for _, i in search.beam(idx, qp, L, trace=tr, expand=e)]
        assert got == want, (L, e)
        if n_exp is not None:
            assert (tr.n_exp, tr.n_dist) == (n_exp, n_dist), (L, e)


@pytest.mark.parametrize("expand", [2, 4])
def test_expand_variant_invariants(tiny, expand):
    wl, idx, Q, Qp = tiny
    k = wl.k
    S = idx.sec.astype(np.float64) @ Q.astype(np.float64).T
    for i in range(2):
        # a window holding every node: brute force whatever the expansion order
        ids, _ = search.search_one(idx, Q[i], Qp[i], k, idx.N, expand=expand)
        assert ids.tolist() == sorted(range(idx.N), key=lambda j: (-S[j, i], j))[:k]
        # the final list is the top L of what was scored, and a bounded visited
        # set does not change it
        tr = search.Trace(scored={})
        lst = search.beam(idx, Qp[i], 24, trace=tr, expand=expand)
        top = sorted(tr.scored.items(), key=lambda kv: (-kv[1], kv[0]))[:24]
        assert [j for j, _ in top] == [j for _, j in lst]
        assert search.beam(idx, Qp[i], 24, visited_cap=40, expand=expand) == lst


def _resid_index(tiny):
    """The tiny workload with residual secondaries: P_full = all D eigenvectors,
    primaries from the first d rows, secondaries = the other D - d coordinates."""
    wl, idx, Q, Qp = tiny
    mix = gen.mixture(wl)
    X = gen.database(wl, mix)
    Pf = ofit.fit_id(ofit.second_moment(X), wl.D)
    P, Pp = Pf[:wl.d], Pf[wl.d:]
    Y = ofit.project(X, P).astype(np.float32)
    mu = ofit.mean_reduced(X, P).astype(np.float32)
    codes, delta, lo = lvq.encode(Y, mu, wl.bits)
    sec = ofit.project(X, Pp)  # float64 residual coordinates
    ridx = search.Index(idx.adj, idx.entry, codes, delta, lo, mu, sec, sec_resid=True)
    return ridx, X, P, Pp


def test_residual_secondaries_decompose_the_inner_product(tiny):
    wl, _, Q, _ = tiny
    ridx, X, P, Pp = _resid_index(tiny)
    # the basis is orthonormal and complete
    Pf = np.vstack([P, Pp])
    assert np.allclose(Pf @ Pf.T, np.eye(wl.D), atol=1e-10)
    ids = np.arange(0, ridx.N, 7)
    for q in Q[:3].astype(np.float64):
        qp, qr = P @ q, Pp @ q
        got = search.secondary_scores(ridx, qr, ids, qp)
        # = primary score + <P_perp q, P_perp x>, and the exact inner product
        # differs from it by the LVQ error of the primary part only
        prim = search.primary_scores(ridx, qp, ids)
        exact_ip = X[ids].astype(np.float64) @ q
        true_prim = (X[ids].astype(np.float64) @ P.T) @ qp
        assert np.allclose(got - prim, exact_ip - true_prim, rtol=0, atol=1e-9)


def test_residual_secondaries_full_window_equals_brute_force(tiny):
    wl, _, Q, _ = tiny
    ridx, X, P, Pp = _resid_index(tiny)
    for q in Q[:3].astype(np.float32):
        qp = (P @ q.astype(np.float64)).astype(np.float32)
        qr = (Pp @ q.astype(np.float64)).astype(np.float32)
        ids, sc = search.search_one(ridx, qr, qp, wl.k, ridx.N)
        s = search.secondary_scores(ridx, qr.astype(np.float64), np.arange(ridx.N),
                                    qp.astype(np.float64))
        want = np.lexsort((np.arange(ridx.N), -s))[:wl.k]
        assert ids.tolist() == want.tolist()


def _two_level_index(tiny, bits):
    """The tiny workload with primaries of `bits` bits and their 8-bit second
    level as the re-ranking representation."""
    wl, idx, Q, Qp = tiny
    mix = gen.mixture(wl)
    X = gen.database(wl, mix)
    P = ofit.fit_id(ofit.second_moment(X), wl.d)
    Y = ofit.project(X, P).astype(np.float32)
    mu = idx.mu
    codes, delta, lo = lvq.encode(Y, mu, bits)
    c2, d2, l2 = lvq.encode_residual(Y, mu, codes, delta, lo)
    tidx = search.Index(idx.adj, idx.entry, codes, delta, lo, mu, c2, d2, l2,
                        sec_two_level=True)
    return tidx, Y, mu


@pytest.mark.parametrize("bits", [4, 8])
def test_two_level_full_window_equals_brute_force(tiny, bits):
    """With L >= N the re-rank returns the exact top-k of <q', y^> over the
    two-level reconstructions (brute force with a full sort), and its scores
    are those inner products."""
    wl, _, Q, Qp = tiny
    tidx, Y, mu = _two_level_index(tiny, bits)
    yhat = lvq.decode_two_level(tidx.codes, tidx.delta, tidx.lo, tidx.sec, tidx.sec_delta,
                                tidx.sec_lo, mu)
    y1 = lvq.decode(tidx.codes, tidx.delta, tidx.lo, mu).astype(np.float64)
    for i in range(3):
        # first level on the query's grid, second level with the query as given
        qp = Qp[i].astype(np.float64)
        S = y1 @ search.grid_query(qp) + (yhat - y1) @ qp
        ids, sc = search.search_one(tidx, None, Qp[i], wl.k, tidx.N)
        order = np.lexsort((np.arange(tidx.N), -S))[:wl.k]
        assert ids.tolist() == order.tolist()
        assert np.allclose(sc, S[order], rtol=0, atol=1e-9)


def test_two_level_scores_closer_to_the_reduced_inner_product(tiny):
    """The second level shrinks the score error against <q', y> to at most
    sum |q'_j| * delta2 / 2 (plus rounding), far below the first level's."""
    wl, _, Q, Qp = tiny
    tidx, Y, mu = _two_level_index(tiny, 4)
    ids = np.arange(300)
    qp = Qp[0].astype(np.float64)
    want = Y[ids].astype(np.float64) @ qp
    two = search.two_level_scores(tidx, qp, ids)
    one = search.primary_scores(tidx, qp, ids)
    # the first level's part is taken on the query's grid (half a step per
    # component at most)
    y1 = lvq.decode(tidx.codes[ids], tidx.delta[ids], tidx.lo[ids], mu).astype(np.float64)
    grid = np.abs(y1) @ np.abs(search.grid_query(qp) - qp)
    bound = (tidx.sec_delta[ids].astype(np.float64) / 2 + 1e-6 * tidx.delta[ids]) \
        * np.abs(qp).sum() + grid
    assert np.all(np.abs(two - want) <= bound + 1e-9)
    assert np.abs(two - want).max() < np.abs(one - want).max() / 20


def test_two_level_parallel_matches_serial(tiny):
    wl, _, Q, Qp = tiny
    tidx, _, _ = _two_level_index(tiny, 4)
    a = search.search_many(tidx, Q, Qp, wl.k, 24, procs=1)
    b = search.search_many(tidx, Q, Qp, wl.k, 24, procs=2, chunk=3)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
