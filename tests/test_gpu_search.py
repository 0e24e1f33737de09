"""GPU parity of the graph search against the float64 oracle.

Inputs come from synth (data, graph) and the oracle (projection, LVQ codes);
both sides walk the same graph with the same reduced vectors.  Bar: ids equal
the oracle's (ties resolved by the same total order), scores within 1e-4
relative, expansion counts equal (exact visited set) and primary-scoring
counts equal with an exact-size visited set, >= with a small one.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import Case, make_case, stride_for
from oracle import exact
from oracle import fit as ofit
from oracle import lvq as olvq
from oracle import search as osearch
from synth import gen, graph

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def lv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2312_16335_amd as lv

    lv.load()
    return lv


def gpu_index(lv, c: Case):
    Yd = torch.from_numpy(c.Y).to(DEV)
    mud = torch.from_numpy(c.mu).to(DEV)
    rec = torch.empty((c.wl.N, c.stride), dtype=torch.uint8, device=DEV)
    lv.lv_lvq_encode(Yd, mud, c.wl.bits, rec)
    sec = torch.from_numpy(c.sec).to(DEV)
    adj = torch.from_numpy(c.adj.view(np.int32)).to(DEV)
    Pb = torch.from_numpy(lv.lv_to_bf16(c.P).view(np.int16)).to(DEV)
    return lv.Index(rec, mud, sec, adj, c.entry, c.wl.bits, c.wl.d, A_bf16=Pb), rec


def run_projected(lv, index, c: Case, k, L, hash_slots=0, Q=None, Qp=None, expand=0,
                  launch=0):
    Q = c.Q if Q is None else Q
    Qp = c.Qp if Qp is None else Qp
    m = len(Q)
    ids = torch.full((m, k), 7, dtype=torch.int32, device=DEV)
    sc = torch.full((m, k), 7.0, dtype=torch.float32, device=DEV)
    cnt = torch.zeros((m, 2), dtype=torch.int32, device=DEV)
    lv.lv_search_projected(index, torch.from_numpy(Q).to(DEV), torch.from_numpy(Qp).to(DEV), k, L,
                           ids, sc, cnt, hash_slots=hash_slots, expand=expand, launch=launch)
    torch.cuda.synchronize()
    return (ids.cpu().numpy().view(np.uint32).astype(np.int64), sc.cpu().numpy(),
            cnt.cpu().numpy())


def assert_parity(c, oidx, got_ids, got_sc, want_ids, want_sc):
    sent = osearch.SENTINEL
    mism = got_ids != want_ids
    if mism.any():
        # tolerate only swaps of exactly tied secondary scores
        for qi in np.unique(np.nonzero(mism)[0]):
            g = [int(x) for x in got_ids[qi] if x != sent]
            w = [int(x) for x in want_ids[qi] if x != sent]
            sg = osearch.secondary_scores(oidx, c.Q[qi].astype(np.float64), g)
            sw = osearch.secondary_scores(oidx, c.Q[qi].astype(np.float64), w)
            assert np.allclose(np.sort(sg), np.sort(sw), rtol=0, atol=1e-12), f"query {qi}"
    finite = np.isfinite(want_sc)
    assert np.array_equal(np.isfinite(got_sc), finite)
    scale = np.maximum(np.abs(want_sc[finite]), 1.0)
    assert np.all(np.abs(got_sc[finite] - want_sc[finite]) <= 1e-4 * scale)


@pytest.fixture(scope="module")
def small():
    return make_case(gen.WORKLOADS["id-small"])


def test_encoded_records_match_oracle(lv, small):
    index, rec = gpu_index(lv, small)
    c, dl, lo = olvq.encode(small.Y, small.mu, small.wl.bits)
    assert np.array_equal(rec.cpu().numpy(), olvq.pack_records(c, dl, lo, small.wl.bits,
                                                               small.stride))


@pytest.mark.parametrize("k,L", [(10, 50), (1, 1), (10, 10), (100, 128), (5, 300)])
def test_search_parity_small(lv, small, k, L):
    index, _ = gpu_index(lv, small)
    oidx = small.oracle_index()
    want_ids, want_sc, want_cnt = osearch.search_many(oidx, small.Q, small.Qp, k, L)
    got_ids, got_sc, got_cnt = run_projected(lv, index, small, k, L, hash_slots=8192)
    assert_parity(small, oidx, got_ids, got_sc, want_ids, want_sc)
    assert np.array_equal(got_cnt[:, 0], want_cnt[:, 0])
    assert np.array_equal(got_cnt[:, 1], want_cnt[:, 1])


@pytest.mark.parametrize("expand", [1, 3])
def test_small_visited_hash_changes_nothing(lv, small, expand):
    """Visited sets of any multiple of 256 slots (powers of two and others,
    whose home slots come from the multiply-high range reduction) forget ids
    differently but return the same ids, scores and expansions; only the
    scorings of forgotten ids grow."""
    index, _ = gpu_index(lv, small)
    ref = run_projected(lv, index, small, 10, 200, hash_slots=8192, expand=expand)
    for hs in (256, 768, 1024, 1280, 1536, 2816):
        got = run_projected(lv, index, small, 10, 200, hash_slots=hs, expand=expand)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), hs
        assert np.array_equal(got[2][:, 0], ref[2][:, 0]), hs
        assert np.all(got[2][:, 1] >= ref[2][:, 1]), hs


def test_full_window_is_exact_knn(lv):
    wl = gen.WORKLOADS["id-small"].scaled(N=900, m_test=8)
    c = make_case(wl)
    assert graph.reachable(c.adj, c.entry).all()
    index, _ = gpu_index(lv, c)
    got_ids, got_sc, _ = run_projected(lv, index, c, 10, 1024)
    truth = exact.ground_truth(c.Q, c.X, 10)
    assert np.array_equal(got_ids, truth)


def test_ragged_and_empty_batches(lv, small):
    index, _ = gpu_index(lv, small)
    oidx = small.oracle_index()
    for m in (1, 3, 65):
        Q, Qp = small.Q[:m], small.Qp[:m]
        want = osearch.search_many(oidx, Q, Qp, 10, 50)
        got = run_projected(lv, index, small, 10, 50, Q=Q, Qp=Qp)
        assert np.array_equal(got[0], want[0])
    z = run_projected(lv, index, small, 10, 50, Q=small.Q[:0], Qp=small.Qp[:0])
    assert z[0].shape == (0, 10)


def test_unreachable_tail_is_padded(lv):
    # a graph where the entry reaches only 3 nodes: results pad with sentinel / -inf
    wl = gen.WORKLOADS["id-small"].scaled(N=64, m_test=2)
    c = make_case(wl)
    adj = np.full_like(c.adj, osearch.SENTINEL)
    others = [i for i in range(wl.N) if i != c.entry][:2]
    adj[c.entry, :2] = others
    c.adj = adj
    index, _ = gpu_index(lv, c)
    got_ids, got_sc, _ = run_projected(lv, index, c, 5, 8)
    want_ids, want_sc, _ = osearch.search_many(c.oracle_index(), c.Q, c.Qp, 5, 8)
    assert np.array_equal(got_ids, want_ids)
    assert np.all(got_ids[:, 3:] == osearch.SENTINEL) and np.all(np.isneginf(got_sc[:, 3:]))


@pytest.mark.parametrize("name,N", [("ood-1m-512", 6000), ("id-1m-768", 6000)])
def test_search_parity_lvq4_and_f16(lv, name, N):
    wl = gen.WORKLOADS[name].scaled(N=N, m_test=40)
    c = make_case(wl)
    index, _ = gpu_index(lv, c)
    oidx = c.oracle_index()
    for L in (20, 60):
        want_ids, want_sc, want_cnt = osearch.search_many(oidx, c.Q, c.Qp, wl.k, L)
        got_ids, got_sc, got_cnt = run_projected(lv, index, c, wl.k, L, hash_slots=8192)
        assert_parity(c, oidx, got_ids, got_sc, want_ids, want_sc)
        assert np.array_equal(got_cnt, want_cnt)


@pytest.mark.parametrize("name,N", [("ood-1m-512", 6000), ("id-1m-768", 6000)])
def test_search_parity_lvq8_secondaries(lv, name, N):
    """Re-ranking with LVQ-8 secondary vectors: encoded rows bit-exact, search
    ids, scores and counters equal to the oracle's (secondary score of the
    LVQ-8 reconstruction)."""
    from dataclasses import replace

    wl = gen.WORKLOADS[name].scaled(N=N, m_test=40)
    c = make_case(wl)
    D = wl.D
    smu = c.X.astype(np.float64).mean(axis=0).astype(np.float32)
    rb = lv.lv_secondary_row_bytes(D, lv.LV_LVQ8)
    assert rb == D + 16
    rows = torch.full((wl.N, rb), 0xAB, dtype=torch.uint8, device=DEV)
    smud = torch.from_numpy(smu).to(DEV)
    lv.lv_lvq_encode(torch.from_numpy(c.X).to(DEV), smud, 8, rows)
    sc_, sd_, sl_ = olvq.encode(c.X, smu, 8)
    assert np.array_equal(rows.cpu().numpy(), olvq.pack_records(sc_, sd_, sl_, 8, rb))
    Yd = torch.from_numpy(c.Y).to(DEV)
    mud = torch.from_numpy(c.mu).to(DEV)
    rec = torch.empty((wl.N, c.stride), dtype=torch.uint8, device=DEV)
    lv.lv_lvq_encode(Yd, mud, wl.bits, rec)
    adj = torch.from_numpy(c.adj.view(np.int32)).to(DEV)
    index = lv.Index(rec, mud, rows, adj, c.entry, wl.bits, wl.d, sec_mu=smud)
    oidx = replace(c.oracle_index(), sec=sc_, sec_delta=sd_, sec_lo=sl_, sec_mu=smu)
    for L in (20, 60):
        want_ids, want_sc, want_cnt = osearch.search_many(oidx, c.Q, c.Qp, wl.k, L)
        got_ids, got_sc, got_cnt = run_projected(lv, index, c, wl.k, L, hash_slots=8192)
        assert_parity(c, oidx, got_ids, got_sc, want_ids, want_sc)
        assert np.array_equal(got_cnt, want_cnt)
        # team launch (LVQ-8 re-ranking in slices): identical
        team = run_projected(lv, index, c, wl.k, L, hash_slots=8192, launch=lv.LV_LAUNCH_TEAM)
        for g, o in zip(team, (got_ids, got_sc, got_cnt)):
            assert np.array_equal(g, o)
    index.close()


def test_full_path_recall_matches_oracle(lv, small):
    # end to end: GPU projection (bfloat16) + search vs oracle float64 projection
    index, _ = gpu_index(lv, small)
    m, k, L = len(small.Q), 10, 50
    ids = torch.empty((m, k), dtype=torch.int32, device=DEV)
    sc = torch.empty((m, k), dtype=torch.float32, device=DEV)
    ws = torch.empty(lv.lv_search_workspace_size(index, m), dtype=torch.uint8, device=DEV)
    lv.lv_search(index, torch.from_numpy(small.Q).to(DEV), k, L, ids, sc, ws=ws)
    torch.cuda.synchronize()
    got = ids.cpu().numpy().view(np.uint32).astype(np.int64)
    want, _, _ = osearch.search_many(small.oracle_index(), small.Q, small.Qp, k, L)
    truth = exact.ground_truth(small.Q, small.X, k)
    r_gpu = exact.recall_at_k(got, truth, k)
    r_orc = exact.recall_at_k(want, truth, k)
    assert abs(r_gpu - r_orc) <= 0.005 + 1e-12, (r_gpu, r_orc)


def test_ood_projections_end_to_end(lv):
    """LeanVec-OOD index with A != B (the oracle's Frank-Wolfe): records encode
    B x, the GPU projects queries with A.  With the oracle's A q supplied the
    search equals the oracle's; with the GPU's bfloat16 projection the recall
    is within 0.5 points of the oracle's."""
    from gpu_common import graph_cached

    wl = gen.WORKLOADS["ood-1m-512"].scaled(N=6000, m_test=100)
    mix = gen.mixture(wl)
    X = gen.database(wl, mix)
    Q = gen.queries(wl, "test", mix=mix)
    Ql = gen.queries(wl, "learn", mix=mix)
    A, B, _ = ofit.frank_wolfe(ofit.second_moment(Ql), len(Ql), ofit.second_moment(X), len(X),
                               wl.d)
    assert not np.allclose(A, B)
    adj, entry = graph_cached(wl, X)
    c = Case(wl, X, Q, A, ofit.project(X, B).astype(np.float32),
             ofit.project(Q, A).astype(np.float32), ofit.mean_reduced(X, B).astype(np.float32),
             adj, entry, X.astype(np.float16), stride_for(wl.d, wl.bits))
    index, _ = gpu_index(lv, c)  # A_bf16 = A: the query side
    oidx = c.oracle_index()
    k, L = wl.k, 60
    want_ids, want_sc, want_cnt = osearch.search_many(oidx, c.Q, c.Qp, k, L)
    got_ids, got_sc, got_cnt = run_projected(lv, index, c, k, L, hash_slots=8192)
    assert_parity(c, oidx, got_ids, got_sc, want_ids, want_sc)
    assert np.array_equal(got_cnt, want_cnt)
    m = len(Q)
    ids = torch.empty((m, k), dtype=torch.int32, device=DEV)
    sc = torch.empty((m, k), dtype=torch.float32, device=DEV)
    ws = torch.empty(lv.lv_search_workspace_size(index, m), dtype=torch.uint8, device=DEV)
    lv.lv_search(index, torch.from_numpy(Q).to(DEV), k, L, ids, sc, ws=ws)
    torch.cuda.synchronize()
    truth = exact.ground_truth(Q, X, k)
    r_gpu = exact.recall_at_k(ids.cpu().numpy().view(np.uint32).astype(np.int64), truth, k)
    r_orc = exact.recall_at_k(want_ids, truth, k)
    assert abs(r_gpu - r_orc) <= 0.005 + 1e-12, (r_gpu, r_orc)
    index.close()


@pytest.mark.parametrize("expand", [2, 4, 8])
@pytest.mark.parametrize("name,N", [("id-1m-768", 6000), ("ood-1m-512", 6000)])
def test_expand_variant_parity(lv, name, N, expand):
    """Several expansions per iteration (throughput variant) against the
    oracle's same variant: ids, scores and expansion / scoring counts."""
    wl = gen.WORKLOADS[name].scaled(N=N, m_test=40)
    c = make_case(wl)
    index, _ = gpu_index(lv, c)
    oidx = c.oracle_index()
    for L in (20, 60):
        want_ids = np.empty((len(c.Q), wl.k), np.int64)
        want_sc = np.empty((len(c.Q), wl.k))
        want_cnt = np.empty((len(c.Q), 2), np.int64)
        for i in range(len(c.Q)):
            tr = osearch.Trace()
            want_ids[i], want_sc[i] = osearch.search_one(oidx, c.Q[i], c.Qp[i], wl.k, L, trace=tr,
                                                         expand=expand)
            want_cnt[i] = (tr.n_exp, tr.n_dist)
        got_ids, got_sc, got_cnt = run_projected(lv, index, c, wl.k, L, hash_slots=8192,
                                                 expand=expand)
        assert_parity(c, oidx, got_ids, got_sc, want_ids, want_sc)
        assert np.array_equal(got_cnt, want_cnt)
        # a small visited set changes nothing but the number of scorings
        got2 = run_projected(lv, index, c, wl.k, L, hash_slots=256, expand=expand)
        assert np.array_equal(got2[0], got_ids) and np.array_equal(got2[1], got_sc)
        assert np.array_equal(got2[2][:, 0], got_cnt[:, 0])


def _oracle_expand(oidx, c, k, L, expand):
    ids = np.empty((len(c.Q), k), np.int64)
    sc = np.empty((len(c.Q), k))
    cnt = np.empty((len(c.Q), 2), np.int64)
    for i in range(len(c.Q)):
        tr = osearch.Trace()
        ids[i], sc[i] = osearch.search_one(oidx, c.Q[i], c.Qp[i], k, L, trace=tr, expand=expand)
        cnt[i] = (tr.n_exp, tr.n_dist)
    return ids, sc, cnt


@pytest.mark.parametrize("expand", [1, 3, 8])
@pytest.mark.parametrize("name,N,d", [("id-1m-768", 6000, 0), ("ood-1m-512", 6000, 0),
                                      ("id-1m-768", 3000, 256), ("id-1m-768", 3000, 112),
                                      ("id-1m-768", 3000, 64)],
                         ids=["lvq8-g16x12", "lvq4-g8x12", "lvq8-g64x8", "lvq8-g16x8",
                              "lvq8-g8x12"])
def test_team_launch_parity(lv, name, N, d, expand):
    """Four wavefronts per query (team launch): the oracle's traversal with the
    same number of expansions per iteration (one: the paper's), and
    bit-for-bit the one-wavefront kernel's ids, scores and counters."""
    from dataclasses import replace

    wl = gen.WORKLOADS[name].scaled(N=N, m_test=40)
    if d:
        wl = replace(wl, d=d)
    c = make_case(wl)
    index, _ = gpu_index(lv, c)
    oidx = c.oracle_index()
    for L in (20, 60):
        want_ids, want_sc, want_cnt = _oracle_expand(oidx, c, wl.k, L, expand)
        got = run_projected(lv, index, c, wl.k, L, hash_slots=8192, expand=expand,
                            launch=lv.LV_LAUNCH_TEAM)
        assert_parity(c, oidx, got[0], got[1], want_ids, want_sc)
        assert np.array_equal(got[2], want_cnt)
        one = run_projected(lv, index, c, wl.k, L, hash_slots=8192, expand=expand)
        for g, o in zip(got, one):
            assert np.array_equal(g, o)
        # small visited set: same results, scorings may repeat
        got2 = run_projected(lv, index, c, wl.k, L, hash_slots=256, expand=expand,
                             launch=lv.LV_LAUNCH_TEAM)
        assert np.array_equal(got2[0], got[0]) and np.array_equal(got2[1], got[1])
        assert np.array_equal(got2[2][:, 0], got[2][:, 0])


@pytest.mark.parametrize("k,L", [(1, 1), (100, 128), (5, 300)])
def test_team_launch_edges(lv, small, k, L):
    """Team launch at the window extremes, one query, and no query."""
    index, _ = gpu_index(lv, small)
    oidx = small.oracle_index()
    want_ids, want_sc, want_cnt = osearch.search_many(oidx, small.Q, small.Qp, k, L)
    got_ids, got_sc, got_cnt = run_projected(lv, index, small, k, L, hash_slots=8192,
                                             launch=lv.LV_LAUNCH_TEAM)
    assert_parity(small, oidx, got_ids, got_sc, want_ids, want_sc)
    assert np.array_equal(got_cnt, want_cnt)
    one = run_projected(lv, index, small, k, L, hash_slots=8192, Q=small.Q[7:8],
                        Qp=small.Qp[7:8], launch=lv.LV_LAUNCH_TEAM)
    assert np.array_equal(one[0], got_ids[7:8]) and np.array_equal(one[1], got_sc[7:8])
    none = run_projected(lv, index, small, k, L, Q=small.Q[:0], Qp=small.Qp[:0],
                         launch=lv.LV_LAUNCH_TEAM)
    assert none[0].shape == (0, k)


@pytest.mark.parametrize("expand", [1, 3])
def test_team_launch_at_the_largest_window(lv, small, expand):
    """L = 1024 (the largest window) and k = 100: the team launch equals the
    one-wavefront kernel bit for bit (ids, scores, counters)."""
    index, _ = gpu_index(lv, small)
    team = run_projected(lv, index, small, 100, 1024, hash_slots=8192, expand=expand,
                         launch=lv.LV_LAUNCH_TEAM)
    one = run_projected(lv, index, small, 100, 1024, hash_slots=8192, expand=expand)
    for g, o in zip(team, one):
        assert np.array_equal(g, o)
    assert (team[0] != osearch.SENTINEL).all()  # 10,000 nodes: every query finds 100


def _resid_case(lv, N=6000):
    """id-1m-768 at N = 6000 with residual secondaries: P_full = all D
    eigenvectors of the oracle's fit, primaries from its first d rows,
    secondaries = float16 of the other D - d coordinates."""
    wl = gen.WORKLOADS["id-1m-768"].scaled(N=N, m_test=40)
    c = make_case(wl)
    Pf = ofit.fit_id(ofit.second_moment(c.X), wl.D)
    P, Pp = Pf[:wl.d], Pf[wl.d:]
    Y = ofit.project(c.X, P).astype(np.float32)
    mu = ofit.mean_reduced(c.X, P).astype(np.float32)
    sec = ofit.project(c.X, Pp).astype(np.float16)
    Qf = ofit.project(c.Q, Pf).astype(np.float32)  # P q then P_perp q
    codes, delta, lo = olvq.encode(Y, mu, wl.bits)
    oidx = osearch.Index(c.adj, c.entry, codes, delta, lo, mu, sec, sec_resid=True)
    Yd = torch.from_numpy(Y).to(DEV)
    mud = torch.from_numpy(mu).to(DEV)
    rec = torch.empty((wl.N, c.stride), dtype=torch.uint8, device=DEV)
    lv.lv_lvq_encode(Yd, mud, wl.bits, rec)
    secd = torch.from_numpy(sec).to(DEV)
    adj = torch.from_numpy(c.adj.view(np.int32)).to(DEV)
    Pb = torch.from_numpy(lv.lv_to_bf16(Pf).view(np.int16)).to(DEV)
    index = lv.Index(rec, mud, secd, adj, c.entry, wl.bits, wl.d, A_bf16=Pb, residual=True)
    return wl, c, oidx, index, Qf, (rec, mud, secd, adj, Pb)


def test_search_parity_residual_secondaries(lv):
    wl, c, oidx, index, Qf, keep = _resid_case(lv)
    m, k = len(c.Q), wl.k
    for L in (20, 60):
        want_ids = np.empty((m, k), np.int64)
        want_sc = np.empty((m, k))
        want_cnt = np.empty((m, 2), np.int64)
        for i in range(m):
            tr = osearch.Trace()
            want_ids[i], want_sc[i] = osearch.search_one(oidx, Qf[i, wl.d:], Qf[i, :wl.d], k, L,
                                                         trace=tr)
            want_cnt[i] = (tr.n_exp, tr.n_dist)
        ids = torch.empty((m, k), dtype=torch.int32, device=DEV)
        sc = torch.empty((m, k), dtype=torch.float32, device=DEV)
        cnt = torch.zeros((m, 2), dtype=torch.int32, device=DEV)
        Qfd = torch.from_numpy(Qf).to(DEV)
        lv.lv_search_projected(index, Qfd, Qfd, k, L, ids, sc, cnt, hash_slots=8192)
        torch.cuda.synchronize()
        got_ids = ids.cpu().numpy().view(np.uint32).astype(np.int64)
        got_sc = sc.cpu().numpy()
        assert np.array_equal(cnt.cpu().numpy(), want_cnt)
        mism = np.nonzero((got_ids != want_ids).any(axis=1))[0]
        for qi in mism:  # only swaps of exactly tied scores
            g = osearch.secondary_scores(oidx, Qf[qi, wl.d:].astype(np.float64), got_ids[qi],
                                         Qf[qi, :wl.d].astype(np.float64))
            w = osearch.secondary_scores(oidx, Qf[qi, wl.d:].astype(np.float64), want_ids[qi],
                                         Qf[qi, :wl.d].astype(np.float64))
            assert np.allclose(np.sort(g), np.sort(w), rtol=0, atol=1e-12), qi
        assert np.all(np.abs(got_sc - want_sc) <= 1e-4 * np.maximum(np.abs(want_sc), 1.0))
        # the team launch re-ranks the residual part in slices: same results
        ids_t = torch.empty_like(ids)
        sc_t = torch.empty_like(sc)
        cnt_t = torch.zeros_like(cnt)
        lv.lv_search_projected(index, Qfd, Qfd, k, L, ids_t, sc_t, cnt_t, hash_slots=8192,
                               launch=lv.LV_LAUNCH_TEAM)
        torch.cuda.synchronize()
        assert torch.equal(ids_t, ids) and torch.equal(sc_t, sc) and torch.equal(cnt_t, cnt)
    index.close()


def test_residual_secondaries_batched_equals_plain(lv):
    wl, c, oidx, index, Qf, keep = _resid_case(lv, N=4000)
    m, k, L = len(c.Q), wl.k, 50
    Qd = torch.from_numpy(c.Q).to(DEV)
    ids_p = torch.empty((m, k), dtype=torch.int32, device=DEV)
    sc_p = torch.empty((m, k), dtype=torch.float32, device=DEV)
    ws = torch.empty(lv.lv_search_workspace_size(index, m), dtype=torch.uint8, device=DEV)
    lv.lv_search(index, Qd, k, L, ids_p, sc_p, None, ws=ws)
    multi = lv.Multi([index])
    batch = lv.Batch(multi, max_requests=4, max_queries=m, max_L=L)
    reqs = [(0, k, L, 13), (0, k, L, m - 13)]
    ids_b = torch.full((m * k,), -7, dtype=torch.int32, device=DEV)
    sc_b = torch.zeros((m * k,), dtype=torch.float32, device=DEV)
    batch.step(reqs, Qd, ids_b, sc_b)
    torch.cuda.synchronize()
    assert torch.equal(ids_b.view(m, k), ids_p) and torch.equal(sc_b.view(m, k), sc_p)
    # end to end (GPU projection of the full basis): recall against exact neighbours
    truth = exact.ground_truth(c.Q, c.X, k)
    got = ids_p.cpu().numpy().view(np.uint32).astype(np.int64)
    rec = sum(len(set(g) & set(t)) for g, t in zip(got, truth)) / (m * k)
    assert rec >= 0.9
    batch.close()
    multi.close()
    index.close()


def _level2_case(lv, name, bits, N=6000, d=0):
    """A workload with `bits`-bit primaries and their 8-bit second level as
    the re-ranking rows (LVQ4x8 at bits = 4).  d: the workload's if 0, D if -1
    (the baseline's own setting, the full eigenbasis as the projection), else
    that value."""
    from dataclasses import replace

    wl = replace(gen.WORKLOADS[name].scaled(N=N, m_test=40), bits=bits)
    if d:
        wl = replace(wl, d=wl.D if d < 0 else d)
    c = make_case(wl)
    codes, delta, lo = olvq.encode(c.Y, c.mu, bits)
    c2, d2, l2 = olvq.encode_residual(c.Y, c.mu, codes, delta, lo)
    oidx = osearch.Index(c.adj, c.entry, codes, delta, lo, c.mu, c2, d2, l2,
                         sec_two_level=True)
    Yd = torch.from_numpy(c.Y).to(DEV)
    mud = torch.from_numpy(c.mu).to(DEV)
    rec = torch.empty((wl.N, c.stride), dtype=torch.uint8, device=DEV)
    lv.lv_lvq_encode(Yd, mud, bits, rec)
    rb = lv.lv_secondary_row_bytes(wl.d, lv.LV_LVQ8_LEVEL2)
    assert rb == (wl.d + 15) // 16 * 16 + 16
    rows = torch.full((wl.N, rb), 0xAB, dtype=torch.uint8, device=DEV)
    lv.lv_lvq_encode_level2(Yd, mud, bits, rec, rows)
    torch.cuda.synchronize()
    want = olvq.pack_level2_rows(c2, d2, l2)
    adj = torch.from_numpy(c.adj.view(np.int32)).to(DEV)
    Pb = torch.from_numpy(lv.lv_to_bf16(c.P).view(np.int16)).to(DEV)
    index = lv.Index(rec, mud, rows, adj, c.entry, bits, wl.d, A_bf16=Pb, level2=True)
    return wl, c, oidx, index, rows, want, (rec, mud, rows, adj, Pb)


@pytest.mark.parametrize("name,bits,d", [("id-1m-768", 4, 0), ("ood-1m-512", 4, 0),
                                         ("id-1m-768", 8, 0), ("id-small", 4, -1),
                                         ("id-small", 8, 88)])
def test_search_parity_level2_secondaries(lv, name, bits, d):
    """Two-level LVQ (the second level re-ranks): rows bit-exact against the
    oracle's encoding; ids, scores and counters equal to the oracle's
    (primary score plus the second level's inner product with A q); the
    team launch identical; the batched step identical to the plain search."""
    wl, c, oidx, index, rows, want, keep = _level2_case(lv, name, bits, d=d)
    assert np.array_equal(rows.cpu().numpy(), want)
    m, k = len(c.Q), wl.k
    for L in (20, 60):
        want_ids, want_sc, want_cnt = osearch.search_many(oidx, c.Q, c.Qp, k, L)
        got_ids, got_sc, got_cnt = run_projected(lv, index, c, k, L, hash_slots=8192)
        mism = np.nonzero((got_ids != want_ids).any(axis=1))[0]
        for qi in mism:  # only swaps of exactly tied scores
            qp = c.Qp[qi].astype(np.float64)
            g = osearch.two_level_scores(oidx, qp, got_ids[qi])
            w = osearch.two_level_scores(oidx, qp, want_ids[qi])
            assert np.allclose(np.sort(g), np.sort(w), rtol=0, atol=1e-12), qi
        assert np.all(np.abs(got_sc - want_sc) <= 1e-4 * np.maximum(np.abs(want_sc), 1.0))
        assert np.array_equal(got_cnt, want_cnt)
        team = run_projected(lv, index, c, k, L, hash_slots=8192, launch=lv.LV_LAUNCH_TEAM)
        for g, o in zip(team, (got_ids, got_sc, got_cnt)):
            assert np.array_equal(g, o)
    # batched step (device projection) equals the plain search with the same projection
    L = 50
    Qd = torch.from_numpy(c.Q).to(DEV)
    ids_p = torch.empty((m, k), dtype=torch.int32, device=DEV)
    sc_p = torch.empty((m, k), dtype=torch.float32, device=DEV)
    ws = torch.empty(lv.lv_search_workspace_size(index, m), dtype=torch.uint8, device=DEV)
    lv.lv_search(index, Qd, k, L, ids_p, sc_p, None, ws=ws)
    multi = lv.Multi([index])
    batch = lv.Batch(multi, max_requests=2, max_queries=m, max_L=L)
    ids_b = torch.full((m * k,), -7, dtype=torch.int32, device=DEV)
    sc_b = torch.zeros((m * k,), dtype=torch.float32, device=DEV)
    batch.step([(0, k, L, 11), (0, k, L, m - 11)], Qd, ids_b, sc_b)
    torch.cuda.synchronize()
    assert torch.equal(ids_b.view(m, k), ids_p) and torch.equal(sc_b.view(m, k), sc_p)
    batch.close()
    multi.close()
    index.close()


def test_level2_rows_edges(lv):
    """Second-level rows for a ragged count of vectors with d not a multiple
    of 16 (zero padding), a vector equal to mu (delta2 = 0: all codes zero) and
    the 4-bit nibble order; bit-exact against the oracle."""
    rng = np.random.default_rng(77)
    for bits, d, n in ((4, 88, 37), (8, 8, 5), (4, 1008, 3), (8, 120, 130)):
        Y = (rng.standard_normal((n, d)) * rng.uniform(0.01, 5, (n, 1))).astype(np.float32)
        mu = rng.standard_normal(d).astype(np.float32)
        Y[0] = mu  # exact at the first level: residual 0, delta2 = 0
        Yd, mud = torch.from_numpy(Y).to(DEV), torch.from_numpy(mu).to(DEV)
        stride = lv.lv_record_stride(d, bits)
        rec = torch.empty((n, stride), dtype=torch.uint8, device=DEV)
        lv.lv_lvq_encode(Yd, mud, bits, rec)
        rb = lv.lv_secondary_row_bytes(d, lv.LV_LVQ8_LEVEL2)
        rows = torch.full((n, rb), 0x5A, dtype=torch.uint8, device=DEV)
        lv.lv_lvq_encode_level2(Yd, mud, bits, rec, rows)
        torch.cuda.synchronize()
        codes, delta, lo = olvq.encode(Y, mu, bits)
        c2, d2, l2 = olvq.encode_residual(Y, mu, codes, delta, lo)
        assert np.array_equal(rows.cpu().numpy(), olvq.pack_level2_rows(c2, d2, l2)), (bits, d)


def test_single_vector_index(lv):
    """N = 1: the entry is the only result; the rest of every list is padding."""
    rng = np.random.default_rng(31)
    D, d, k = 32, 8, 4
    X = rng.standard_normal((1, D)).astype(np.float32)
    P = np.linalg.qr(rng.standard_normal((D, d)))[0].T
    Y = ofit.project(X, P).astype(np.float32)
    mu = Y.mean(axis=0).astype(np.float32)
    codes, delta, lo = olvq.encode(Y, mu, 8)
    stride = stride_for(d, 8)
    rec = torch.from_numpy(olvq.pack_records(codes, delta, lo, 8, stride)).to(DEV)
    adj = np.full((1, 4), osearch.SENTINEL, dtype=np.uint32)
    sec = X.astype(np.float16)
    index = lv.Index(rec, torch.from_numpy(mu).to(DEV), torch.from_numpy(sec).to(DEV),
                     torch.from_numpy(adj.view(np.int32)).to(DEV), 0, 8, d)
    Q = rng.standard_normal((3, D)).astype(np.float32)
    Qp = ofit.project(Q, P).astype(np.float32)
    ids = torch.empty((3, k), dtype=torch.int32, device=DEV)
    sc = torch.empty((3, k), dtype=torch.float32, device=DEV)
    lv.lv_search_projected(index, torch.from_numpy(Q).to(DEV), torch.from_numpy(Qp).to(DEV), k, 5,
                           ids, sc)
    torch.cuda.synchronize()
    got = ids.cpu().numpy().view(np.uint32)
    oidx = osearch.Index(adj, 0, codes, delta, lo, mu, sec)
    for i in range(3):
        wi, ws = osearch.search_one(oidx, Q[i], Qp[i], k, 5)
        assert got[i].astype(np.int64).tolist() == wi.tolist()
        assert np.isneginf(sc[i, 1:].cpu().numpy()).all()
        assert abs(float(sc[i, 0]) - ws[0]) <= 1e-4 * max(1.0, abs(ws[0]))
    index.close()


# Record layouts and graph degrees beyond the benchmark's: every record
# stride the library accepts with 8- and 4-bit codes (8-bit records of up to
# four 64-byte chunks take the matrix-core scoring, including the 96-byte
# stride whose last chunk is partial; wider ones and all 4-bit ones the lane
# groups), and out-degrees above 64 (R = 128, the paper's construction
# setting, and R = 100, not a multiple of 64), with one and three expansions
# per iteration.  Ids, scores and both counters against the oracle.
LAYOUTS = [
    # bits, d, D, R
    (8, 160, 256, 128), (8, 160, 256, 100), (8, 32, 128, 64), (8, 88, 128, 64),
    (8, 120, 128, 64), (8, 240, 256, 64), (8, 384, 512, 64), (8, 752, 768, 64),
    (8, 1016, 1024, 64), (4, 32, 128, 64), (4, 160, 256, 128), (4, 240, 256, 64),
    (4, 368, 512, 64), (4, 480, 512, 64), (4, 1000, 1024, 64),
]


@pytest.mark.parametrize("bits,d,D,R", LAYOUTS,
                         ids=lambda v: str(v))
def test_search_parity_record_layouts_and_degrees(lv, bits, d, D, R):
    from dataclasses import replace

    base = gen.WORKLOADS["id-small"]
    wl = replace(base, name=f"layout-b{bits}-d{d}-D{D}", D=D, d=d, N=1500, m_test=24,
                 bits=bits, sec_dtype="f16", R=R)
    c = make_case(wl)
    assert c.stride == stride_for(d, bits) and c.adj.shape[1] == R
    index, _ = gpu_index(lv, c)
    oidx = c.oracle_index()
    for L, E in ((32, 1), (100, 1), (100, 3)):
        want_ids, want_sc, want_cnt = osearch.search_many(oidx, c.Q, c.Qp, 10, L, expand=E)
        got_ids, got_sc, got_cnt = run_projected(lv, index, c, 10, L, hash_slots=8192,
                                                 expand=E)
        assert_parity(c, oidx, got_ids, got_sc, want_ids, want_sc)
        assert np.array_equal(got_cnt, want_cnt), (L, E)
    # the team launch (four wavefronts per query) takes the same decisions
    team = run_projected(lv, index, c, 10, 100, hash_slots=8192, expand=3, launch=2)
    assert np.array_equal(team[0], got_ids) and np.array_equal(team[1], got_sc)
