"""GPU tests of the batched persistent search: identical results to the plain
search request by request (several sub-indexes, uneven batch sizes, mixed k
and L), consecutive captured steps, validation, and the autotuner."""
from dataclasses import replace

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import make_case
from oracle import exact
from synth import gen

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def lv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2312_16335_amd as lv

    lv.load()
    return lv


@pytest.fixture(scope="module")
def subs(lv):
    base = gen.WORKLOADS["id-1m-768"]
    out = []
    for s, n in enumerate((3000, 5000, 8000)):
        wl = replace(base, name=f"sub{s}", N=n, m_test=300, m_learn=300, seed_data=4000 + s,
                     seed_test=4100 + s, seed_learn=4200 + s)
        c = make_case(wl)
        Yd = torch.from_numpy(c.Y).to(DEV)
        mud = torch.from_numpy(c.mu).to(DEV)
        rec = torch.empty((wl.N, c.stride), dtype=torch.uint8, device=DEV)
        lv.lv_lvq_encode(Yd, mud, wl.bits, rec)
        sec = torch.from_numpy(c.sec).to(DEV)
        adj = torch.from_numpy(c.adj.view(np.int32)).to(DEV)
        Pb = torch.from_numpy(lv.lv_to_bf16(c.P).view(np.int16)).to(DEV)
        ix = lv.Index(rec, mud, sec, adj, c.entry, wl.bits, wl.d, A_bf16=Pb)
        out.append((c, ix))
    return out


def plain(lv, ix, Q, k, L, hash_slots=0, expand=0):
    m = len(Q)
    ids = torch.empty((m, k), dtype=torch.int32, device=DEV)
    sc = torch.empty((m, k), dtype=torch.float32, device=DEV)
    cnt = torch.zeros((m, 2), dtype=torch.int32, device=DEV)
    ws = torch.empty(lv.lv_search_workspace_size(ix, m), dtype=torch.uint8, device=DEV)
    lv.lv_search(ix, Q, k, L, ids, sc, cnt, ws=ws, hash_slots=hash_slots, expand=expand)
    return ids, sc, cnt


def run_step(lv, batch, subs, reqs, cursor):
    """Pack queries per request (taken from each sub-index's pool) and run one step."""
    Qs, spans = [], []
    for sub, k, L, count in reqs:
        c = subs[sub][0]
        lo = cursor[sub]
        Qs.append(c.Q[lo:lo + count])
        cursor[sub] += count
        spans.append((sub, k, L, count))
    Q = torch.from_numpy(np.concatenate(Qs)).to(DEV)
    nout = sum(k * count for _, k, _, count in reqs)
    ids = torch.full((nout,), -7, dtype=torch.int32, device=DEV)
    sc = torch.zeros((nout,), dtype=torch.float32, device=DEV)
    cnt = torch.zeros((len(Q), 2), dtype=torch.int32, device=DEV)
    batch.step(reqs, Q, ids, sc, cnt)
    return Q, ids, sc, cnt


def check_against_plain(lv, subs, reqs, Q, ids, sc, cnt, expand=0):
    torch.cuda.synchronize()
    q0 = o0 = 0
    for sub, k, L, count in reqs:
        pi, ps, pc = plain(lv, subs[sub][1], Q[q0:q0 + count], k, L, expand=expand)
        torch.cuda.synchronize()
        bi = ids[o0:o0 + count * k].view(count, k)
        bs = sc[o0:o0 + count * k].view(count, k)
        assert torch.equal(bi, pi), (sub, k, L, count)
        assert torch.equal(bs, ps), (sub, k, L, count)
        assert torch.equal(cnt[q0:q0 + count], pc)
        q0 += count
        o0 += count * k


@pytest.mark.parametrize("launch", [0, 1], ids=["per_query", "persistent"])
def test_batched_equals_plain_over_consecutive_steps(lv, subs, launch):
    multi = lv.Multi([ix for _, ix in subs])
    batch = lv.Batch(multi, max_requests=16, max_queries=1024, max_L=200, launch=launch)
    cursor = [0, 0, 0]
    steps = [
        [(0, 10, 40, 1), (1, 1, 20, 33), (2, 100, 128, 70), (0, 10, 60, 5), (1, 10, 40, 64)],
        [(2, 10, 200, 31), (2, 1, 1, 2)],
        [(1, 10, 30, 100), (0, 5, 5, 7), (2, 10, 50, 3), (1, 100, 100, 9)],
    ]
    for reqs in steps:
        out = run_step(lv, batch, subs, reqs, cursor)
        check_against_plain(lv, subs, reqs, *out)
    batch.close()
    multi.close()


@pytest.mark.parametrize("expand", [2, 4])
def test_batched_equals_plain_with_several_expansions_per_step(lv, subs, expand):
    multi = lv.Multi([ix for _, ix in subs])
    batch = lv.Batch(multi, max_requests=8, max_queries=512, max_L=128, expand=expand)
    cursor = [0, 0, 0]
    for reqs in ([(0, 10, 40, 17), (1, 1, 20, 33), (2, 100, 128, 70)],
                 [(2, 10, 64, 31), (0, 5, 5, 3), (1, 10, 96, 50)]):
        out = run_step(lv, batch, subs, reqs, cursor)
        check_against_plain(lv, subs, reqs, *out, expand=expand)
    batch.close()
    multi.close()


def test_batch_validation(lv, subs):
    multi = lv.Multi([ix for _, ix in subs])
    batch = lv.Batch(multi, max_requests=4, max_queries=100, max_L=64)
    Q = torch.zeros((200, 768), device=DEV)
    ids = torch.zeros((2000,), dtype=torch.int32, device=DEV)
    sc = torch.zeros((2000,), dtype=torch.float32, device=DEV)
    for bad in ([(0, 10, 65, 5)], [(3, 10, 20, 5)], [(0, 10, 5, 5)], [(0, 10, 20, 0)],
                [(0, 10, 20, 101)], [(0, 10, 20, 1)] * 5, []):
        with pytest.raises((lv.LVError, ValueError)):
            batch.step(bad, Q, ids, sc)
    batch.close()
    with pytest.raises(lv.LVError):
        lv.Batch(multi, max_requests=0, max_queries=10, max_L=10)
    with pytest.raises(lv.LVError):
        lv.Batch(multi, max_requests=4, max_queries=10, max_L=10, launch=2)
    multi.close()


def test_autotune_window_is_minimal(lv, subs):
    c, ix = subs[2]
    multi = lv.Multi([ix])
    Ql = c.Q[:200]
    truth = exact.ground_truth(Ql, c.X, 10).astype(np.uint32)
    Qd = torch.from_numpy(Ql).to(DEV)
    L, rec = lv.lv_autotune_window(multi, 0, Qd, truth, 10, 0.9, 512)
    assert rec >= 0.9 and 10 <= L <= 512

    def recall_at(L):
        ids, _, _ = plain(lv, ix, Qd, 10, L)
        torch.cuda.synchronize()
        return exact.recall_at_k(ids.cpu().numpy().view(np.uint32).astype(np.int64),
                                 truth.astype(np.int64), 10)

    assert recall_at(L) == pytest.approx(rec)
    if L > 10:
        assert recall_at(L - 1) < 0.9
    multi.close()


def test_autotune_knobs_returns_a_valid_choice(lv, subs):
    multi = lv.Multi([ix for _, ix in subs])
    reqs = [(0, 10, 40, 50), (1, 10, 40, 50), (2, 10, 40, 50)]
    Q = torch.from_numpy(np.concatenate([subs[s][0].Q[:50] for s in range(3)])).to(DEV)
    ids = torch.zeros((1500,), dtype=torch.int32, device=DEV)
    sc = torch.zeros((1500,), dtype=torch.float32, device=DEV)
    best, ms = lv.lv_autotune_knobs(multi, 4, 256, 64, reqs, Q, ids, sc, reps=2)
    assert best["hash_slots"] in (1024, 1280, 1536, 2048, 4096, 8192) and ms > 0
    assert best["launch"] in (0, 1)
    multi.close()


def test_timed_step_equals_untimed_and_brackets_the_traversal(lv, subs):
    multi = lv.Multi([ix for _, ix in subs])
    batch = lv.Batch(multi, max_requests=4, max_queries=512, max_L=100)
    reqs = [(0, 10, 60, 200), (2, 10, 100, 150), (1, 1, 20, 100)]
    Q = torch.from_numpy(np.concatenate([subs[0][0].Q[:200], subs[2][0].Q[:150],
                                         subs[1][0].Q[:100]])).to(DEV)
    nout = 200 * 10 + 150 * 10 + 100
    outs = []
    for timed in (False, True, True):
        ids = torch.full((nout,), -7, dtype=torch.int32, device=DEV)
        sc = torch.zeros((nout,), dtype=torch.float32, device=DEV)
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        batch.step(reqs, Q, ids, sc, events=ev if timed else None)
        t1.record()
        torch.cuda.synchronize()
        if timed:
            kernel_ms, step_ms = ev[0].elapsed_time(ev[1]), t0.elapsed_time(t1)
            assert 0 < kernel_ms <= step_ms
        outs.append((ids, sc))
    for ids, sc in outs[1:]:
        assert torch.equal(ids, outs[0][0]) and torch.equal(sc, outs[0][1])
    batch.close()
    multi.close()


@pytest.mark.parametrize("launch", [0, 1], ids=["per_query", "persistent"])
def test_consecutive_steps_on_several_streams(lv, subs, launch):
    """Steps issued in turn on three streams run concurrently on rotating
    device state; every step still equals the plain search."""
    multi = lv.Multi([ix for _, ix in subs])
    batch = lv.Batch(multi, max_requests=4, max_queries=600, max_L=128, launch=launch)
    streams = [torch.cuda.current_stream(), torch.cuda.Stream(), torch.cuda.Stream()]
    cursor = [0, 0, 0]
    plan = [
        [(0, 10, 60, 150), (2, 10, 100, 200)],
        [(1, 10, 40, 250), (0, 1, 10, 40)],
        [(2, 100, 128, 90), (1, 10, 80, 160)],
        [(0, 10, 50, 60), (2, 5, 20, 300), (1, 10, 30, 7)],
        [(1, 10, 64, 120)],
        [(2, 10, 90, 64), (0, 10, 30, 33)],
        [(0, 1, 1, 5), (1, 100, 100, 20)],
    ]
    # 3 in flight at first; later a device set is reused from another stream
    order = [0, 1, 2, 1, 2, 0, 1]
    runs = []
    for i, reqs in enumerate(plan):
        Qs = []
        for sub, k, L, count in reqs:
            pool = subs[sub][0].Q
            Qs.append(pool[(cursor[sub] + np.arange(count)) % len(pool)])
            cursor[sub] += count
        Q = torch.from_numpy(np.concatenate(Qs)).to(DEV)
        nout = sum(k * c for _, k, _, c in reqs)
        ids = torch.full((nout,), -7, dtype=torch.int32, device=DEV)
        sc = torch.zeros((nout,), dtype=torch.float32, device=DEV)
        cnt = torch.zeros((len(Q), 2), dtype=torch.int32, device=DEV)
        st = streams[order[i]]
        if st is not streams[0]:
            st.wait_stream(streams[0])  # inputs were made on stream 0
        batch.step(reqs, Q, ids, sc, cnt, stream=st)
        runs.append((reqs, Q, ids, sc, cnt))
    for st in streams[1:]:
        streams[0].wait_stream(st)
    torch.cuda.synchronize()
    for reqs, Q, ids, sc, cnt in runs:
        check_against_plain(lv, subs, reqs, Q, ids, sc, cnt)
    batch.close()
    multi.close()
