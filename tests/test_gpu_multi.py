"""Batched search over many sub-indexes at a reduced scale of the multi-index
workload: 64 sub-indexes with log-uniform sizes (the 1e4..5e5 range divided
by 50), each with its own ID fit, LVQ-8 records, float16 secondaries and
R = 64 graph; a seeded stream of requests (sub-index, batch size, k in
{1, 10, 100}) packed greedily into captured steps; window L per
(sub-index, k) from the autotuner on learning queries.

Checks: every request of every step equals the plain search of the same
queries on its sub-index (ids and scores), the autotuned windows are the
smallest reaching the target on the learning queries, and test recall is
close to the target.
"""
from dataclasses import replace

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import graph_cached
from oracle import exact
from oracle import fit as ofit
from oracle import lvq as olvq
from oracle import search as osearch
from synth import gen

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
N_SUB = 64
SIZE_DIV = 50
POOL = 512        # test queries per sub-index
LEARN = 256       # learning queries per sub-index
MAX_BATCH = 256
CAPACITY = 4096   # queries per step
N_REQ = 96
TARGET = 0.90


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
    sizes = np.maximum(gen.subindex_sizes(N_SUB) // SIZE_DIV, 200)
    out = []
    for s in range(N_SUB):
        wl = replace(base, name=f"multi{s}", N=int(sizes[s]), m_test=POOL, m_learn=LEARN,
                     seed_data=4000 + s, seed_test=4100 + s, seed_learn=4200 + s)
        mix = gen.mixture(wl)
        X = gen.database(wl, mix)
        Q = gen.queries(wl, "test", mix=mix)
        Ql = gen.queries(wl, "learn", mix=mix)
        P = ofit.fit_id(ofit.second_moment(X), wl.d)
        Y = ofit.project(X, P).astype(np.float32)
        mu = ofit.mean_reduced(X, P).astype(np.float32)
        adj, entry = graph_cached(wl, X)
        mud = torch.from_numpy(mu).to(DEV)
        rec = torch.empty((wl.N, lv.lv_record_stride(wl.d, wl.bits)), dtype=torch.uint8,
                          device=DEV)
        lv.lv_lvq_encode(torch.from_numpy(Y).to(DEV), mud, wl.bits, rec)
        sec = torch.from_numpy(X.astype(np.float16)).to(DEV)
        adjd = torch.from_numpy(adj.view(np.int32)).to(DEV)
        Pb = torch.from_numpy(lv.lv_to_bf16(P).view(np.int16)).to(DEV)
        ix = lv.Index(rec, mud, sec, adjd, entry, wl.bits, wl.d, A_bf16=Pb)
        out.append(dict(wl=wl, X=X, Q=Q, Ql=Ql, ix=ix, keep=(rec, mud, sec, adjd, Pb),
                        P=P, Y=Y, mu=mu, adj=adj, entry=entry, Pb=Pb,
                        truth=exact.ground_truth(Q, X, 100),
                        truth_l=exact.ground_truth(Ql, X, 100).astype(np.uint32)))
    yield out
    for d in out:
        d["ix"].close()


def test_multi_index_stream(lv, subs):
    multi = lv.Multi([d["ix"] for d in subs])
    sub, cnt, kk, off = gen.request_stream(N_REQ, N_SUB, POOL, max_batch=MAX_BATCH)

    # autotuned window per (sub-index, k) on the learning queries
    Lsk = {}
    for s, k in sorted(set(zip(sub.tolist(), kk.tolist()))):
        Qld = torch.from_numpy(subs[s]["Ql"]).to(DEV)
        L, r = lv.lv_autotune_window(multi, s, Qld, subs[s]["truth_l"], k, TARGET, 512)
        assert r >= TARGET or L == 512
        Lsk[(s, k)] = L
    print("autotuned windows:", sorted(set(Lsk.values())))

    # greedy packing of consecutive requests into steps
    steps, curr, nq = [], [], 0
    for i in range(N_REQ):
        if curr and nq + cnt[i] > CAPACITY:
            steps.append(curr)
            curr, nq = [], 0
        curr.append(i)
        nq += int(cnt[i])
    steps.append(curr)
    max_req = max(len(st) for st in steps)
    batch = lv.Batch(multi, max_requests=max_req, max_queries=CAPACITY,
                     max_L=max(Lsk.values()))
    hits = total = 0
    for st in steps:
        reqs, Qs = [], []
        for i in st:
            s, k = int(sub[i]), int(kk[i])
            rows = (int(off[i]) + np.arange(int(cnt[i]))) % POOL
            Qs.append(subs[s]["Q"][rows])
            reqs.append((s, k, Lsk[(s, k)], int(cnt[i])))
        Q = torch.from_numpy(np.concatenate(Qs)).to(DEV)
        nout = sum(k * c for _, k, _, c in reqs)
        ids = torch.full((nout,), -7, dtype=torch.int32, device=DEV)
        sc = torch.zeros((nout,), dtype=torch.float32, device=DEV)
        batch.step(reqs, Q, ids, sc)
        torch.cuda.synchronize()
        q0 = o0 = 0
        for (s, k, L, c), i in zip(reqs, st):
            pi = torch.empty((c, k), dtype=torch.int32, device=DEV)
            ps = torch.empty((c, k), dtype=torch.float32, device=DEV)
            ws = torch.empty(lv.lv_search_workspace_size(subs[s]["ix"], c), dtype=torch.uint8,
                             device=DEV)
            lv.lv_search(subs[s]["ix"], Q[q0:q0 + c], k, L, pi, ps, None, ws=ws)
            torch.cuda.synchronize()
            bi = ids[o0:o0 + c * k].view(c, k)
            assert torch.equal(bi, pi), (s, k, L, c)
            assert torch.equal(sc[o0:o0 + c * k].view(c, k), ps), (s, k, L, c)
            got = bi.cpu().numpy().view(np.uint32).astype(np.int64)
            rows = (int(off[i]) + np.arange(c)) % POOL
            tr = subs[s]["truth"][rows, :k]
            hits += sum(len(set(a) & set(b)) for a, b in zip(got.tolist(), tr.tolist()))
            total += c * k
            q0 += c
            o0 += c * k
    rec = hits / total
    print(f"{len(steps)} steps, {N_REQ} requests, test recall {rec:.4f}")
    assert rec >= TARGET - 0.03
    batch.close()
    multi.close()


def test_batched_step_against_oracle(lv, subs):
    """One captured step of eight requests on eight sub-indexes of uneven
    sizes, k in {1, 10, 100}, against the float64 oracle directly:

    * given the same projected queries (the device projection, whose bits the
      step's grouped projection reproduces; lv_project computes them here),
      the oracle's ids, scores and expansion and scoring counts, request by
      request (exact visited set);
    * each side with its own projection (the oracle's in float64), recall@k
      of the step within 0.5 points of the oracle's, over all requests."""
    chosen = [3, 11, 17, 25, 34, 42, 50, 61]
    ks = [1, 10, 100, 10, 1, 100, 10, 10]
    counts = [37, 128, 64, 1, 90, 50, 128, 7]
    Ls = {1: 24, 10: 48, 100: 128}
    multi = lv.Multi([d["ix"] for d in subs])
    batch = lv.Batch(multi, max_requests=len(chosen), max_queries=sum(counts), max_L=128,
                     hash_slots=8192)
    reqs, Qs = [], []
    for s, k, c in zip(chosen, ks, counts):
        reqs.append((s, k, Ls[k], c))
        Qs.append(subs[s]["Q"][:c])
    Q = np.concatenate(Qs)
    Qd = torch.from_numpy(Q).to(DEV)
    nout = sum(k * c for _, k, _, c in reqs)
    ids = torch.full((nout,), -7, dtype=torch.int32, device=DEV)
    sc = torch.zeros((nout,), dtype=torch.float32, device=DEV)
    cnt = torch.zeros((len(Q), 2), dtype=torch.int32, device=DEV)
    batch.step(reqs, Qd, ids, sc, cnt)
    torch.cuda.synchronize()
    ids = ids.cpu().numpy().view(np.uint32).astype(np.int64)
    sc = sc.cpu().numpy()
    cnt = cnt.cpu().numpy()
    hits_gpu = hits_orc = total = 0
    q0 = o0 = 0
    for (s, k, L, c) in reqs:
        d = subs[s]
        codes, delta, lo = olvq.encode(d["Y"], d["mu"], d["wl"].bits)
        oidx = osearch.Index(d["adj"], d["entry"], codes, delta, lo, d["mu"],
                             d["X"].astype(np.float16))
        Qp = torch.empty((c, d["wl"].d), dtype=torch.float32, device=DEV)
        lv.lv_project(Qd[q0:q0 + c], d["Pb"], Qp)
        torch.cuda.synchronize()
        Qp = Qp.cpu().numpy()
        w_ids, w_sc, w_cnt = osearch.search_many(oidx, Q[q0:q0 + c], Qp, k, L)
        g_ids = ids[o0:o0 + c * k].reshape(c, k)
        g_sc = sc[o0:o0 + c * k].reshape(c, k)
        assert np.array_equal(g_ids, w_ids), (s, k, L, c)
        assert np.all(np.abs(g_sc - w_sc) <= 1e-4 * np.maximum(np.abs(w_sc), 1.0)), (s, k)
        assert np.array_equal(cnt[q0:q0 + c], w_cnt), (s, k)
        # recall: the oracle with its own float64 projection
        o_ids, _, _ = osearch.search_many(oidx, Q[q0:q0 + c],
                                          ofit.project(Q[q0:q0 + c], d["P"]).astype(np.float32),
                                          k, L)
        tr = d["truth"][:c, :k]
        hits_gpu += sum(len(set(a) & set(b)) for a, b in zip(g_ids.tolist(), tr.tolist()))
        hits_orc += sum(len(set(a) & set(b)) for a, b in zip(o_ids.tolist(), tr.tolist()))
        total += c * k
        q0 += c
        o0 += c * k
    r_gpu, r_orc = hits_gpu / total, hits_orc / total
    print(f"batched step recall {r_gpu:.4f}, oracle {r_orc:.4f} over {len(reqs)} requests")
    assert abs(r_gpu - r_orc) <= 0.005
    batch.close()
    multi.close()
