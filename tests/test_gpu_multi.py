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
