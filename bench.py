"""Benchmark: LeanVec search QPS at 10-recall@10 = 0.90 on one MI355X.

Workload (synthetic stand-in for the paper's rqa-768-1M, Table 1): 1M
database vectors of dimension 768 drawn from a 1,000-cluster mixture with a
1/i spectrum (L2-normalised), 10,000 test queries from the same mixture,
LeanVec-ID projection to d = 160, LVQ-8 primary records, float16 secondary
vectors, graph out-degree 64.  Index preparation (data, fit, projection,
encoding, graph, ground truth) is untimed.

A step is one pass of the hot path over the whole query set: query
projection on the matrix cores, then the per-query traversal + re-ranking
kernel, at the smallest window L whose recall reaches 0.90 (found by a sweep
before the timed region).  The query set arrives as a stream of requests of
uneven size (uniform in [1, 4096]); "plain" launches one search per request.

Prints one JSON line (rank 0).  Extra fields: the recall/QPS sweep, the
interpolated QPS at exactly 0.90, the roofline of the traversal kernel, and
the float64 CPU oracle timed on a bounded sample (cpu_baseline).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import threading
import time
from dataclasses import replace

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=None,
                    help="id-1m-768 (default); with --fit: ood-1m-512 (default)")
    ap.add_argument("--n", type=int, default=0, help="override database size (testing)")
    ap.add_argument("--target", type=float, default=0.90)
    ap.add_argument("--hash-slots", type=int, default=0,
                    help="visited-set slots (with --launch, skips the knob search)")
    ap.add_argument("--launch", choices=("per_query", "persistent"), default="per_query",
                    help="batched traversal launch when --hash-slots is given")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ood", action="store_true",
                    help="skip the cross-modal workload's sub-record (ood-1m-512)")
    ap.add_argument("--no-mfma", action="store_true",
                    help="skip the matrix-core kernels' sub-record (projections, refinement "
                         "step, GEMM; the same figures as --mfma)")
    ap.add_argument("--sec", choices=("f16", "lvq8", "resid", "level2"), default="f16",
                    help="secondary vectors: float16 (the benchmark configuration), LVQ-8, "
                         "float16 residual coordinates only (D - d per vector), or the 8-bit "
                         "second level of the primaries' LVQ (two-level LVQ; LVQ4x8 with "
                         "--bits 4); all but the first without CPU baseline")
    ap.add_argument("--bits", type=int, choices=(0, 4, 8), default=0,
                    help="LVQ bits of the primaries (0: the workload's)")
    ap.add_argument("--cpu-sample", type=int, default=10000)
    ap.add_argument("--only-steps", action="store_true",
                    help="skip the sweep refinement (profiling runs)")
    ap.add_argument("--L", type=int, default=0, help="fixed window (skips the sweep)")
    ap.add_argument("--expand", type=int, default=3,
                    help="entries expanded per traversal iteration (beam width of a step): "
                         "1 = the paper's one-at-a-time traversal; 2..8 = several best "
                         "unexpanded entries per iteration (3 measured fastest at recall 0.90)")
    ap.add_argument("--no-variant", action="store_true",
                    help="skip timing the other traversal (one expansion per iteration when "
                         "--expand > 1, three otherwise) beside the main value")
    ap.add_argument("--graph", choices=("cpu", "gpu"), default="cpu",
                    help="index graph: the host builder on float16 vectors (cached), or "
                         "lv_graph_build on the primary vectors (timed)")
    ap.add_argument("--build-L", type=int, default=0,
                    help="search window of the GPU graph build (default R, as the host builder)")
    ap.add_argument("--build-batch", type=int, default=0,
                    help="largest insertion batch of the GPU graph build (default N/50)")
    ap.add_argument("--mfma", action="store_true",
                    help="only time the matrix-core kernels (projections, refinement step, a "
                         "large GEMM) against the bf16 peak and HBM, print one JSON line, exit")
    ap.add_argument("--fit", action="store_true",
                    help="only time and compare the projection fits (host float64: ID, "
                         "eigenvector search, Frank-Wolfe; library and oracle) and their "
                         "brute-force recall in the reduced space, print one JSON line, exit")
    ap.add_argument("--refine", type=int, default=0, metavar="STEPS",
                    help="only run the differentiable refinement (Adam, STEPS steps from the "
                         "LeanVec-ID fit) on the OOD refinement workload, compare it with the "
                         "OOD fits on loss and reduced-space recall, print one JSON line, exit")
    ap.add_argument("--multi", action="store_true",
                    help="only run the multi-index workload at full size (64 sub-indexes of "
                         "log-uniform sizes in [1e4, 5e5], 1,024 requests with batch sizes "
                         "in [1, 4096] and k in {1, 10, 100}, autotuned windows), print one "
                         "JSON line, exit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration) and exit")
    return ap.parse_args()


def cache_dir():
    d = os.environ.get("LV_CACHE", "/tmp/lv_cache")
    os.makedirs(d, exist_ok=True)
    return d


def build_graph_cached(wl, X, out):
    from synth import graph

    key = f"{wl.name}_s{wl.seed_data}_n{wl.N}_R{wl.R}_a{'-'.join(map(str, wl.graph_alphas))}_v6"
    p = os.path.join(cache_dir(), key + ".npz")
    if os.path.exists(p):
        z = np.load(p)
        out["adj"], out["entry"] = z["adj"], int(z["entry"])
        out["graph_s"] = 0.0
        return
    t = time.time()
    adj, entry = graph.build_graph(X, wl.R, alphas=wl.graph_alphas)
    out["graph_s"] = time.time() - t
    np.savez(p + ".tmp.npz", adj=adj, entry=np.int64(entry))
    os.replace(p + ".tmp.npz", p)
    out["adj"], out["entry"] = adj, entry


def build_graph_gpu(lv, torch, wl, X, rec, args, out):
    """lv_graph_build over the primary records; entry = medoid of the database
    (as for the host builder), insertion order = a seeded permutation."""
    from synth import graph as sgraph

    entry = sgraph.medoid(X)
    order = np.random.default_rng(wl.seed_data + 17).permutation(wl.N).astype(np.uint32)
    bL = args.build_L or wl.R
    mb = args.build_batch or max(1, wl.N // 50)
    adjd = torch.empty((wl.N, wl.R), dtype=torch.int32, device=rec.device)
    bp = lv.build_params(wl.R, bL, wl.graph_alphas, mb)
    torch.cuda.synchronize()
    t = time.time()
    lv.lv_graph_build(rec, wl.N, wl.d, wl.bits, order, entry, bp, adjd)
    torch.cuda.synchronize()
    out["graph_s"] = time.time() - t
    # again with the work counters (a second, untimed build; must be identical)
    again = torch.empty_like(adjd)
    out["stats"] = lv.lv_graph_build(rec, wl.N, wl.d, wl.bits, order, entry, bp, again,
                                     stats=True)
    torch.cuda.synchronize()
    out["deterministic"] = bool(torch.equal(adjd, again))
    del again
    out["kind"] = (f"lv_graph_build on the primary vectors (window {bL}, batches up to {mb}, "
                   f"alphas {list(wl.graph_alphas)})")
    return adjd, entry


def oracle_build_sample(wl, X, bL, n=1000):
    """The oracle's construction (same R, window and alphas; batches up to
    n / 50) on the first n database vectors, with the oracle's own fit,
    projection and encoding: host nodes per second, one thread, for scale
    beside the GPU build (the work per node grows slowly with N)."""
    from oracle import fit as ofit
    from oracle import graph as og
    from oracle import lvq as olvq

    Xs = X[:n]
    P = ofit.fit_id(ofit.second_moment(Xs), wl.d)
    Y = ofit.project(Xs, P).astype(np.float32)
    mu = Y.astype(np.float64).mean(axis=0).astype(np.float32)
    codes, delta, lo = olvq.encode(Y, mu, wl.bits)
    prim = og.Primaries(codes, delta, lo)
    order = np.random.default_rng(wl.seed_data + 17).permutation(n).astype(np.uint32)
    t = time.time()
    og.build(prim, order, int(order[0]), wl.R, bL, wl.graph_alphas, max(1, n // 50))
    sec = time.time() - t
    return {"kind": "oracle", "nodes": n, "s": sec, "nodes_per_s": n / sec, "cores": 1,
            "sample": f"first {n} database vectors, oracle fit / projection / LVQ encoding"}


def fit_report(lv, wl, n_s=100_000, m_test=1000, k=10):
    """Projection fits of Section 2 on one workload, host float64: second
    moments of n_s database vectors (the first n_s rows of the seeded
    generator, a uniform sample) and of the learning queries, then LeanVec-ID
    (top-d eigenvectors of K_X), eigenvector search (Algorithm 2), Frank-Wolfe
    (Algorithm 1) from its default start (the eigenvectors of K_Q/m + K_X/n),
    from zero, and from the eigenvector search's result.  Each is timed
    in the library and in the oracle on the same moments; reported with its
    loss (Problem leanvec_efficient, normalised moments) and the 10-recall@10
    of exact search with <A q, B x> over the n_s vectors for m_test test
    queries (the paper compares the fits by loss and brute-force accuracy)."""
    from oracle import fit as ofit
    from synth import gen

    t0 = time.time()
    mix = gen.mixture(wl)
    X = gen.database(wl.scaled(N=n_s), mix)
    Ql = gen.queries(wl, "learn", mix=mix)
    Qt = gen.queries(wl, "test", m=m_test, mix=mix)
    log(f"fit data: {X.shape} database sample, {Ql.shape} learning queries "
        f"in {time.time() - t0:.1f}s")
    D, d, m = wl.D, wl.d, len(Ql)

    def timed(fn):
        t = time.time()
        r = fn()
        return r, time.time() - t

    KX = np.zeros((D, D))
    KQ = np.zeros((D, D))
    _, t_kx = timed(lambda: lv.lv_second_moment(X, KX))
    _, t_kq = timed(lambda: lv.lv_second_moment(Ql, KQ))
    KXo, t_kxo = timed(lambda: ofit.second_moment(X))
    KQo, t_kqo = timed(lambda: ofit.second_moment(Ql))
    moments = {"lib_s": t_kx + t_kq, "oracle_s": t_kxo + t_kqo,
               "max_rel_diff": float(max(np.abs(KX - KXo).max() / np.abs(KXo).max(),
                                         np.abs(KQ - KQo).max() / np.abs(KQo).max()))}

    import torch

    def recall(A, B):
        return reduced_recall(torch, Qt, X, {"f": (A, B)}, k)["f"]

    def loss(A, B):
        return lv.lv_ood_loss(KQ, m, KX, n_s, A, B)

    rows = {}
    P, t = timed(lambda: lv.lv_fit_id(KX, d))
    Po, to = timed(lambda: ofit.fit_id(KXo, d))
    rows["id"] = {"lib_s": t, "oracle_s": to, "loss": loss(P, P), "recall": recall(P, P),
                  "max_abs_diff_vs_oracle": float(np.abs(P - Po).max())}
    (P, beta), t = timed(lambda: lv.lv_fit_es(KQ, m, KX, n_s, d))
    (Po, beta_o), to = timed(lambda: ofit.eigsearch(KQo, m, KXo, n_s, d))
    rows["es"] = {"lib_s": t, "oracle_s": to, "beta": beta, "beta_oracle": beta_o,
                  "loss": loss(P, P), "loss_oracle": loss(Po, Po), "recall": recall(P, P)}
    P_es, Po_es = P, Po
    for name, init in (("fw", lv.LV_FW_INIT_ES), ("fw_from_zero", lv.LV_FW_INIT_ZERO),
                       ("es_then_fw", lv.LV_FW_INIT_GIVEN)):
        given = init == lv.LV_FW_INIT_GIVEN
        (A, B, info), t = timed(lambda: lv.lv_fit_ood(
            KQ, m, KX, n_s, d, init=init, A0=P_es if given else None,
            B0=P_es if given else None))
        (Ao, Bo, rep), to = timed(lambda: ofit.frank_wolfe(
            KQo, m, KXo, n_s, d, init="zero" if init == lv.LV_FW_INIT_ZERO else "es",
            A0=Po_es if given else None, B0=Po_es if given else None))
        rows[name] = {"lib_s": t, "oracle_s": to, "iters": info["iters"],
                      "iters_oracle": rep.iters, "converged": info["converged"],
                      "loss": loss(A, B), "loss_oracle": loss(Ao, Bo), "recall": recall(A, B)}
    for r in rows.values():
        log("fit " + ", ".join(f"{k_}={v:.4g}" if isinstance(v, float) else f"{k_}={v}"
                               for k_, v in r.items()))
    return {"fit": wl.name, "D": D, "d": d, "database_sample": n_s, "learning_queries": m,
            "test_queries": m_test, "k": k, "threads": int(os.environ.get("OMP_NUM_THREADS")
                                                          or os.cpu_count()),
            "timing": "host wall seconds (library: C++ float64, OpenMP; oracle: numpy/scipy)",
            "second_moments": moments, "fits": rows,
            "recall_full_dimension": 1.0}


def multi_report(lv, torch, args, n_sub=64, pool=4096, learn=4096, n_req=1024,
                 capacity=65536, target=0.90, L_max=512, in_flight=2):
    """The multi-index workload at full size.  Per sub-index s (sizes
    log-uniform in [1e4, 5e5], the id-1m-768 distribution with data seed
    4000 + s): LeanVec-ID fit on up to 100,000 vectors (host float64),
    projection and LVQ-8 encoding on the GPU, float16 secondaries, graph by
    lv_graph_build (R = 64, window R, two passes at alpha = 1), a pool of
    4,096 test and 4,096 learning queries with exact top-100 ids.  Windows L
    per (sub-index, k) from lv_autotune_window on the learning queries; the
    request stream (seed 401) is packed greedily into steps of at most
    65,536 queries; the steps run back to back, two in flight, queries
    resident.  Reported: whole-stream QPS (batched), the same requests as
    one plain search per request, and k-recall@k against the exact ids."""
    from dataclasses import replace

    from synth import gen
    from synth import graph as sgraph

    dev = torch.device("cuda:0")
    base = gen.WORKLOADS["id-1m-768"]
    sizes = gen.subindex_sizes(n_sub)
    subs, keep = [], []
    t0 = time.time()
    build_s = 0.0
    for s_ in range(n_sub):
        wl = replace(base, name=f"multi{s_}", N=int(sizes[s_]), m_test=pool, m_learn=learn,
                     seed_data=4000 + s_, seed_test=4100 + s_, seed_learn=4200 + s_)
        mix = gen.mixture(wl)
        X = gen.database(wl, mix)
        Q = gen.queries(wl, "test", mix=mix)
        Ql = gen.queries(wl, "learn", mix=mix)
        ns = min(wl.N, 100_000)
        K = np.zeros((wl.D, wl.D))
        ssum = np.zeros(wl.D)
        lv.lv_second_moment(X[:ns], K, ssum)
        P = lv.lv_fit_id(K, wl.d)
        mu = lv.lv_mean_reduced(P, ssum, ns)
        Xd = torch.from_numpy(X).to(dev)
        Pb = torch.from_numpy(lv.lv_to_bf16(P).view(np.int16)).to(dev)
        mud = torch.from_numpy(mu).to(dev)
        Y = torch.empty((wl.N, wl.d), dtype=torch.float32, device=dev)
        lv.lv_project(Xd, Pb, Y)
        rec = torch.empty((wl.N, lv.lv_record_stride(wl.d, wl.bits)), dtype=torch.uint8,
                          device=dev)
        lv.lv_lvq_encode(Y, mud, wl.bits, rec)
        sec = torch.empty((wl.N, wl.D), dtype=torch.float16, device=dev)
        lv.lv_to_f16(Xd, sec)
        del Y
        entry = sgraph.medoid(X)
        order = np.random.default_rng(wl.seed_data + 17).permutation(wl.N).astype(np.uint32)
        adjd = torch.empty((wl.N, wl.R), dtype=torch.int32, device=dev)
        bp = lv.build_params(wl.R, wl.R, wl.graph_alphas, max(1, wl.N // 50))
        torch.cuda.synchronize()
        tb = time.time()
        lv.lv_graph_build(rec, wl.N, wl.d, wl.bits, order, entry, bp, adjd)
        torch.cuda.synchronize()
        build_s += time.time() - tb
        truth = ground_truth_gpu(torch, Xd, Q, 100)
        truth_l = ground_truth_gpu(torch, Xd, Ql, 100).astype(np.uint32)
        del Xd
        ix = lv.Index(rec, mud, sec, adjd, entry, wl.bits, wl.d, A_bf16=Pb)
        keep.append((rec, mud, sec, adjd, Pb))
        subs.append(dict(N=wl.N, Q=Q, Ql=Ql, truth=truth, truth_l=truth_l, ix=ix))
    n_total = int(sum(d_["N"] for d_ in subs))
    log(f"multi: {n_sub} sub-indexes, {n_total} vectors ready in {time.time() - t0:.1f}s "
        f"(graph builds {build_s:.1f}s)")

    multi = lv.Multi([d_["ix"] for d_ in subs])
    sub, cnt, kk, off = gen.request_stream(n_req, n_sub, pool)
    t1 = time.time()
    Lsk = {}
    for s_, k_ in sorted(set(zip(sub.tolist(), kk.tolist()))):
        Qld = torch.from_numpy(subs[s_]["Ql"]).to(dev)
        Lsk[(s_, k_)], _ = lv.lv_autotune_window(multi, s_, Qld, subs[s_]["truth_l"], k_,
                                                 target, L_max)
    tune_s = time.time() - t1
    log(f"multi: {len(Lsk)} windows autotuned in {tune_s:.1f}s "
        f"(L from {min(Lsk.values())} to {max(Lsk.values())})")

    steps, curr, nq = [], [], 0
    for i in range(n_req):
        if curr and nq + cnt[i] > capacity:
            steps.append(curr)
            curr, nq = [], 0
        curr.append(i)
        nq += int(cnt[i])
    steps.append(curr)
    staged = []
    for st in steps:
        reqs, Qs = [], []
        for i in st:
            s_, k_ = int(sub[i]), int(kk[i])
            rows = (int(off[i]) + np.arange(int(cnt[i]))) % pool
            Qs.append(subs[s_]["Q"][rows])
            reqs.append((s_, k_, Lsk[(s_, k_)], int(cnt[i])))
        nout = sum(k_ * c_ for _, k_, _, c_ in reqs)
        staged.append(dict(reqs=reqs, rows=[(int(off[i]) + np.arange(int(cnt[i]))) % pool
                                            for i in st],
                           Q=torch.from_numpy(np.concatenate(Qs)).to(dev),
                           ids=torch.empty((nout,), dtype=torch.int32, device=dev),
                           sc=torch.empty((nout,), dtype=torch.float32, device=dev)))
    m_total = int(cnt.sum())
    max_req = max(len(st) for st in steps)
    batch = lv.Batch(multi, max_requests=max_req, max_queries=capacity,
                     max_L=max(Lsk.values()), expand=args.expand)
    stream = torch.cuda.current_stream()
    strs = [stream] + [torch.cuda.Stream() for _ in range(in_flight - 1)]

    def run_stream():
        for s_ in strs[1:]:
            s_.wait_stream(stream)
        for j, stg in enumerate(staged):
            batch.step(stg["reqs"], stg["Q"], stg["ids"], stg["sc"], stream=strs[j % in_flight])
        for s_ in strs[1:]:
            stream.wait_stream(s_)

    run_stream()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    e0.record(stream)
    for _ in range(reps):
        run_stream()
    e1.record(stream)
    torch.cuda.synchronize()
    batched_ms = e0.elapsed_time(e1) / reps

    # recall (k-recall@k per request, pooled) and the plain search of the same requests
    hits = total = 0
    plain_ids = []
    for stg in staged:
        o0 = 0
        for (s_, k_, L_, c_), rows in zip(stg["reqs"], stg["rows"]):
            got = stg["ids"][o0:o0 + c_ * k_].view(c_, k_).cpu().numpy().view(np.uint32)
            tr = subs[s_]["truth"][rows, :k_]
            hits += sum(len(set(a) & set(b)) for a, b in zip(got.tolist(), tr.tolist()))
            total += c_ * k_
            o0 += c_ * k_
    ws = torch.empty(lv.lv_search_workspace_size(subs[0]["ix"], capacity), dtype=torch.uint8,
                     device=dev)
    pouts = [(torch.empty((c_, k_), dtype=torch.int32, device=dev),
              torch.empty((c_, k_), dtype=torch.float32, device=dev))
             for stg in staged for (_, k_, _, c_) in stg["reqs"]]

    def run_plain():
        j = 0
        for stg in staged:
            q0 = 0
            for (s_, k_, L_, c_) in stg["reqs"]:
                lv.lv_search(subs[s_]["ix"], stg["Q"][q0:q0 + c_], k_, L_, pouts[j][0],
                             pouts[j][1], None, ws=ws, expand=args.expand)
                q0 += c_
                j += 1

    run_plain()
    torch.cuda.synchronize()
    e0.record(stream)
    run_plain()
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1)
    j = 0
    same = True
    for stg in staged:
        o0 = 0
        for (_, k_, _, c_) in stg["reqs"]:
            same &= bool(torch.equal(stg["ids"][o0:o0 + c_ * k_].view(c_, k_), pouts[j][0]))
            o0 += c_ * k_
            j += 1
    batch.close()
    multi.close()
    for d_ in subs:
        d_["ix"].close()
    qps = m_total / (batched_ms / 1e3)
    log(f"multi: {len(steps)} steps, {m_total} queries: batched {qps:.0f} QPS, plain "
        f"{m_total / (plain_ms / 1e3):.0f} QPS, recall {hits / total:.4f}")
    return {"multi": "id-1m-768 distribution, 64 sub-indexes", "sub_indexes": n_sub,
            "vectors": n_total, "D": base.D, "d": base.d, "requests": n_req,
            "steps": len(steps), "queries": m_total, "capacity": capacity,
            "expand": max(1, args.expand), "in_flight": in_flight,
            "windows": {"min": min(Lsk.values()), "max": max(Lsk.values()),
                        "median": float(np.median(list(Lsk.values()))), "count": len(Lsk)},
            "batched": {"qps": qps, "ms_per_stream": batched_ms, "reps": reps},
            "plain": {"qps": m_total / (plain_ms / 1e3), "ms_per_stream": plain_ms},
            "batched_over_plain": plain_ms / batched_ms,
            "batched_equals_plain": same, "recall": hits / total, "target": target,
            "prepare_s": time.time() - t0, "graph_build_s": build_s, "autotune_s": tune_s}


def reduced_recall(torch, Qt, X, fits, k=10):
    """10-recall@10 of exact search with <A q, B x> over the rows of X, for
    each (A, B) of fits, against the exact top k of <q, x> (host float64;
    torch's top-k only for speed)."""
    def top_k(Qm, Xm):
        Xt = torch.from_numpy(np.ascontiguousarray(Xm, np.float64))
        out = []
        for i in range(0, len(Qm), 100):
            S = torch.from_numpy(np.ascontiguousarray(Qm[i:i + 100], np.float64)) @ Xt.T
            out.append(torch.topk(S, k, dim=1).indices.numpy())
        return np.concatenate(out)

    truth = top_k(Qt, X)
    res = {}
    for name, (A, B) in fits.items():
        got = top_k(Qt.astype(np.float64) @ A.T, X.astype(np.float64) @ B.T)
        res[name] = float(np.mean([len(set(g) & set(t)) / k for g, t in zip(got, truth)]))
    return res


def refine_report(lv, torch, wl, steps, n_s=100_000, m_test=1000, bq=1024, bx=4096):
    """Differentiable refinement (the sampled-pair + trace loss, Adam with the
    projection onto the spectral-norm ball after each step) from the
    LeanVec-ID fit, against the OOD fits (Frank-Wolfe, eigenvector search) on
    the loss of Problem leanvec_efficient and on reduced-space recall.
    Database: the first n_s vectors of the workload's generator (a uniform
    sample); learning queries: the workload's; blocks of bq learning queries
    and bx database vectors drawn per step (seed 506)."""
    from paper_2312_16335_amd.autograd import refine
    from synth import gen

    t0 = time.time()
    mix = gen.mixture(wl)
    X = gen.database(wl.scaled(N=n_s), mix)
    Ql = gen.queries(wl, "learn", mix=mix)
    Qt = gen.queries(wl, "test", m=m_test, mix=mix)
    D, d, m = wl.D, wl.d, len(Ql)
    log(f"refine data: {X.shape} database sample, {Ql.shape} learning queries "
        f"in {time.time() - t0:.1f}s")
    KX = np.zeros((D, D))
    KQ = np.zeros((D, D))
    lv.lv_second_moment(X, KX)
    lv.lv_second_moment(Ql, KQ)
    KQn, KXn = KQ / m, KX / n_s
    fits = {}
    P = lv.lv_fit_id(KX, d)
    fits["id"] = (P, P)
    t = time.time()
    A, B, info = lv.lv_fit_ood(KQ, m, KX, n_s, d)
    t_fw = time.time() - t
    fits["fw"] = (A, B)
    Pe, beta = lv.lv_fit_es(KQ, m, KX, n_s, d)
    fits["es"] = (Pe, Pe)

    dev = torch.device("cuda:0")
    Qd = torch.from_numpy(Ql).to(dev)
    Xd = torch.from_numpy(X).to(dev)
    KQd = torch.from_numpy(KQn.astype(np.float32)).to(dev)
    KXd = torch.from_numpy(KXn.astype(np.float32)).to(dev)
    tc = float(np.trace(KQn @ KXn))
    rng = np.random.default_rng(506)

    def sample_block(step):
        qi = torch.from_numpy(np.sort(rng.choice(m, bq, replace=False))).to(dev)
        xi = torch.from_numpy(np.sort(rng.choice(n_s, bx, replace=False))).to(dev)
        return Qd.index_select(0, qi).contiguous(), Xd.index_select(0, xi).contiguous()

    trace = []

    def cb(step, loss):
        if step == 1 or step % 100 == 0:
            trace.append((step, [float(v) for v in loss.cpu()]))

    torch.cuda.synchronize()
    t = time.time()
    Ar, Br = refine(P, P, sample_block, steps, lr=1e-3, KQn=KQd, KXn=KXd, trace_const=tc,
                    lam=1.0, callback=cb)
    torch.cuda.synchronize()
    t_ref = time.time() - t
    fits["refined_from_id"] = (Ar, Br)
    rec = reduced_recall(torch, Qt, X, fits)
    rows = {name: {"loss": lv.lv_ood_loss(KQ, m, KX, n_s, A_, B_), "recall": rec[name]}
            for name, (A_, B_) in fits.items()}
    for name, r in rows.items():
        log(f"refine {name}: loss {r['loss']:.4e}, recall {r['recall']:.4f}")
    return {"refine": wl.name, "D": D, "d": d, "database_sample": n_s, "learning_queries": m,
            "test_queries": m_test, "b_q": bq, "b_x": bx, "steps": steps, "lr": 1e-3,
            "lam": 1.0, "refine_wall_s": t_ref, "refine_ms_per_step": 1e3 * t_ref / steps,
            "per_step": "block gather, forward + backward kernels, two Adam kernels, host "
                        "float64 spectral clip of A and B (device-host copies included)",
            "fw_s": t_fw, "fw_iters": info["iters"], "es_beta": beta,
            "loss_trace": [{"step": s_, "total": v[0], "pairs": v[1], "trace": v[2]}
                           for s_, v in trace],
            "fits": rows}


MFMA_PEAK_TFLOPS = 2500.0  # dense bf16 on MI355X


def mfma_report(lv, torch, reps=10):
    """Matrix-core kernels on synthetic operands of the workloads' shapes: the
    database projection (1M x 768 -> 160) and the query projection (10,000
    queries), one refinement step (forward + backward, b_q = 1024, b_x = 4096,
    D = 768, d = 128, with the trace term) and one 8192^3 GEMM (float32
    operands rounded when staged, and bfloat16 operands in memory).  Flops are the
    products' own (2 M N K each); bytes are the projections' operands and outputs."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(5)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def entry(ms, flops, nbytes=None):
        e = {"ms": ms, "tflops": flops / (ms / 1e3) / 1e12}
        e["frac_bf16_peak"] = e["tflops"] / MFMA_PEAK_TFLOPS
        if nbytes is not None:
            e["GBs"] = nbytes / (ms / 1e3) / 1e9
            e["frac_hbm_peak"] = e["GBs"] / HBM_PEAK_GBS
        return e

    out = {"peaks": {"bf16_tflops": MFMA_PEAK_TFLOPS, "hbm_GBs": HBM_PEAK_GBS}}
    D, d = 768, 160
    M = torch.randn((d, D), device=dev, generator=g).to(torch.bfloat16).view(torch.int16)
    for name, rows in (("database_projection", 1_000_000), ("query_projection", 10_000)):
        V = torch.randn((rows, D), device=dev, generator=g)
        Y = torch.empty((rows, d), device=dev)
        ms = timed(lambda: lv.lv_project(V, M, Y))
        out[name] = dict(rows=rows, D=D, d=d, **entry(ms, 2.0 * rows * D * d,
                                                         4.0 * rows * (D + d) + 2.0 * d * D))
        if rows == 1_000_000:
            # one pass: LVQ-8 records (192-byte stride) straight from the products,
            # against the projection followed by the encoder
            mu = torch.randn(d, device=dev, generator=g) * 0.1
            rec = torch.empty((rows, 192), dtype=torch.uint8, device=dev)
            ms1 = timed(lambda: lv.lv_project_encode(V, M, mu, 8, rec))
            ms_enc = timed(lambda: lv.lv_lvq_encode(Y, mu, 8, rec))
            out["database_projection_encode"] = dict(
                rows=rows, D=D, d=d, bits=8, record_stride=192,
                two_kernels_ms=ms + ms_enc, encode_kernel_ms=ms_enc,
                **entry(ms1, 2.0 * rows * D * d, 4.0 * rows * D + 2.0 * d * D + 168.0 * rows))
            del mu, rec
        del V, Y
    bq, bx, D2, d2 = 1024, 4096, 768, 128
    A = torch.randn((d2, D2), device=dev, generator=g) * 0.03
    B = torch.randn((d2, D2), device=dev, generator=g) * 0.03
    Qb = torch.randn((bq, D2), device=dev, generator=g)
    Xb = torch.randn((bx, D2), device=dev, generator=g)
    KQ = torch.eye(D2, device=dev)
    KX = torch.eye(D2, device=dev)
    loss = torch.zeros(3, device=dev)
    dA, dB = torch.empty_like(A), torch.empty_like(B)
    ws = torch.empty(lv.lv_projloss_workspace_size(bq, bx, D2, d2), dtype=torch.uint8,
                     device=dev)

    def step():
        lv.lv_projloss_fwd(A, B, Qb, Xb, loss, ws, KQ, KX)
        lv.lv_projloss_bwd(A, B, Qb, Xb, dA, dB, ws, KQ, KX)

    pair_f = 2.0 * (bq * d2 * D2 + bx * d2 * D2 + bq * bx * D2 + bq * bx * d2)
    pair_b = 2.0 * (2 * bq * bx * d2 + d2 * D2 * bq + d2 * D2 * bx)
    trace = 2.0 * (2 * d2 * D2 * D2 + 2 * d2 * d2 * D2) * 2
    out["refinement_step"] = dict(b_q=bq, b_x=bx, D=D2, d=d2,
                                  **entry(timed(step), pair_f + pair_b + trace))
    # the same step captured once in a HIP graph (its second stream included)
    # and replayed: the host's launch work leaves the loop
    gstream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gstream):
        step()
    torch.cuda.synchronize()
    out["refinement_step_graph"] = dict(b_q=bq, b_x=bx, D=D2, d=d2,
                                        **entry(timed(graph.replay), pair_f + pair_b + trace))
    del graph
    # the float64 oracle beside them (host cores): projection + LVQ-8 encoding of
    # a 20,000-row sample, and one refinement step (loss and gradients)
    from oracle import fit as ofit
    from oracle import lvq as olvq
    from oracle import projloss as oproj

    rows_o = 20_000
    Vo = torch.randn((rows_o, D), generator=torch.Generator().manual_seed(5)).numpy()
    Mo = np.asarray(M.view(torch.bfloat16).float().cpu().numpy(), np.float64)
    muo = np.zeros(d, np.float32)
    t = time.perf_counter()
    Yo = ofit.project(Vo, Mo).astype(np.float32)
    olvq.encode(Yo, muo, 8)
    dt = time.perf_counter() - t
    out["database_projection_encode"]["oracle"] = {
        "rows_per_s": rows_o / dt, "sample": f"{rows_o} rows, float64 numpy on the host",
        "gpu_rows_per_s": 1_000_000 / (out["database_projection_encode"]["ms"] / 1e3)}
    Ah, Bh, Qh, Xh = (x.double().cpu().numpy() for x in (A, B, Qb, Xb))
    KQh, KXh = KQ.double().cpu().numpy(), KX.double().cpu().numpy()
    t = time.perf_counter()
    oproj.loss(Ah, Bh, Qh, Xh, KQh, KXh)
    oproj.grads(Ah, Bh, Qh, Xh, KQh, KXh)
    out["refinement_step"]["oracle"] = {"ms": (time.perf_counter() - t) * 1e3,
                                        "sample": "one step at the same block sizes, float64 "
                                                  "numpy on the host (its BLAS threads)"}
    n = 8192
    Ga = torch.randn((n, n), device=dev, generator=g)
    Gb = torch.randn((n, n), device=dev, generator=g)
    Gc = torch.empty((n, n), device=dev)
    ms = timed(lambda: lv.lv_gemm(Ga, Gb, Gc, n, n, n))
    out["gemm_8192"] = entry(ms, 2.0 * n ** 3)
    # the same product with the operands held as bfloat16 (converted once,
    # outside the timed region): half the bytes staged per flop
    Ha, Hb = Ga.to(torch.bfloat16), Gb.to(torch.bfloat16)
    del Ga, Gb
    ms = timed(lambda: lv.lv_gemm_bf16(Ha, Hb, Gc, n, n, n))
    out["gemm_8192_bf16_operands"] = entry(ms, 2.0 * n ** 3)
    return out


def ground_truth_gpu(torch, Xd, Q, k):
    """Exact top-k ids by <q, x> (float32 candidates, float64 re-scoring)."""
    dev = Xd.device
    m = len(Q)
    cand_k = max(64, k + 28)
    Qd = torch.from_numpy(Q).to(dev)
    best_s = torch.full((m, 0), -math.inf, device=dev)
    best_i = torch.zeros((m, 0), dtype=torch.int64, device=dev)
    for lo in range(0, Xd.shape[0], 1 << 18):
        S = Qd @ Xd[lo:lo + (1 << 18)].T
        s, i = torch.topk(S, min(cand_k, S.shape[1]), dim=1)
        best_s = torch.cat([best_s, s], 1)
        best_i = torch.cat([best_i, i + lo], 1)
        s, j = torch.topk(best_s, min(cand_k, best_s.shape[1]), dim=1)
        best_s, best_i = s, torch.gather(best_i, 1, j)
    # float64 re-score of the candidates, ties to the smaller id
    cand = best_i
    Xc = Xd[cand.reshape(-1)].reshape(m, cand.shape[1], -1).double()
    s64 = torch.einsum("mkd,md->mk", Xc, Qd.double())
    s64 = s64.cpu().numpy()
    ci = cand.cpu().numpy()
    out = np.empty((m, k), dtype=np.int64)
    for r in range(m):
        order = np.lexsort((ci[r], -s64[r]))[:k]
        out[r] = ci[r][order]
    return out


def recall(ids, truth, k):
    hit = 0
    for a, b in zip(ids[:, :k], truth[:, :k]):
        hit += len(set(a.tolist()) & set(b.tolist()))
    return hit / (k * len(truth))


def profile_traffic(kernel_src, L, slots, launch, expand):
    """HBM bytes per launch from committed counter runs, if the kernel is unchanged and
    counters were taken in this configuration (window, visited-set size, launch, expand)."""
    p = os.path.join(ROOT, "profiles", "batched_kernel_id-1m-768_counters.md")
    if not os.path.exists(p):
        return None
    sha = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    want = {"window_L": str(L), "visited_slots": str(slots), "launch": launch,
            "expand": str(expand)}
    src_ok = False
    for line in open(p):
        if line.startswith("- kernel_source_sha256:"):
            src_ok = line.split(":", 1)[1].strip() == sha
        elif line.startswith("- traffic:") and src_ok:
            kv = dict(f.split("=", 1) for f in line.split(":", 1)[1].split())
            if all(kv.get(k_) == v_ for k_, v_ in want.items()):
                try:
                    return float(kv["hbm_bytes_per_launch"])
                except (KeyError, ValueError):
                    return None
    return None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on exactly one GPU; "
                                   "--gpus %d is not supported (query or database sharding "
                                   "across GPUs is a design only, not built)" % args.gpus}))
        sys.exit(2)
    import torch

    import paper_2312_16335_amd as lv
    from synth import gen

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.calibrate_copy:
        # 1 GiB read + 1 GiB written per copy, three copies
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read_per_copy": 1 << 30,
                          "bytes_written_per_copy": 1 << 30, "copies": 3}))
        return
    lv.load()
    if args.mfma:
        print(json.dumps(mfma_report(lv, torch)))
        return
    if args.fit:
        print(json.dumps(fit_report(lv, gen.WORKLOADS[args.workload or "ood-1m-512"])))
        return
    if args.multi:
        print(json.dumps(multi_report(lv, torch, args)))
        return
    if args.refine:
        print(json.dumps(refine_report(lv, torch, gen.WORKLOADS[args.workload or "ood-1m-768"],
                                       args.refine)))
        return
    dev = torch.device("cuda:0")
    wl = gen.WORKLOADS[args.workload or "id-1m-768"]
    if args.n:
        wl = wl.scaled(N=args.n)
    if args.bits:
        wl = replace(wl, bits=args.bits)
    k = wl.k
    t0 = time.time()
    mix = gen.mixture(wl)
    X = gen.database(wl, mix)
    Q = gen.queries(wl, "test", mix=mix)
    log(f"data {X.shape} queries {Q.shape} in {time.time() - t0:.1f}s")

    g = {}
    th = None
    if args.graph == "cpu":
        th = threading.Thread(target=build_graph_cached, args=(wl, X, g))
        th.start()

    # ---- index side: fit (host float64), projection + encoding (GPU)
    rng = np.random.default_rng(7)
    ns = min(wl.N, 100_000)  # uniform subsample for the second moment (Section 2.2)
    sub = np.sort(rng.choice(wl.N, size=ns, replace=False))
    Xs = np.ascontiguousarray(X[sub])
    K = np.zeros((wl.D, wl.D))
    ssum = np.zeros(wl.D)
    lv.lv_second_moment(Xs, K, ssum)
    resid = args.sec == "resid"
    ood = wl.fit == "ood"
    if ood and resid:
        raise SystemExit("residual secondaries need A = B (LeanVec-ID)")
    fit_info = {"kind": "id (top-d eigenvectors of the database second moment)"}
    if ood:
        # LeanVec-OOD (Algorithm 1): queries projected with A, the database with B
        Ql = gen.queries(wl, "learn", mix=mix)
        KQ = np.zeros((wl.D, wl.D))
        lv.lv_second_moment(Ql, KQ)
        tf = time.time()
        Aq, P, info = lv.lv_fit_ood(KQ, len(Ql), K, ns, wl.d)
        fit_info = {"kind": "ood (Frank-Wolfe, Algorithm 1)", "iters": info["iters"],
                    "seconds": time.time() - tf, "learning_queries": len(Ql)}
        Pf = P
        Pqb = torch.from_numpy(lv.lv_to_bf16(Aq).view(np.int16)).to(dev)
    else:
        # residual secondaries: all D eigenvectors, the first d are the projection
        Pf = lv.lv_fit_id(K, wl.D if resid else wl.d)
        P = np.ascontiguousarray(Pf[:wl.d])
    mu = lv.lv_mean_reduced(P, ssum, ns)
    Pb = torch.from_numpy(lv.lv_to_bf16(P).view(np.int16)).to(dev)
    if not ood:
        Pqb = torch.from_numpy(lv.lv_to_bf16(Pf).view(np.int16)).to(dev) if resid else Pb
    mud = torch.from_numpy(mu).to(dev)
    Xd = torch.from_numpy(X).to(dev)
    stride = lv.lv_record_stride(wl.d, wl.bits)
    rec = torch.empty((wl.N, stride), dtype=torch.uint8, device=dev)
    Y = torch.empty((wl.N, wl.d), dtype=torch.float32, device=dev)
    smud = None
    if args.sec == "lvq8":
        # LVQ-8 secondaries centred on the sample mean of the database
        smud = torch.from_numpy((ssum / ns).astype(np.float32)).to(dev)
        sec = torch.empty((wl.N, lv.lv_secondary_row_bytes(wl.D, lv.LV_LVQ8)), dtype=torch.uint8,
                          device=dev)
    elif resid:
        sec = torch.empty((wl.N, wl.D - wl.d), dtype=torch.float16, device=dev)
    elif args.sec == "level2":
        sec = torch.empty((wl.N, lv.lv_secondary_row_bytes(wl.d, lv.LV_LVQ8_LEVEL2)),
                          dtype=torch.uint8, device=dev)
    else:
        sec = torch.empty((wl.N, wl.D), dtype=torch.float16, device=dev)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    if args.sec == "level2":  # the second level needs the reduced vectors themselves
        lv.lv_project(Xd, Pb, Y)
        lv.lv_lvq_encode(Y, mud, wl.bits, rec)
        ev1.record()
    else:  # records in one pass (the reduced vectors never go through memory)
        lv.lv_project_encode(Xd, Pb, mud, wl.bits, rec)
        ev1.record()
    if smud is not None:
        lv.lv_lvq_encode(Xd, smud, 8, sec)
    elif resid:
        Pp = torch.from_numpy(lv.lv_to_bf16(np.ascontiguousarray(Pf[wl.d:])).view(np.int16)).to(dev)
        Yr = torch.empty((wl.N, wl.D - wl.d), dtype=torch.float32, device=dev)
        lv.lv_project(Xd, Pp, Yr)
        lv.lv_to_f16(Yr, sec)
        del Yr, Pp
    elif args.sec == "level2":
        lv.lv_lvq_encode_level2(Y, mud, wl.bits, rec, sec)
    else:
        lv.lv_to_f16(Xd, sec)
    torch.cuda.synchronize()
    db_proj_ms = ev0.elapsed_time(ev1)
    truth = ground_truth_gpu(torch, Xd, Q, k)
    del Y
    Xd = None
    torch.cuda.empty_cache()
    log(f"fit + encode + ground truth done at {time.time() - t0:.1f}s")
    if th is not None:
        th.join()
        adj, entry = g["adj"], g["entry"]
        adjd = torch.from_numpy(adj.view(np.int32)).to(dev)
    else:
        adjd, entry = build_graph_gpu(lv, torch, wl, X, rec, args, g)
        adj = adjd.cpu().numpy().view(np.uint32)
        from synth import graph as sgraph

        g["reachable"] = float(sgraph.reachable(adj, entry).mean())
        st = g.get("stats") or {}
        if st:
            # construction-search bytes (per search: the node's record, its row,
            # the pool row written; per expansion a row; per scoring a record)
            cb = wl.d * wl.bits // 8 + 8
            bL = args.build_L or wl.R
            nb = (4 * wl.R * st["expansions"] + cb * st["scorings"]
                  + st["searches"] * (cb + 4 * wl.R + 4 * (bL + wl.R)))
            g["rates"] = {"nodes_per_s": wl.N / g["graph_s"],
                          "search_alg_bytes": nb,
                          "search_alg_GBs_over_whole_build": nb / g["graph_s"] / 1e9}
        if not args.no_cpu_baseline:
            g["oracle_sample"] = oracle_build_sample(wl, X, args.build_L or wl.R)
            log(f"oracle construction: {g['oracle_sample']['nodes']} nodes in "
                f"{g['oracle_sample']['s']:.1f}s")
    log(f"graph ready at {time.time() - t0:.1f}s (build {g['graph_s']:.1f}s)")
    index = lv.Index(rec, mud, sec, adjd, entry, wl.bits, wl.d, A_bf16=Pqb, sec_mu=smud,
                     residual=resid, level2=args.sec == "level2")

    # ---- request stream over the test queries (uneven batches)
    m = len(Q)
    sizes = []
    rs = np.random.Generator(np.random.PCG64(401))
    left = m
    while left > 0:
        b = int(min(left, rs.integers(1, 4097)))
        sizes.append(b)
        left -= b
    offs = np.concatenate([[0], np.cumsum(sizes)])
    Qd = torch.from_numpy(Q).to(dev)
    Qp = torch.empty((m, wl.D if resid else wl.d), dtype=torch.float32, device=dev)
    ids = torch.empty((m, k), dtype=torch.int32, device=dev)
    scores = torch.empty((m, k), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    knob_hs = [args.hash_slots]  # visited-set slots (result-neutral knob)

    def step(L, ev=None):
        """One pass over the request stream; optional per-kernel events."""
        for i, b in enumerate(sizes):
            lo, hi = int(offs[i]), int(offs[i + 1])
            if ev is not None:
                ev[0][i].record(stream)
            lv.lv_project(Qd[lo:hi], Pqb, Qp[lo:hi])
            if ev is not None:
                ev[1][i].record(stream)
            lv.lv_search_projected(index, Qd[lo:hi], Qp[lo:hi], k, L, ids[lo:hi],
                                   scores[lo:hi], hash_slots=knob_hs[0], expand=args.expand)
            if ev is not None:
                ev[2][i].record(stream)

    def measure(L, reps=3):
        step(L)
        torch.cuda.synchronize()
        best = math.inf
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            step(L)
            b.record()
            torch.cuda.synchronize()
            best = min(best, a.elapsed_time(b))
        got = ids.cpu().numpy().view(np.uint32).astype(np.int64)
        return recall(got, truth, k), m / (best / 1e3)

    sweep = {}
    if args.L:
        L_star = args.L
        sweep[L_star] = measure(L_star)
    else:
        for L in sorted(set(list(wl.L_list) + [k])):
            if L < k:
                continue
            sweep[L] = measure(L)
            log(f"L={L}: recall {sweep[L][0]:.4f}, {sweep[L][1]:.0f} QPS")
            if sweep[L][0] >= args.target:
                break
        reach = [L for L, (r, _) in sweep.items() if r >= args.target]
        if not reach:
            L = max(sweep)
            while L < 1024:
                L = min(1024, int(L * 1.5))
                sweep[L] = measure(L)
                log(f"L={L}: recall {sweep[L][0]:.4f}")
                if sweep[L][0] >= args.target:
                    break
            reach = [L for L, (r, _) in sweep.items() if r >= args.target]
        L_hi = min(reach) if reach else max(sweep)
        lower = [L for L in sweep if L < L_hi]
        L_lo = max(lower) if lower else L_hi
        if not args.only_steps:
            # refine: smallest window in (L_lo, L_hi] reaching the target
            lo_, hi_ = L_lo, L_hi
            while hi_ - lo_ > 1:
                mid = (lo_ + hi_) // 2
                sweep[mid] = measure(mid)
                if sweep[mid][0] >= args.target:
                    hi_ = mid
                else:
                    lo_ = mid
            L_hi = hi_
        L_star = L_hi

    # interpolated QPS at exactly the target recall, in (recall, log QPS)
    pts = sorted(sweep.items())
    qps_interp = None
    for (La, (ra, qa)), (Lb, (rb, qb)) in zip(pts, pts[1:]):
        if ra < args.target <= rb and rb > ra:
            w = (args.target - ra) / (rb - ra)
            qps_interp = math.exp(math.log(qa) + w * (math.log(qb) - math.log(qa)))
    log(f"operating window L={L_star}")

    # ---- algorithmic bytes per query at L* from the debug counters (exact visited set)
    cnt = torch.zeros((m, 2), dtype=torch.int32, device=dev)
    lv.lv_search_projected(index, Qd, Qp, k, L_star, ids, scores, cnt, hash_slots=8192,
                           expand=args.expand)
    torch.cuda.synchronize()
    c = cnt.cpu().numpy().astype(np.float64)
    n_exp, n_dist = c[:, 0], c[:, 1]
    n_rr = np.minimum(L_star, n_dist)
    code_bytes = wl.d * wl.bits // 8
    # bytes of one secondary row: float16, LVQ-8 codes + delta + lo, residual float16, or
    # second-level codes + delta2 + lo2
    sec_row = (wl.D + 8 if smud is not None else 2 * (wl.D - wl.d) if resid else
               wl.d + 8 if args.sec == "level2" else 2 * wl.D)
    bytes_q = (4 * wl.D + n_exp * 4 * wl.R + n_dist * (code_bytes + 8) + n_rr * sec_row
               + 8 * k)
    alg_bytes_total = float(bytes_q.sum())

    # ---- batched persistent form (one captured step = the whole request stream)
    nreq = len(sizes)
    multi = lv.Multi([index])
    reqs = [(0, k, L_star, b) for b in sizes]
    ids_flat, scores_flat = ids.view(-1), scores.view(-1)
    if args.hash_slots:
        hs = args.hash_slots
        launch = lv.LV_LAUNCH_PERSISTENT if args.launch == "persistent" else lv.LV_LAUNCH_PER_QUERY
        how = "given"
    else:
        knobs, _ = lv.lv_autotune_knobs(multi, nreq, m, L_star, reqs, Qd, ids_flat, scores_flat,
                                        reps=6, expand=args.expand)
        hs, launch = knobs["hash_slots"], knobs["launch"]
        how = "chosen by the autotuner"
    launch_name = "persistent" if launch == lv.LV_LAUNCH_PERSISTENT else "per_query"
    knob_hs[0] = hs
    batch = lv.Batch(multi, max_requests=nreq, max_queries=m, max_L=L_star, hash_slots=hs,
                     launch=launch, expand=args.expand)
    log(f"batched step captured (visited-set slots {hs}, {launch_name} launch, {how})")

    def step_batched(ev=None):
        batch.step(reqs, Qd, ids_flat, scores_flat, events=ev)

    def timed(fn, evs):
        for _ in range(args.warmup):
            fn(None) if evs else fn()
        torch.cuda.synchronize()
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        per = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        wall0 = time.perf_counter()
        t_start.record()
        for sidx in range(args.steps):
            per[sidx][0].record(stream)
            if evs:
                fn(evs[sidx])
            else:
                fn()
            per[sidx][1].record(stream)
        t_end.record()
        torch.cuda.synchronize()
        return t_start.elapsed_time(t_end), time.perf_counter() - wall0, per

    def step_stats(per):
        t = sorted(a_.elapsed_time(b_) for a_, b_ in per)
        return {"best_ms": t[0], "median_ms": float(np.median(t)), "worst_ms": t[-1]}

    # plain: one projection + one traversal launch per request, events per kernel
    evs = [[[torch.cuda.Event(enable_timing=True) for _ in range(nreq)] for _ in range(3)]
           for _ in range(args.steps)]
    plain_ms, plain_wall, plain_per = timed(lambda e: step(L_star, e), evs)
    got = ids.cpu().numpy().view(np.uint32).astype(np.int64)
    rec_plain = recall(got, truth, k)
    proj_ms = sum(evs[s_][0][i].elapsed_time(evs[s_][1][i]) for s_ in range(args.steps)
                  for i in range(nreq))
    beam_ms = sum(evs[s_][1][i].elapsed_time(evs[s_][2][i]) for s_ in range(args.steps)
                  for i in range(nreq))
    plain_qps = m * args.steps / (plain_ms / 1e3)

    # batched: two graph launches per step (request-table copy + grouped projection;
    # counter reset + persistent traversal), events around the traversal graph
    ids.fill_(-1)
    trav = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(args.steps)]
    total_ms, wall, batched_per = timed(step_batched, trav)
    got = ids.cpu().numpy().view(np.uint32).astype(np.int64)
    rec_star = recall(got, truth, k)
    serial_qps = m * args.steps / (total_ms / 1e3)
    kernel_ms = sum(a_.elapsed_time(b_) for a_, b_ in trav) / args.steps

    # batched, pipelined: consecutive steps rotate over two streams (and two
    # output buffers), so a step's wavefronts start while earlier steps' slowest
    # queries finish; the timed region still spans exactly K whole steps
    IN_FLIGHT = 2  # steps in flight (the batch rotates four state sets: 2 divides 4)
    strs = [stream] + [torch.cuda.Stream() for _ in range(IN_FLIGHT - 1)]
    outs = [(ids_flat, scores_flat)] + [(torch.empty_like(ids_flat), torch.empty_like(scores_flat))
                                        for _ in range(IN_FLIGHT - 1)]

    def run_pipelined(n, evs=None, b=None):
        b = batch if b is None else b
        for i_ in range(n):
            o_ = outs[i_ % IN_FLIGHT]
            b.step(reqs, Qd, o_[0], o_[1], stream=strs[i_ % IN_FLIGHT],
                   events=None if evs is None else evs[i_])

    for s_ in strs[1:]:
        s_.wait_stream(stream)
    run_pipelined(max(IN_FLIGHT, args.warmup))
    for s_ in strs[1:]:
        stream.wait_stream(s_)
    torch.cuda.synchronize()
    for o_ in outs:
        o_[0].fill_(-1)
    trav_p = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall_p0 = time.perf_counter()
    p0.record(stream)
    for s_ in strs[1:]:
        s_.wait_event(p0)
    run_pipelined(args.steps, trav_p)
    for s_ in strs[1:]:
        stream.wait_stream(s_)
    p1.record(stream)
    torch.cuda.synchronize()
    wall_p = time.perf_counter() - wall_p0
    total_p_ms = p0.elapsed_time(p1)
    qps = m * args.steps / (total_p_ms / 1e3)
    ms_per_step = total_p_ms / args.steps
    for o_ in outs[: min(IN_FLIGHT, args.steps)]:
        got_p = o_[0].view(m, k).cpu().numpy().view(np.uint32).astype(np.int64)
        assert np.array_equal(got_p, got), "pipelined steps differ from serial steps"
    # effective launch duration with several launches in flight: span of the K traversals / K
    span_ms = trav_p[0][0].elapsed_time(trav_p[-1][1])
    launch_eff_ms = span_ms / args.steps
    achieved = alg_bytes_total / (launch_eff_ms / 1e3) / 1e9
    achieved_serial = alg_bytes_total / (kernel_ms / 1e3) / 1e9
    beam_launch_ms = beam_ms / (args.steps * nreq)
    achieved_plain = (alg_bytes_total / nreq) / (beam_launch_ms / 1e3) / 1e9
    # the committed counter runs are of the id-1m-768 workload with float16 secondaries
    traffic = None
    if wl.name == "id-1m-768" and args.sec == "f16" and not args.n:
        traffic = profile_traffic(os.path.join(ROOT, "paper_2312_16335_amd", "csrc",
                                               "lv_search.hip"),
                                  L_star, hs, launch_name, max(1, args.expand))
    batch.close()

    # the other traversal at the same window, timed the same way and reported
    # beside `value`: one expansion per iteration (the paper's traversal) when
    # the main run expands several, three otherwise
    variant = None
    if not args.no_variant:
        other = 1 if args.expand > 1 else 3
        bv = lv.Batch(multi, max_requests=nreq, max_queries=m, max_L=L_star, hash_slots=hs,
                      launch=launch, expand=other)
        for s_ in strs[1:]:
            s_.wait_stream(stream)
        run_pipelined(max(IN_FLIGHT, args.warmup), b=bv)
        for s_ in strs[1:]:
            stream.wait_stream(s_)
        torch.cuda.synchronize()
        tv = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        v0, v1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        v0.record(stream)
        for s_ in strs[1:]:
            s_.wait_event(v0)
        run_pipelined(args.steps, tv, b=bv)
        for s_ in strs[1:]:
            stream.wait_stream(s_)
        v1.record(stream)
        torch.cuda.synchronize()
        vgot = outs[0][0].view(m, k).cpu().numpy().view(np.uint32).astype(np.int64)
        vms = v0.elapsed_time(v1)
        variant = {"expand": other, "L": L_star, "recall": recall(vgot, truth, k),
                   "qps": m * args.steps / (vms / 1e3), "ms_per_step": vms / args.steps,
                   "traversal_launch_ms": tv[0][0].elapsed_time(tv[-1][1]) / args.steps}
        bv.close()
        log(f"other traversal expand={other} at L={L_star}: recall {variant['recall']:.4f}, "
            f"{variant['qps']:.0f} QPS")
    multi.close()

    # reference: the plain path as one launch pair over all queries
    def single():
        lv.lv_project(Qd, Pqb, Qp)
        lv.lv_search_projected(index, Qd, Qp, k, L_star, ids, scores, hash_slots=hs,
                               expand=args.expand)

    single()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        single()
    e1.record()
    torch.cuda.synchronize()
    single_qps = m * 5 / (e0.elapsed_time(e1) / 1e3)
    small_batches = small_batch_report(lv, torch, index, Qd, Qp, k, L_star, hs,
                                       sorted({1, max(1, args.expand)}))

    # ---- CPU oracle on a bounded sample
    cpu = None
    if not args.no_cpu_baseline and args.sec == "f16":
        cpu = cpu_baseline(wl, X, Xs, Q, adj, entry, L_star, args.cpu_sample, truth,
                           max(1, args.expand), mix)
        if cpu["sample"].startswith("all") and abs(cpu["recall"] - rec_star) > 0.005:
            log(f"WARNING: GPU recall {rec_star:.4f} vs oracle {cpu['recall']:.4f}")

    ood = None
    if (not args.no_ood and wl.name == "id-1m-768" and not args.n and args.sec == "f16"
            and not args.bits):
        # the cross-modal workload as a compact sub-record (its own index)
        index.close()
        torch.cuda.empty_cache()
        ood = ood_report(lv, torch, args)
    mfma = None
    if (not args.no_mfma and wl.name == "id-1m-768" and not args.n and args.sec == "f16"
            and not args.bits):
        # the matrix-core kernels (database and query projections, one refinement
        # step of the differentiable projection, a large GEMM) as a sub-record
        torch.cuda.empty_cache()
        mfma = mfma_report(lv, torch)

    out = {
        "metric": ("QPS at 10-recall@10=0.90 (1M x 768, d=160), batched vs plain; HBM GB/s"
                   if wl.name == "id-1m-768" and not args.n else
                   f"QPS at 10-recall@10=0.90 ({wl.N} x {wl.D}, d={wl.d}), batched vs plain; "
                   f"HBM GB/s"),
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "N": wl.N, "D": wl.D, "d": wl.d, "lvq_bits": wl.bits,
                   "secondary": args.sec, "R": wl.R, "k": k, "queries": m, "L": L_star,
                   "requests": nreq, "mode": "batched, 2 steps in flight",
                   "visited_slots": hs, "launch": launch_name,
                   "expand": max(1, args.expand), "fit": fit_info},
        "recall_at_L": rec_star,
        "plain": {"qps": plain_qps, "recall": rec_plain, "ms_per_step": plain_ms / args.steps,
                  "traversal_kernel_GBs": achieved_plain,
                  "traversal_kernel_frac": achieved_plain / HBM_PEAK_GBS},
        "batched_over_plain": qps / plain_qps,
        "batched_serial": {"qps": serial_qps, "ms_per_step": total_ms / args.steps,
                           "step_ms": step_stats(batched_per), "traversal_launch_ms": kernel_ms,
                           "traversal_GBs": achieved_serial,
                           "traversal_frac": achieved_serial / HBM_PEAK_GBS,
                           "wall_s_timed": wall},
        "plain_step_ms": step_stats(plain_per),
        "plain_single_launch_qps": single_qps,
        "qps_interp_at_target": qps_interp,
        "sweep": {str(L): {"recall": r, "qps": q} for L, (r, q) in sorted(sweep.items())},
        "wall_s_timed": wall_p,
        "wall_s_timed_plain": plain_wall,
        "per_query": {"expansions": float(n_exp.mean()), "primary_scorings": float(n_dist.mean()),
                      "reranked": float(n_rr.mean()), "alg_bytes": float(bytes_q.mean())},
        "kernels_ms_per_step": {"query_projection": proj_ms / args.steps,
                                "traversal": beam_ms / args.steps},
        "roofline": {"bound": "hbm", "achieved": achieved_serial, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved_serial / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled)",
                     "alg_bytes_per_launch": alg_bytes_total, "launch_ms": kernel_ms,
                     "kernel": "batched_kernel (traversal + re-rank), one launch per step",
                     "traversal": ("%d expansions per iteration (throughput variant; the "
                                   "paper's one-at-a-time traversal is in traversal_compare)"
                                   % max(1, args.expand)) if args.expand > 1 else
                                  "one expansion per iteration (the paper's traversal)",
                     "launch_timing": "launch_ms: average duration of the K serial launches "
                                      "(one step after another), HIP events around each "
                                      "traversal graph on its launch stream",
                     "pipelined": {"launch_ms": launch_eff_ms, "achieved": achieved,
                                   "frac": achieved / HBM_PEAK_GBS,
                                   "how": "two steps in flight: (last traversal end - first "
                                          "traversal start) / K; the launches overlap, so "
                                          "this is the throughput per launch, not one "
                                          "launch's duration"}},
        "index_build": {"db_projection_encode_ms": db_proj_ms, "graph_build_s": g.get("graph_s"),
                        "graph": g.get("kind", "host builder, float16 vectors"),
                        "graph_build_threads": (None if args.graph == "gpu" else
                                                int(os.environ.get("OMP_NUM_THREADS") or
                                                    os.cpu_count())),
                        "graph_cached": g.get("graph_s") == 0.0,
                        "graph_reachable": g.get("reachable"),
                        "graph_build_work": g.get("stats"),
                        "graph_build_repeatable": g.get("deterministic"),
                        "graph_build_rates": g.get("rates"),
                        "graph_build_oracle_sample": g.get("oracle_sample")},
        "cpu_baseline": cpu,
        "traversal_compare": variant,
        "small_batches": small_batches,
        "ood": ood,
        "mfma": mfma,
    }
    print(json.dumps(out))


def ood_report(lv, torch, args, steps=40, in_flight=2, target=0.90, expand=5,
               hash_slots=0, cpu_sample=1000):
    """Compact run of the cross-modal workload (ood-1m-512: 1M x 512 database,
    10,000 out-of-distribution test queries): LeanVec-OOD fit (Algorithm 1, host
    float64, on 10,000 learning queries and a 100,000-vector sample), A q for the
    queries and B x for the database on the GPU, LVQ-4 primaries (d = 128),
    float16 secondaries, the host-built graph (R = 64).  The smallest window
    reaching 10-recall@10 = 0.90 is found with the plain search, then batched
    steps over the uneven request stream run one after another (each launch's
    own duration, for the roofline) and two in flight (the throughput), with five
    expansions per iteration (this workload's deeper searches: QPS at recall 0.90
    for E = 3, 4, 5, 6, 8 measured 7.80, 8.06, 8.11-8.12, 8.11, 8.00 M).  The
    float64 oracle, with its own Frank-Wolfe fit and encoding, searches a sample
    of the queries at the same window for its recall."""
    from synth import gen

    dev = torch.device("cuda:0")
    wl = gen.WORKLOADS["ood-1m-512"]
    k = wl.k
    t0 = time.time()
    mix = gen.mixture(wl)
    X = gen.database(wl, mix)
    Q = gen.queries(wl, "test", mix=mix)
    Ql = gen.queries(wl, "learn", mix=mix)
    g = {}
    th = threading.Thread(target=build_graph_cached, args=(wl, X, g))
    th.start()
    rng = np.random.default_rng(7)
    ns = min(wl.N, 100_000)
    sub = np.sort(rng.choice(wl.N, size=ns, replace=False))
    Xs = np.ascontiguousarray(X[sub])
    KX = np.zeros((wl.D, wl.D))
    ssum = np.zeros(wl.D)
    lv.lv_second_moment(Xs, KX, ssum)
    KQ = np.zeros((wl.D, wl.D))
    lv.lv_second_moment(Ql, KQ)
    tf = time.time()
    A, B, info = lv.lv_fit_ood(KQ, len(Ql), KX, ns, wl.d)
    fit = {"iters": info["iters"], "seconds": time.time() - tf}
    mu = lv.lv_mean_reduced(B, ssum, ns)
    Ab = torch.from_numpy(lv.lv_to_bf16(A).view(np.int16)).to(dev)
    Bb = torch.from_numpy(lv.lv_to_bf16(B).view(np.int16)).to(dev)
    mud = torch.from_numpy(mu).to(dev)
    Xd = torch.from_numpy(X).to(dev)
    Y = torch.empty((wl.N, wl.d), dtype=torch.float32, device=dev)
    lv.lv_project(Xd, Bb, Y)
    rec = torch.empty((wl.N, lv.lv_record_stride(wl.d, wl.bits)), dtype=torch.uint8, device=dev)
    lv.lv_lvq_encode(Y, mud, wl.bits, rec)
    sec = torch.empty((wl.N, wl.D), dtype=torch.float16, device=dev)
    lv.lv_to_f16(Xd, sec)
    torch.cuda.synchronize()
    truth = ground_truth_gpu(torch, Xd, Q, k)
    del Y, Xd
    torch.cuda.empty_cache()
    th.join()
    adj, entry = g["adj"], g["entry"]
    adjd = torch.from_numpy(adj.view(np.int32)).to(dev)
    index = lv.Index(rec, mud, sec, adjd, entry, wl.bits, wl.d, A_bf16=Ab)
    log(f"ood index ready at {time.time() - t0:.1f}s (graph {g['graph_s']:.1f}s)")
    m = len(Q)
    Qd = torch.from_numpy(Q).to(dev)
    Qp = torch.empty((m, wl.d), dtype=torch.float32, device=dev)
    lv.lv_project(Qd, Ab, Qp)
    ids = torch.empty((m, k), dtype=torch.int32, device=dev)
    sc = torch.empty((m, k), dtype=torch.float32, device=dev)

    def rec_at(L):
        lv.lv_search_projected(index, Qd, Qp, k, L, ids, sc, hash_slots=hash_slots,
                               expand=expand)
        torch.cuda.synchronize()
        return recall(ids.cpu().numpy().view(np.uint32).astype(np.int64), truth, k)

    sweep = {}
    lo_, hi_ = 10, 256
    sweep[hi_] = rec_at(hi_)
    while sweep[hi_] < target and hi_ < 1024:
        lo_, hi_ = hi_, min(1024, 2 * hi_)
        sweep[hi_] = rec_at(hi_)
    while hi_ - lo_ > 1:  # smallest window reaching the target
        mid = (lo_ + hi_) // 2
        sweep[mid] = rec_at(mid)
        if sweep[mid] >= target:
            hi_ = mid
        else:
            lo_ = mid
    L = hi_
    cnt = torch.zeros((m, 2), dtype=torch.int32, device=dev)
    lv.lv_search_projected(index, Qd, Qp, k, L, ids, sc, cnt, hash_slots=8192, expand=expand)
    torch.cuda.synchronize()
    c = cnt.cpu().numpy().astype(np.float64)
    n_rr = np.minimum(L, c[:, 1])
    bytes_q = (4 * wl.D + c[:, 0] * 4 * wl.R + c[:, 1] * (wl.d * wl.bits // 8 + 8)
               + n_rr * 2 * wl.D + 8 * k)
    alg = float(bytes_q.sum())
    rs = np.random.Generator(np.random.PCG64(401))
    sizes, left = [], m
    while left > 0:
        b = int(min(left, rs.integers(1, 4097)))
        sizes.append(b)
        left -= b
    reqs = [(0, k, L, b) for b in sizes]
    multi = lv.Multi([index])
    stream = torch.cuda.current_stream()
    strs = [stream] + [torch.cuda.Stream() for _ in range(in_flight - 1)]
    outs = [(torch.empty(m * k, dtype=torch.int32, device=dev),
             torch.empty(m * k, dtype=torch.float32, device=dev)) for _ in range(in_flight)]
    if not hash_slots:  # visited-set size: the autotuner's choice, as for the main record
        knobs, _ = lv.lv_autotune_knobs(multi, len(reqs), m, L, reqs, Qd, outs[0][0], outs[0][1],
                                        reps=6, expand=expand)
        hash_slots = knobs["hash_slots"]
    batch = lv.Batch(multi, max_requests=len(reqs), max_queries=m, max_L=L,
                     hash_slots=hash_slots, expand=expand)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    for _ in range(2):
        batch.step(reqs, Qd, *outs[0])
    torch.cuda.synchronize()
    ser = [(ev(), ev()) for _ in range(steps)]
    for i in range(steps):  # serial: each launch's own duration
        batch.step(reqs, Qd, *outs[0], events=ser[i])
    torch.cuda.synchronize()
    launch_ms = sum(a.elapsed_time(b) for a, b in ser) / steps
    got = outs[0][0].view(m, k).cpu().numpy().view(np.uint32).astype(np.int64)
    rec_b = recall(got, truth, k)
    for s_ in strs[1:]:
        s_.wait_stream(stream)
    pip = [(ev(), ev()) for _ in range(steps)]
    p0, p1 = ev(), ev()
    p0.record(stream)
    for s_ in strs[1:]:
        s_.wait_event(p0)
    for i in range(steps):
        batch.step(reqs, Qd, *outs[i % in_flight], stream=strs[i % in_flight], events=pip[i])
    for s_ in strs[1:]:
        stream.wait_stream(s_)
    p1.record(stream)
    torch.cuda.synchronize()
    ms = p0.elapsed_time(p1) / steps
    span = pip[0][0].elapsed_time(pip[-1][1]) / steps
    batch.close()
    multi.close()
    # the oracle at the same window on a sample, with its own fit and encoding
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import fit as ofit
        from oracle import lvq as olvq
        from oracle import search as osearch

        t = time.perf_counter()
        Ao, Bo, _ = ofit.frank_wolfe(ofit.second_moment(Ql), len(Ql), ofit.second_moment(Xs),
                                     len(Xs), wl.d)
        muo = ofit.mean_reduced(Xs, Bo).astype(np.float32)
        Yo = np.empty((wl.N, wl.d), dtype=np.float32)
        for lo in range(0, wl.N, 1 << 17):
            Yo[lo:lo + (1 << 17)] = ofit.project(X[lo:lo + (1 << 17)], Bo)
        codes, delta, lo4 = olvq.encode(Yo, muo, wl.bits)
        oidx = osearch.Index(adj, entry, codes, delta, lo4, muo, X.astype(np.float16))
        n = min(cpu_sample, m)
        Qpo = ofit.project(Q[:n], Ao).astype(np.float32)
        procs = max(1, min(16, len(os.sched_getaffinity(0))))
        t1 = time.perf_counter()
        o_ids, _, _ = osearch.search_many(oidx, Q[:n], Qpo, k, L, procs=procs, chunk=16,
                                          expand=expand)
        dt = time.perf_counter() - t1
        cpu = {"value": n / dt, "unit": "queries/s", "cores": procs, "kind": "oracle",
               "sample": f"first {n} of {m} test queries at window L={L}, {expand} expansions "
                         "per iteration, float64 oracle with its own Frank-Wolfe fit and "
                         "encoding, one process per core",
               "recall": recall(np.asarray(o_ids).astype(np.int64), truth[:n], k),
               "gpu_recall_same_sample": recall(got[:n], truth[:n], k),
               "setup_s": t1 - t}
        log(f"ood oracle: recall {cpu['recall']:.4f} on {n} queries")
    index.close()
    frac = alg / (launch_ms / 1e3) / 1e9 / HBM_PEAK_GBS
    out = {"workload": wl.name, "N": wl.N, "D": wl.D, "d": wl.d, "lvq_bits": wl.bits,
           "secondary": "f16", "R": wl.R, "k": k, "queries": m, "L": L, "recall_at_L": rec_b,
           "fit": dict(kind="ood (Frank-Wolfe, Algorithm 1)", **fit), "expand": expand,
           "visited_slots": hash_slots, "qps": m / (ms / 1e3), "ms_per_step": ms,
           "window_sweep": {str(x): r for x, r in sorted(sweep.items())},
           "per_query": {"expansions": float(c[:, 0].mean()),
                         "primary_scorings": float(c[:, 1].mean()),
                         "alg_bytes": float(bytes_q.mean())},
           "roofline": {"bound": "hbm", "achieved": frac * HBM_PEAK_GBS, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": frac, "alg_bytes_per_launch": alg,
                        "launch_ms": launch_ms,
                        "kernel": "batched_kernel (LVQ-4 records in 96-byte slots)",
                        "launch_timing": "average of the serial launches' own durations",
                        "pipelined": {"launch_ms": span,
                                      "frac": alg / (span / 1e3) / 1e9 / HBM_PEAK_GBS}},
           "cpu_baseline": cpu, "prep_s": time.time() - t0}
    log(f"ood: L={L} recall {rec_b:.4f}, {out['qps']:.0f} QPS, frac {frac:.3f}")
    return out


def small_batch_report(lv, torch, index, Qd, Qp, k, L, hs, expands, reps=20):
    """Latency of one plain search call over b queries (projection excluded,
    projected queries resident), one wavefront per query against the team
    launch (four wavefronts per query), at the benchmark's window.  The two
    launches must return identical ids."""
    rows = []
    for b in (1, 16, 64, 256, 1024):
        for e in expands:
            res = {}
            for name, launch in (("one_wave", lv.LV_LAUNCH_PER_QUERY),
                                 ("team", lv.LV_LAUNCH_TEAM)):
                ids = torch.empty((b, k), dtype=torch.int32, device=Qd.device)
                sc = torch.empty((b, k), dtype=torch.float32, device=Qd.device)

                def call():
                    lv.lv_search_projected(index, Qd[:b], Qp[:b], k, L, ids, sc, hash_slots=hs,
                                           expand=e, launch=launch)

                call()
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    call()
                e1.record()
                torch.cuda.synchronize()
                us = e0.elapsed_time(e1) * 1e3 / reps
                res[name] = (us, ids.cpu().numpy().copy())
            rows.append({"queries": b, "expand": e, "one_wave_us": res["one_wave"][0],
                         "team_us": res["team"][0],
                         "team_speedup": res["one_wave"][0] / res["team"][0],
                         "identical": bool(np.array_equal(res["one_wave"][1], res["team"][1]))})
            log(f"small batch b={b} E={e}: one wave {res['one_wave'][0]:.1f} us, "
                f"team {res['team'][0]:.1f} us")
    return {"L": L, "k": k, "visited_slots": hs, "reps": reps,
            "timing": "HIP events around reps calls of lv_search_projected (traversal + "
                      "re-rank), current stream", "rows": rows}


def cpu_model_name():
    """The host CPU's model name as lscpu prints it (else /proc/cpuinfo's)."""
    import subprocess

    try:
        out = subprocess.run(["lscpu"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL,
                             text=True, timeout=20).stdout
        f = {}
        for line in out.splitlines():
            k, _, v = line.partition(":")
            f.setdefault(k.strip(), v.strip())
        if f.get("Model name"):
            # the name a virtual machine reports can be short ("AMD EPYC"): the
            # family, model and stepping numbers identify the part
            ids = ", ".join(f"{k.lower()} {f[k]}" for k in ("CPU family", "Model", "Stepping")
                            if f.get(k))
            return f["Model name"] + (f" ({ids})" if ids else "")
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def cpu_baseline(wl, X, Xs, Q, adj, entry, L, sample, truth, expand=1, mix=None):
    """The float64 oracle (its own fit, projection and encoding), timed on a bounded
    query sample over all host cores; also its recall on that sample."""
    from oracle import fit as ofit
    from oracle import lvq as olvq
    from oracle import search as osearch
    from synth import gen

    t = time.time()
    if wl.fit == "ood":
        Ql = gen.queries(wl, "learn", mix=mix)
        A, P, _ = ofit.frank_wolfe(ofit.second_moment(Ql), len(Ql), ofit.second_moment(Xs),
                                   len(Xs), wl.d)
    else:
        P = ofit.fit_id(ofit.second_moment(Xs), wl.d)
        A = P
    mu = ofit.mean_reduced(Xs, P).astype(np.float32)
    Y = np.empty((wl.N, wl.d), dtype=np.float32)
    for lo in range(0, wl.N, 1 << 17):
        Y[lo:lo + (1 << 17)] = ofit.project(X[lo:lo + (1 << 17)], P)
    Qp = ofit.project(Q, A).astype(np.float32)
    codes, delta, lo_ = olvq.encode(Y, mu, wl.bits)
    index = osearch.Index(adj, entry, codes, delta, lo_, mu, X.astype(np.float16))
    log(f"oracle index ready in {time.time() - t:.1f}s")
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    n = min(sample, len(Q))
    dt = math.inf
    for _ in range(3):  # best of three (the runs are short)
        t = time.perf_counter()
        got, _, _ = osearch.search_many(index, Q[:n], Qp[:n], wl.k, L, procs=procs, chunk=16,
                                        expand=expand)
        dt = min(dt, time.perf_counter() - t)
    rec = recall(np.asarray(got).astype(np.int64), truth[:n], wl.k)
    model = cpu_model_name()
    log(f"oracle: {n} queries in {dt:.1f}s on {procs} processes")
    which = f"all {n}" if n == len(Q) else f"first {n} of {len(Q)}"
    return {"value": n / dt, "unit": "queries/s", "cores": procs, "kind": "oracle",
            "sample": f"{which} test queries, window L={L}, {expand} expansion(s) per iteration, "
                      f"float64 numpy oracle with its own "
                      f"projection and encoding, one process per core (process start-up "
                      f"included), best of 3 runs",
            "recall": rec, "cpu_model": model}


if __name__ == "__main__":
    main()
