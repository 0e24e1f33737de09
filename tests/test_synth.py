"""Input module checks: seeded generators and graph invariants."""
import numpy as np
import pytest

from synth import gen, graph


def test_generators_deterministic_unit_norm_and_chunked():
    wl = gen.WORKLOADS["id-small"]
    a = gen.database(wl)
    b = gen.database(wl)
    assert a.dtype == np.float32 and a.shape == (wl.N, wl.D)
    assert np.array_equal(a, b)
    assert np.allclose(np.linalg.norm(a.astype(np.float64), axis=1), 1, atol=1e-6)
    # a larger set's first rows do not depend on how many rows were asked for
    wl2 = gen.WORKLOADS["id-1m-768"].scaled(N=70_000, m_test=5)
    mix = gen.mixture(wl2)
    x1 = gen.database(wl2, mix)
    x2 = gen.database(wl2.scaled(N=66_000), mix)
    assert np.array_equal(x1[:66_000], x2)
    q = gen.queries(wl2, "test", mix=mix)
    assert q.shape == (5, 768)


def test_ood_queries_differ_from_database_distribution():
    wl = gen.WORKLOADS["ood-1m-512"].scaled(N=4000, m_test=4000)
    mix = gen.mixture(wl)
    X = gen.database(wl, mix).astype(np.float64)
    Q = gen.queries(wl, "test", mix=mix).astype(np.float64)
    # the mean shift is visible in the query mean, not in the database mean
    assert np.linalg.norm(Q.mean(0)) > 3 * np.linalg.norm(X.mean(0))


def test_request_stream_ranges():
    sub, cnt, k, off = gen.request_stream(200, 8, 4096)
    assert sub.min() >= 0 and sub.max() < 8
    assert cnt.min() >= 1 and cnt.max() <= 4096
    assert set(k.tolist()) <= {1, 10, 100}
    sizes = gen.subindex_sizes()
    assert len(sizes) == 64 and sizes.min() >= 10_000 and sizes.max() <= 500_000


@pytest.mark.parametrize("name", ["id-small", "id-1m-768"])
def test_graph_invariants_and_determinism(name):
    wl = gen.WORKLOADS[name].scaled(N=3000)
    X = gen.database(wl)
    adj, entry = graph.build_graph(X, wl.R, threads=4)
    n, R = adj.shape
    assert R == wl.R
    valid = adj != graph.SENTINEL
    # valid entries first, then padding
    assert np.all(np.diff(valid.astype(np.int8), axis=1) <= 0)
    for i in range(n):
        row = adj[i][valid[i]]
        assert len(set(row.tolist())) == len(row)
        assert i not in row
        assert row.max(initial=0) < n
    assert graph.reachable(adj, entry).all()
    adj2, entry2 = graph.build_graph(X, wl.R, threads=2)
    assert entry2 == entry and np.array_equal(adj, adj2)
    assert entry == graph.medoid(X)
