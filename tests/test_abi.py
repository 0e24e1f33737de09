"""C-ABI checks that need no GPU: exported symbols, host-side validation (every
error returns before any device work), and the host float64 fitting routines
against the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2312_16335_amd as lv
from oracle import fit as ofit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "leanvec.h")
FAKE = 0x100000  # never dereferenced: validation must fail first


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lv_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_function_is_exported_and_bound():
    lib = lv.load()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(lv.exported_names())


def _desc(**kw):
    base = dict(N=100, D=128, d=32, bits=8, record_stride=64, records=FAKE, mu=FAKE,
                sec_dtype=lv.LV_F32, secondaries=FAKE, R=32, adjacency=FAKE, entry=0, A=FAKE)
    base.update(kw)
    return lv.IndexDesc(**base)


def _create(desc):
    h = ctypes.c_void_p()
    rc = lv.load().lv_index_create(ctypes.byref(desc), ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("kw,code", [
    (dict(N=0), lv.LV_EINVAL), (dict(d=12), lv.LV_EINVAL), (dict(bits=3), lv.LV_EINVAL),
    (dict(entry=100), lv.LV_EINVAL), (dict(record_stride=32), lv.LV_EINVAL),
    (dict(record_stride=160), lv.LV_EUNSUPPORTED), (dict(records=None), lv.LV_EINVAL),
    (dict(R=0), lv.LV_EINVAL), (dict(R=2000), lv.LV_EINVAL), (dict(sec_dtype=7), lv.LV_EINVAL),
    (dict(D=2000), lv.LV_EUNSUPPORTED), (dict(D=20), lv.LV_EINVAL)])
def test_index_descriptor_validation(kw, code):
    rc, h = _create(_desc(**kw))
    assert rc == code and not h.value
    assert lv.load().lv_last_error()


def test_secondary_row_bytes_and_lvq8_descriptor():
    rb = lv.lv_secondary_row_bytes
    assert rb(768, lv.LV_F16) == 1536 and rb(256, lv.LV_F32) == 1024
    assert rb(768, lv.LV_LVQ8) == 784 and rb(1008, lv.LV_LVQ8) == 1024
    assert rb(1024, lv.LV_LVQ8) == 0 and rb(100, lv.LV_LVQ8) == 0   # > 1008, D % 16
    assert rb(1032, lv.LV_F16) == 0 and rb(12, lv.LV_F16) == 0      # > 2 KiB, not 16-B rows
    assert rb(0, lv.LV_F32) == 0 and rb(64, 7) == 0
    rc, h = _create(_desc(sec_dtype=lv.LV_LVQ8))                     # no sec_mu
    assert rc == lv.LV_EINVAL and not h.value
    rc, h = _create(_desc(sec_dtype=lv.LV_LVQ8, sec_mu=FAKE, D=136))  # D % 16 != 0
    assert rc == lv.LV_EUNSUPPORTED and not h.value
    rc, h = _create(_desc(sec_dtype=lv.LV_LVQ8, sec_mu=FAKE))
    assert rc == lv.LV_OK
    lv.load().lv_index_destroy(h)


def test_search_argument_validation_before_launch():
    rc, h = _create(_desc())
    assert rc == lv.LV_OK
    lib = lv.load()
    prm = lv.SearchParams(0, 0, 0)
    cases = [(10, 0, 50), (10, 5, 3), (10, 5, 2000), (-1, 5, 50), (10, 2000, 3000)]
    for m, k, L in cases:
        rc = lib.lv_search_projected(h, FAKE, FAKE, m, k, L, FAKE, FAKE, None,
                                     ctypes.byref(prm), None)
        assert rc == lv.LV_EINVAL, (m, k, L)
    for bad in (lv.SearchParams(1000, 0, 0),   # slots not a multiple of 256
                lv.SearchParams(128, 0, 0),    # too few slots
                lv.SearchParams(65792, 0, 0),  # too many slots
                lv.SearchParams(1024, 17, 0),  # too many probes
                lv.SearchParams(1024, -1, 0),
                lv.SearchParams(1024, 0, 0, 9),    # more expansions per step than allowed
                lv.SearchParams(1024, 0, 0, -1),
                lv.SearchParams(1024, 0, 3),       # no such launch
                lv.SearchParams(1024, 0, -1)):
        assert lib.lv_search_projected(h, FAKE, FAKE, 10, 5, 50, FAKE, FAKE, None,
                                       ctypes.byref(bad), None) == lv.LV_EINVAL
        # refused before the query projection is launched
        ws = lib.lv_search_workspace_size(h, 10)
        assert lib.lv_search(h, FAKE, 10, 5, 50, FAKE, FAKE, None, FAKE, ws,
                             ctypes.byref(bad), None) == lv.LV_EINVAL
    # workspace too small
    assert lib.lv_search(h, FAKE, 10, 5, 50, FAKE, FAKE, None, FAKE, 16,
                         ctypes.byref(prm), None) == lv.LV_EINVAL
    assert lib.lv_search_workspace_size(h, 10) >= 10 * 32 * 4
    # zero queries: valid, nothing to do (also with the team launch)
    assert lib.lv_search_projected(h, FAKE, FAKE, 0, 5, 50, FAKE, FAKE, None,
                                   ctypes.byref(prm), None) == lv.LV_OK
    team = lv.SearchParams(0, 0, lv.LV_LAUNCH_TEAM, 3)
    assert lib.lv_search_projected(h, FAKE, FAKE, 0, 5, 50, FAKE, FAKE, None,
                                   ctypes.byref(team), None) == lv.LV_OK
    lib.lv_index_destroy(h)


def test_encode_and_project_validation():
    lib = lv.load()
    assert lib.lv_lvq_encode(FAKE, 10, 32, FAKE, 3, FAKE, 64, None) == lv.LV_EINVAL
    assert lib.lv_lvq_encode(FAKE, 10, 36, FAKE, 8, FAKE, 64, None) == lv.LV_EINVAL
    assert lib.lv_lvq_encode(FAKE, 10, 160, FAKE, 8, FAKE, 160, None) == lv.LV_EINVAL
    assert lib.lv_lvq_encode(None, 10, 32, FAKE, 8, FAKE, 64, None) == lv.LV_EINVAL
    assert lib.lv_lvq_encode(FAKE, 0, 32, FAKE, 8, FAKE, 64, None) == lv.LV_OK
    # decode: the encoder's checks
    dec = lib.lv_lvq_decode
    assert dec(FAKE, 10, 32, 3, 64, FAKE, FAKE, None) == lv.LV_EINVAL
    assert dec(FAKE, 10, 36, 8, 64, FAKE, FAKE, None) == lv.LV_EINVAL
    assert dec(FAKE, 10, 160, 8, 160, FAKE, FAKE, None) == lv.LV_EINVAL
    assert dec(None, 10, 32, 8, 64, FAKE, FAKE, None) == lv.LV_EINVAL
    assert dec(FAKE, 10, 32, 8, 64, FAKE, None, None) == lv.LV_EINVAL
    assert dec(FAKE, -1, 32, 8, 64, FAKE, FAKE, None) == lv.LV_EINVAL
    assert dec(FAKE, 0, 32, 8, 64, FAKE, FAKE, None) == lv.LV_OK
    # one-pass projection and encoding: d in [8, 256], stride checks, NULLs
    pe = lib.lv_project_encode
    assert pe(FAKE, 10, 768, FAKE, 264, FAKE, 8, FAKE, 512, None) == lv.LV_EINVAL
    assert pe(FAKE, 10, 768, FAKE, 12, FAKE, 8, FAKE, 64, None) == lv.LV_EINVAL
    assert pe(FAKE, 10, 768, FAKE, 160, FAKE, 3, FAKE, 192, None) == lv.LV_EINVAL
    assert pe(FAKE, 10, 768, FAKE, 160, FAKE, 8, FAKE, 164, None) == lv.LV_EINVAL
    assert pe(FAKE, 10, 768, FAKE, 160, FAKE, 8, FAKE, 170, None) == lv.LV_EINVAL
    assert pe(FAKE, 10, 12, FAKE, 160, FAKE, 8, FAKE, 192, None) == lv.LV_EINVAL
    assert pe(FAKE, -1, 768, FAKE, 160, FAKE, 8, FAKE, 192, None) == lv.LV_EINVAL
    assert pe(FAKE, 10, 768, FAKE, 160, None, 8, FAKE, 192, None) == lv.LV_EINVAL
    assert pe(FAKE, 10, 768, FAKE, 160, FAKE, 8, None, 192, None) == lv.LV_EINVAL
    assert pe(FAKE, 0, 768, FAKE, 160, FAKE, 8, FAKE, 192, None) == lv.LV_OK
    # second level: same checks, d <= 1008 and rows of exactly the level-2 width
    rb = lib.lv_secondary_row_bytes(32, lv.LV_LVQ8_LEVEL2)
    assert lib.lv_lvq_encode_level2(FAKE, 10, 32, FAKE, 3, FAKE, 64, FAKE, rb, None) == lv.LV_EINVAL
    assert lib.lv_lvq_encode_level2(FAKE, 10, 36, FAKE, 8, FAKE, 64, FAKE, rb, None) == lv.LV_EINVAL
    assert lib.lv_lvq_encode_level2(FAKE, 10, 1016, FAKE, 4, FAKE, 1024, FAKE,
                                    1040, None) == lv.LV_EINVAL
    assert lib.lv_lvq_encode_level2(FAKE, 10, 32, FAKE, 8, FAKE, 32, FAKE, rb, None) == lv.LV_EINVAL
    assert lib.lv_lvq_encode_level2(FAKE, 10, 32, FAKE, 8, FAKE, 64, FAKE, rb + 16,
                                    None) == lv.LV_EINVAL
    assert lib.lv_lvq_encode_level2(FAKE, 10, 32, FAKE, 8, None, 64, FAKE, rb, None) == lv.LV_EINVAL
    assert lib.lv_lvq_encode_level2(FAKE, 10, 32, FAKE, 8, FAKE, 64, None, rb, None) == lv.LV_EINVAL
    assert lib.lv_lvq_encode_level2(FAKE, -1, 32, FAKE, 8, FAKE, 64, FAKE, rb, None) == lv.LV_EINVAL
    assert lib.lv_lvq_encode_level2(FAKE, 0, 32, FAKE, 8, FAKE, 64, FAKE, rb, None) == lv.LV_OK
    assert lib.lv_project(FAKE, 10, 12, FAKE, 4, FAKE, None) == lv.LV_EINVAL
    assert lib.lv_project(FAKE, 10, 16, FAKE, 0, FAKE, None) == lv.LV_EINVAL
    assert lib.lv_project(FAKE, -1, 16, FAKE, 4, FAKE, None) == lv.LV_EINVAL
    assert lib.lv_to_f16(FAKE, -5, FAKE, None) == lv.LV_EINVAL
    assert lv.lv_record_stride(160, 8) == 192 and lv.lv_record_stride(128, 4) == 96
    assert lv.lv_record_stride(112, 8) == 128 and lv.lv_record_stride(64, 8) == 96
    assert lv.lv_record_stride(32, 8) == 64 and lv.lv_record_stride(3000, 8) == 0


def test_gemm_validation_and_workspace_size():
    lib = lv.load()
    assert lib.lv_gemm(FAKE, 1, 8, FAKE, 1, 8, FAKE, 4, 4, 4, 8, 1.0, 0.0, None, 64,
                       None) == lv.LV_EINVAL
    assert "workspace" in lib.lv_last_error().decode()
    assert lib.lv_gemm(FAKE, 1, 8, FAKE, 1, 8, FAKE, 4, 4, 4, 8, 1.0, 0.0, FAKE + 2, 64,
                       None) == lv.LV_EINVAL
    assert lib.lv_gemm(FAKE, 1, 7, FAKE, 1, 8, FAKE, 4, 4, 4, 8, 1.0, 0.0, None, 0,
                       None) == lv.LV_EINVAL
    assert lib.lv_gemm(FAKE, 1, 8, FAKE, 1, 8, FAKE, 4, -1, 4, 8, 1.0, 0.0, None, 0,
                       None) == lv.LV_EINVAL
    # at most 16 parts of M x N floats; nothing for an empty product
    assert lv.lv_gemm_workspace_size(128, 768) == 16 * 128 * 768 * 4
    assert lv.lv_gemm_workspace_size(0, 768) == 0


def test_device_clip_validation_and_workspace_size():
    lib = lv.load()
    ws = lv.lv_clip_spectral_device_workspace_size(128, 768)
    assert ws == 2 * 128 * 128 * 8 + 128 * 768 * 4
    assert lv.lv_clip_spectral_device_workspace_size(0, 768) == 0
    assert lib.lv_clip_spectral_device(None, 128, 768, FAKE, ws, None) == lv.LV_EINVAL
    assert lib.lv_clip_spectral_device(FAKE, 128, 768, FAKE, ws - 1, None) == lv.LV_EINVAL
    assert lib.lv_clip_spectral_device(FAKE, 2000, 768, FAKE, 1 << 30, None) == lv.LV_EINVAL
    assert lib.lv_clip_spectral_device(FAKE, 128, 768, FAKE + 4, ws, None) == lv.LV_EINVAL


def test_batch_step_validation_without_a_device():
    lib = lv.load()
    one = (lv.Request * 1)(lv.Request(0, 10, 20, 5))
    assert lib.lv_batch_step(None, one, 1, FAKE, FAKE, FAKE, None, None) == lv.LV_EINVAL
    assert lib.lv_batch_step_timed(None, one, 1, FAKE, FAKE, FAKE, None, FAKE, FAKE,
                                   None) == lv.LV_EINVAL
    # a NULL timing event is refused before the batch is looked at
    assert lib.lv_batch_step_timed(FAKE, one, 1, FAKE, FAKE, FAKE, None, None, FAKE,
                                   None) == lv.LV_EINVAL
    assert "event" in lib.lv_last_error().decode()


def test_bf16_conversion_is_round_to_nearest_even():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-5, 5, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0]])
    got = lv.lv_to_bf16(x)
    f = x.astype(np.float32).view(np.uint32).astype(np.uint64)
    keep = f >> 16
    rest = f & 0xFFFF
    up = (rest > 0x8000) | ((rest == 0x8000) & (keep & 1 == 1))
    want = (keep + up).astype(np.uint16)
    assert np.array_equal(got, want)


def _moments(D=24, n=700, m=500, seed=0):
    rng = np.random.default_rng(seed)
    sc = 1.0 / np.sqrt(np.arange(1, D + 1))
    X = (rng.standard_normal((n, D)) * sc).astype(np.float32)
    Rot, _ = np.linalg.qr(rng.standard_normal((D, D)))
    Q = ((rng.standard_normal((m, D)) * sc) @ Rot.T + 0.2).astype(np.float32)
    return X, Q


def test_mean_reduced_matches_oracle():
    X, _ = _moments(D=24, n=500)
    P = ofit.fit_id(ofit.second_moment(X), 6)
    s = X.astype(np.float64).sum(0)
    mu = lv.lv_mean_reduced(np.ascontiguousarray(P), s, len(X))
    want = ofit.mean_reduced(X, P)
    assert np.allclose(mu, want, rtol=1e-6, atol=1e-7)
    assert mu.dtype == np.float32


def test_second_moment_matches_oracle():
    X, _ = _moments()
    K = np.zeros((X.shape[1],) * 2)
    s = np.zeros(X.shape[1])
    lv.lv_second_moment(X[:300], K, s)
    lv.lv_second_moment(X[300:], K, s)
    assert np.allclose(K, ofit.second_moment(X), rtol=1e-12, atol=1e-12)
    assert np.allclose(s, X.astype(np.float64).sum(0), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("D,d", [(24, 5), (64, 16), (7, 7), (1, 1)])
def test_fit_id_matches_oracle(D, d):
    X, _ = _moments(D=D)
    K = ofit.second_moment(X)
    P, ev = lv.lv_fit_id(np.ascontiguousarray(K), d, with_evals=True)
    Po = ofit.fit_id(K, d)
    assert np.linalg.norm(P.T @ P - Po.T @ Po) < 1e-10 * max(1, d)
    assert np.allclose(P @ P.T, np.eye(d), atol=1e-12)
    assert np.allclose(ev, np.sort(np.linalg.eigvalsh(K))[::-1], rtol=1e-10, atol=1e-10 * ev[0])
    # same sign convention as the oracle on a well-separated spectrum
    assert np.allclose(P, Po, atol=1e-8)


def test_fit_id_larger_matrix():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((300, 300))
    K = A @ A.T
    P, ev = lv.lv_fit_id(np.ascontiguousarray(K), 40, with_evals=True)
    Po = ofit.fit_id(K, 40)
    assert np.linalg.norm(P.T @ P - Po.T @ Po) < 1e-8
    assert np.allclose(ev, np.sort(np.linalg.eigvalsh(K))[::-1], rtol=1e-9)


def test_fit_ood_matches_oracle_frank_wolfe():
    X, Q = _moments(D=24, n=700, m=500, seed=1)
    KQ, KX = ofit.second_moment(Q), ofit.second_moment(X)
    A, B, info = lv.lv_fit_ood(KQ, len(Q), KX, len(X), 6)
    Ao, Bo, rep = ofit.frank_wolfe(KQ, len(Q), KX, len(X), 6)
    assert info["iters"] == rep.iters and info["converged"] == rep.converged
    assert np.allclose(info["f"], rep.f, rtol=1e-7)
    assert np.allclose(A, Ao, atol=1e-6) and np.allclose(B, Bo, atol=1e-6)
    f = lv.lv_ood_loss(KQ, len(Q), KX, len(X), A, B)
    assert f == pytest.approx(ofit.loss_trace(A, B, KQ / len(Q), KX / len(X)), rel=1e-10)


def test_fit_ood_zero_start_and_not_converged_warning():
    X, Q = _moments(D=16, n=400, m=300, seed=2)
    KQ, KX = ofit.second_moment(Q), ofit.second_moment(X)
    A, B, info = lv.lv_fit_ood(KQ, len(Q), KX, len(X), 4, init=lv.LV_FW_INIT_ZERO,
                               max_iter=2, tol=0.0)
    assert info["status"] == lv.LV_WNOTCONVERGED and info["iters"] == 2
    Ao, Bo, rep = ofit.frank_wolfe(KQ, len(Q), KX, len(X), 4, init="zero", T=1, tol=0.0)
    assert np.allclose(A, Ao, atol=1e-9) and np.allclose(B, Bo, atol=1e-9)
    with pytest.raises(lv.LVError):
        lv.lv_fit_ood(KQ, len(Q), KX, len(X), 4, alpha=1.5)


def test_fit_es_matches_oracle():
    X, Q = _moments(D=20, n=600, m=400, seed=4)
    KQ, KX = ofit.second_moment(Q), ofit.second_moment(X)
    P, beta = lv.lv_fit_es(KQ, len(Q), KX, len(X), 5, xtol=1e-6)
    Po, bo = ofit.eigsearch(KQ, len(Q), KX, len(X), 5, xtol=1e-6)
    fo = ofit.equalised_loss(Po, KQ, len(Q), KX, len(X))
    f = ofit.equalised_loss(P, KQ, len(Q), KX, len(X))
    assert abs(beta - bo) < 1e-3
    assert f <= fo + 1e-9 * abs(fo)


def test_clip_spectral_against_svd():
    rng = np.random.default_rng(8)
    M = rng.standard_normal((6, 20)) * 0.25
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    assert s.max() > 1 and s.min() < 1
    got = lv.lv_clip_spectral(M)
    want = U @ np.diag(np.minimum(s, 1.0)) @ Vt
    assert np.allclose(got, want, atol=1e-10)
    inside = M / (2 * s.max())
    assert np.array_equal(lv.lv_clip_spectral(inside), inside)


def test_graph_build_validation_without_a_device():
    lib = lv.load()
    order = np.arange(100, dtype=np.uint32)
    op = order.ctypes.data

    def call(records=FAKE, stride=64, N=100, d=32, bits=8, order_p=op, entry=0, adj=FAKE,
             **kw):
        base = dict(R=16, L=32, alphas=(1.0, 1.0), max_batch=8)
        base.update(kw)
        bp = lv.build_params(**base)
        return lib.lv_graph_build(records, stride, N, d, bits, order_p, entry, ctypes.byref(bp),
                                  adj, None)

    assert call(records=None) == lv.LV_EINVAL
    assert call(adj=None) == lv.LV_EINVAL
    assert call(order_p=None) == lv.LV_EINVAL
    assert call(N=0) == lv.LV_EINVAL
    assert call(d=12) == lv.LV_EINVAL
    assert call(bits=3) == lv.LV_EINVAL
    assert call(d=512, stride=1024) == lv.LV_EUNSUPPORTED  # 512 code bytes per record
    assert call(stride=160) == lv.LV_EUNSUPPORTED
    assert call(d=64, stride=64) == lv.LV_EINVAL  # no room for delta and lo
    assert call(R=65) == lv.LV_EUNSUPPORTED
    assert call(R=0) == lv.LV_EUNSUPPORTED
    assert call(L=0) == lv.LV_EINVAL
    assert call(alphas=(1.0, -0.5)) == lv.LV_EINVAL
    assert call(alphas=(float("nan"),)) == lv.LV_EINVAL
    assert call(max_batch=0) == lv.LV_EINVAL
    assert call(stop_after=-1) == lv.LV_EINVAL
    assert call(entry=100) == lv.LV_EINVAL
    assert call(hash_slots=1000) == lv.LV_EINVAL
    dup = order.copy()
    dup[5] = 4
    assert call(order_p=dup.ctypes.data) == lv.LV_EINVAL
    assert "permutation" in lib.lv_last_error().decode()
    big = order.copy()
    big[7] = 100
    assert call(order_p=big.ctypes.data) == lv.LV_EINVAL
    with pytest.raises(ValueError):
        lv.build_params(16, 32, alphas=(1.0,) * 9)


def test_residual_secondaries_descriptor():
    assert lv.lv_secondary_row_bytes(608, lv.LV_F16_RESID) == 1216
    rc, h = _create(_desc(sec_dtype=lv.LV_F16_RESID, D=32, d=32))   # nothing left over
    assert rc == lv.LV_EINVAL and not h.value
    rc, h = _create(_desc(sec_dtype=lv.LV_F16_RESID, D=128, d=32))
    assert rc == lv.LV_OK
    lib = lv.load()
    # the workspace holds P q and P_perp q: D floats per query
    assert lib.lv_search_workspace_size(h, 10) >= 10 * 128 * 4
    lib.lv_index_destroy(h)


def test_level2_secondaries_descriptor():
    # d code bytes padded to 16, then delta2, lo2 and 8 zero bytes
    for d, want in ((8, 32), (88, 112), (160, 176), (1008, 1024), (1016, 0)):
        assert lv.lv_secondary_row_bytes(d, lv.LV_LVQ8_LEVEL2) == want, d
    rc, h = _create(_desc(sec_dtype=lv.LV_LVQ8_LEVEL2, D=128, d=32))
    assert rc == lv.LV_OK
    lib = lv.load()
    assert lib.lv_search_workspace_size(h, 10) == (10 * 32 * 4 + 255) // 256 * 256
    lib.lv_index_destroy(h)
    rc, h = _create(_desc(sec_dtype=5, D=128, d=32))
    assert rc == lv.LV_EINVAL and not h.value


def test_binding_checks_buffer_sizes_before_any_call():
    """The C ABI cannot see buffer sizes, so the binding checks shapes and
    element counts first: an undersized output raises ValueError before a
    pointer is taken (host tensors stand in for device ones; with the right
    shapes the same calls stop at the device-tensor check instead)."""
    import types

    torch = pytest.importorskip("torch")
    f32, i32, u8 = torch.float32, torch.int32, torch.uint8
    z = lambda *s, dt=f32: torch.zeros(s, dtype=dt)  # noqa: E731

    with pytest.raises(ValueError):   # out holds 10 x 3 < 10 x 4
        lv.lv_project(z(10, 16), z(4, 16, dt=torch.int16), z(10, 3))
    with pytest.raises(ValueError):   # M has 12 columns, V has 16
        lv.lv_project(z(10, 16), z(4, 12, dt=torch.int16), z(10, 4))
    with pytest.raises(TypeError):    # shapes fine: refused as host tensors
        lv.lv_project(z(10, 16), z(4, 16, dt=torch.int16), z(10, 4))
    with pytest.raises(ValueError):   # 9 record rows for 10 vectors
        lv.lv_lvq_encode(z(10, 32), z(32), 8, z(9, 64, dt=u8))
    with pytest.raises(ValueError):
        lv.lv_lvq_encode(z(10, 32), z(16), 8, z(10, 64, dt=u8))
    with pytest.raises(ValueError):
        lv.lv_to_f16(z(10, 8), z(79, dt=torch.float16))

    N, D, d, R = 100, 128, 32, 32
    good = dict(records=z(N, 64, dt=u8), mu=z(d), secondaries=z(N, D), adjacency=z(N, R, dt=i32),
                entry=0, bits=8, d=d)
    for bad in (dict(records=z(N - 1, 64, dt=u8)), dict(mu=z(d - 1)),
                dict(adjacency=z(N - 1, R, dt=i32)), dict(entry=N),
                dict(A_bf16=z(d, D - 1, dt=torch.int16)),
                dict(secondaries=z(N, D + 8, dt=u8), sec_mu=z(D))):  # LVQ-8 rows are D + 16 B
        with pytest.raises(ValueError):
            lv.Index(**{**good, **bad})
    with pytest.raises(TypeError):
        lv.Index(**good)

    rc, h = _create(_desc(N=N, D=D, d=d, R=R))
    assert rc == lv.LV_OK
    ix = types.SimpleNamespace(handle=h, D=D, d=d, qp_width=d)
    m, k, L = 10, 5, 50
    ws = z(lv.lv_search_workspace_size(ix, m), dt=u8)
    ok = dict(ids=z(m, k, dt=i32), scores=z(m, k), counters=z(m, 2, dt=i32))
    for bad in (dict(ids=z(m * k - 1, dt=i32)), dict(scores=z(m, k - 1)),
                dict(counters=z(2 * m - 1, dt=i32))):
        args = {**ok, **bad}
        with pytest.raises(ValueError):
            lv.lv_search(ix, z(m, D), k, L, args["ids"], args["scores"], args["counters"], ws=ws)
        with pytest.raises(ValueError):
            lv.lv_search_projected(ix, z(m, D), z(m, d), k, L, args["ids"], args["scores"],
                                   args["counters"])
    with pytest.raises(ValueError):   # queries of the wrong dimension
        lv.lv_search(ix, z(m, D - 1), k, L, ok["ids"], ok["scores"], ws=ws)
    with pytest.raises(ValueError):   # workspace one byte short
        lv.lv_search(ix, z(m, D), k, L, ok["ids"], ok["scores"], ws=z(ws.numel() - 1, dt=u8))
    with pytest.raises(ValueError):   # projected queries of the wrong width
        lv.lv_search_projected(ix, z(m, D), z(m, d + 1), k, L, ok["ids"], ok["scores"])
    with pytest.raises(TypeError):
        lv.lv_search(ix, z(m, D), k, L, ok["ids"], ok["scores"], ws=ws)
    lv.load().lv_index_destroy(h)

    multi = types.SimpleNamespace(D=D)
    reqs = [(0, 10, 50, 7), (0, 100, 120, 3)]      # 10 queries, 370 results
    from paper_2312_16335_amd._lib import _step_buffers
    _step_buffers(multi, reqs, z(10, D), z(370, dt=i32), z(370), z(20, dt=i32))
    for args in ((z(9, D), z(370, dt=i32), z(370)), (z(10, D), z(369, dt=i32), z(370)),
                 (z(10, D), z(370, dt=i32), z(369)), (z(10, D + 1), z(370, dt=i32), z(370))):
        with pytest.raises(ValueError):
            _step_buffers(multi, reqs, *args)
    with pytest.raises(ValueError):
        _step_buffers(multi, reqs, z(10, D), z(370, dt=i32), z(370), z(19, dt=i32))

    with pytest.raises(ValueError):   # C [M][N] with M = N = K = 8 needs 64 elements
        lv.lv_gemm(z(64), z(64), z(63), 8, 8, 8)
    with pytest.raises(ValueError):   # B read with ldb = 16: (8 - 1) * 16 + 8 elements
        lv.lv_gemm(z(64), z(64), z(64), 8, 8, 8, ldb=16)
    bf = torch.bfloat16
    with pytest.raises(TypeError):    # bfloat16 operands only
        lv.lv_gemm_bf16(z(64), z(64, dt=bf), z(64), 8, 8, 8)
    with pytest.raises(ValueError):   # A [8][8] needs 64 elements
        lv.lv_gemm_bf16(z(63, dt=bf), z(64, dt=bf), z(64), 8, 8, 8)
    with pytest.raises(ValueError):   # C [8][8] needs 64 elements
        lv.lv_gemm_bf16(z(64, dt=bf), z(64, dt=bf), z(63), 8, 8, 8)
    Dr, dr, bq, bx = 16, 4, 5, 7
    pws = z(lv.lv_projloss_workspace_size(bq, bx, Dr, dr), dt=u8)
    A, B, Qb, Xb = z(dr, Dr), z(dr, Dr), z(bq, Dr), z(bx, Dr)
    with pytest.raises(ValueError):
        lv.lv_projloss_fwd(A, B, Qb, Xb, z(2), pws)
    with pytest.raises(ValueError):
        lv.lv_projloss_fwd(A, B, Qb, Xb, z(3), pws, KQn=z(Dr, Dr))
    with pytest.raises(ValueError):
        lv.lv_projloss_fwd(A, B, Qb, Xb, z(3), z(pws.numel() - 1, dt=u8))
    with pytest.raises(ValueError):
        lv.lv_projloss_bwd(A, B, Qb, Xb, z(dr, Dr), z(dr, Dr - 1), pws)
    with pytest.raises(TypeError):
        lv.lv_projloss_bwd(A, B, Qb, Xb, z(dr, Dr), z(dr, Dr), pws)
    with pytest.raises(ValueError):
        lv.lv_adam_step(z(10), z(10), z(9), z(10), 1e-3, 1)
    with pytest.raises(ValueError):
        lv.lv_clip_spectral_device(z(dr, Dr), z(1, dt=u8))


def test_fit_ood_hand_worked_trace():
    """lv_fit_ood from a given start against Algorithm 1 worked by hand on
    D = 2, d = 1 (tests/golden/fw_hand.json): iterates, losses and the sum of
    the two linear steps' gaps per iteration; the early stop's denominator is
    the loss before the iteration."""
    import json

    g = json.load(open(os.path.join(ROOT, "tests", "golden", "fw_hand.json")))
    KQ, KX = np.array(g["KQ"]), np.array(g["KX"])
    its = g["iterations"]
    for n_it in range(1, len(its)):
        A, B, info = lv.lv_fit_ood(KQ, 1, KX, 1, 1, alpha=g["alpha"], tol=0.0, max_iter=n_it,
                                   init=lv.LV_FW_INIT_GIVEN, A0=[g["A0"]], B0=[g["B0"]])
        want = its[n_it]
        assert info["iters"] == n_it and not info["converged"]
        np.testing.assert_allclose(A[0], want["A"], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(B[0], want["B"], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(info["f"], g["f"][:n_it + 1], rtol=1e-12)
        np.testing.assert_allclose(info["gap"][-1], want["gap_A"] + want["gap_B"], rtol=1e-11)
    for s in g["stops"]:
        _, _, info = lv.lv_fit_ood(KQ, 1, KX, 1, 1, alpha=g["alpha"], tol=s["tol"], max_iter=50,
                                   init=lv.LV_FW_INIT_GIVEN, A0=[g["A0"]], B0=[g["B0"]])
        assert info["converged"] and info["iters"] == s["iters"]


def test_mean_reduced_hand_example():
    """mu = B * (sum of rows / n): rows (1, 2), (3, 4), (5, 9) sum to (9, 15);
    B = [[1, 0], [1, 1], [2, -1]] maps their mean (3, 5) to (3, 8, 1)."""
    B = np.array([[1.0, 0.0], [1.0, 1.0], [2.0, -1.0]])
    mu = lv.lv_mean_reduced(B, np.array([9.0, 15.0]), 3)
    np.testing.assert_array_equal(mu, np.array([3.0, 8.0, 1.0], np.float32))
