"""The allocation-free search entry point (lv_search_noalloc) against
lv_search through the C ABI: identical ids, scores and counters on two
calls in a row, the second with fewer queries (the shared scratch array
keeps the first call's contents), with one and three expansions; a batch
too large for the scratch array is refused before any launch."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import make_case
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
def case(lv):
    wl = gen.WORKLOADS["id-1m-768"].scaled(N=6000, m_test=300)
    c = make_case(wl)
    Yd = torch.from_numpy(c.Y).to(DEV)
    mud = torch.from_numpy(c.mu).to(DEV)
    rec = torch.empty((wl.N, c.stride), dtype=torch.uint8, device=DEV)
    lv.lv_lvq_encode(Yd, mud, wl.bits, rec)
    sec = torch.from_numpy(c.sec).to(DEV)
    adj = torch.from_numpy(c.adj.view(np.int32)).to(DEV)
    Pb = torch.from_numpy(lv.lv_to_bf16(c.P).view(np.int16)).to(DEV)
    ix = lv.Index(rec, mud, sec, adj, c.entry, wl.bits, wl.d, A_bf16=Pb)
    yield c, ix, (rec, mud, sec, adj, Pb)
    ix.close()


def _run(lv, ix, Q, k, L, expand, noalloc):
    m = len(Q)
    ids = torch.full((m, k), 7, dtype=torch.int32, device=DEV)
    sc = torch.full((m, k), 7.0, dtype=torch.float32, device=DEV)
    cnt = torch.zeros((m, 2), dtype=torch.int32, device=DEV)
    Qd = torch.from_numpy(Q).to(DEV)
    if noalloc:
        lv.lv_search_noalloc(ix, Qd, k, L, ids, sc, cnt, expand=expand)
    else:
        ws = torch.empty(lv.lv_search_workspace_size(ix, m), dtype=torch.uint8, device=DEV)
        lv.lv_search(ix, Qd, k, L, ids, sc, cnt, ws=ws, expand=expand)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), sc.cpu().numpy(), cnt.cpu().numpy()


@pytest.mark.parametrize("expand", [1, 3])
def test_noalloc_equals_workspace_search_twice(lv, case, expand):
    c, ix, _ = case
    k, L = 10, 64
    for m in (300, 37):  # second call smaller: stale scratch rows past m are never read
        Q = c.Q[:m]
        want = _run(lv, ix, Q, k, L, expand, noalloc=False)
        got = _run(lv, ix, Q, k, L, expand, noalloc=True)
        for g, w in zip(got, want):
            assert np.array_equal(g, w), (m, expand)


def test_noalloc_refuses_batches_beyond_the_scratch_array(lv, case):
    c, ix, _ = case
    lib = lv.load()
    limit = lv.LV_NOALLOC_SCRATCH_BYTES // (4 * c.wl.d)
    prm = lv.SearchParams(0, 0, 0, 0)
    FAKE = 0x100000  # never dereferenced: the size check fails first
    rc = lib.lv_search_noalloc(ix.handle, FAKE, limit + 1, 10, 64, FAKE, FAKE, None,
                               ctypes.byref(prm), None)
    assert rc == lv.LV_EINVAL and b"at most" in lib.lv_last_error()
    # zero queries: valid, nothing launched
    assert lib.lv_search_noalloc(ix.handle, FAKE, 0, 10, 64, FAKE, FAKE, None,
                                 ctypes.byref(prm), None) == lv.LV_OK
