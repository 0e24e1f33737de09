"""GPU tests of the differentiable projection path: the matrix-core GEMM (exact on
bfloat16-representable inputs), the sampled-pair + trace loss and its gradients
against the float64 oracle at the refinement shape (bfloat16 error stated),
the autograd wrapper, and Adam."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fit as ofit
from oracle import projloss as opl
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


def t(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


# shapes whose leading dimensions are multiples of 4 take the vector-load kernel
# (full and partial tiles in M, N and K); the others the element-wise one
@pytest.mark.parametrize("M,N,K", [(70, 130, 45), (128, 128, 32), (1, 300, 7), (257, 3, 100),
                                   (200, 136, 100), (256, 256, 128), (132, 260, 196)])
@pytest.mark.parametrize("ak,bk", [(True, True), (True, False), (False, True), (False, False)])
def test_gemm_exact_on_small_integers(lv, M, N, K, ak, bk):
    rng = np.random.default_rng(M * 7 + N + K)
    a = rng.integers(-6, 7, size=(M, K)).astype(np.float64)
    b = rng.integers(-6, 7, size=(N, K)).astype(np.float64)
    c0 = rng.integers(-3, 4, size=(M, N)).astype(np.float64)
    A = a if ak else a.T.copy()
    B = b if bk else b.T.copy()
    C = t(c0)
    lv.lv_gemm(t(A), t(B), C, M, N, K, a_kcont=ak, b_kcont=bk, alpha=2.0, beta=-1.0)
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy().astype(np.float64), 2.0 * a @ b.T - c0)


# few output tiles and K >= 512 with a workspace: the product is split over K
# (ragged last part included) and the parts added in order; integer operands
# keep every partial sum exact, so the result must equal a @ b^T exactly.
# A workspace too small for any split gives the unsplit kernel, same result.
@pytest.mark.parametrize("M,N,K", [(128, 768, 4096), (100, 200, 1000), (64, 64, 513),
                                   (8, 12, 2048), (256, 512, 700)])
@pytest.mark.parametrize("ak,bk", [(True, True), (True, False), (False, False)])
@pytest.mark.parametrize("ws", ["full", "tiny"])
def test_gemm_split_over_k_is_exact(lv, M, N, K, ak, bk, ws):
    rng = np.random.default_rng(M + 3 * N + 5 * K)
    a = rng.integers(-6, 7, size=(M, K)).astype(np.float64)
    b = rng.integers(-6, 7, size=(N, K)).astype(np.float64)
    c0 = rng.integers(-3, 4, size=(M, N)).astype(np.float64)
    A = a if ak else a.T.copy()
    B = b if bk else b.T.copy()
    nbytes = lv.lv_gemm_workspace_size(M, N) if ws == "full" else 4 * M * N
    W = torch.full((nbytes // 4,), float("nan"), dtype=torch.float32, device=DEV)
    C = t(c0)
    lv.lv_gemm(t(A), t(B), C, M, N, K, a_kcont=ak, b_kcont=bk, alpha=2.0, beta=-1.0,
               workspace=W)
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy().astype(np.float64), 2.0 * a @ b.T - c0)
    # a second call with beta = 0 reuses the workspace's stale parts
    C2 = torch.full((M, N), float("nan"), dtype=torch.float32, device=DEV)
    lv.lv_gemm(t(A), t(B), C2, M, N, K, a_kcont=ak, b_kcont=bk, workspace=W)
    torch.cuda.synchronize()
    assert np.array_equal(C2.cpu().numpy().astype(np.float64), a @ b.T)


@pytest.fixture(scope="module")
def block():
    wl = gen.WORKLOADS["ood-1m-768"].scaled(N=8192, m_test=2048)
    mix = gen.mixture(wl)
    X = gen.database(wl, mix)
    Q = gen.queries(wl, "test", mix=mix)
    KX = ofit.second_moment(X) / len(X)
    KQ = ofit.second_moment(Q) / len(Q)
    P = ofit.fit_id(ofit.second_moment(X), wl.d)
    rng = np.random.default_rng(3)
    A = P + 0.01 * rng.standard_normal(P.shape)
    B = P + 0.01 * rng.standard_normal(P.shape)
    return A, B, Q[:1024], X[:4096], KQ, KX


def test_projloss_forward_backward_against_float64(lv, block):
    A, B, Qb, Xb, KQ, KX = block
    d, D = A.shape
    lam = 1.0
    tc = float(np.trace(KQ @ KX))
    ws = torch.empty(lv.lv_projloss_workspace_size(len(Qb), len(Xb), D, d), dtype=torch.uint8,
                     device=DEV)
    loss = torch.empty(3, dtype=torch.float32, device=DEV)
    dA, dB = torch.empty((d, D), device=DEV), torch.empty((d, D), device=DEV)
    At, Bt, Qt, Xt, KQt, KXt = t(A), t(B), t(Qb), t(Xb), t(KQ), t(KX)
    lv.lv_projloss_fwd(At, Bt, Qt, Xt, loss, ws, KQt, KXt, tc, lam)
    lv.lv_projloss_bwd(At, Bt, Qt, Xt, dA, dB, ws, KQt, KXt, lam, 1.0)
    torch.cuda.synchronize()
    # the oracle on the same float32-rounded inputs, in float64
    A32, B32 = A.astype(np.float32), B.astype(np.float32)
    pair = opl.pair_loss(A32, B32, Qb, Xb)
    tr = ofit.loss_trace(A32, B32, KQ.astype(np.float32), KX.astype(np.float32))
    gA, gB = opl.grads(A32, B32, Qb, Xb, KQ.astype(np.float32), KX.astype(np.float32), lam)
    got = loss.cpu().numpy().astype(np.float64)
    err = {
        "pair": abs(got[1] - pair) / pair,
        "trace": abs(got[2] - tr) / abs(tr),
        "dA": np.linalg.norm(dA.cpu().numpy() - gA) / np.linalg.norm(gA),
        "dB": np.linalg.norm(dB.cpu().numpy() - gB) / np.linalg.norm(gB),
    }
    print("bfloat16 relative errors vs float64:", err)
    # bfloat16 operands (2^-9 relative rounding) with float32 accumulation
    assert err["pair"] < 2e-2 and err["dA"] < 5e-2 and err["dB"] < 5e-2
    assert err["trace"] < 5e-2
    assert abs(got[0] - (got[1] + lam * got[2])) <= 1e-6 * abs(got[0])


def test_autograd_function_matches_kernels(lv, block):
    from paper_2312_16335_amd.autograd import ProjLoss

    A, B, Qb, Xb, KQ, KX = block
    d, D = A.shape
    At = t(A).requires_grad_(True)
    Bt = t(B).requires_grad_(True)
    tc = float(np.trace(KQ @ KX))
    loss = ProjLoss.apply(At, Bt, t(Qb), t(Xb), t(KQ), t(KX), tc, 0.5)
    (3.0 * loss).backward()
    ws = torch.empty(lv.lv_projloss_workspace_size(len(Qb), len(Xb), D, d), dtype=torch.uint8,
                     device=DEV)
    out = torch.empty(3, device=DEV)
    dA, dB = torch.empty((d, D), device=DEV), torch.empty((d, D), device=DEV)
    lv.lv_projloss_fwd(t(A), t(B), t(Qb), t(Xb), out, ws, t(KQ), t(KX), tc, 0.5)
    lv.lv_projloss_bwd(t(A), t(B), t(Qb), t(Xb), dA, dB, ws, t(KQ), t(KX), 0.5, 3.0)
    torch.cuda.synchronize()
    assert torch.equal(loss.detach(), out[0])
    assert torch.equal(At.grad, dA) and torch.equal(Bt.grad, dB)


def test_adam_step_matches_definition(lv):
    rng = np.random.default_rng(4)
    p = rng.standard_normal(1000).astype(np.float32)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    pt, mt, vt = t(p), t(m), t(v)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    for step in range(1, 4):
        g = rng.standard_normal(1000).astype(np.float32)
        lv.lv_adam_step(pt, t(g), mt, vt, lr, step, b1, b2, eps)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        p = p - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
    torch.cuda.synchronize()
    assert np.allclose(pt.cpu().numpy(), p, rtol=1e-5, atol=1e-6)


def test_refinement_reduces_the_loss(lv, block):
    from paper_2312_16335_amd.autograd import refine

    A, B, Qb, Xb, KQ, KX = block
    Qt, Xt = t(Qb), t(Xb)
    tc = float(np.trace(KQ @ KX))
    losses = []

    def blocks(step):
        return Qt, Xt

    refine(A, B, blocks, 30, lr=1e-3, KQn=t(KQ), KXn=t(KX), trace_const=tc, lam=1.0,
           callback=lambda s, l: losses.append(float(l[0])))
    assert losses[-1] < losses[0]


@pytest.mark.parametrize("d,D,scale", [(128, 768, 3.0), (160, 768, 0.5), (7, 33, 2.0)])
def test_device_clip_matches_host(lv, d, D, scale):
    """Projection onto the spectral-norm ball on the device against the host
    float64 routine (itself pinned against an SVD): equal to float32
    rounding; a matrix already inside the ball is left bit for bit."""
    rng = np.random.default_rng(d + D)
    U, _ = np.linalg.qr(rng.standard_normal((D, d)))
    sv = scale * np.linspace(0.2, 1.8, d)  # singular values on both sides of 1 (scale 1)
    Vt, _ = np.linalg.qr(rng.standard_normal((d, d)))
    M = ((Vt * sv) @ U.T).astype(np.float32)
    Md = t(M)
    ws = torch.empty(lv.lv_clip_spectral_device_workspace_size(d, D), dtype=torch.uint8,
                     device=DEV)
    lv.lv_clip_spectral_device(Md, ws)
    torch.cuda.synchronize()
    want = lv.lv_clip_spectral(M.astype(np.float64))
    got = Md.cpu().numpy().astype(np.float64)
    assert np.abs(got - want).max() <= 4e-6 * max(1.0, np.abs(want).max())
    assert np.linalg.svd(got, compute_uv=False).max() <= 1.0 + 1e-5
    if sv.max() <= 1.0:
        assert np.array_equal(got, M.astype(np.float64))


def test_gemm_unaligned_operands_take_the_elementwise_kernel(lv):
    # operands starting one float past a 16-byte boundary: same exact result
    rng = np.random.default_rng(17)
    M, N, K = 96, 80, 64
    a = rng.integers(-6, 7, size=(M, K)).astype(np.float64)
    b = rng.integers(-6, 7, size=(N, K)).astype(np.float64)
    Ab = torch.zeros(M * K + 1, dtype=torch.float32, device=DEV)
    Bb = torch.zeros(N * K + 1, dtype=torch.float32, device=DEV)
    Ab[1:] = t(a).view(-1)
    Bb[1:] = t(b).view(-1)
    C = torch.zeros((M, N), dtype=torch.float32, device=DEV)
    lv.load().lv_gemm(Ab[1:].data_ptr(), 1, K, Bb[1:].data_ptr(), 1, K, C.data_ptr(), N, M, N, K,
                      1.0, 0.0, None, 0, None)
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy().astype(np.float64), a @ b.T)
