"""GPU tests of the differentiable projection path: the matrix-core GEMM (exact on
bfloat16-representable inputs, plain and split precision), the sampled-pair +
trace loss and its gradients against the float64 oracle at the refinement
shape, element by element within derived bounds, the autograd wrapper, and
Adam."""
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


# products with at least 128 tiles of 256 x 256 take the large-tile kernel:
# ragged m, n and k edges, every operand layout, exact on small integers
@pytest.mark.parametrize("M,N,K", [(3000, 2900, 70), (4096, 2048, 256)])
@pytest.mark.parametrize("ak,bk", [(True, True), (True, False), (False, True), (False, False)])
def test_gemm_large_tile_exact_on_small_integers(lv, M, N, K, ak, bk):
    rng = np.random.default_rng(M + N + K + 2 * ak + bk)
    a = rng.integers(-6, 7, size=(M, K)).astype(np.float32)
    b = rng.integers(-6, 7, size=(N, K)).astype(np.float32)
    c0 = rng.integers(-3, 4, size=(M, N)).astype(np.float32)
    A = a if ak else np.ascontiguousarray(a.T)
    B = b if bk else np.ascontiguousarray(b.T)
    C = torch.from_numpy(c0).to(DEV)
    lv.lv_gemm(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV), C, M, N, K, a_kcont=ak,
               b_kcont=bk, alpha=2.0, beta=-1.0)
    torch.cuda.synchronize()
    want = 2.0 * (a.astype(np.float64) @ b.astype(np.float64).T) - c0
    assert np.array_equal(C.cpu().numpy().astype(np.float64), want)


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


# Split precision: one operand of 12-bit integers (not representable in
# bfloat16, but exactly hi + lo), the other of small integers (exact in
# bfloat16, lo = 0), so hi*hi + hi*lo + lo*hi is the exact product and every
# float32 partial sum is an exact integer; plain bfloat16 rounds the wide
# operand and misses.  Both orders (the hi*lo and the lo*hi pass), both
# kernels (aligned and element-wise shapes) and the split over K.
@pytest.mark.parametrize("M,N,K", [(70, 130, 45), (256, 256, 128), (128, 768, 1100)])
@pytest.mark.parametrize("wide", ["A", "B"])
@pytest.mark.parametrize("ak,bk", [(True, True), (False, True), (True, False)])
def test_gemm_split_precision_is_exact_on_wide_integers(lv, M, N, K, wide, ak, bk):
    rng = np.random.default_rng(M + N + K + (wide == "A"))
    big = lambda r, c: rng.integers(-2048, 2049, size=(r, c)).astype(np.float64)  # noqa: E731
    small = lambda r, c: rng.integers(-6, 7, size=(r, c)).astype(np.float64)  # noqa: E731
    a = big(M, K) if wide == "A" else small(M, K)
    b = small(N, K) if wide == "A" else big(N, K)
    c0 = rng.integers(-3, 4, size=(M, N)).astype(np.float64)
    A = a if ak else a.T.copy()
    B = b if bk else b.T.copy()
    W = torch.empty(lv.lv_gemm_workspace_size(M, N) // 4, dtype=torch.float32, device=DEV)
    C = t(c0)
    lv.lv_gemm(t(A), t(B), C, M, N, K, a_kcont=ak, b_kcont=bk, alpha=2.0, beta=-1.0,
               workspace=W, split=True)
    P = torch.zeros((M, N), dtype=torch.float32, device=DEV)
    lv.lv_gemm(t(A), t(B), P, M, N, K, a_kcont=ak, b_kcont=bk, workspace=W)
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy().astype(np.float64), 2.0 * a @ b.T - c0)
    assert not np.array_equal(P.cpu().numpy().astype(np.float64), a @ b.T)


# bfloat16 operands in memory: whole 256 x 256 tiles, ragged m, n and k edges
# (element-wise edge loads), a row stride past K, exact on small integers
@pytest.mark.parametrize("M,N,K,ld", [(512, 768, 256, None), (300, 520, 100, 104),
                                      (1, 7, 5, 8), (257, 255, 33, 48), (1024, 1024, 1024, None)])
def test_gemm_bf16_exact_on_small_integers(lv, M, N, K, ld):
    rng = np.random.default_rng(M + 3 * N + 7 * K)
    lda = ldb = ld if ld is not None else K
    a = rng.integers(-8, 9, size=(M, K)).astype(np.float32)
    b = rng.integers(-8, 9, size=(N, K)).astype(np.float32)
    c0 = rng.integers(-3, 4, size=(M, N)).astype(np.float32)
    A = torch.zeros((M, lda), dtype=torch.bfloat16, device=DEV)
    B = torch.zeros((N, ldb), dtype=torch.bfloat16, device=DEV)
    A[:, :K] = t(a).to(torch.bfloat16)
    B[:, :K] = t(b).to(torch.bfloat16)
    if lda > K:  # values past K in a row must not enter the product
        A[:, K:] = 1e4
        B[:, K:] = -1e4
    C = t(c0)
    lv.lv_gemm_bf16(A, B, C, M, N, K, lda=lda, ldb=ldb, alpha=2.0, beta=-1.0)
    torch.cuda.synchronize()
    want = 2.0 * a.astype(np.float64) @ b.astype(np.float64).T - c0
    assert np.array_equal(C.cpu().numpy().astype(np.float64), want)


@pytest.mark.parametrize("M,N,K", [(4096, 2048, 256), (3000, 2900, 70)])
def test_gemm_bf16_equals_float32_operands_bit_for_bit(lv, M, N, K):
    """Products with at least 128 tiles of 256 x 256 take the large-tile kernel
    in both entry points: on values that bfloat16 holds exactly, the float32
    operands round to the same bfloat16 and each output gets the same MFMA
    sequence, so lv_gemm_bf16 must equal lv_gemm bit for bit (random values,
    not integers: any staging or layout slip changes the sums)."""
    g = torch.Generator(device=DEV)
    g.manual_seed(M + N + K)
    lda = ldb = (K + 7) // 8 * 8
    Ab = torch.randn((M, lda), device=DEV, generator=g).to(torch.bfloat16)
    Bb = torch.randn((N, ldb), device=DEV, generator=g).to(torch.bfloat16)
    C16 = torch.empty((M, N), device=DEV)
    C32 = torch.empty((M, N), device=DEV)
    lv.lv_gemm_bf16(Ab, Bb, C16, M, N, K, lda=lda, ldb=ldb)
    lv.lv_gemm(Ab.float(), Bb.float(), C32, M, N, K, lda=lda, ldb=ldb)
    torch.cuda.synchronize()
    assert torch.equal(C16, C32)


def test_gemm_bf16_rejects_unaligned_rows(lv):
    A = torch.zeros((16, 12), dtype=torch.bfloat16, device=DEV)
    B = torch.zeros((16, 16), dtype=torch.bfloat16, device=DEV)
    C = torch.zeros((16, 16), device=DEV)
    with pytest.raises(lv.LVError):  # lda = 12 is not a multiple of 8
        lv.lv_gemm_bf16(A, B, C, 16, 16, 12, lda=12, ldb=16)
    with pytest.raises(lv.LVError):  # A one element past an aligned start
        lv.lv_gemm_bf16(A.view(-1)[1:], B, C, 15, 16, 8, lda=8, ldb=16)


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


def _gpu_projloss(lv, A, B, Qb, Xb, KQ, KX, lam):
    d, D = A.shape
    tc = float(np.trace(KQ.astype(np.float64) @ KX.astype(np.float64))) if KQ is not None else 0.0
    ws = torch.empty(lv.lv_projloss_workspace_size(len(Qb), len(Xb), D, d), dtype=torch.uint8,
                     device=DEV)
    loss = torch.empty(3, dtype=torch.float32, device=DEV)
    dA, dB = torch.empty((d, D), device=DEV), torch.empty((d, D), device=DEV)
    KQt = t(KQ) if KQ is not None else None
    KXt = t(KX) if KX is not None else None
    At, Bt, Qt, Xt = t(A), t(B), t(Qb), t(Xb)
    lv.lv_projloss_fwd(At, Bt, Qt, Xt, loss, ws, KQt, KXt, tc, lam)
    lv.lv_projloss_bwd(At, Bt, Qt, Xt, dA, dB, ws, KQt, KXt, lam, 1.0)
    torch.cuda.synchronize()
    return (loss.cpu().numpy().astype(np.float64), dA.cpu().numpy().astype(np.float64),
            dB.cpu().numpy().astype(np.float64))


def _bounds(A, B, Qb, Xb, KQ, KX, lam):
    """Element-wise error bounds of the GPU gradients, from float64 magnitudes.

    Pair part, -(2/P) (Rm H)^T Qb (and the same for B with G, Xb): the two
    backward products round their operands to bfloat16 (2^-9 each), so the
    error is at most about 2 * 2^-8 (2/P) (|H| |Rm|^T |Qb|)_ij; Rm itself is
    formed with split precision (relative 2^-16 of |Qb Xb^T| + |G H^T|, far
    below).  Trace part, 2 lam (M2 A - B K_X) K_Q with M2 = B K_X B^T: every
    product has split operands, so the error is about 2^-15 of the chain of
    magnitudes (|B| |K_X| |B|^T |A| + |B| |K_X|) |K_Q|.  Both are widened by
    4 (pair) and 8 (trace)."""
    A, B, Qb, Xb = (np.asarray(v, np.float64) for v in (A, B, Qb, Xb))
    P = len(Qb) * len(Xb)
    G, H = A @ Qb.T, B @ Xb.T
    Rm = Qb @ Xb.T - G.T @ H
    bA = 4 * 2 * 2.0 ** -8 * (2.0 / P) * (np.abs(H) @ np.abs(Rm).T) @ np.abs(Qb)
    bB = 4 * 2 * 2.0 ** -8 * (2.0 / P) * (np.abs(G) @ np.abs(Rm)) @ np.abs(Xb)
    if KQ is not None:
        aA, aB = np.abs(A), np.abs(B)
        aQ, aX = np.abs(np.asarray(KQ, np.float64)), np.abs(np.asarray(KX, np.float64))
        UB, UA = aB @ aX, aA @ aQ  # |B| |K_X|, |A| |K_Q|: the magnitudes along each chain
        bA = bA + 8 * 2.0 ** -15 * 2 * lam * ((UB @ aB.T) @ aA + UB) @ aQ
        bB = bB + 8 * 2.0 ** -15 * 2 * lam * ((UA @ aA.T) @ aB + UA) @ aX
    return bA, bB


@pytest.mark.parametrize("case", ["pair-only", "full", "trace-dominated"])
def test_projloss_elementwise_against_float64(lv, block, case):
    """Loss and gradients against the float64 oracle on the same
    float32-rounded inputs, element by element within the bounds of
    `_bounds`: the pair part alone (no moments), pair and trace part with
    lam = 1, and a trace-dominated case (lam = 100) in which a sign or scale
    error of the trace gradient would exceed the bound by orders of
    magnitude.  Relative Frobenius errors are printed and bounded too."""
    A, B, Qb, Xb, KQ, KX = block
    lam = {"pair-only": 1.0, "full": 1.0, "trace-dominated": 100.0}[case]
    if case == "pair-only":
        KQ = KX = None
    A32, B32 = A.astype(np.float32), B.astype(np.float32)
    K32 = (None, None) if KQ is None else (KQ.astype(np.float32), KX.astype(np.float32))
    got, dA, dB = _gpu_projloss(lv, A32, B32, Qb, Xb, K32[0], K32[1], lam)
    pA, pB = opl.pair_grads(A32, B32, Qb, Xb)
    gA, gB = pA, pB
    pair = opl.pair_loss(A32, B32, Qb, Xb)
    if KQ is not None:
        KQ64, KX64 = K32[0].astype(np.float64), K32[1].astype(np.float64)
        tA = lam * ofit.grad_A(A32, B32, KQ64, KX64)
        tB = lam * ofit.grad_B(A32, B32, KQ64, KX64)
        gA, gB = pA + tA, pB + tB
        tr = ofit.loss_trace(A32, B32, KQ64, KX64)
    bA, bB = _bounds(A32, B32, Qb, Xb, K32[0], K32[1], lam)
    err = {"pair": abs(got[1] - pair) / pair,
           "dA": np.linalg.norm(dA - gA) / np.linalg.norm(gA),
           "dB": np.linalg.norm(dB - gB) / np.linalg.norm(gB),
           "dA/bound": float(np.max(np.abs(dA - gA) / bA)),
           "dB/bound": float(np.max(np.abs(dB - gB) / bB))}
    if KQ is not None:
        err["trace"] = abs(got[2] - tr) / abs(tr)
        err["trace part of dA"] = np.linalg.norm(tA) / np.linalg.norm(gA)
    print(case, "errors vs float64:", err)
    assert np.all(np.abs(dA - gA) <= bA), err
    assert np.all(np.abs(dB - gB) <= bB), err
    # split-precision residuals: the pair loss to about 2^-15 relative
    assert err["pair"] < 1e-4
    assert err["dA"] < 2e-3 and err["dB"] < 2e-3
    if KQ is not None:
        # f = <M1, M2> + tr(K_Q K_X) - 2 <A K_Q, B K_X>: error relative to the terms
        Av, Bv = A32.astype(np.float64), B32.astype(np.float64)
        terms = (abs(np.trace(Av @ KQ64 @ Av.T @ Bv @ KX64 @ Bv.T)) + abs(np.trace(KQ64 @ KX64))
                 + 2 * abs(np.trace(KQ64 @ Av.T @ Bv @ KX64)))
        assert abs(got[2] - tr) <= 2.0 ** -12 * terms
    assert abs(got[0] - (got[1] + lam * got[2])) <= 1e-6 * abs(got[0])


# (bq, bx, D, d): partial tiles in every dimension and K of neither segment a
# multiple of the K step (vector-load kernels); a row length not a multiple of
# 4 (the element-wise kernel, the residual's two K segments as two products)
@pytest.mark.parametrize("bq,bx,D,d", [(70, 196, 100, 12), (130, 260, 36, 20), (33, 70, 45, 13)])
def test_projloss_ragged_shapes(lv, bq, bx, D, d):
    """Loss and gradients of the pair part at shapes that are not multiples of
    the tiles, against the float64 oracle within the bounds of `_bounds`."""
    rng = np.random.default_rng(bq + bx + D + d)
    Qb = rng.standard_normal((bq, D)).astype(np.float32)
    Xb = rng.standard_normal((bx, D)).astype(np.float32)
    A = (rng.standard_normal((d, D)) / np.sqrt(D)).astype(np.float32)
    B = (A + 0.05 * rng.standard_normal((d, D)) / np.sqrt(D)).astype(np.float32)
    got, dA, dB = _gpu_projloss(lv, A, B, Qb, Xb, None, None, 1.0)
    gA, gB = opl.pair_grads(A, B, Qb, Xb)
    pair = opl.pair_loss(A, B, Qb, Xb)
    bA, bB = _bounds(A, B, Qb, Xb, None, None, 1.0)
    err = {"pair": abs(got[1] - pair) / pair,
           "dA/bound": float(np.max(np.abs(dA - gA) / bA)),
           "dB/bound": float(np.max(np.abs(dB - gB) / bB))}
    print((bq, bx, D, d), "errors vs float64:", err)
    assert np.all(np.abs(dA - gA) <= bA), err
    assert np.all(np.abs(dB - gB) <= bB), err
    assert err["pair"] < 1e-4


def test_projloss_on_a_caller_stream_is_bit_identical(lv, block):
    """The loss forks its independent products onto a second stream of its
    own and joins it back: on a stream of the caller's, with a long kernel
    queued before it that rewrites the inputs, the results must equal those
    on the default stream bit for bit (a missing wait would read the old
    inputs or a half-computed intermediate)."""
    A, B, Qb, Xb, KQ, KX = block
    d, D = A.shape
    tc = float(np.trace(KQ @ KX))
    ref = _gpu_projloss(lv, A, B, Qb, Xb, KQ, KX, 1.0)
    ws = torch.empty(lv.lv_projloss_workspace_size(len(Qb), len(Xb), D, d), dtype=torch.uint8,
                     device=DEV)
    loss = torch.empty(3, device=DEV)
    dA, dB = torch.empty((d, D), device=DEV), torch.empty((d, D), device=DEV)
    At, Bt, Qt, Xt, KQt, KXt = (t(v) for v in (A, B, Qb, Xb, KQ, KX))
    Az, Bz = torch.zeros_like(At), torch.zeros_like(Bt)
    big = torch.randn((4096, 4096), device=DEV)
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        for _ in range(3):  # keep the stream busy before the inputs are written
            big = big @ big
            big = big / big.norm()
        Az.copy_(At)
        Bz.copy_(Bt)
        lv.lv_projloss_fwd(Az, Bz, Qt, Xt, loss, ws, KQt, KXt, tc, 1.0)
        lv.lv_projloss_bwd(Az, Bz, Qt, Xt, dA, dB, ws, KQt, KXt, 1.0, 1.0)
    st.synchronize()
    got = (loss.cpu().numpy().astype(np.float64), dA.cpu().numpy().astype(np.float64),
           dB.cpu().numpy().astype(np.float64))
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)


def test_projloss_graph_replays_are_bit_identical(lv, block):
    """The forward and backward captured in one HIP graph (the library's
    second stream joins the capture through its events) and replayed three
    times, with eager work and synchronisations between the replays and the
    outputs cleared before each: every replay equals the eager results."""
    A, B, Qb, Xb, KQ, KX = block
    d, D = A.shape
    tc = float(np.trace(KQ @ KX))
    ws = torch.empty(lv.lv_projloss_workspace_size(len(Qb), len(Xb), D, d), dtype=torch.uint8,
                     device=DEV)
    loss = torch.empty(3, device=DEV)
    dA, dB = torch.empty((d, D), device=DEV), torch.empty((d, D), device=DEV)
    At, Bt, Qt, Xt, KQt, KXt = (t(v) for v in (A, B, Qb, Xb, KQ, KX))

    def step():
        lv.lv_projloss_fwd(At, Bt, Qt, Xt, loss, ws, KQt, KXt, tc, 1.0)
        lv.lv_projloss_bwd(At, Bt, Qt, Xt, dA, dB, ws, KQt, KXt, 1.0, 1.0)

    step()  # eager (also creates the second stream outside the capture)
    torch.cuda.synchronize()
    ref = (loss.clone(), dA.clone(), dB.clone())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=torch.cuda.Stream()):
        step()
    torch.cuda.synchronize()
    for i in range(3):
        loss.fill_(float("nan"))
        dA.fill_(float("nan"))
        dB.fill_(float("nan"))
        x = torch.randn((512, 512), device=DEV)
        (x @ x).sum().item()  # eager work between the replays
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(loss, ref[0]) and torch.equal(dA, ref[1]) and torch.equal(dB, ref[2]), i


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
