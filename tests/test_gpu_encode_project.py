"""GPU parity: LVQ encoding (bit-exact), float16 secondaries (bit-exact), and the
bfloat16 matrix-core projection (exact on bfloat16-representable inputs,
stated error bound otherwise)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import fit as ofit
from oracle import lvq as olvq

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2312_16335_amd as lv

    lv.load()
    return lv


DEV = "cuda:0"


@pytest.mark.parametrize("bits,d,n", [(8, 160, 3001), (8, 32, 777), (4, 128, 2049), (4, 8, 65),
                                      (8, 512, 130), (8, 1024, 33)])
def test_lvq_encode_bit_exact(lv, bits, d, n):
    rng = np.random.default_rng(d + bits)
    Y = (rng.standard_normal((n, d)) * rng.uniform(1e-3, 10, (n, 1))).astype(np.float32)
    Y[0] = 0.25  # constant row: delta = 0
    mu = (0.1 * rng.standard_normal(d)).astype(np.float32)
    # the search's stride where one exists, else any multiple of 4 that fits
    stride = lv.lv_record_stride(d, bits) or (d * bits // 8 + 12)
    c, delta, lo = olvq.encode(Y, mu, bits)
    want = olvq.pack_records(c, delta, lo, bits, stride)
    rec = torch.full((n, stride), 0xAB, dtype=torch.uint8, device=DEV)
    lv.lv_lvq_encode(torch.from_numpy(Y).to(DEV), torch.from_numpy(mu).to(DEV), bits, rec)
    got = rec.cpu().numpy()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("D,d,bits,rows,stride", [
    (768, 160, 8, 3001, 192), (512, 128, 4, 2049, 96), (64, 8, 4, 65, 64),
    (128, 256, 8, 300, 512), (96, 40, 8, 17, 52), (1024, 256, 4, 1000, 136), (64, 32, 8, 1, 64)])
def test_project_encode_equals_project_then_encode(lv, D, d, bits, rows, stride):
    """The one-pass database encoding writes exactly the records of the
    projection followed by the LVQ encoder, and the oracle's encoding of the
    device projection (ragged row tails, d short of a whole 32-column tile,
    strides with padding, a zero row with mu = 0 giving delta = 0)."""
    rng = np.random.default_rng(D + d + bits)
    V = (rng.standard_normal((rows, D)) * rng.uniform(0.1, 4, (rows, 1))).astype(np.float32)
    mu = (0.2 * rng.standard_normal(d)).astype(np.float32)
    if rows > 5:
        V[5] = 0.0
        mu[:] = 0.0
    M = torch.from_numpy(lv.lv_to_bf16(rng.standard_normal((d, D)) / np.sqrt(D)).view(np.int16))
    Vd, Md, mud = torch.from_numpy(V).to(DEV), M.to(DEV), torch.from_numpy(mu).to(DEV)
    Y = torch.empty((rows, d), dtype=torch.float32, device=DEV)
    lv.lv_project(Vd, Md, Y)
    two = torch.full((rows, stride), 0xAB, dtype=torch.uint8, device=DEV)
    lv.lv_lvq_encode(Y, mud, bits, two)
    one = torch.full((rows, stride), 0xCD, dtype=torch.uint8, device=DEV)
    lv.lv_project_encode(Vd, Md, mud, bits, one)
    torch.cuda.synchronize()
    got = one.cpu().numpy()
    assert np.array_equal(got, two.cpu().numpy())
    c, delta, lo = olvq.encode(Y.cpu().numpy(), mu, bits)
    assert np.array_equal(got, olvq.pack_records(c, delta, lo, bits, stride))
    if rows > 5:
        assert delta[5] == 0.0 and not got[5, :d * bits // 8].any()


def test_project_encode_empty(lv):
    V = torch.zeros((0, 64), device=DEV)
    M = torch.zeros((32, 64), dtype=torch.int16, device=DEV)
    mu = torch.zeros(32, device=DEV)
    lv.lv_project_encode(V, M, mu, 8, torch.zeros((0, 64), dtype=torch.uint8, device=DEV))
    torch.cuda.synchronize()


@pytest.mark.parametrize("bits,d,n", [(8, 160, 3001), (4, 128, 2049), (4, 8, 65), (8, 1024, 33)])
def test_lvq_decode_bit_exact(lv, bits, d, n):
    """Device reconstruction equals the oracle's float64 decode rounded to
    float32, and lies within half a step (plus rounding) of the encoded rows."""
    rng = np.random.default_rng(3 * d + bits)
    Y = (rng.standard_normal((n, d)) * rng.uniform(1e-3, 10, (n, 1))).astype(np.float32)
    Y[0] = 0.25
    mu = (0.1 * rng.standard_normal(d)).astype(np.float32)
    stride = lv.lv_record_stride(d, bits) or (d * bits // 8 + 12)
    c, delta, lo = olvq.encode(Y, mu, bits)
    rec = torch.from_numpy(olvq.pack_records(c, delta, lo, bits, stride)).to(DEV)
    out = torch.full((n, d), float("nan"), dtype=torch.float32, device=DEV)
    lv.lv_lvq_decode(rec, d, bits, torch.from_numpy(mu).to(DEV), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = olvq.decode(c, delta, lo, mu).astype(np.float32)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    err = np.abs(got.astype(np.float64) - Y)
    bound = delta.astype(np.float64)[:, None] / 2 + 4 * np.spacing(np.abs(Y).max(axis=1))[:, None]
    assert np.all(err <= bound + 1e-12)


def test_lvq_encode_empty_and_errors(lv):
    Y = torch.zeros((0, 16), device=DEV)
    mu = torch.zeros(16, device=DEV)
    rec = torch.zeros((0, 64), dtype=torch.uint8, device=DEV)
    lv.lv_lvq_encode(Y, mu, 8, rec)
    with pytest.raises(lv.LVError):
        lv.lv_lvq_encode(torch.zeros((4, 16), device=DEV), mu, 3,
                         torch.zeros((4, 64), dtype=torch.uint8, device=DEV))


def test_f16_secondaries_bit_exact(lv):
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(100_003).astype(np.float32),
                        np.array([65504, 65520, 1e-8, -6e-8, 3e-5, 0.0, -0.0], np.float32)])
    out = torch.empty(x.size, dtype=torch.float16, device=DEV)
    lv.lv_to_f16(torch.from_numpy(x).to(DEV), out)
    assert np.array_equal(out.cpu().numpy().view(np.uint16), x.astype(np.float16).view(np.uint16))


@pytest.mark.parametrize("rows,D,d", [(1000, 768, 160), (77, 128, 32), (300, 512, 128),
                                      (33, 64, 300), (5, 8, 1)])
def test_projection_exact_on_bf16_integers(lv, rows, D, d):
    # small integers are exact in bfloat16 and their products sum exactly in
    # float32, so any lane-layout or indexing mistake shows up as a mismatch
    rng = np.random.default_rng(rows + D)
    V = rng.integers(-8, 9, size=(rows, D)).astype(np.float32)
    M = rng.integers(-4, 5, size=(d, D)).astype(np.float64)
    want = V.astype(np.float64) @ M.T
    assert np.abs(want).max() < 2 ** 24
    Mb = torch.from_numpy(lv.lv_to_bf16(M).view(np.int16)).to(DEV)
    out = torch.full((rows, d), np.nan, dtype=torch.float32, device=DEV)
    lv.lv_project(torch.from_numpy(V).to(DEV), Mb, out)
    assert np.array_equal(out.cpu().numpy().astype(np.float64), want)


@pytest.mark.parametrize("D,d", [(256, 160), (128, 520), (64, 1)])
def test_projection_row_and_column_kernels_agree(lv, D, d):
    """More than 65,536 rows take the row-tiled kernel, fewer the
    column-tiled one: the same MFMA sequence per output, so the same bits;
    integer inputs on the large side check it exactly."""
    rng = np.random.default_rng(D + d)
    rows = 70_001
    V = rng.standard_normal((rows, D)).astype(np.float32)
    M = rng.standard_normal((d, D))
    Mb = torch.from_numpy(lv.lv_to_bf16(M).view(np.int16)).to(DEV)
    Vd = torch.from_numpy(V).to(DEV)
    big = torch.full((rows, d), np.nan, dtype=torch.float32, device=DEV)
    lv.lv_project(Vd, Mb, big)
    for lo, n in ((0, 4099), (65_000, 5_001)):
        part = torch.full((n, d), np.nan, dtype=torch.float32, device=DEV)
        lv.lv_project(Vd[lo:lo + n], Mb, part)
        torch.cuda.synchronize()
        assert torch.equal(part, big[lo:lo + n])
    Vi = rng.integers(-8, 9, size=(rows, D)).astype(np.float32)
    Mi = rng.integers(-4, 5, size=(d, D)).astype(np.float64)
    Mib = torch.from_numpy(lv.lv_to_bf16(Mi).view(np.int16)).to(DEV)
    lv.lv_project(torch.from_numpy(Vi).to(DEV), Mib, big)
    torch.cuda.synchronize()
    assert np.array_equal(big.cpu().numpy().astype(np.float64), Vi.astype(np.float64) @ Mi.T)


def test_projection_error_against_float64(lv):
    rng = np.random.default_rng(9)
    V = rng.standard_normal((4096, 768)).astype(np.float32)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    M, _ = np.linalg.qr(rng.standard_normal((768, 160)))
    M = M.T
    Mb = torch.from_numpy(lv.lv_to_bf16(M).view(np.int16)).to(DEV)
    out = torch.empty((4096, 160), dtype=torch.float32, device=DEV)
    lv.lv_project(torch.from_numpy(V).to(DEV), Mb, out)
    got = out.cpu().numpy().astype(np.float64)
    want = ofit.project(V, M)
    # each product carries at most two bfloat16 roundings (2 * 2^-9 relative)
    # plus float32 accumulation: bound by 2^-7 * sum_j |v_j m_j|
    bound = 2.0 ** -7 * (np.abs(V.astype(np.float64)) @ np.abs(M).T) + 1e-6
    assert np.all(np.abs(got - want) <= bound)
    rel_rms = np.sqrt(np.mean((got - want) ** 2) / np.mean(want ** 2))
    assert rel_rms < 5e-3
