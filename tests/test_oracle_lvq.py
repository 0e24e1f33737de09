"""Pins for the LVQ oracle: hand-worked cases, error bound, range, fixed point."""
import json
import os

import numpy as np
import pytest

from oracle import lvq

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lvq_hand.json")


def test_hand_worked_cases():
    for case in json.load(open(GOLDEN))["cases"]:
        y = np.array([case["y"]], dtype=np.float32)
        mu = np.array(case["mu"], dtype=np.float32)
        c, delta, lo = lvq.encode(y, mu, case["bits"])
        assert c[0].tolist() == case["codes"], case["why"]
        assert float(delta[0]) == pytest.approx(case["delta"], rel=0, abs=0)
        assert float(lo[0]) == case["lo"]


@pytest.mark.parametrize("bits", [4, 8])
def test_half_step_bound_and_range(bits):
    rng = np.random.default_rng(1)
    Y = (rng.standard_normal((500, 40)) * rng.uniform(0.01, 10, (500, 1))).astype(np.float32)
    mu = rng.standard_normal(40).astype(np.float32)
    c, delta, lo = lvq.encode(Y, mu, bits)
    levels = (1 << bits) - 1
    assert c.max() <= levels
    r = Y.astype(np.float64) - mu.astype(np.float64)
    rec = lo.astype(np.float64)[:, None] + delta.astype(np.float64)[:, None] * c
    mag = np.maximum(np.abs(r.min(1)), np.abs(r.max(1)))
    ulp = np.spacing(mag.astype(np.float32)).astype(np.float64)
    bound = delta.astype(np.float64) / 2 + 2 * ulp
    assert np.all(np.abs(r - rec) <= bound[:, None] * (1 + 1e-12))
    rows = np.arange(len(Y))
    assert np.all(c[rows, r.argmin(1)] == 0)
    assert np.all(c[rows, r.argmax(1)] == levels)


@pytest.mark.parametrize("bits", [4, 8])
def test_reencode_fixed_point(bits):
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((300, 32)).astype(np.float32)
    mu = (0.1 * rng.standard_normal(32)).astype(np.float32)
    c, delta, lo = lvq.encode(Y, mu, bits)
    Yhat = lvq.decode(c, delta, lo, mu).astype(np.float32)
    c2, _, _ = lvq.encode(Yhat, mu, bits)
    assert np.array_equal(c, c2)


def test_constant_vector_all_zero():
    Y = np.full((3, 16), 0.5, dtype=np.float32)
    c, delta, lo = lvq.encode(Y, np.zeros(16, np.float32), 8)
    assert not c.any() and not delta.any()


def test_pack_layout_and_roundtrip():
    c = np.array([[1, 2, 15, 0, 7, 8, 3, 4]], dtype=np.uint8)
    rec = lvq.pack_records(c, np.array([0.5], np.float32), np.array([-2.0], np.float32), 4, 16)
    # component 2i in the low nibble, 2i+1 in the high nibble
    assert rec[0, :4].tolist() == [0x21, 0x0F, 0x87, 0x43]
    assert rec[0, 4:8].view(np.float32)[0] == 0.5
    assert rec[0, 8:12].view(np.float32)[0] == -2.0
    assert not rec[0, 12:].any()
    c2, d2, l2 = lvq.unpack_records(rec, 8, 4)
    assert np.array_equal(c, c2) and d2[0] == 0.5 and l2[0] == -2.0
    c8 = np.arange(16, dtype=np.uint8).reshape(1, 16)
    rec8 = lvq.pack_records(c8, np.array([1.0], np.float32), np.array([0.0], np.float32), 8, 32)
    assert rec8[0, :16].tolist() == list(range(16))


def test_two_level_hand_worked_case():
    for case in json.load(open(GOLDEN))["two_level_cases"]:
        y = np.array([case["y"]], dtype=np.float32)
        mu = np.array(case["mu"], dtype=np.float32)
        c, delta, lo = lvq.encode(y, mu, case["bits"])
        assert c[0].tolist() == case["codes"] and float(delta[0]) == case["delta"]
        assert float(lo[0]) == case["lo"]
        assert lvq.residual(y, mu, c, delta, lo)[0].tolist() == case["residual"]
        c2, d2, l2 = lvq.encode_residual(y, mu, c, delta, lo)
        assert c2[0].tolist() == case["codes2"], case["why"]
        assert float(d2[0]) == case["delta2"] and float(l2[0]) == case["lo2"]
        rec = lvq.decode_two_level(c, delta, lo, c2, d2, l2, mu)
        assert rec[0].tolist() == case["reconstruction"]


@pytest.mark.parametrize("bits", [4, 8])
def test_two_level_error_bounds(bits):
    """The second level is within half its own step of the residual, its step
    is at most 1/255 of the first level's (plus float32 rounding), and codes
    use the full range."""
    rng = np.random.default_rng(3 + bits)
    Y = (rng.standard_normal((400, 48)) * rng.uniform(0.01, 10, (400, 1))).astype(np.float32)
    mu = rng.standard_normal(48).astype(np.float32)
    c, delta, lo = lvq.encode(Y, mu, bits)
    c2, d2, l2 = lvq.encode_residual(Y, mu, c, delta, lo)
    r2 = lvq.residual(Y, mu, c, delta, lo)
    rec2 = l2.astype(np.float64)[:, None] + d2.astype(np.float64)[:, None] * c2
    mag = np.maximum(np.abs(r2.min(1)), np.abs(r2.max(1)))
    ulp = np.spacing(mag.astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(r2 - rec2) <= (d2.astype(np.float64) / 2 + 2 * ulp)[:, None])
    first_ulp = np.spacing(np.maximum(np.abs(lo), np.abs(lo + 15 * delta))).astype(np.float64)
    assert np.all(d2.astype(np.float64) <= (delta.astype(np.float64) / 2 + 2 * first_ulp)
                  * 2 / 255 * (1 + 1e-6))
    rows = np.arange(len(Y))
    assert np.all(c2[rows, r2.argmin(1)] == 0) and np.all(c2[rows, r2.argmax(1)] == 255)
    full = Y.astype(np.float64) - lvq.decode_two_level(c, delta, lo, c2, d2, l2, mu)
    one = Y.astype(np.float64) - lvq.decode(c, delta, lo, mu)
    assert np.abs(full).max() < np.abs(one).max()
