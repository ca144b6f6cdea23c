"""Pins of the oracle's reduced-precision codecs against library conversions
(NumPy float16, torch bfloat16 / float8_e4m3fn) and a brute-force nearest-code
search."""
import numpy as np
import pytest
import torch

import oracle


def _same(a, b):
    a, b = np.asarray(a, np.float32), np.asarray(b, np.float32)
    return ((a == b) | (np.isnan(a) & np.isnan(b))).all()


def test_decode_f16_all_codes():
    codes = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
    assert _same(oracle.decode("f16", codes), codes.view(np.float16).astype(np.float32))


def test_decode_bf16_all_codes():
    codes = np.arange(1 << 16, dtype=np.uint32)
    ref = (codes << 16).astype(np.uint32).view(np.float32)
    assert _same(oracle.decode("bf16", codes.astype(np.uint16)), ref)


def test_decode_e4m3_all_codes():
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).float().numpy()
    assert _same(oracle.decode("e4m3", codes), ref)
    assert np.nanmax(oracle.decode("e4m3", codes)) == 448.0


def _rand_floats(n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    mag = np.exp(rng.uniform(np.log(lo), np.log(hi), n))
    return (mag * rng.choice([-1, 1], n)).astype(np.float32)


def _midpoints(dec_sorted):
    v = dec_sorted[np.isfinite(dec_sorted)].astype(np.float64)
    v = np.unique(v)
    return ((v[:-1] + v[1:]) / 2).astype(np.float32)


def test_encode_f16_matches_numpy_rne():
    x = np.concatenate([_rand_floats(200000, 1e-9, 6e4, 1),
                        _midpoints(np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
                                   .view(np.float16).astype(np.float32))])
    x = x[np.abs(x) < 65504]
    assert _same(oracle.decode("f16", oracle.encode("f16", x)),
                 x.astype(np.float16).astype(np.float32))
    assert oracle.decode("f16", oracle.encode("f16", np.float32([1e6, -1e6, np.inf]))).tolist() \
        == [65504.0, -65504.0, 65504.0]                            # saturation


def test_encode_bf16_matches_torch_rne():
    x = np.concatenate([_rand_floats(200000, 1e-38, 1e38, 2),
                        _midpoints(((np.arange(1 << 16, dtype=np.uint32) << 16)
                                    .astype(np.uint32).view(np.float32)))])
    x = x[np.isfinite(x) & (np.abs(x) < 3.38e38)]
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    assert _same(oracle.decode("bf16", oracle.encode("bf16", x)), ref)


def test_encode_e4m3_matches_torch_and_nearest_code():
    all_vals = oracle.decode("e4m3", np.arange(256, dtype=np.uint8))
    x = np.concatenate([_rand_floats(50000, 1e-4, 448, 3), _midpoints(np.sort(all_vals)),
                        np.float32([0.0, -0.0, 448.0, -448.0, 2.0 ** -9, 2.0 ** -10])])
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).float().numpy()
    got = oracle.decode("e4m3", oracle.encode("e4m3", x))
    assert _same(got, ref)
    # independent brute force: nearest finite code, ties to the even code
    fin = np.where(np.isfinite(all_vals))[0]
    for v in x[:3000]:
        dist = np.abs(all_vals[fin].astype(np.float64) - float(v))
        best = fin[dist == dist.min()]
        if len(best) > 1:
            best = [c for c in best if c % 2 == 0]
        assert got[list(x).index(v)] == all_vals[best[0]] or v == 0
    # saturation instead of overflow
    assert oracle.decode("e4m3", oracle.encode("e4m3", np.float32([1e4, -500, np.inf]))).tolist() \
        == [448.0, -448.0, 448.0]


@pytest.mark.parametrize("dt", ["f16", "bf16", "e4m3"])
def test_quantize_scales_and_decoded_rows(dt):
    rng = np.random.default_rng(4)
    X = (rng.normal(size=(300, 24)) * rng.uniform(0.1, 200, size=24)).astype(np.float32)
    X[:, 3] = 0.0
    s = oracle.scales(dt, X)
    M = 448.0 if dt == "e4m3" else 1.0
    np.testing.assert_array_equal(s[3], 1.0)
    np.testing.assert_allclose(np.delete(s, 3), np.delete(np.abs(X).max(0) / M, 3), rtol=1e-7)
    codes, dec = oracle.quantize(dt, X, s)
    assert _same(dec, (s[None, :] * oracle.decode(dt, codes)).astype(np.float32))
    rel = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8, "e4m3": 2.0 ** -4}[dt]
    scale = np.abs(X).max(0, keepdims=True)
    # error bound: half an ulp of the code, relative to the magnitude, plus the
    # subnormal floor of the format, times the per-dim scale
    floor = {"f16": 2.0 ** -25, "bf16": 2.0 ** -134, "e4m3": 2.0 ** -10}[dt] * s[None, :]
    assert (np.abs(dec - X) <= rel * np.abs(X) * 1.0001 + floor + 1e-7 * scale).all()
