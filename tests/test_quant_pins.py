"""Pins of the reference quantisers against torch's CPU casts (library routines).

BF16 is round-to-nearest-even from FP32.  FP8 is OCP E4M3 ("e4m3fn"), the
format gfx950's FP8 instructions use; torch's cast is non-saturating above the
largest finite value, so saturation is checked separately, from the format's
definition.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import quant


def _sweep(seed=0, count=200_000):
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 2 ** 32, size=count, dtype=np.uint64).astype(np.uint32)
    v = bits.view(np.float32)
    v = v[np.isfinite(v)]
    specials = np.array([0.0, -0.0, 1.0, -1.0, 1e-40, -1e-40, 3.4e38, -3.4e38,
                         np.float32(1.00390625), np.float32(1.01171875)], np.float32)
    return np.concatenate([v, specials, rng.standard_normal(count).astype(np.float32)])


def test_bf16_matches_torch():
    v = _sweep()
    ref = torch.from_numpy(v).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    got = quant.bf16_codes(v)
    assert np.array_equal(got, ref)
    assert np.array_equal(quant.bf16_decode(got).view(np.uint32),
                          torch.from_numpy(v).to(torch.bfloat16).float().numpy().view(np.uint32))


def test_fp8_decode_all_codes_match_torch():
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).float().numpy()
    got = quant.fp8_decode(codes)
    nan = np.isnan(ref)
    assert np.array_equal(nan, np.isnan(got))
    assert nan.sum() == 2 and nan[0x7F] and nan[0xFF]
    assert np.array_equal(got[~nan].view(np.uint32), ref[~nan].view(np.uint32))


def test_fp8_encode_matches_torch_in_range():
    rng = np.random.default_rng(1)
    vals = quant.fp8_decode(np.arange(256, dtype=np.uint8)).astype(np.float64)
    vals = np.unique(vals[np.isfinite(vals)])
    mids = 0.5 * (vals[1:] + vals[:-1])          # exact ties: RNE decides
    v = np.concatenate([
        vals, mids, np.nextafter(mids, np.inf), np.nextafter(mids, -np.inf),
        rng.uniform(-448, 448, 100_000), rng.standard_normal(100_000) * 1e-2,
        rng.standard_normal(100_000) * 1e-3,
    ]).astype(np.float32)
    v = v[np.abs(v) <= 448]
    ref = torch.from_numpy(v).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = quant.fp8_codes(v)
    assert np.array_equal(got, ref)


def test_fp8_saturates():
    v = np.array([448.0, 449.0, 464.0, 500.0, 1e6, 3e38, -500.0, -3e38], np.float32)
    got = quant.fp8_codes(v)
    assert got.tolist() == [0x7E] * 6 + [0xFE] * 2


@pytest.mark.parametrize("seed", [0, 1])
def test_fp8_column_round_trip(seed):
    """Per-column scale s = amax/448: the column's largest entry maps to 448,
    and every entry is within half an e4m3 step of its scaled value."""
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal((256, 64)).astype(np.float32)
    psi /= np.linalg.norm(psi, axis=0)
    psi[:, 5] = 0.0
    codes, s = quant.fp8_quantise(psi)
    assert s[5] == 1.0 and not codes[:, 5].any()
    deq = quant.fp8_decode(codes).astype(np.float64) * s[None, :].astype(np.float64)
    q = psi.astype(np.float64) / s[None, :]
    # e4m3 spacing: 2^(e-3) for normals, 2^-9 for subnormals
    e = np.floor(np.log2(np.maximum(np.abs(q), 2.0 ** -6)))
    half_step = 0.5 * np.exp2(e - 3)
    assert np.all(np.abs(quant.fp8_decode(codes) - q) <= half_step * (1 + 1e-6) + 1e-7)
    assert np.all(np.max(np.abs(codes.astype(np.int32) & 0x7F), axis=0)[[0, 1, 2]] == 0x7E)
    assert np.allclose(deq, psi, atol=0.07 * np.abs(psi).max())
