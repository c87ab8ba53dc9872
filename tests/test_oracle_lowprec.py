"""Pins for the oracle's BF16 / FP8-E4M3 storage: against torch's CPU
conversions (library routines) and the format's own properties."""
import numpy as np
import pytest
import torch

from oracle import lowprec


def test_e4m3_decode_covers_the_format():
    codes = np.arange(256, dtype=np.uint8)
    finite = (codes & 0x7F) != 0x7F
    vals = lowprec.e4m3_decode(codes[finite])
    assert vals.max() == 448.0 and vals.min() == -448.0
    pos = np.sort(vals[vals > 0])
    assert pos[0] == 2.0 ** -9                       # smallest subnormal
    assert 2.0 ** -6 in pos                           # smallest normal
    # decode agrees with torch's float8_e4m3fn view of the same bytes
    t = torch.from_numpy(codes[finite].copy()).view(torch.float8_e4m3fn).float().numpy()
    np.testing.assert_array_equal(vals.astype(np.float32), t)


def test_e4m3_encode_roundtrip_and_torch_rounding():
    codes = np.arange(256, dtype=np.uint8)
    finite = codes[(codes & 0x7F) != 0x7F]
    back = lowprec.e4m3_encode(lowprec.e4m3_decode(finite))
    # +0 and -0 both encode to a zero code
    nz = lowprec.e4m3_decode(finite) != 0
    np.testing.assert_array_equal(back[nz], finite[nz])
    x = np.random.default_rng(0).standard_normal(20000) * np.exp(
        np.random.default_rng(1).uniform(-9, 6, 20000))
    x = np.clip(x, -448, 448).astype(np.float32)
    ours = lowprec.e4m3_encode(x)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(ours, ref)


def test_e4m3_ties_to_even():
    # 1 + 1/16 lies halfway between 1 (code 0x38) and 1 + 1/8 (code 0x39)
    assert lowprec.e4m3_encode(np.array([1.0625]))[0] == 0x38
    assert lowprec.e4m3_encode(np.array([1.1875]))[0] == 0x3A


def test_bf16_against_torch():
    x = (np.random.default_rng(2).standard_normal(10000) * 1e3).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy().astype(np.float64)
    np.testing.assert_array_equal(lowprec.bf16_round(x), ref)


@pytest.mark.parametrize("seed", [0, 1])
def test_fp8_scales_bracket_the_column_max(seed):
    SA = np.random.default_rng(seed).standard_normal((50, 30)) * np.exp2(
        np.random.default_rng(seed + 5).integers(-20, 20, 30))[None, :]
    SA[:, 3] = 0.0
    codes, s, deq = lowprec.fp8_quantize(SA)
    mx = np.abs(SA).max(0)
    ok = mx > 0
    assert np.all(mx[ok] / s[ok] <= 448) and np.all(mx[ok] / s[ok] > 224)
    assert s[3] == 1.0 and np.all(deq[:, 3] == 0)
    assert np.all(np.log2(s) == np.round(np.log2(s)))
    # relative error of a 3-bit mantissa, away from the subnormal range
    big = np.abs(SA) > 2.0 ** -6 * s[None, :]
    assert np.max(np.abs(deq - SA)[big] / np.abs(SA)[big]) <= 2.0 ** -4 + 1e-12
