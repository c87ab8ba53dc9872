"""Low-precision storage formats of the sketch (oracle side).

Test infrastructure: see the package docstring.

BF16: FP32 with the low 16 bits rounded off to nearest even.
FP8 E4M3 (OCP 8-bit floating point, "FN" flavour): 1 sign, 4 exponent bits with
bias 7, 3 mantissa bits, subnormals M * 2^-9, largest finite value 448, no
infinities.  Encoding rounds to nearest, ties to even.  The sketch's columns
carry power-of-two scales s_j = 2^ceil(log2(max_k |SA[k, j]| / 448)) (1 for a
zero column), so stored codes are e4m3(SA[k, j] / s_j).
"""
import numpy as np


def e4m3_decode(code):
    code = np.asarray(code, dtype=np.uint8)
    s = np.where(code & 0x80, -1.0, 1.0)
    E = (code >> 3) & 0xF
    M = (code & 7).astype(np.float64)
    val = np.where(E == 0, M * 2.0 ** -9, (1.0 + M / 8.0) * np.exp2(E.astype(np.float64) - 7.0))
    return s * val


def _all_finite_codes():
    codes = np.arange(256, dtype=np.uint8)
    keep = (codes & 0x7F) != 0x7F        # 0x7f / 0xff are NaN
    return codes[keep]


_POS = None


def e4m3_encode(x):
    """Round to the nearest representable E4M3 value (ties to the even code);
    magnitudes above 448 saturate to 448."""
    global _POS
    if _POS is None:
        codes = np.arange(0, 0x7F, dtype=np.uint8)        # non-negative finite codes
        _POS = (codes, e4m3_decode(codes))
    codes, vals = _POS
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), 448.0)
    idx = np.searchsorted(vals, a)                        # vals ascending with the code
    idx = np.clip(idx, 1, len(vals) - 1)
    lo, hi = vals[idx - 1], vals[idx]
    pick_hi = (a - lo > hi - a) | ((a - lo == hi - a) & (codes[idx] % 2 == 0))
    c = np.where(pick_hi, codes[idx], codes[idx - 1]).astype(np.uint8)
    c = np.where(a == 0.0, 0, c).astype(np.uint8)
    return np.where(x < 0, c | 0x80, c).astype(np.uint8)


def pow2_scales(SA):
    """Per-column power-of-two scales mapping the column maximum into (224, 448]."""
    mx = np.max(np.abs(np.asarray(SA, dtype=np.float64)), axis=0)
    s = np.ones_like(mx)
    nz = mx > 0
    s[nz] = np.exp2(np.ceil(np.log2(mx[nz] / 448.0)))
    return s


def fp8_quantize(SA, scales=None):
    """(codes, scales, dequantized values) of a sketch stored in E4M3."""
    SA = np.asarray(SA, dtype=np.float64)
    s = pow2_scales(SA) if scales is None else np.asarray(scales, dtype=np.float64)
    codes = e4m3_encode(SA / s[None, :])
    return codes, s, e4m3_decode(codes) * s[None, :]


def bf16_round(x):
    """Round FP32 values to BF16 (nearest even), returned as float64."""
    f = np.asarray(x, dtype=np.float32).copy()
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
