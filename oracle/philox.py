"""Philox4x32-10 and the draws the sketches take from it (oracle side).

Test infrastructure: see the package docstring.

The paper draws its sketches at random (Section 1: i.i.d. N(0, 1/m) Gaussian
entries; Appendix C.2: Rademacher signs and a uniform row subset drawn without
replacement) but names no generator.  Both this oracle and the GPU library
implement, independently, the counter-based generator Philox4x32-10 from its
published definition (J. Salmon, M. Moraes, R. Dror, D. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11): four 32-bit counter words, a 64-bit key,
ten rounds of two 32x32->64 multiplies with the key bumped by the Weyl
constants between rounds.

Stream map (counter word 2):
    4 = SRHT Rademacher signs, 5 = SRHT row keys, 6 = Gaussian sketch entries,
    7 = Hutchinson probe signs, 8 = CountSketch bucket and sign.
Counter = (idx mod 2^32, idx div 2^32, stream, sketch_id); key = (seed mod 2^32,
seed div 2^32).
"""
import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK32 = 0xFFFFFFFF

STREAM_SIGNS = 4
STREAM_ROWKEYS = 5
STREAM_GAUSS = 6
STREAM_PROBE = 7
STREAM_COUNT = 8


def philox4x32_10_scalar(counter, key):
    """One Philox4x32-10 block on Python ints: counter (4 words), key (2 words)."""
    c0, c1, c2, c3 = (int(v) & _MASK32 for v in counter)
    k0, k1 = (int(v) & _MASK32 for v in key)
    for rnd in range(10):
        prod0 = PHILOX_M0 * c0
        prod1 = PHILOX_M1 * c2
        hi0, lo0 = prod0 >> 32, prod0 & _MASK32
        hi1, lo1 = prod1 >> 32, prod1 & _MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
        if rnd != 9:
            k0 = (k0 + PHILOX_W0) & _MASK32
            k1 = (k1 + PHILOX_W1) & _MASK32
    return c0, c1, c2, c3


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 over numpy arrays of counter words.

    All arguments broadcast; each is interpreted as uint32.  Products are taken
    in uint64, which holds a 32x32-bit product exactly.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.uint64(int(k0) & _MASK32)
    k1 = np.uint64(int(k1) & _MASK32)
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    s32 = np.uint64(32)
    mask = np.uint64(_MASK32)
    for rnd in range(10):
        prod0 = m0 * c0
        prod1 = m1 * c2
        hi0, lo0 = prod0 >> s32, prod0 & mask
        hi1, lo1 = prod1 >> s32, prod1 & mask
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
        if rnd != 9:
            k0 = (k0 + np.uint64(PHILOX_W0)) & mask
            k1 = (k1 + np.uint64(PHILOX_W1)) & mask
    return c0, c1, c2, c3


def draw(seed, stream, sketch_id, idx):
    """Philox block for counter (idx, stream, sketch_id) under key=seed.

    ``idx`` is an array of non-negative int64 indices.  Returns four uint64
    arrays holding 32-bit words.
    """
    idx = np.asarray(idx, dtype=np.uint64)
    seed = int(seed)
    return philox4x32_10(idx & np.uint64(_MASK32), idx >> np.uint64(32),
                         np.uint64(stream), np.uint64(int(sketch_id) & _MASK32),
                         seed & _MASK32, (seed >> 32) & _MASK32)


def rademacher_signs(seed, sketch_id, n):
    """SRHT signs: eps_i = 1 - 2 * (word0 & 1), i = 0..n-1 (float64 +-1)."""
    w0, _, _, _ = draw(seed, STREAM_SIGNS, sketch_id, np.arange(n, dtype=np.uint64))
    return 1.0 - 2.0 * (w0 & np.uint64(1)).astype(np.float64)


def row_keys(seed, sketch_id, n):
    """SRHT row keys: key_i = word1 * 2^32 + word0 (uint64), i = 0..n-1."""
    w0, w1, _, _ = draw(seed, STREAM_ROWKEYS, sketch_id, np.arange(n, dtype=np.uint64))
    return (w1 << np.uint64(32)) | w0


def gaussian_entries(seed, sketch_id, idx, precision):
    """Standard normal draws by the Box-Muller transform, one per counter index.

    precision "f64": u1 from words (0,1), u2 from words (2,3), each as
        ((w_a >> 6) * 2^26 + (w_b >> 6) + 1/2) * 2^-52, which is exact in FP64
        and lies strictly inside (0, 1).
    precision "f32": u1 = ((w0 >> 9) + 1/2) * 2^-23, u2 = ((w1 >> 9) + 1/2) * 2^-23,
        exact in FP32.  The GPU evaluates the transform in FP32; here it is
        evaluated in FP64 from the same uniforms.
    z = sqrt(-2 ln u1) * cos(2 pi u2).
    """
    w0, w1, w2, w3 = draw(seed, STREAM_GAUSS, sketch_id, idx)
    if precision == "f64":
        u1 = ((w0 >> np.uint64(6)).astype(np.float64) * 2.0 ** 26
              + (w1 >> np.uint64(6)).astype(np.float64) + 0.5) * 2.0 ** -52
        u2 = ((w2 >> np.uint64(6)).astype(np.float64) * 2.0 ** 26
              + (w3 >> np.uint64(6)).astype(np.float64) + 0.5) * 2.0 ** -52
    elif precision == "f32":
        u1 = ((w0 >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23
        u2 = ((w1 >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23
    else:
        raise ValueError(precision)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def count_sketch_hash(seed, sketch_id, n, m):
    """CountSketch column of each row i = 0..n-1: bucket h_i = (word0 * m) >> 32
    (the high word of the product, uniform on [0, m) and refined by doubling m:
    h_i at 2m is 2 h_i or 2 h_i + 1) and sign s_i = 1 - 2 * (word1 & 1)."""
    w0, w1, _, _ = draw(seed, STREAM_COUNT, sketch_id, np.arange(n, dtype=np.uint64))
    h = ((w0 * np.uint64(m)) >> np.uint64(32)).astype(np.int64)
    return h, 1.0 - 2.0 * (w1 & np.uint64(1)).astype(np.float64)
