"""Pins for the oracle's generator and embeddings (CPU only).

Every check here is anchored outside the oracle's own formulas: published
known-answer vectors, a library Hadamard construction, exact orthogonality
identities, and distributional properties of the embeddings.
"""
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from oracle import philox, sketch

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(v, 16) for v in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat_rows())
def test_philox_known_answers_scalar(ctr, key, out):
    assert list(philox.philox4x32_10_scalar(ctr, key)) == out


@pytest.mark.parametrize("ctr,key,out", _kat_rows())
def test_philox_known_answers_vectorised(ctr, key, out):
    got = philox.philox4x32_10(*[np.array([c]) for c in ctr], key[0], key[1])
    assert [int(g[0]) for g in got] == out


def test_philox_vectorised_matches_scalar_on_draw_counters():
    idx = np.array([0, 1, 2, 12345, 2**32 - 1, 2**32, 2**40 + 7], dtype=np.uint64)
    seed = 0x123456789ABCDEF0
    w = philox.draw(seed, philox.STREAM_ROWKEYS, 9, idx)
    for j, i in enumerate(idx):
        i = int(i)
        ref = philox.philox4x32_10_scalar(
            (i & 0xFFFFFFFF, i >> 32, philox.STREAM_ROWKEYS, 9),
            (seed & 0xFFFFFFFF, seed >> 32))
        assert tuple(int(x[j]) for x in w) == ref


def test_signs_are_balanced_rademacher():
    eps = philox.rademacher_signs(3, 0, 1 << 16)
    assert set(np.unique(eps)) == {-1.0, 1.0}
    # binomial: mean within 5 sigma of 0
    assert abs(eps.mean()) < 5.0 / np.sqrt(eps.size)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gaussian_entries_are_standard_normal(prec):
    z = philox.gaussian_entries(11, 2, np.arange(200000, dtype=np.uint64), prec)
    assert np.all(np.isfinite(z))
    ks = scipy.stats.kstest(z, "norm")
    assert ks.pvalue > 1e-4
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 0.02


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64, 128])
def test_hadamard_entries_match_sylvester_library(n):
    idx = np.arange(n)
    H = sketch.hadamard_entries(idx, idx)
    assert np.array_equal(H, scipy.linalg.hadamard(n).astype(np.float64))


def test_hadamard_orthogonality_and_involution():
    n = 256
    idx = np.arange(n)
    H = sketch.hadamard_entries(idx, idx)
    assert np.array_equal(H @ H.T, n * np.eye(n))
    x = np.random.default_rng(0).integers(-50, 50, size=(n, 3)).astype(np.float64)
    assert np.array_equal(H @ (H @ x), n * x)


@pytest.mark.parametrize("n,m", [(64, 1), (64, 7), (100, 33), (128, 128), (1000, 1024)])
def test_srht_rows_without_replacement_ascending(n, m):
    rows = sketch.srht_rows(5, 3, n, m)
    npad = sketch.next_pow2(n)
    assert rows.size == m
    assert np.all(np.diff(rows) > 0)
    assert rows.min() >= 0 and rows.max() < npad


def test_srht_rows_are_smallest_keys_brute_force():
    n, m, seed, sid = 37, 11, 17, 4
    npad = sketch.next_pow2(n)
    keys = [philox.philox4x32_10_scalar((i, 0, philox.STREAM_ROWKEYS, sid), (seed, 0))
            for i in range(npad)]
    keys = [(k[1] << 32) | k[0] for k in keys]
    want = sorted(sorted(range(npad), key=lambda i: (keys[i], i))[:m])
    assert list(sketch.srht_rows(seed, sid, n, m)) == want


def test_srht_nested_rows_are_supersets():
    prev = None
    for m in [1, 2, 4, 8, 16, 32, 64]:
        rows = set(sketch.srht_rows(1, 0, 64, m))
        if prev is not None:
            assert prev <= rows
        prev = rows


def test_srht_rows_uniform_inclusion():
    n, m, trials = 32, 8, 3000
    counts = np.zeros(n)
    for sid in range(trials):
        counts[sketch.srht_rows(2, sid, n, m)] += 1
    expect = trials * m / n
    # each index is included w.p. m/n; 6 sigma band
    sd = np.sqrt(trials * (m / n) * (1 - m / n))
    assert np.all(np.abs(counts - expect) < 6 * sd)


def _srht_matrix(seed, sid, n, m):
    """S built by sketching the identity with the oracle's SRHT."""
    SA, _ = sketch.srht_sketch(np.eye(n), seed, sid, m)
    return SA


@pytest.mark.parametrize("n,m", [(64, 8), (64, 64), (128, 20)])
def test_srht_rows_orthogonal(n, m):
    S = _srht_matrix(7, 1, n, m)
    np.testing.assert_allclose(S @ S.T, (n / m) * np.eye(m), atol=1e-12)


def test_srht_full_sample_is_isometry():
    n = 64
    S = _srht_matrix(7, 2, n, n)
    np.testing.assert_allclose(S.T @ S, np.eye(n), atol=1e-12)


def test_srht_padding_ignores_padded_rows():
    rng = np.random.default_rng(1)
    n, d, m = 100, 5, 40
    A = rng.standard_normal((n, d))
    Apad = np.vstack([A, np.zeros((28, d))])
    SA, _ = sketch.srht_sketch(A, 3, 0, m)
    SAp, _ = sketch.srht_sketch(Apad, 3, 0, m)
    np.testing.assert_allclose(SA, SAp, atol=1e-12)


def test_srht_expectation_is_identity_monte_carlo():
    n, m, trials = 32, 4, 2000
    acc = np.zeros((n, n))
    for sid in range(trials):
        S = _srht_matrix(9, sid, n, m)
        acc += S.T @ S
    acc /= trials
    assert np.max(np.abs(acc - np.eye(n))) < 0.25
    assert abs(np.trace(acc) - n) < 1e-9 * n    # trace(S^T S) = n exactly


def test_srht_rows_are_sign_flipped_hadamard_rows():
    n, m = 16, 5
    S = _srht_matrix(4, 6, n, m)
    rows = sketch.srht_rows(4, 6, n, m)
    eps = sketch.srht_signs(4, 6, n)
    H = scipy.linalg.hadamard(n).astype(np.float64)
    np.testing.assert_allclose(S, H[rows] * eps[None, :] / np.sqrt(m), atol=1e-15)


def test_gaussian_sketch_variance_and_expectation():
    n, m = 40, 50
    S = sketch.gaussian_matrix(1, 0, m, n)
    # entries N(0, 1/m)
    assert abs(S.var() * m - 1.0) < 0.05
    acc = np.zeros((n, n))
    trials = 200
    for sid in range(trials):
        S = sketch.gaussian_matrix(2, sid, 8, n)
        acc += S.T @ S
    acc /= trials
    assert np.max(np.abs(acc - np.eye(n))) < 0.5
    assert abs(np.trace(acc) / n - 1.0) < 0.05


def test_gaussian_sketch_equals_matrix_product():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((30, 4))
    SA = sketch.gaussian_sketch(A, 5, 1, 7)
    S = sketch.gaussian_matrix(5, 1, 7, 30)
    np.testing.assert_allclose(SA, S @ A, atol=1e-12)


def test_gaussian_marchenko_pastur_edges():
    # Remark 3.1: spectrum of U^T S^T S U approaches (1 +- sqrt(d/m))^2
    rng = np.random.default_rng(5)
    n, d, m = 2048, 20, 400
    U, _ = np.linalg.qr(rng.standard_normal((n, d)))
    SU = sketch.gaussian_sketch(U, 3, 0, m)
    ev = np.linalg.eigvalsh(SU.T @ SU)
    r = d / m
    assert ev.min() > (1 - np.sqrt(r)) ** 2 - 0.1
    assert ev.max() < (1 + np.sqrt(r)) ** 2 + 0.1
