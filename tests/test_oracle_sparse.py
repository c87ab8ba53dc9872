"""Pins for the oracle's CountSketch and the sparse-A solve (CPU only)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import ihs, philox, ridge, sketch


@pytest.fixture(scope="module")
def sparse_problem():
    rng = np.random.default_rng(3)
    A = sp.random(3000, 60, density=0.08, random_state=4, format="csr",
                  data_rvs=rng.standard_normal)
    b = rng.standard_normal(3000)
    return A, b, 1.0


def test_count_sketch_matches_scatter_of_signed_rows(sparse_problem):
    # brute force: SA[h_i] += s_i * A[i], row by row
    A, _, _ = sparse_problem
    m = 37
    h, s = philox.count_sketch_hash(5, 2, A.shape[0], m)
    ref = np.zeros((m, A.shape[1]))
    Ad = A.toarray()
    for i in range(A.shape[0]):
        ref[h[i]] += s[i] * Ad[i]
    np.testing.assert_allclose(sketch.count_sketch(A, 5, 2, m), ref, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(sketch.count_sketch(Ad, 5, 2, m), ref, rtol=1e-13, atol=1e-13)


def test_count_sketch_hash_distribution_and_nesting():
    n, m = 200000, 64
    h, s = philox.count_sketch_hash(1, 0, n, m)
    assert h.min() >= 0 and h.max() < m
    counts = np.bincount(h, minlength=m)
    chi2 = np.sum((counts - n / m) ** 2 / (n / m))
    assert chi2 < 130                     # 63 degrees of freedom: p ~ 1e-6 cut
    assert abs(s.mean()) < 5 / np.sqrt(n)
    h2, s2 = philox.count_sketch_hash(1, 0, n, 2 * m)
    assert np.all(h2 // 2 == h) and np.array_equal(s2, s)


def test_count_sketch_is_unbiased():
    # S^T S has a unit diagonal exactly and E[(SA)^T SA] = A^T A
    rng = np.random.default_rng(2)
    A = rng.standard_normal((200, 5))
    acc = np.zeros((5, 5))
    trials = 400
    for sid in range(trials):
        SA = sketch.count_sketch(A, 9, sid, 16)
        acc += SA.T @ SA
    G = A.T @ A
    assert np.max(np.abs(acc / trials - G)) <= 0.1 * np.max(np.abs(G))
    h, s = philox.count_sketch_hash(9, 0, 200, 16)
    S = np.zeros((16, 200))
    S[h, np.arange(200)] = s
    np.testing.assert_array_equal(np.diag(S.T @ S), np.ones(200))


def test_single_bucket_sums_signed_rows(sparse_problem):
    A, _, _ = sparse_problem
    h, s = philox.count_sketch_hash(3, 0, A.shape[0], 1)
    assert np.all(h == 0)
    np.testing.assert_allclose(sketch.count_sketch(A, 3, 0, 1)[0], A.T @ s, rtol=1e-12,
                               atol=1e-12)


def test_sparse_gradient_equals_dense(sparse_problem):
    A, b, nu2 = sparse_problem
    x = np.random.default_rng(8).standard_normal(A.shape[1])
    np.testing.assert_allclose(ridge.sparse_gradient(A, b, nu2, x),
                               ridge.gradient(A.toarray(), b, nu2, x), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("variant", ["gd", "polyak"])
@pytest.mark.parametrize("resample", ["fresh", "nested"])
def test_sparse_solve_reaches_direct_solution(sparse_problem, variant, resample):
    A, b, nu2 = sparse_problem
    x, info = ihs.adaptive_solve_sparse(A, b, nu2, ihs.Options(kind="count", variant=variant,
                                                               resample=resample, tol=1e-10))
    assert info.status == "ok"
    Ad = A.toarray()
    assert ridge.relative_error(ridge.hessian(Ad, nu2), x, ridge.solve_direct(Ad, b, nu2)) <= 1e-8
    assert info.m_final == min(2 ** info.doublings, A.shape[0])
    # the same run on the dense copy takes the same steps
    xd, infod = ihs.adaptive_solve(Ad, b, nu2, ihs.Options(kind="count", variant=variant,
                                                           resample=resample, tol=1e-10))
    assert infod.events == info.events
    np.testing.assert_allclose(x, xd, rtol=1e-9, atol=1e-12)
