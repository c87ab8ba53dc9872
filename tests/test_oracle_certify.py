"""Pins of the streamed error certificate (oracle/certify.py), CPU only.

The certificate replaces x* at sizes where the FP64 Gram is out of reach, so it is
pinned against the direct solution on small problems:
* with k = d the Nystrom approximation is A^T A itself, so the upper bound equals
  delta(x) = 1/2 (x - x*)^T H (x - x*) (Section 1.1) for any x, and the dual lower
  bound equals delta(0) at x = x*;
* with k < d the ratio never falls below the exact delta(x) / delta(0), for points
  far from and near x*, and stays within the (lambda_{k+1} + nu^2) / nu^2 factor;
* the sums do not depend on how the rows are split into blocks.
"""
import numpy as np
import pytest

from oracle import ridge
from oracle.certify import StreamedCertificate
from synth import make_problem, spectrum


def _problem(n=600, d=48, nu2=1e-3, seed=3):
    p = make_problem(n, d, spectrum("poly", d, 1.0), nu2, 0.1, seed, dtype=np.float64)
    return p.A, p.b, nu2


def _points(A, b, nu2, rng):
    xs = ridge.solve_svd(A, b, nu2)
    d = A.shape[1]
    pts = [np.zeros(d), rng.standard_normal(d),
           xs + 1e-3 * rng.standard_normal(d), xs + 1e-6 * rng.standard_normal(d), xs]
    return xs, np.stack(pts, axis=1)


def _exact(A, nu2, x, xs):
    return ridge.delta(ridge.hessian(A, nu2), x, xs)


@pytest.mark.parametrize("nu2", [1e-2, 1e-4])
def test_full_rank_nystrom_is_exact(nu2):
    A, b, _ = _problem(nu2=nu2)
    rng = np.random.default_rng(1)
    xs, X = _points(A, b, nu2, rng)
    C = StreamedCertificate(A.shape[1], X, k=A.shape[1], seed=7)
    C.add(A, b)
    d0 = _exact(A, nu2, np.zeros_like(xs), xs)
    for j, (up, lo, ratio) in enumerate(C.bounds(nu2)):
        want = _exact(A, nu2, X[:, j], xs)
        assert abs(up - want) <= 1e-8 * want + 1e-18
        assert lo <= d0 * (1 + 1e-12)
    # the dual bound is exact at x = x*
    _, lo_star, _ = C.bounds(nu2, cols=[X.shape[1] - 1])[0]
    assert abs(lo_star - d0) <= 1e-10 * d0


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("k", [4, 16, 32])
def test_bound_never_below_exact(seed, k):
    nu2 = 1e-4
    A, b, _ = _problem(nu2=nu2, seed=seed + 10)
    rng = np.random.default_rng(seed)
    xs, X = _points(A, b, nu2, rng)
    C = StreamedCertificate(A.shape[1], X[:, :-1], k=k, seed=seed)
    C.add(A, b)
    d0 = _exact(A, nu2, np.zeros_like(xs), xs)
    s = np.linalg.svd(A, compute_uv=False)
    lam_next = s[k] ** 2 if k < len(s) else 0.0
    for j, (up, lo, ratio) in enumerate(C.bounds(nu2)):
        want = _exact(A, nu2, X[:, j], xs) / d0
        assert ratio >= want * (1 - 1e-10)
        # loose by at most (lambda_{k+1} + nu^2) / nu^2 on delta(x), and by the
        # dual bound's own slack on delta(0) (small near x*)
        if j >= 2:
            assert ratio <= want * 1.01 * (lam_next + nu2) / nu2 * (d0 / max(lo, 1e-300))


def test_row_blocks_do_not_change_the_sums():
    A, b, nu2 = _problem()
    rng = np.random.default_rng(5)
    _, X = _points(A, b, nu2, rng)
    one = StreamedCertificate(A.shape[1], X, k=20, seed=9)
    one.add(A, b)
    many = StreamedCertificate(A.shape[1], X, k=20, seed=9)
    for r0, r1 in ((0, 77), (77, 300), (300, 301), (301, A.shape[0])):
        many.add(A[r0:r1], b[r0:r1])
    for a, c in zip(one.bounds(nu2), many.bounds(nu2)):
        np.testing.assert_allclose(a, c, rtol=1e-9, atol=1e-20)


def test_per_column_nu2():
    """Points of different nu^2 in one pass: each column uses its own shift."""
    A, b, _ = _problem()
    rng = np.random.default_rng(8)
    nus = (1e-2, 1e-4)
    xs = [ridge.solve_svd(A, b, nu) + 1e-4 * rng.standard_normal(A.shape[1]) for nu in nus]
    C = StreamedCertificate(A.shape[1], np.stack(xs, axis=1), k=A.shape[1], seed=2)
    C.add(A, b)
    got = C.bounds(np.array(nus))
    for j, nu in enumerate(nus):
        xst = ridge.solve_svd(A, b, nu)
        want = _exact(A, nu, xs[j], xst)
        assert abs(got[j][0] - want) <= 1e-8 * want
