"""Pins for the oracle's underdetermined case (appendix: the dual problem), CPU only."""
import numpy as np
import pytest

from oracle import ihs, ridge
from synth import make_problem, spectrum


@pytest.fixture(scope="module")
def wide():
    # n < d: the transpose of a tall problem with sigma_i = 0.9^i
    p = make_problem(1024, 64, spectrum("geom", 64, 0.9), 1e-2, 0.01, 5, dtype=np.float64)
    A = np.ascontiguousarray(p.A.T)              # 64 x 1024
    rng = np.random.default_rng(9)
    b = rng.standard_normal(64)
    return A, b, 1e-2


def test_dual_optimum_maps_to_the_primal_solution(wide):
    # x* = A^T z*, against the primal normal equations and the SVD closed form
    A, b, nu2 = wide
    x = A.T @ ridge.solve_dual_direct(A, b, nu2)
    np.testing.assert_allclose(x, ridge.solve_svd(A, b, nu2), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(x, ridge.solve_direct(A, b, nu2), rtol=1e-8, atol=1e-11)


def test_dual_gradient_is_the_dual_objectives_gradient(wide):
    A, b, nu2 = wide

    def g(z):
        return 0.5 * np.sum((A.T @ z) ** 2) + 0.5 * nu2 * np.sum(z ** 2) - b @ z

    z = np.random.default_rng(1).standard_normal(A.shape[0])
    h = 1e-5
    fd = np.array([(g(z + h * e) - g(z - h * e)) / (2 * h) for e in np.eye(A.shape[0])])
    np.testing.assert_allclose(ridge.dual_gradient(A, b, nu2, z), fd, rtol=1e-6, atol=1e-6)
    zs = ridge.solve_dual_direct(A, b, nu2)
    assert np.linalg.norm(ridge.dual_gradient(A, b, nu2, zs)) <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("kind", ["srht", "gaussian"])
@pytest.mark.parametrize("variant", ["polyak", "gd"])
def test_dual_solve_reaches_the_primal_solution(wide, kind, variant):
    A, b, nu2 = wide
    x, z, info = ihs.adaptive_solve_dual(A, b, nu2, ihs.Options(kind=kind, variant=variant,
                                                                  tol=1e-10))
    assert info.status == "ok"
    H = ridge.hessian(A, nu2)
    assert ridge.relative_error(H, x, ridge.solve_svd(A, b, nu2)) <= 1e-8
    # the sketch acts on the d rows of A^T: m is bounded by the padded d
    assert info.m_final <= 1024


def test_dual_is_the_primal_algorithm_on_the_transpose_with_pseudo_inverse_rhs(wide):
    # the appendix: the dual equals the primal problem with data A^T and b^ = A^+ b,
    # so Algorithm 1 takes the same steps on both (same sketches: same seed, same rows)
    A, b, nu2 = wide
    bh = np.linalg.pinv(A) @ b
    opts = ihs.Options(tol=1e-9, seed=4)
    x, z, info = ihs.adaptive_solve_dual(A, b, nu2, opts)
    zp, infop = ihs.adaptive_solve(A.T, bh, nu2, opts)
    assert info.events == infop.events
    np.testing.assert_allclose(z, zp, rtol=1e-7, atol=1e-10)


def test_primal_error_of_a_dual_iterate(wide):
    # delta(A^T z) = 1/2 |A A^T (z - z*)|^2 + nu^2/2 |A^T (z - z*)|^2 <= sigma_1^2 eps(z)
    A, b, nu2 = wide
    zs = ridge.solve_dual_direct(A, b, nu2)
    xs = A.T @ zs
    s1 = np.linalg.svd(A, compute_uv=False)[0]
    for tol in (1e-2, 1e-4, 1e-6):
        _, z, _ = ihs.adaptive_solve_dual(A, b, nu2, ihs.Options(tol=tol, seed=2))
        e = z - zs
        eps = 0.5 * np.sum((A.T @ e) ** 2) + 0.5 * nu2 * np.sum(e ** 2)
        x = A.T @ z
        delta = 0.5 * np.sum((A @ (x - xs)) ** 2) + 0.5 * nu2 * np.sum((x - xs) ** 2)
        assert delta == pytest.approx(0.5 * np.sum((A @ A.T @ e) ** 2)
                                      + 0.5 * nu2 * np.sum((A.T @ e) ** 2), rel=1e-9)
        assert delta <= s1 ** 2 * eps * (1 + 1e-12)


def test_dual_start_at_origin_has_reference_minus_b(wide):
    # z_0 = 0: g(0) = -b, so r_1 = 1/2 b^T H_S^-1 b under the first sketch
    A, b, nu2 = wide
    _, _, info = ihs.adaptive_solve_dual(A, b, nu2, ihs.Options(m_init=1024, tol=1e-3))
    Hs = A @ A.T + nu2 * np.eye(A.shape[0])      # m = padded d: the SRHT is exact
    assert info.r_history[0] == pytest.approx(0.5 * b @ np.linalg.solve(Hs, b), rel=1e-10)
