"""Pins for the oracle's ridge solution, Hessian sketch and Algorithm 1 (CPU only)."""
import math

import numpy as np
import pytest

from oracle import ihs, ridge, sketch
from synth import config_c1, make_problem, spectrum


@pytest.fixture(scope="module")
def small():
    return make_problem(256, 16, spectrum("geom", 16, 0.8), 1e-2, 0.05, 3,
                        dtype=np.float64)


def test_direct_solution_matches_svd_closed_form(small):
    x1 = ridge.solve_direct(small.A, small.b, small.nu2)
    x2 = ridge.solve_svd(small.A, small.b, small.nu2)
    np.testing.assert_allclose(x1, x2, rtol=1e-11, atol=1e-13)


def test_gradient_vanishes_at_solution(small):
    xs = ridge.solve_direct(small.A, small.b, small.nu2)
    g = ridge.gradient(small.A, small.b, small.nu2, xs)
    assert np.linalg.norm(g) < 1e-13 * np.linalg.norm(small.A.T @ small.b)


def test_gradient_matches_finite_differences(small):
    rng = np.random.default_rng(0)
    x = rng.standard_normal(small.A.shape[1])

    def f(v):
        r = small.A @ v - small.b
        return 0.5 * r @ r + 0.5 * small.nu2 * v @ v

    g = ridge.gradient(small.A, small.b, small.nu2, x)
    h = 1e-6
    for j in range(small.A.shape[1]):
        e = np.zeros_like(x)
        e[j] = h
        assert abs((f(x + e) - f(x - e)) / (2 * h) - g[j]) < 1e-6


def test_effective_dimension_trace_matches_svd(small):
    a = ridge.effective_dimension_trace(small.A, small.nu2)
    b = ridge.effective_dimension_svd(small.A, small.nu2)
    assert abs(a - b) < 1e-10 * b
    # ratio form differs by the factor ||D||_2^2 <= 1
    c = ridge.effective_dimension_ratio(small.A, small.nu2)
    s1 = np.linalg.svd(small.A, compute_uv=False)[0]
    assert abs(c - b * (s1 * s1 + small.nu2) / (s1 * s1)) < 1e-10 * c


def test_delta_is_stacked_norm(small):
    xs = ridge.solve_direct(small.A, small.b, small.nu2)
    x = xs + np.random.default_rng(1).standard_normal(xs.size)
    Abar = np.vstack([small.A, math.sqrt(small.nu2) * np.eye(xs.size)])
    want = 0.5 * np.linalg.norm(Abar @ (x - xs)) ** 2
    H = ridge.hessian(small.A, small.nu2)
    assert abs(ridge.delta(H, x, xs) - want) < 1e-12 * want


def test_stacked_svd_reconstructs_abar(small):
    Ubar, sbar, V = ridge.stacked_svd(small.A, small.nu2)
    Abar = np.vstack([small.A, math.sqrt(small.nu2) * np.eye(V.shape[0])])
    np.testing.assert_allclose(Ubar * sbar[None, :] @ V.T, Abar, atol=1e-12)
    np.testing.assert_allclose(Ubar.T @ Ubar, np.eye(V.shape[0]), atol=1e-12)


# ------------------------------------------------------------- parameters
@pytest.mark.parametrize("rho", [0.05, 0.1, 0.25, 0.5, 0.9])
def test_srht_rate_equals_rho(rho):
    # proof of Theorem 7: c_gd(rho) = rho; Definition 3.2 gives mu_gd = 1 - rho
    p = ihs.params_for("srht", rho)
    assert abs(p.cbar_gd - rho) < 1e-14
    assert abs(p.mu_gd - (1 - rho)) < 1e-14


def test_gaussian_parameters_limits():
    p = ihs.params_for("gaussian", 0.1, 0.01)
    s2 = 1.69 * 0.1
    # Theorem 2 at lambda, Lambda = (1 -+ s)^2: the momentum equals s^2
    assert abs(p.beta_p - s2) < 1e-14 and abs(p.cbar_p - s2) < 1e-14
    assert 0 < p.cbar_gd < 1 and 0 < p.mu_gd < 1
    with pytest.raises(ValueError):
        ihs.params_for("gaussian", 0.5, 0.01)


def test_parameter_optimality_of_gradient_step():
    # mu_gd minimises max(|1 - mu/Lambda|, |1 - mu/lambda|) (proof of Theorem 1)
    lam, Lam = 0.4, 2.3
    mus = np.linspace(0.01, 2 * Lam, 20001)
    worst = np.maximum(np.abs(1 - mus / Lam), np.abs(1 - mus / lam))
    j = np.argmin(worst)
    mu = ihs.mu_gd(lam, Lam)
    assert abs(mus[j] - mu) < 2 * (mus[1] - mus[0])
    at_mu = max(abs(1 - mu / Lam), abs(1 - mu / lam))
    assert at_mu <= worst.min() + 1e-15
    assert abs(at_mu ** 2 - ihs.c_gd(lam, Lam)) < 1e-14


def test_polyak_spectral_radius():
    # Theorem 2: spectral radius of the heavy-ball matrix over [lambda, Lambda]
    # at (mu_p, beta_p) squared equals c_p.
    lam, Lam = 0.5, 1.7
    mu, beta = ihs.mu_p(lam, Lam), ihs.beta_p(lam, Lam)
    worst = 0.0
    for g in np.linspace(lam, Lam, 101):
        M = np.array([[1 + beta - mu / g, -beta], [1.0, 0.0]])
        worst = max(worst, np.max(np.abs(np.linalg.eigvals(M))))
    assert abs(worst ** 2 - ihs.c_p(lam, Lam)) < 1e-6


# --------------------------------------------------------- sketched Hessian
@pytest.mark.parametrize("m", [3, 16, 40])
def test_woodbury_matches_direct_solve(small, m):
    SA, _ = sketch.srht_sketch(small.A, 1, 0, m)
    P = ihs.SketchedHessian(SA, small.nu2)
    assert P.woodbury == (m < small.A.shape[1])
    g = np.random.default_rng(2).standard_normal(small.A.shape[1])
    HS = SA.T @ SA + small.nu2 * np.eye(small.A.shape[1])
    np.testing.assert_allclose(P.solve(g), np.linalg.solve(HS, g), rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("kind", ["srht", "gaussian"])
def test_newton_decrement_identity(small, kind):
    # Lemma 1: 1/2 g^T H_S^-1 g = 1/2 || C_S^{-1/2} Ubar^T Abar (x - x*) ||^2
    A, nu2 = small.A, small.nu2
    n, d = A.shape
    m = 24
    if kind == "srht":
        S = sketch.srht_sketch(np.eye(n), 5, 0, m)[0]
    else:
        S = sketch.gaussian_matrix(5, 0, m, n)
    P = ihs.SketchedHessian(S @ A, nu2)
    xs = ridge.solve_direct(A, small.b, nu2)
    x = xs + np.random.default_rng(3).standard_normal(d)
    _, r = P.decrement(ridge.gradient(A, small.b, nu2, x))
    Ubar, _, _ = ridge.stacked_svd(A, nu2)
    Abar = np.vstack([A, math.sqrt(nu2) * np.eye(d)])
    e = Ubar.T @ Abar @ (x - xs)
    C = ridge.c_matrix(A, nu2, S)
    want = 0.5 * e @ np.linalg.solve(C, e)
    assert abs(r - want) < 1e-9 * want


def test_error_recursion_predicts_polyak_step(small):
    # e_{t+1} = ((1+beta) I - mu C_S^-1) e_t - beta e_{t-1}  (proofs of Theorems 1-2)
    A, b, nu2 = small.A, small.b, small.nu2
    n, d = A.shape
    S = sketch.srht_sketch(np.eye(n), 2, 0, 32)[0]
    P = ihs.SketchedHessian(S @ A, nu2)
    xs = ridge.solve_direct(A, b, nu2)
    rng = np.random.default_rng(4)
    x_prev, x = rng.standard_normal(d), rng.standard_normal(d)
    mu, beta = 0.8, 0.3
    gt = P.solve(ridge.gradient(A, b, nu2, x))
    x_new = ihs.polyak_candidate(x, x_prev, gt, mu, beta)
    Ubar, _, _ = ridge.stacked_svd(A, nu2)
    Abar = np.vstack([A, math.sqrt(nu2) * np.eye(d)])
    E = lambda v: Ubar.T @ Abar @ (v - xs)
    C = ridge.c_matrix(A, nu2, S)
    pred = (1 + beta) * E(x) - mu * np.linalg.solve(C, E(x)) - beta * E(x_prev)
    np.testing.assert_allclose(E(x_new), pred, rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("m", [4, 12, 64])
def test_theorem1_per_step_bound_with_exact_extremes(small, m):
    A, b, nu2 = small.A, small.b, small.nu2
    n, d = A.shape
    S = sketch.srht_sketch(np.eye(n), 8, 1, m)[0]
    P = ihs.SketchedHessian(S @ A, nu2)
    ev = np.linalg.eigvalsh(ridge.c_matrix(A, nu2, S))
    lam, Lam = ev.min(), ev.max()
    mu = ihs.mu_gd(lam, Lam)
    H = ridge.hessian(A, nu2)
    xs = ridge.solve_direct(A, b, nu2)
    x = np.random.default_rng(m).standard_normal(d)
    for _ in range(5):
        x_new = ihs.gd_candidate(x, P.solve(ridge.gradient(A, b, nu2, x)), mu)
        ratio = ridge.delta(H, x_new, xs) / ridge.delta(H, x, xs)
        assert ratio <= ihs.c_gd(lam, Lam) * (1 + 1e-9)
        x = x_new


def test_full_srht_gradient_step_lands_on_solution(small):
    # m = n: S^T S = I, so H_S = H and one step with mu = 1 is exact
    A, b, nu2 = small.A, small.b, small.nu2
    n, d = A.shape
    SA, _ = sketch.srht_sketch(A, 0, 0, n)
    P = ihs.SketchedHessian(SA, nu2)
    x = np.random.default_rng(5).standard_normal(d)
    x1 = ihs.gd_candidate(x, P.solve(ridge.gradient(A, b, nu2, x)), 1.0)
    np.testing.assert_allclose(x1, ridge.solve_direct(A, b, nu2), rtol=1e-9, atol=1e-11)


# ------------------------------------------------------------- Algorithm 1
@pytest.fixture(scope="module")
def c1():
    p = config_c1()
    xs = ridge.solve_direct(p.A, p.b, p.nu2)
    return p, xs, ridge.hessian(p.A, p.nu2)


@pytest.mark.parametrize("kind", ["srht", "gaussian"])
@pytest.mark.parametrize("variant", ["polyak", "gd"])
@pytest.mark.parametrize("resample", ["fresh", "nested"])
def test_algorithm1_reaches_tolerance_and_invariants(c1, kind, variant, resample):
    p, xs, H = c1
    opts = ihs.Options(kind=kind, variant=variant, resample=resample, tol=1e-7)
    x, info = ihs.adaptive_solve(p.A, p.b, p.nu2, opts)
    assert info.status == "ok"
    assert ridge.relative_error(H, x, xs) <= 1e-6
    # m = m_init * 2^K
    assert info.m_final == opts.m_init * 2 ** info.doublings
    prm = ihs.params_for(kind, opts.rho, opts.eta)
    # replay the recorded r values against the tests the events claim
    r1 = info.r_history[0]
    k = 0
    for (t, ev, m) in info.events:
        if ev in ("polyak", "gd"):
            r_now = info.r_history[k]
            r_next = info.r_history[k + 1]
            if ev == "polyak":
                assert (r_next / r1) ** (1.0 / t) <= prm.cbar_p
            else:
                assert r_next / r_now <= prm.cbar_gd or m == info.m_final
            k += 1
        elif ev == "double":
            k += 1
    if variant == "gd":
        assert info.accepted_polyak == 0
    # the r proxy tracks the true error at the stop (within Lambda/lambda)
    assert info.r_history[-1] <= opts.tol * 10 * info.r_history[0] or info.doublings


def test_algorithm1_from_full_sketch_never_doubles(c1):
    p, xs, H = c1
    opts = ihs.Options(kind="srht", variant="gd", m_init=1024)
    x, info = ihs.adaptive_solve(p.A, p.b, p.nu2, opts)
    assert info.doublings == 0 and info.status == "ok"
    # C_S = I: each gradient step contracts delta by exactly rho^2
    assert info.t_final - 1 == math.ceil(math.log(opts.tol) / math.log(opts.rho ** 2))


def test_algorithm1_zero_rhs_stops_immediately(c1):
    # b = 0: x* = 0 = x_1, the gradient is exactly zero and so is r_1
    p, xs, H = c1
    x, info = ihs.adaptive_solve(p.A, np.zeros_like(p.b), p.nu2, ihs.Options())
    assert info.grad_evals == 1 and info.events[-1][1] == "stop"
    assert np.all(x == 0)


def test_algorithm1_cap_reports_no_convergence_when_stuck(c1):
    p, _, _ = c1
    opts = ihs.Options(kind="srht", variant="gd", m_max=2, max_iter=50)
    _, info = ihs.adaptive_solve(p.A, p.b, p.nu2, opts)
    assert info.m_final == 2
    assert info.status in ("ok", "no_convergence")
    assert info.status == "no_convergence" or info.r_history[-1] <= opts.tol * info.r_history[0]


def test_iteration_count_bound_after_last_doubling(c1):
    # proof of Theorem 7: T = ceil((log 2 + log(1 + s1^2/nu^2) + log(1/eps)) / log(1/rho))
    p, xs, H = c1
    opts = ihs.Options(kind="srht", variant="gd", tol=1e-7)
    x, info = ihs.adaptive_solve(p.A, p.b, p.nu2, opts)
    s1 = np.linalg.svd(p.A, compute_uv=False)[0]
    T = math.ceil((math.log(2) + math.log(1 + s1 * s1 / p.nu2) + math.log(1e7)) / math.log(10))
    last_double = max([i for i, e in enumerate(info.events) if e[1] == "double"], default=-1)
    accepted_after = sum(1 for e in info.events[last_double + 1:] if e[1] in ("gd", "polyak"))
    assert accepted_after <= T


# --- regularization path with warm starts (Section 4) ---------------------------

PATH_NU2 = [1e-1, 3e-2, 1e-2, 3e-3, 1e-3]


def test_path_reaches_direct_solution_at_every_nu(c1):
    p, _, _ = c1
    X, infos = ihs.solve_path(p.A, p.b, PATH_NU2, ihs.Options(tol=1e-8))
    for j, nu2 in enumerate(PATH_NU2):
        xs = ridge.solve_direct(p.A, p.b, nu2)
        assert infos[j].status == "ok"
        assert ridge.relative_error(ridge.hessian(p.A, nu2), X[j], xs) <= 1e-6


def test_path_first_point_is_the_cold_nested_solve(c1):
    # at x = 0 the origin reference is the start's own gradient: same arithmetic
    p, _, _ = c1
    X, infos = ihs.solve_path(p.A, p.b, PATH_NU2[:1], ihs.Options())
    x, info = ihs.adaptive_solve(p.A, p.b, PATH_NU2[0], ihs.Options(resample="nested"))
    assert np.array_equal(X[0], x)
    assert infos[0].events == info.events
    assert infos[0].grad_evals == info.grad_evals


def test_path_sketch_size_never_shrinks_and_warm_starts_pay(c1):
    p, _, _ = c1
    X, infos = ihs.solve_path(p.A, p.b, PATH_NU2, ihs.Options())
    ms = [inf.m_final for inf in infos]
    assert ms == sorted(ms)
    cold = sum(ihs.adaptive_solve(p.A, p.b, nu2, ihs.Options(resample="nested"))[1].grad_evals
               for nu2 in PATH_NU2)
    assert sum(inf.grad_evals for inf in infos) < cold


def test_path_rejects_increasing_nu(c1):
    p, _, _ = c1
    with pytest.raises(ValueError):
        ihs.solve_path(p.A, p.b, [1e-3, 1e-2], ihs.Options())


def test_warm_start_at_solution_stops_with_origin_reference(c1):
    # delta(x*) = 0 < tol * delta(0): the origin-referenced test stops at once; the
    # start-referenced test compares the (rounding-level) decrement with itself
    p, xs, _ = c1
    x, info = ihs.adaptive_solve(p.A, p.b, p.nu2, ihs.Options(ref_at_zero=True), x_init=xs)
    # g(x*) and the reference g(0), then the stop
    assert info.grad_evals == 2 and info.events == [(1, "stop", 1)]
    assert np.array_equal(x, xs)
    _, info0 = ihs.adaptive_solve(p.A, p.b, p.nu2, ihs.Options(), x_init=xs)
    assert info0.grad_evals > 1


def test_origin_reference_is_the_cold_first_decrement(c1):
    # r_ref from g(0) = -A^T b under the same sketch equals the cold run's r_1
    p, xs, _ = c1
    x0 = 0.5 * xs
    _, warm = ihs.adaptive_solve(p.A, p.b, p.nu2, ihs.Options(ref_at_zero=True, tol=1e-3), x_init=x0)
    _, cold = ihs.adaptive_solve(p.A, p.b, p.nu2, ihs.Options(tol=1e-3))
    r_cold_1 = cold.r_history[0]
    # the warm run stops once r_t <= tol * r_ref(0); r_ref(0) is the cold r_1 when
    # both runs still hold the first sketch
    if warm.doublings == 0:
        assert warm.r_history[-1] <= 1e-3 * r_cold_1 * (1 + 1e-12)
    # half-way start: delta(x0) = delta(0) / 4 exactly, so the warm r_1 is a
    # quarter of the cold one under the same sketch
    assert warm.r_history[0] == pytest.approx(r_cold_1 / 4, rel=1e-10)


# --- refreshed embeddings (Section 1, other versions of the IHS) -------------------

def test_refreshed_full_srht_contracts_by_rho_squared(c1):
    # m = padded n: every refreshed sketch is exact (H_S = H), so the gradient
    # variant contracts delta by exactly (1 - mu_gd)^2 = rho^2 per step
    p, xs, H = c1
    x = np.zeros(64)
    errs = []
    for steps in range(1, 5):
        x, info = ihs.refreshed_ihs(p.A, p.b, p.nu2, 1024, ihs.Options(variant="gd",
                                                                        max_iter=steps, tol=0.0))
        errs.append(ridge.relative_error(H, x, xs))
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 / e0 == pytest.approx(0.01, rel=1e-6)


def test_refreshed_step_follows_the_error_recursion(c1):
    # x_{t+1} - x* = (I - mu H_t^-1 H)(x_t - x*) + beta (x_t - x_{t-1}), H_t from S_t
    p, xs, H = c1
    opts = ihs.Options(kind="gaussian", variant="polyak", max_iter=2, tol=0.0, seed=6)
    m = 200
    x1, _ = ihs.refreshed_ihs(p.A, p.b, p.nu2, m, ihs.Options(**{**opts.__dict__, "max_iter": 1}))
    x2, _ = ihs.refreshed_ihs(p.A, p.b, p.nu2, m, opts)
    SA = ihs.make_sketch(p.A, "gaussian", 6, 1, m)
    Ht = SA.T @ SA + p.nu2 * np.eye(64)
    prm = ihs.params_for("gaussian", opts.rho, opts.eta)
    pred = xs + (np.eye(64) - prm.mu_p * np.linalg.solve(Ht, H)) @ (x1 - xs) + prm.beta_p * x1
    np.testing.assert_allclose(x2, pred, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("kind", ["srht", "gaussian"])
def test_refreshed_reaches_solution_and_stops_on_its_rule(c1, kind):
    p, xs, H = c1
    x, info = ihs.refreshed_ihs(p.A, p.b, p.nu2, 512, ihs.Options(kind=kind, variant="gd",
                                                                  tol=1e-9))
    assert info.status == "ok"
    assert ridge.relative_error(H, x, xs) <= 1e-7
    assert info.r_history[-1] <= 1e-9 * info.r_history[0]
    assert all(r > 1e-9 * info.r_history[0] for r in info.r_history[:-1])
    assert len(info.r_history) == info.steps + 1
