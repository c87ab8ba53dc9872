"""The synthetic input recipe (CPU only): each generator draws what its docstring
states (spectrum, planted model, noise level, CSR structure and column
popularity), and the same seed draws the same problem."""
import numpy as np
import pytest

import synth
from synth import problems

torch = pytest.importorskip("torch")


def gauss_factor_bounds(n, d):
    # extreme singular values of an n x d matrix with N(0, 1/n) entries lie near
    # 1 -+ sqrt(d/n) (Marchenko-Pastur edges); 0.1 of slack covers the sampling
    r = np.sqrt(d / n)
    return 1.0 - r - 0.1, 1.0 + r + 0.1


def sv_ratio(A, sigma):
    s = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    return s / np.sort(sigma)[::-1]


@pytest.mark.parametrize("kind,rate", [("geom", 0.9), ("poly", 1.0), ("exp", 10.0)])
def test_spectrum_kinds(kind, rate):
    s = problems.spectrum(kind, 40, rate)
    assert s.shape == (40,) and np.all(np.diff(s) < 0)
    first = {"geom": 1.0, "poly": 1.0, "exp": np.exp(-1.0 / rate)}[kind]
    last = {"geom": rate ** 39, "poly": 40.0 ** -rate, "exp": np.exp(-40.0 / rate)}[kind]
    assert s[0] == pytest.approx(first) and s[-1] == pytest.approx(last)


def test_haar_factor_is_orthogonal_with_uniform_signs():
    rng = np.random.default_rng(1)
    V = problems.haar_orthogonal(rng, 50)
    np.testing.assert_allclose(V.T @ V, np.eye(50), atol=1e-12)
    # the sign fix makes the distribution Haar: E[V] = 0 entrywise
    acc = sum(problems.haar_orthogonal(rng, 4) for _ in range(4000)) / 4000
    assert np.max(np.abs(acc)) < 0.05


def test_make_problem_spectrum_plant_and_noise():
    n, d = 8192, 32
    sigma = problems.spectrum("geom", d, 0.85)
    p = problems.make_problem(n, d, sigma, 1e-2, 0.5, 3, dtype=np.float64)
    assert p.A.shape == (n, d) and p.A.flags.c_contiguous and p.b.shape == (n,)
    lo, hi = gauss_factor_bounds(n, d)
    r = sv_ratio(p.A, sigma)
    assert np.all(r > lo) and np.all(r < hi)
    resid = p.b - p.A @ p.x_pl
    assert np.std(resid) == pytest.approx(0.5, rel=0.05)
    # same seed, same draw; another seed, another draw
    q = problems.make_problem(n, d, sigma, 1e-2, 0.5, 3, dtype=np.float64)
    np.testing.assert_array_equal(p.A, q.A)
    np.testing.assert_array_equal(p.b, q.b)
    assert not np.array_equal(problems.make_problem(n, d, sigma, 1e-2, 0.5, 4,
                                                    dtype=np.float64).A, p.A)


def test_named_configs():
    c1 = synth.config_c1()
    assert c1.A.shape == (1024, 64) and c1.A.dtype == np.float64 and c1.nu2 == 1e-2
    np.testing.assert_allclose(c1.sigma, 0.9 ** np.arange(64))
    nus = synth.config_path_nu2()
    np.testing.assert_allclose(np.sqrt(nus), [1.0, 1e-1, 1e-2, 1e-3, 1e-4])
    grid = problems.config_c4a_nu2()
    assert grid.size == 64 and grid[0] == pytest.approx(1e-6) and grid[-1] == pytest.approx(1.0)
    specs = problems.config_c4b_specs()
    assert len(specs) == 256 and specs == problems.config_c4b_specs()
    assert all(s["n"] in (4096, 8192, 16384, 32768, 65536) and 128 <= s["d"] <= 1024
               and s["nu2"] == 1e-3 for s in specs)
    assert len({s["seed"] for s in specs}) == 256
    assert len({s["n"] for s in specs}) == 5


def test_device_generator_spectrum_and_repeatability():
    n, d = 16384, 48
    sigma = problems.spectrum("poly", d, 1.0)
    A, b, x_pl = problems.make_problem_torch(n, d, sigma, 0.1, 7, "cpu", row_block=5000)
    assert A.shape == (n, d) and A.dtype == torch.float32 and b.shape == (n,)
    lo, hi = gauss_factor_bounds(n, d)
    r = sv_ratio(A.numpy(), sigma)
    assert np.all(r > lo) and np.all(r < hi)
    resid = b.double() - A.double() @ x_pl
    assert float(resid.std()) == pytest.approx(0.1, rel=0.05)
    A2, b2, _ = problems.make_problem_torch(n, d, sigma, 0.1, 7, "cpu", row_block=5000)
    assert torch.equal(A, A2) and torch.equal(b, b2)


def test_wide_generator_is_a_transposed_draw():
    n, d = 40, 12000
    sigma = problems.spectrum("poly", n, 1.0)
    A, b = problems.make_wide_problem_torch(n, d, sigma, 0.1, 5, "cpu")
    assert A.shape == (n, d) and A.is_contiguous() and b.shape == (n,)
    T = problems.make_problem_torch(d, n, sigma, 0.1, 5, "cpu")[0]
    assert torch.equal(A, T.t())
    lo, hi = gauss_factor_bounds(d, n)
    r = sv_ratio(A.numpy(), sigma)
    assert np.all(r > lo) and np.all(r < hi)


def test_sparse_generator_csr_structure_and_popularity():
    n, d, per_row, alpha = 20000, 300, 9, 0.8
    rowptr, col, val, b = problems.make_sparse_problem(n, d, per_row, alpha, 0.1, 5)
    assert rowptr.dtype == np.int64 and col.dtype == np.int32 and val.dtype == np.float32
    assert rowptr[0] == 0 and rowptr[-1] == col.size == val.size and np.all(np.diff(rowptr) >= 0)
    assert b.shape == (n,) and col.min() >= 0 and col.max() < d
    counts = np.diff(rowptr)
    assert counts.min() >= 1 and counts.max() <= per_row
    # columns strictly increase within a row: distinct, as the CSR entry point requires
    row_of = np.repeat(np.arange(n), counts)
    same_row = row_of[1:] == row_of[:-1]
    assert np.all(col[1:][same_row] > col[:-1][same_row])
    # column popularity follows P(j) ~ (j + 1)^-alpha before repeats are dropped: the
    # first column is far more common than the last ones, and a row holds it with
    # probability 1 - (1 - P(0))^per_row
    pop = np.bincount(col, minlength=d)
    assert pop[0] > 10 * pop[-20:].mean()
    assert pop[0] / n == pytest.approx(1 - (1 - 1 / np.sum(np.arange(1, d + 1.0) ** -alpha))
                                       ** per_row, rel=0.05)
    assert np.std(val) * np.sqrt(n) == pytest.approx(1.0, rel=0.05)
    r2 = problems.make_sparse_problem(n, d, per_row, alpha, 0.1, 5)
    assert all(np.array_equal(u, v) for u, v in zip((rowptr, col, val, b), r2))


def test_sparse_workload_constants():
    assert (problems.SPARSE_N, problems.SPARSE_D, problems.SPARSE_PER_ROW) == (1 << 20, 1024, 16)
    assert (problems.PATH_N, problems.PATH_D) == (65536, 1024)
    assert (problems.DUAL_N, problems.DUAL_D) == (1024, 65536)
