"""GPU parity of the regularization path (rs_solve_path, Section 4 warm starts):
each nu follows the oracle's warm-started trajectory (FP64), equals the chain of
single warm-started solves it is defined by, reaches the direct solution at the
full 65536 x 1024 FP32 size, and bad arguments are rejected."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ihs, ridge  # noqa: E402
from synth import config_c1, config_path_nu2, make_path_problem, make_problem, spectrum  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_05874_amd import rs as _rs
    _rs.load()
    return _rs


def dev_padded(A, rs):
    dt = torch.float64 if A.dtype == np.float64 else torch.float32
    T = rs.padded(A.shape[0], A.shape[1], dtype=dt)
    T.copy_(torch.from_numpy(A))
    return T


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("kind,variant", [("srht", "polyak"), ("srht", "gd"),
                                          ("gaussian", "polyak"), ("gaussian", "gd")])
def test_path_fp64_trajectories(rs, kind, variant):
    # the paper's synthetic path nu = 10^0 .. 10^-4 at eps = 1e-10 on the
    # exponential-decay problem
    p = config_c1()
    nus = list(config_path_nu2())
    X, infos = rs.rs_solve_path(dev_padded(p.A, rs), torch.from_numpy(p.b).cuda(), nus,
                                kind=kind, variant=variant, tol=1e-10, seed=3)
    Xo, io = ihs.solve_path(p.A, p.b, nus, ihs.Options(kind=kind, variant=variant, tol=1e-10,
                                                       seed=3))
    Xh = host(X)
    for k, nu2 in enumerate(nus):
        assert infos[k]["events"] == [e for e in io[k].events if e[1] != "stop"], k
        assert infos[k]["m_final"] == io[k].m_final and infos[k]["status"] == "ok"
        np.testing.assert_allclose(Xh[k], Xo[k], rtol=1e-8, atol=1e-12)
        xs = ridge.solve_direct(p.A, p.b, nu2)
        assert ridge.relative_error(ridge.hessian(p.A, nu2), Xh[k], xs) <= 1e-9


@pytest.mark.parametrize("dtype,sketch_dtype", [(np.float64, None), (np.float32, "bf16")])
def test_path_equals_chain_of_warm_solves(rs, dtype, sketch_dtype):
    # ragged shape (n not a power of two, d not a multiple of 64)
    p = make_problem(3000, 70, spectrum("poly", 70, 1.0), 1e-3, 0.1, 7, dtype=dtype)
    nus = [1.0, 1e-2, 1e-2, 1e-4, 1e-6]   # a repeated nu starts at its own solution
    A = dev_padded(p.A, rs)
    b = torch.from_numpy(p.b).cuda()
    X, infos = rs.rs_solve_path(A, b, nus, sketch_dtype=sketch_dtype, tol=1e-9, seed=11)
    x = torch.zeros(70, dtype=torch.float64, device="cuda")
    m = 1
    for k, nu2 in enumerate(nus):
        x, i1 = rs.rs_adaptive_solve(A, b, nu2, resample="nested", sketch_dtype=sketch_dtype,
                                     tol=1e-9, seed=11, m_init=m, x0=x, ref_at_zero=True)
        assert infos[k]["events"] == i1["events"], k
        assert infos[k]["m_final"] == i1["m_final"]
        np.testing.assert_array_equal(host(X[k]), host(x))
        m = i1["m_final"]
    # the repeated nu: its start is already within tol, so it stops at once
    assert infos[2]["events"] == [] and infos[2]["grad_passes"] == 1


def test_origin_reference_leaves_a_cold_start_unchanged(rs):
    p = config_c1()
    A = dev_padded(p.A, rs)
    b = torch.from_numpy(p.b).cuda()
    x0, i0 = rs.rs_adaptive_solve(A, b, p.nu2, resample="nested", seed=5)
    x1, i1 = rs.rs_adaptive_solve(A, b, p.nu2, resample="nested", seed=5, ref_at_zero=True)
    assert i0["events"] == i1["events"] and i0["r_ref"] == pytest.approx(i1["r_ref"], rel=1e-13)
    np.testing.assert_allclose(host(x1), host(x0), rtol=1e-12, atol=1e-15)


def test_path_full_size_reaches_direct_solutions(rs):
    # 65536 x 1024 FP32, sigma_i = 1/i, nu = 10^0 .. 10^-4 at eps = 1e-10
    A0, b = make_path_problem("cuda")
    A = rs.padded(A0.shape[0], A0.shape[1], dtype=torch.float32)
    A.copy_(A0)
    del A0
    nus = list(config_path_nu2())
    X, infos = rs.rs_solve_path(A, b, nus, tol=1e-10)
    assert all(i["status"] == "ok" for i in infos)
    assert [i["m_final"] for i in infos] == sorted(i["m_final"] for i in infos)
    d = A.shape[1]
    G = np.zeros((d, d))
    Atb = np.zeros(d)
    for r0 in range(0, A.shape[0], 16384):
        Ac = host(A[r0:r0 + 16384]).astype(np.float64)
        G += Ac.T @ Ac
        Atb += Ac.T @ host(b[r0:r0 + 16384]).astype(np.float64)
    Xh = host(X)
    for k, nu2 in enumerate(nus):
        xs = ridge.solve_direct_from_gram(G, Atb, nu2)
        assert ridge.relative_error(G + nu2 * np.eye(d), Xh[k], xs) <= 1e-9, k


def test_path_argument_errors(rs):
    p = config_c1()
    A = dev_padded(p.A, rs)
    b = torch.from_numpy(p.b).cuda()
    with pytest.raises(rs.RsError) as e:
        rs.rs_solve_path(A, b, [1e-2, 1e-1])
    assert e.value.name == "arg"
    with pytest.raises(rs.RsError) as e:
        rs.rs_solve_path(A, b, [1e-2, -1.0])
    assert e.value.name == "not_spd"
    X, infos = rs.rs_solve_path(A, b, [])
    assert X.shape == (0, 64) and infos == []


def test_path_single_nu_and_warm_first_start(rs):
    p = config_c1()
    A = dev_padded(p.A, rs)
    b = torch.from_numpy(p.b).cuda()
    # one nu: the cold nested solve with the origin reference (same steps)
    X, infos = rs.rs_solve_path(A, b, [p.nu2], seed=5)
    x1, i1 = rs.rs_adaptive_solve(A, b, p.nu2, resample="nested", seed=5)
    assert infos[0]["events"] == i1["events"]
    # a nonzero first start: the oracle's warm solve from that point
    xs = ridge.solve_direct(p.A, p.b, 0.1)
    X2, inf2 = rs.rs_solve_path(A, b, [p.nu2, 1e-3], x0=torch.from_numpy(xs).cuda(), seed=5)
    o = ihs.Options(resample="nested", ref_at_zero=True, seed=5)
    xa, ia = ihs.adaptive_solve(p.A, p.b, p.nu2, o, x_init=xs)
    assert inf2[0]["events"] == [e for e in ia.events if e[1] != "stop"]
    np.testing.assert_allclose(host(X2[0]), xa, rtol=1e-8, atol=1e-12)


def test_path_runs_are_bitwise_repeatable(rs):
    p = make_problem(3000, 70, spectrum("poly", 70, 1.0), 1e-3, 0.1, 7)
    A = dev_padded(p.A, rs)
    b = torch.from_numpy(p.b).cuda()
    nus = [1.0, 1e-2, 1e-4]
    X1, i1 = rs.rs_solve_path(A, b, nus, sketch_dtype="bf16", tol=1e-9, seed=2)
    X2, i2 = rs.rs_solve_path(A, b, nus, sketch_dtype="bf16", tol=1e-9, seed=2)
    assert [i["events"] for i in i1] == [i["events"] for i in i2]
    np.testing.assert_array_equal(host(X1), host(X2))
