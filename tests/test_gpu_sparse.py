"""GPU parity of sparse A with the CountSketch (rs_adaptive_solve_csr): the FP64
event trajectory equals the oracle's sparse solve, ragged FP32/BF16 runs and the
full 2^20 x 1024 problem reach the direct solution, and malformed CSR input is
rejected before any other work."""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

from oracle import ihs, ridge  # noqa: E402
from synth import config_sparse, make_sparse_problem  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_05874_amd import rs as _rs
    _rs.load()
    return _rs


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def as_scipy(rowptr, col, val, n, d):
    return sp.csr_matrix((val.astype(np.float64), col, rowptr), shape=(n, d))


@pytest.mark.parametrize("variant", ["gd", "polyak"])
@pytest.mark.parametrize("resample", ["fresh", "nested"])
def test_sparse_fp64_trajectories(rs, variant, resample):
    n, d = 5000, 80
    rowptr, col, val, b = make_sparse_problem(n, d, 6, 0.8, 0.1, 3, dtype=np.float64)
    nu2 = 0.05
    x, info = rs.rs_adaptive_solve_csr(*dev(rowptr, col, val), d, *dev(b), nu2, variant=variant,
                                       resample=resample, tol=1e-10, seed=4)
    A = as_scipy(rowptr, col, val, n, d)
    xo, io = ihs.adaptive_solve_sparse(A, b, nu2, ihs.Options(kind="count", variant=variant,
                                                              resample=resample, tol=1e-10,
                                                              seed=4))
    assert info["status"] == "ok"
    assert info["events"] == [e for e in io.events if e[1] != "stop"]
    assert info["m_final"] == io.m_final
    np.testing.assert_allclose(host(x), xo, rtol=1e-8, atol=1e-12)
    Ad = A.toarray()
    assert ridge.relative_error(ridge.hessian(Ad, nu2), host(x),
                                ridge.solve_direct(Ad, b, nu2)) <= 1e-8


@pytest.mark.parametrize("n,d,sketch_dtype", [(7001, 129, "f32"), (20000, 300, "bf16")])
def test_sparse_fp32_ragged_reaches_solution(rs, n, d, sketch_dtype):
    rowptr, col, val, b = make_sparse_problem(n, d, 9, 1.0, 0.1, 5)
    nu2 = 0.05
    x, info = rs.rs_adaptive_solve_csr(*dev(rowptr, col, val), d, *dev(b), nu2,
                                       sketch_dtype=sketch_dtype, tol=1e-10)
    assert info["status"] == "ok"
    A = as_scipy(rowptr, col, val, n, d)
    G = (A.T @ A).toarray()
    Atb = A.T @ b.astype(np.float64)
    xs = ridge.solve_direct_from_gram(G, Atb, nu2)
    assert ridge.relative_error(G + nu2 * np.eye(d), host(x), xs) <= 1e-8


def test_sparse_full_size_reaches_solution(rs):
    (rowptr, col, val, b), nu2 = config_sparse()
    n, d = rowptr.size - 1, 1024
    x, info = rs.rs_adaptive_solve_csr(*dev(rowptr, col, val), d, *dev(b), nu2, tol=1e-10)
    assert info["status"] == "ok"
    A = as_scipy(rowptr, col, val, n, d)
    G = (A.T @ A).toarray()
    xs = ridge.solve_direct_from_gram(G, A.T @ b.astype(np.float64), nu2)
    assert ridge.relative_error(G + nu2 * np.eye(d), host(x), xs) <= 1e-8


def test_sparse_malformed_csr_rejected(rs):
    rowptr, col, val, b = make_sparse_problem(500, 20, 4, 0.5, 0.1, 1)
    bad_col = col.copy()
    bad_col[17] = 20                       # column d: out of range
    with pytest.raises(rs.RsError) as e:
        rs.rs_adaptive_solve_csr(*dev(rowptr, bad_col, val), 20, *dev(b), 0.1)
    assert e.value.name == "arg"
    bad_ptr = rowptr.copy()
    bad_ptr[-1] -= 1                       # does not end at nnz
    with pytest.raises(rs.RsError) as e:
        rs.rs_adaptive_solve_csr(*dev(bad_ptr, col, val), 20, *dev(b), 0.1)
    assert e.value.name == "arg"
    # the dense solver does not take the CountSketch
    A = rs.padded(500, 20, dtype=torch.float32)
    A.zero_()
    with pytest.raises(rs.RsError) as e:
        rs.rs_adaptive_solve(A, *dev(b), 0.1, kind="count")
    assert e.value.name == "unsupported"


def test_sparse_empty_rows_and_empty_matrix(rs):
    # rows without entries (every third row emptied) still reach the solution
    n, d = 3001, 40
    rowptr, col, val, b = make_sparse_problem(n, d, 5, 0.5, 0.1, 8, dtype=np.float64)
    keep = np.repeat(np.arange(n) % 3 != 0, np.diff(rowptr))
    counts = np.where(np.arange(n) % 3 != 0, np.diff(rowptr), 0)
    rp2 = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp2[1:])
    col2, val2 = col[keep], val[keep]
    x, info = rs.rs_adaptive_solve_csr(*dev(rp2, col2, val2), d, *dev(b), 0.05, tol=1e-10, seed=2)
    A = as_scipy(rp2, col2, val2, n, d)
    xo, io = ihs.adaptive_solve_sparse(A, b, 0.05, ihs.Options(kind="count", tol=1e-10, seed=2))
    assert info["events"] == [e for e in io.events if e[1] != "stop"]
    np.testing.assert_allclose(host(x), xo, rtol=1e-8, atol=1e-12)
    # no entries at all: A = 0, g(0) = 0, so x* = 0 and the solve stops at once
    rp0 = np.zeros(n + 1, dtype=np.int64)
    x0, i0 = rs.rs_adaptive_solve_csr(*dev(rp0), torch.zeros(0, dtype=torch.int32).cuda(),
                                      torch.zeros(0, dtype=torch.float64).cuda(), d, *dev(b), 0.05)
    assert i0["status"] == "ok" and i0["events"] == []
    assert np.all(host(x0) == 0.0)


def test_sparse_runs_are_bitwise_repeatable(rs):
    # sorts, chunked sums and the column pass all run in a fixed order
    rowptr, col, val, b = make_sparse_problem(20000, 300, 9, 1.0, 0.1, 5)
    args = (*dev(rowptr, col, val), 300, *dev(b), 0.05)
    x1, i1 = rs.rs_adaptive_solve_csr(*args, tol=1e-10, seed=9)
    x2, i2 = rs.rs_adaptive_solve_csr(*args, tol=1e-10, seed=9)
    assert i1["events"] == i2["events"]
    np.testing.assert_array_equal(host(x1), host(x2))
