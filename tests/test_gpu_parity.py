"""GPU parity: every entry point of librs (through the C ABI) against the oracle.

Inputs are seeded synthetic problems; expected values come only from oracle/.
Bars: bit-exact for signs and sampled row indices; FP64 paths within a few
ulps x transform depth; FP32 paths within the tolerance derived in the test
from the arithmetic (stated per check).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ihs, ridge, sketch  # noqa: E402
from synth import config_c1, make_problem, spectrum  # noqa: E402

pytestmark = pytest.mark.gpu


def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def rs():
    _needs_gpu()
    from paper_2006_05874_amd import rs as _rs
    _rs.load()
    return _rs


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def dev_padded(A, rs):
    """Upload a row-major matrix with a 16-byte-multiple leading dimension."""
    dt = torch.float64 if A.dtype == np.float64 else torch.float32
    T = rs.padded(A.shape[0], A.shape[1], dtype=dt)
    T.copy_(torch.from_numpy(A))
    return T


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# ------------------------------------------------------------------ SRHT
SRHT_CASES = [
    # n, d, m, dtype        (single pass n<=1024; two pass above; ragged n and d)
    (1024, 64, 1, np.float64),
    (1024, 64, 37, np.float64),
    (1000, 13, 512, np.float64),
    (1024, 64, 1024, np.float64),
    (4096, 24, 300, np.float64),
    (5000, 40, 2048, np.float64),
    (65536, 8, 64, np.float64),
    (3000, 70, 100, np.float32),
    (16384, 33, 1500, np.float32),
    # padded n above 2^20: the second pass folds 1 or 2 extra high index bits
    (1_500_000, 3, 1500, np.float32),
    ((1 << 21) + 5, 4, 64, np.float64),
]


@pytest.mark.parametrize("n,d,m,dt", SRHT_CASES)
def test_srht_rows_signs_bitwise(rs, n, d, m, dt):
    A = np.random.default_rng(n + d).standard_normal((n, d)).astype(dt)
    SA, rows, signs = rs.rs_sketch_srht(dev_padded(A, rs), m, seed=123, sketch_id=7, rows=True,
                                        signs=True)
    want_rows = sketch.srht_rows(123, 7, n, m)
    want_signs = sketch.srht_signs(123, 7, n)
    assert np.array_equal(host(rows), want_rows)
    assert np.array_equal(host(signs).astype(np.float64), want_signs)


@pytest.mark.parametrize("n,d,m,dt", SRHT_CASES)
def test_srht_values_against_dense_oracle(rs, n, d, m, dt):
    A = np.random.default_rng(n * 3 + d).standard_normal((n, d)).astype(dt)
    SA = host(rs.rs_sketch_srht(dev_padded(A, rs), m, seed=9, sketch_id=2))
    # compare a sample of rows (all when small): each oracle row is a dense sum
    nsample = 64 if n <= (1 << 20) else 6
    which = (np.arange(m) if m <= nsample
             else np.random.default_rng(0).choice(m, nsample, replace=False))
    want = sketch.srht_sketch_rows(A.astype(np.float64), 9, 2, m, which)
    npad = sketch.next_pow2(n)
    # error of a length-npad +-1 sum in the working precision, scaled by 1/sqrt(m)
    eps = np.finfo(dt).eps
    scale = np.sqrt(npad / m) * np.abs(A).max()
    tol = 4 * eps * math.log2(npad) * scale * (1 if dt == np.float64 else 4)
    np.testing.assert_allclose(SA[which], want, rtol=0, atol=tol)


def test_srht_integer_inputs_exact(rs):
    # integer-valued data: every partial sum is exact in FP64, so the fast
    # transform must equal the dense one bit for bit (up to the final scale)
    n, d, m = 8192, 16, 256
    A = np.random.default_rng(4).integers(-8, 9, size=(n, d)).astype(np.float64)
    SA = host(rs.rs_sketch_srht(dev_padded(A, rs), m, seed=1, sketch_id=1))
    want, _ = sketch.srht_sketch(A, 1, 1, m)
    np.testing.assert_array_equal(np.round(SA * np.sqrt(m)), np.round(want * np.sqrt(m)))
    np.testing.assert_allclose(SA, want, rtol=1e-15, atol=0)


def test_srht_integer_inputs_exact_large_n(rs):
    # padded n = 2^22 (two folded high bits in the second pass): sampled rows of
    # integer data are exact
    n, d, m = (1 << 21) + 3, 3, 2048
    A = np.random.default_rng(8).integers(-4, 5, size=(n, d)).astype(np.float64)
    SA = host(rs.rs_sketch_srht(dev_padded(A, rs), m, seed=5, sketch_id=3))
    which = np.array([0, 1, 777, 1500, m - 1])
    want = sketch.srht_sketch_rows(A, 5, 3, m, which)
    np.testing.assert_array_equal(np.round(SA[which] * np.sqrt(m)), np.round(want * np.sqrt(m)))


def test_srht_full_sample_is_isometry(rs):
    n, d = 2048, 12
    A = np.random.default_rng(5).standard_normal((n, d))
    SA = host(rs.rs_sketch_srht(dev_padded(A, rs), n, seed=3, sketch_id=0))
    np.testing.assert_allclose(SA.T @ SA, A.T @ A, rtol=1e-11, atol=1e-11)


def test_srht_nested_prefix_and_bf16(rs):
    n, d = 4096, 40
    A = np.random.default_rng(6).standard_normal((n, d)).astype(np.float32)
    Ad = dev_padded(A, rs)
    S32, r32 = rs.rs_sketch_srht(Ad, 512, seed=2, sketch_id=0, rows=True)
    S16 = rs.rs_sketch_srht(Ad, 512, seed=2, sketch_id=0, sa_dtype="bf16")
    a, b = host(S32), host(S16.float())
    np.testing.assert_allclose(b, a, rtol=2 ** -8, atol=1e-30)
    _, r64 = rs.rs_sketch_srht(Ad, 1024, seed=2, sketch_id=0, rows=True)
    assert set(host(r32)) <= set(host(r64))


# ------------------------------------------------------------------ Gaussian
@pytest.mark.parametrize("n,d,m,dt", [(1024, 64, 1, np.float64), (1024, 64, 100, np.float64),
                                      (777, 19, 65, np.float64), (2048, 130, 70, np.float32)])
def test_gaussian_sketch(rs, n, d, m, dt):
    A = np.random.default_rng(n + m).standard_normal((n, d)).astype(dt)
    SA = host(rs.rs_sketch_gaussian(dev_padded(A, rs), m, seed=5, sketch_id=3))
    prec = "f64" if dt == np.float64 else "f32"
    want = sketch.gaussian_sketch(A.astype(np.float64), 5, 3, m, precision=prec)
    # device log/cos differ from the host's by a few ulps; FP32 adds the MFMA
    # accumulation over n terms
    if dt == np.float64:
        tol = 1e-12 * np.sqrt(n) * np.abs(A).max()
    else:
        tol = 2e-6 * np.sqrt(n) * np.abs(A).max()
    np.testing.assert_allclose(SA, want, rtol=0, atol=tol)


# ------------------------------------------------------------------ gradient
GRAD_CASES = [(1024, 64, 1, np.float64), (1024, 64, 2, np.float64), (777, 13, 2, np.float64),
              (5000, 300, 3, np.float64), (65536, 1024, 2, np.float32), (4099, 1000, 1, np.float32),
              (3000, 2048, 2, np.float32), (2000, 4096, 1, np.float32), (50, 1, 1, np.float32),
              (1, 7, 2, np.float64)]


@pytest.mark.parametrize("n,d,k,dt", GRAD_CASES)
def test_gradient_against_oracle(rs, n, d, k, dt):
    rng = np.random.default_rng(n + d + k)
    A = (rng.standard_normal((n, d)) / np.sqrt(n)).astype(dt)
    b = rng.standard_normal(n).astype(dt)
    X = rng.standard_normal((k, d))
    nu2 = 0.37
    G = host(rs.rs_gradient(dev_padded(A, rs), dev(b), nu2, dev(X)))
    A64, b64 = A.astype(np.float64), b.astype(np.float64)
    for c in range(k):
        if dt == np.float64:
            want = ridge.gradient(A64, b64, nu2, X[c])
            scale = np.abs(A64).sum(0) * (np.abs(A64 @ X[c]) + np.abs(b64)).max()
            tol = 64 * np.finfo(np.float64).eps * (scale + nu2 * np.abs(X[c]))
            assert np.all(np.abs(G[c] - want) <= tol + 1e-300)
        else:
            # the residual is formed in FP32 from FP32 x: compare with the exact
            # gradient at the rounded iterate, within the FP32 residual error
            x32 = X[c].astype(np.float32).astype(np.float64)
            want = A64.T @ (A64 @ x32 - b64) + nu2 * X[c]
            row = np.abs(A64) @ np.abs(x32) + np.abs(b64)
            tol = 8 * np.finfo(np.float32).eps * (np.abs(A64).T @ row) * math.log2(max(d, 2))
            assert np.all(np.abs(G[c] - want) <= tol + 1e-12)


@pytest.mark.parametrize("n,d,k", [(20000, 300, 2), (9000, 1000, 1), (3001, 37, 2)])
def test_gradient_autotune_then_parity(rs, n, d, k):
    # the tuned plan covers the row, is reported back, and the gradient it runs
    # still meets the FP32 bound against the exact gradient at the rounded iterate
    rng = np.random.default_rng(n + d)
    A = (rng.standard_normal((n, d)) / np.sqrt(n)).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    Ad, bd = dev_padded(A, rs), dev(b)
    tpr, nv, grid, rows = rs.rs_gradient_autotune(Ad, bd, k=k)
    assert tpr * nv * 4 >= d and grid >= 1 and rows in (2, 4, 8)
    assert rs.rs_gradient_plan("f32", n, d, k) == (tpr, nv, grid, rows)
    X = rng.standard_normal((k, d))
    G = host(rs.rs_gradient(Ad, bd, 0.37, dev(X)))
    A64, b64 = A.astype(np.float64), b.astype(np.float64)
    for c in range(k):
        x32 = X[c].astype(np.float32).astype(np.float64)
        want = A64.T @ (A64 @ x32 - b64) + 0.37 * X[c]
        row = np.abs(A64) @ np.abs(x32) + np.abs(b64)
        tol = 8 * np.finfo(np.float32).eps * (np.abs(A64).T @ row) * math.log2(max(d, 2))
        assert np.all(np.abs(G[c] - want) <= tol + 1e-12)
    # and a solve with the tuned pass reaches the oracle's solution
    p = make_problem(n, d, spectrum("poly", d, 1.0), 1e-3, 0.1, 3)
    A2 = dev_padded(p.A, rs)
    rs.rs_gradient_autotune(A2, dev(p.b), k=2)
    x, info = rs.rs_adaptive_solve(A2, dev(p.b), p.nu2)
    A64 = p.A.astype(np.float64)
    xs = ridge.solve_direct(A64, p.b.astype(np.float64), p.nu2)
    assert info["status"] == "ok"
    assert ridge.relative_error(ridge.hessian(A64, p.nu2), host(x), xs) <= 1e-6


def _fp32_grad_check(A, b, X, G, nu2):
    A64, b64 = A.astype(np.float64), b.astype(np.float64)
    d = A.shape[1]
    for c in range(X.shape[0]):
        x32 = X[c].astype(np.float32).astype(np.float64)
        want = A64.T @ (A64 @ x32 - b64) + nu2 * X[c]
        row = np.abs(A64) @ np.abs(x32) + np.abs(b64)
        tol = 8 * np.finfo(np.float32).eps * (np.abs(A64).T @ row) * math.log2(max(d, 2))
        assert np.all(np.abs(G[c] - want) <= tol + 1e-12)


WIDE_SHAPES = [(tpr, nv, r) for tpr in (16, 64, 128, 256, 512) for nv in (1, 2, 4, 8)
               for r in (2, 4, 8)]


@pytest.mark.parametrize("d", [8192, 4096])
@pytest.mark.parametrize("k", [1, 2])
def test_gradient_every_built_shape_at_wide_d(rs, d, k):
    """Every partial-sum shape the library builds that covers d (the ones the tuner
    can pick at the 2^21 x 8192 evaluation size among them), forced through
    rs_gradient_set_plan, against the oracle's gradient; ragged n, several grids."""
    n = 3001
    rng = np.random.default_rng(d + k)
    A = (rng.standard_normal((n, d)) / np.sqrt(n)).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    X = rng.standard_normal((k, d))
    Ad, bd, Xd = dev_padded(A, rs), dev(b), dev(X)
    tried = 0
    for (tpr, nv, r) in WIDE_SHAPES:
        for grid in (7, n // 64):          # the library caps a grid at n / 64 blocks
            try:
                rs.rs_gradient_set_plan("f32", n, d, k, (tpr, nv, grid, r))
            except rs.RsError as e:
                assert e.name in ("unsupported", "shape")
                break
            assert rs.rs_gradient_plan("f32", n, d, k) == (tpr, nv, grid, r)
            G = host(rs.rs_gradient(Ad, bd, 0.37, Xd))
            _fp32_grad_check(A, b, X, G, 0.37)
            tried += 1
    assert tried >= 4          # (256, 8, 2) and (256, 8, 4) at d = 8192, two grids each


@pytest.mark.parametrize("n,d,plan", [(3001, 8192, (512, 4, 7, 2)), (4099, 8190, (512, 4, 64, 2)),
                                      (2500, 4093, (512, 2, 39, 4)), (1, 5000, (512, 4, 1, 2))])
def test_gradient_two_equals_two_single_passes(rs, n, d, plan):
    """Two problems on one A and b in one read: each job's G bit for bit what its own
    k = 2 pass gives under the same plan (ragged n and d, a grid that leaves the
    last block short, one row), and within the FP32 bound of the exact gradient."""
    rng = np.random.default_rng(n + d)
    A = (rng.standard_normal((n, d)) / np.sqrt(max(n, 2))).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    X0, X1 = rng.standard_normal((2, d)), rng.standard_normal((2, d))
    Ad, bd = dev_padded(A, rs), dev(b)
    rs.rs_gradient_set_plan("f32", n, d, 2, plan)
    G0, G1 = rs.rs_gradient_two(Ad, bd, (0.37, 1e-4), dev(X0), dev(X1))
    assert torch.equal(G0, rs.rs_gradient(Ad, bd, 0.37, dev(X0)))
    assert torch.equal(G1, rs.rs_gradient(Ad, bd, 1e-4, dev(X1)))
    _fp32_grad_check(A, b, X0, host(G0), 0.37)
    _fp32_grad_check(A, b, X1, host(G1), 1e-4)


def test_gradient_two_needs_the_512_thread_plan(rs):
    n, d = 3001, 4096
    Ad = rs.padded(n, d, dtype=torch.float32)
    Ad.zero_()
    bd = torch.zeros(n, device="cuda", dtype=torch.float32)
    X = torch.zeros(2, d, dtype=torch.float64, device="cuda")
    rs.rs_gradient_set_plan("f32", n, d, 2, (256, 4, 16, 4))
    with pytest.raises(rs.RsError) as e:
        rs.rs_gradient_two(Ad, bd, (1.0, 1.0), X, X)
    assert e.value.name == "unsupported"
    with pytest.raises(ValueError):
        rs.rs_gradient_two(Ad.double(), bd.double(), (1.0, 1.0), X, X)


def test_gradient_set_plan_rejects_bad_plans(rs):
    with pytest.raises(rs.RsError) as e:
        rs.rs_gradient_set_plan("f32", 4096, 8192, 2, (64, 1, 16, 8))     # does not cover d
    assert e.value.name == "shape"
    with pytest.raises(rs.RsError) as e:
        rs.rs_gradient_set_plan("f32", 4096, 8192, 2, (256, 8, 16, 3))    # not built
    assert e.value.name == "unsupported"
    with pytest.raises(rs.RsError) as e:
        rs.rs_gradient_set_plan("f32", 4096, 8192, 2, (256, 8, 0, 4))     # empty grid
    assert e.value.name == "arg"


# ------------------------------------------------------------------ factor
FACTOR_CASES = [(1, 64), (5, 64), (63, 64), (64, 64), (65, 64), (200, 64), (100, 300),
                (512, 1024), (1024, 1024), (2048, 1024), (300, 100)]


@pytest.mark.parametrize("m,d", [(1024, 8192), (520, 8192), (8192, 8192)])
def test_factor_apply_at_evaluation_width(rs, m, d):
    """The factor and apply at d = 8192, the width of the 2^21 x 8192 evaluation
    problem: the m x m Woodbury route with 128 column blocks (m < d) and the
    8192 x 8192 Cholesky route (m = d), FP32 SA as the solver stores it."""
    rng = np.random.default_rng(m + d)
    SA = (rng.standard_normal((m, d)) / np.sqrt(d)).astype(np.float32)
    nu2 = 0.05
    F = rs.rs_factor_woodbury(dev(SA), nu2)
    G = rng.standard_normal((2, d))
    GT, r = F.apply(dev(G))
    GT, r = host(GT), host(r)
    F.close()
    SA64 = SA.astype(np.float64)
    P = ihs.SketchedHessian(SA64, nu2)
    # |SA|_2^2 by power iteration on SA^T SA (converges from below; 1.25x margin)
    v = rng.standard_normal(d)
    for _ in range(30):
        v = SA64.T @ (SA64 @ v)
        v /= np.linalg.norm(v)
    smax2 = 1.25 * float(np.linalg.norm(SA64 @ v) ** 2)
    cond = (smax2 + nu2) / nu2          # H_S = SA^T SA + nu^2 I
    for c in range(2):
        want, rw = P.decrement(G[c])
        err = np.linalg.norm(GT[c] - want) / np.linalg.norm(want)
        # FP32 Gram on the matrix cores: relative error ~ 1e-7 sqrt(q) amplified by cond
        assert err <= 2e-6 * cond, (err, cond)
        assert abs(r[c] - rw) <= 2e-6 * cond * abs(rw)


@pytest.mark.parametrize("m,d", FACTOR_CASES)
def test_factor_apply_against_oracle(rs, m, d):
    rng = np.random.default_rng(m * 7 + d)
    SA = rng.standard_normal((m, d)) / np.sqrt(d)
    nu2 = 0.05
    F = rs.rs_factor_woodbury(dev(SA), nu2)
    G = rng.standard_normal((2, d))
    GT, r = F.apply(dev(G))
    GT, r = host(GT), host(r)
    P = ihs.SketchedHessian(SA, nu2)
    HS = SA.T @ SA + nu2 * np.eye(d)
    cond = np.linalg.cond(HS)
    for c in range(2):
        want, rw = P.decrement(G[c])
        err = np.linalg.norm(GT[c] - want) / np.linalg.norm(want)
        assert err <= 1e-14 * cond * 50, (err, cond)
        assert abs(r[c] - rw) <= 1e-13 * cond * abs(rw)
    F.close()


def test_factor_fp32_and_bf16_inputs(rs):
    rng = np.random.default_rng(11)
    m, d, nu2 = 300, 200, 0.1
    SA = (rng.standard_normal((m, d)) / np.sqrt(d)).astype(np.float32)
    g = rng.standard_normal((1, d))
    for tdt in (torch.float32, torch.bfloat16):
        SAd = dev(SA).to(tdt)
        used = SAd.float().double().cpu().numpy()   # the stored values define the sketch
        F = rs.rs_factor_woodbury(SAd, nu2)
        GT, r = F.apply(dev(g))
        want, rw = ihs.SketchedHessian(used, nu2).decrement(g[0])
        # Gram accumulated in FP32 on the matrix cores
        np.testing.assert_allclose(host(GT)[0], want, rtol=2e-5, atol=2e-5 * np.abs(want).max())
        F.close()


def test_factor_not_spd(rs):
    SA = torch.zeros(8, 16, dtype=torch.float64, device="cuda")
    with pytest.raises(rs.RsError) as e:
        rs.rs_factor_woodbury(SA, 0.0)
    assert e.value.name == "not_spd"


# ------------------------------------------------------------------ one step
def test_ihs_step_matches_oracle(rs):
    p = config_c1()
    n, d = p.A.shape
    A = dev_padded(p.A, rs)
    b = dev(p.b)
    SA = rs.rs_sketch_srht(A, 32, seed=0, sketch_id=0)
    F = rs.rs_factor_woodbury(SA, p.nu2)
    prm = rs.rs_params("srht", 0.1)
    x = torch.zeros(d, dtype=torch.float64, device="cuda")
    g = rs.rs_gradient(A, b, p.nu2, x[None, :])[0].contiguous()
    gt, r = F.apply(g[None, :])
    state = {"x": x, "x_prev": x.clone(), "g": g, "gtilde": gt[0].contiguous(),
             "r_t": float(host(r)[0]), "r_1": float(host(r)[0]), "t": 1}
    P = ihs.SketchedHessian(sketch.srht_sketch(p.A, 0, 0, 32)[0], p.nu2)
    pr = ihs.params_for("srht", 0.1)
    xo, xpo = np.zeros(d), np.zeros(d)
    go = ridge.gradient(p.A, p.b, p.nu2, xo)
    gto, ro = P.decrement(go)
    r1o = ro
    assert abs(state["r_t"] - ro) < 1e-10 * ro
    for t in range(1, 6):
        res = rs.rs_ihs_step(A, b, p.nu2, F, prm, "polyak", state)
        xp = ihs.polyak_candidate(xo, xpo, gto, pr.mu_p, pr.beta_p)
        _, rp = P.decrement(ridge.gradient(p.A, p.b, p.nu2, xp))
        xg = ihs.gd_candidate(xo, gto, pr.mu_gd)
        gg = ridge.gradient(p.A, p.b, p.nu2, xg)
        gtg, rg = P.decrement(gg)
        assert abs(res["r_gd"] - rg) <= 1e-9 * rg
        assert abs(res["r_p"] - rp) <= 1e-9 * rp
        if (rp / r1o) ** (1 / t) <= pr.cbar_p:
            want = 0
            gp = ridge.gradient(p.A, p.b, p.nu2, xp)
            xpo, xo = xo, xp
            go = gp
            gto, ro = P.decrement(gp)
        elif rg / ro <= pr.cbar_gd:
            want = 1
            xpo, xo = xo, xg
            go, gto, ro = gg, gtg, rg
        else:
            want = -1
        assert res["accepted"] == want
        if want == -1:
            break
        np.testing.assert_allclose(host(state["x"]), xo, rtol=1e-9, atol=1e-12)
    F.close()


# ------------------------------------------------------------------ Algorithm 1
@pytest.fixture(scope="module")
def c1_problem():
    p = config_c1()
    xs = ridge.solve_direct(p.A, p.b, p.nu2)
    return p, xs, ridge.hessian(p.A, p.nu2)


@pytest.mark.parametrize("kind", ["srht", "gaussian"])
@pytest.mark.parametrize("variant", ["polyak", "gd"])
@pytest.mark.parametrize("resample", ["fresh", "nested"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_adaptive_solve_fp64_trajectory(rs, c1_problem, kind, variant, resample, seed):
    p, xs, H = c1_problem
    A = dev_padded(p.A, rs)
    x, info = rs.rs_adaptive_solve(A, dev(p.b), p.nu2, kind=kind, variant=variant,
                                   resample=resample, seed=seed)
    xo, io = ihs.adaptive_solve(p.A, p.b, p.nu2, ihs.Options(kind=kind, variant=variant,
                                                           resample=resample, seed=seed))
    ev_o = [e for e in io.events if e[1] != "stop"]
    assert info["events"] == ev_o
    assert info["m_final"] == io.m_final and info["doublings"] == io.doublings
    assert info["status"] == "ok"
    assert ridge.relative_error(H, host(x), xs) <= 1e-6
    np.testing.assert_allclose(host(x), xo, rtol=1e-8, atol=1e-10)


def test_adaptive_solve_fp64_deterministic(rs, c1_problem):
    p, _, _ = c1_problem
    A = dev_padded(p.A, rs)
    x1, i1 = rs.rs_adaptive_solve(A, dev(p.b), p.nu2)
    x2, i2 = rs.rs_adaptive_solve(A, dev(p.b), p.nu2)
    assert torch.equal(x1, x2) and i1["events"] == i2["events"]


def test_adaptive_solve_zero_rhs(rs, c1_problem):
    p, _, _ = c1_problem
    x, info = rs.rs_adaptive_solve(dev_padded(p.A, rs), dev(np.zeros_like(p.b)), p.nu2)
    assert info["status"] == "ok" and info["grad_passes"] == 1
    assert torch.count_nonzero(x) == 0


def test_adaptive_solve_warm_start_and_cap(rs, c1_problem):
    p, xs, H = c1_problem
    A = dev_padded(p.A, rs)
    # m_max = 2 with gradient steps only: stuck at the cap -> no_convergence
    x, info = rs.rs_adaptive_solve(A, dev(p.b), p.nu2, variant="gd", m_max=2, max_iter=50)
    assert info["m_final"] <= 2
    xo, io = ihs.adaptive_solve(p.A, p.b, p.nu2, ihs.Options(variant="gd", m_max=2, max_iter=50))
    assert info["events"] == [e for e in io.events if e[1] != "stop"]
    assert (info["status"] == "ok") == (io.status == "ok")
    # full sketch from the start: no doubling
    x, info = rs.rs_adaptive_solve(A, dev(p.b), p.nu2, variant="gd", m_init=1024)
    assert info["doublings"] == 0 and info["status"] == "ok"


def test_adaptive_solve_max_iter(rs, c1_problem):
    p, _, _ = c1_problem
    x, info = rs.rs_adaptive_solve(dev_padded(p.A, rs), dev(p.b), p.nu2, max_iter=3)
    assert info["status"] == "no_convergence" and info["steps"] == 2


@pytest.mark.parametrize("nu2", [1e-2, 1e-4])
def test_adaptive_solve_fp32_reaches_tolerance(rs, nu2):
    # FP32 problem with the shape and spectrum of the 65536 x 1024 workload,
    # shrunk to n = 8192, d = 256 so the oracle finishes quickly
    p = make_problem(8192, 256, spectrum("poly", 256, 1.0), nu2, 0.1, 0)
    A64 = p.A.astype(np.float64)
    xs = ridge.solve_direct(A64, p.b.astype(np.float64), nu2)
    H = ridge.hessian(A64, nu2)
    x, info = rs.rs_adaptive_solve(dev_padded(p.A, rs), dev(p.b), nu2)
    assert info["status"] == "ok"
    assert ridge.relative_error(H, host(x), xs) <= 1e-6
