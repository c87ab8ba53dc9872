"""GPU parity of the precision form: BF16 / FP8-E4M3 sketches, their Gram on the
matrix cores with FP32 accumulation, FP64 factor, and the outer iteration
reaching the FP64 oracle's solution."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ihs, lowprec, ridge, sketch  # noqa: E402
from synth import make_problem, spectrum  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_05874_amd import rs as _rs
    _rs.load()
    return _rs


def dev_padded(A, rs):
    T = rs.padded(A.shape[0], A.shape[1], dtype=torch.float32)
    T.copy_(torch.from_numpy(A))
    return T


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("n,d,m", [(1024, 64, 48), (4096, 200, 300), (16384, 33, 1024)])
def test_srht_fp8_codes_and_scales(rs, n, d, m):
    A = np.random.default_rng(n + d).standard_normal((n, d)).astype(np.float32)
    (codes, scale), S32 = (rs.rs_sketch_srht(dev_padded(A, rs), m, seed=4, sketch_id=1,
                                             sa_dtype="fp8"),
                           rs.rs_sketch_srht(dev_padded(A, rs), m, seed=4, sketch_id=1))
    S32 = host(S32).astype(np.float64)
    # the device quantizes its own FP32 sketch: same scales, codes within one step
    want_codes, want_scale, _ = lowprec.fp8_quantize(S32)
    np.testing.assert_array_equal(host(scale).astype(np.float64), want_scale)
    got = lowprec.e4m3_decode(host(codes)) * want_scale[None, :]
    ref = lowprec.e4m3_decode(want_codes) * want_scale[None, :]
    assert np.mean(host(codes) == want_codes) > 0.999
    # any differing code is a neighbour (ties met in FP32 vs FP64)
    step = 2.0 ** -3 * np.maximum(np.abs(ref), 2.0 ** -6 * want_scale[None, :])
    assert np.all(np.abs(got - ref) <= step + 1e-30)
    # and the FP32 sketch itself matches the dense oracle
    which = np.arange(min(m, 16))
    np.testing.assert_allclose(S32[which], sketch.srht_sketch_rows(A.astype(np.float64), 4, 1, m,
                                                                    which),
                               rtol=0, atol=1e-4 * np.abs(S32).max())


@pytest.mark.parametrize("n,d,m", [(2048, 72, 40), (3001, 300, 130), (65536, 40, 16)])
def test_gaussian_bf16_matrix_core_product(rs, n, d, m):
    """The BF16 Gaussian sketch is the product of BF16-rounded inputs on the matrix
    cores: SA = bf16(S) bf16(A) / sqrt(m) with FP32 accumulation, stored in BF16.
    Against the oracle's FP64 product of the same rounded inputs; the bound adds
    the FP32 accumulation of n products, the final BF16 rounding and one BF16 step
    of one entry of S per row (the device's FP32 Box-Muller value and the
    oracle's FP64 one can round to neighbouring BF16 values when they straddle a
    rounding midpoint).  Ragged d and n, and n = 65536 with m = 16 (the split over
    A's rows)."""
    rng = np.random.default_rng(n + d + m)
    A = rng.standard_normal((n, d)).astype(np.float32)
    Ad = dev_padded(A, rs)
    S16 = host(rs.rs_sketch_gaussian(Ad, m, seed=3, sketch_id=2, sa_dtype="bf16").float())
    z = sketch.gaussian_matrix(3, 2, m, n, precision="f32") * np.sqrt(m)
    Sq = lowprec.bf16_round(z)
    Aq = lowprec.bf16_round(A.astype(np.float64))
    want = Sq @ Aq / np.sqrt(m)
    absprod = np.abs(Sq) @ np.abs(Aq) / np.sqrt(m)
    flip = 2.0 ** -8 * np.abs(Sq).max(axis=1)[:, None] * np.abs(Aq).max(axis=0)[None, :] / np.sqrt(m)
    tol = 2.0 ** -8 * np.abs(want) + n * 2.0 ** -24 * absprod + flip + 1e-30
    assert np.all(np.abs(S16.astype(np.float64) - want) <= tol)


def test_gaussian_fp8(rs):
    n, d, m = 2048, 72, 40
    A = np.random.default_rng(9).standard_normal((n, d)).astype(np.float32)
    Ad = dev_padded(A, rs)
    S32 = host(rs.rs_sketch_gaussian(Ad, m, seed=3, sketch_id=2)).astype(np.float64)
    codes, scale = rs.rs_sketch_gaussian(Ad, m, seed=3, sketch_id=2, sa_dtype="fp8")
    want_codes, want_scale, _ = lowprec.fp8_quantize(S32)
    np.testing.assert_array_equal(host(scale).astype(np.float64), want_scale)
    assert np.mean(host(codes) == want_codes) > 0.999


@pytest.mark.parametrize("m,d", [(500, 256), (2048, 128)])
def test_factor_lowprec_matrix_core_gram(rs, m, d):
    # m >= d with 64-aligned rows: the Gram runs on the BF16 / FP8 K=32 MFMA path
    rng = np.random.default_rng(m + 3 * d)
    SA = rng.standard_normal((m, d)) / np.sqrt(m)
    g = rng.standard_normal((1, d))
    for dt in ("bf16", "fp8"):
        if dt == "bf16":
            dev = torch.from_numpy(SA.astype(np.float32)).cuda().to(torch.bfloat16)
            used = dev.float().double().cpu().numpy()
            arg = dev
        else:
            codes, s, used = lowprec.fp8_quantize(SA)
            arg = (torch.from_numpy(codes).cuda(), torch.from_numpy(s.astype(np.float32)).cuda())
        F = rs.rs_factor_woodbury(arg, 0.05)
        GT, r = F.apply(torch.from_numpy(g).cuda())
        want, rw = ihs.SketchedHessian(used, 0.05).decrement(g[0])
        # BF16 products are summed exactly in FP32 (Gram error ~1e-8, times
        # cond(H_S) ~ 1e2 here).  The FP8 K=32 instruction sums less exactly
        # (Gram error ~1e-6 measured against the dequantized values), so its
        # bound is 50x wider; H_S stays SPD and the outer iteration absorbs it.
        tol = 2e-5 if dt == "bf16" else 1e-3
        np.testing.assert_allclose(host(GT)[0], want, rtol=tol, atol=tol * np.abs(want).max())
        assert abs(host(r)[0] - rw) <= tol * rw
        F.close()


@pytest.mark.parametrize("m,d", [(40, 100), (300, 200)])
def test_factor_fp8_against_oracle(rs, m, d):
    rng = np.random.default_rng(m + d)
    SA = rng.standard_normal((m, d)) / np.sqrt(d)
    codes, s, deq = lowprec.fp8_quantize(SA)
    F = rs.rs_factor_woodbury((torch.from_numpy(codes).cuda(),
                               torch.from_numpy(s.astype(np.float32)).cuda()), 0.1)
    g = rng.standard_normal((1, d))
    GT, r = F.apply(torch.from_numpy(g).cuda())
    want, rw = ihs.SketchedHessian(deq, 0.1).decrement(g[0])
    np.testing.assert_allclose(host(GT)[0], want, rtol=3e-5, atol=3e-5 * np.abs(want).max())
    F.close()


@pytest.fixture(scope="module")
def problem():
    # the precision workload's spectrum shape (exponential decay), shrunk so the
    # oracle finishes in seconds
    p = make_problem(8192, 256, spectrum("exp", 256, 25.0), 1e-3, 0.1, 0)
    A64 = p.A.astype(np.float64)
    xs = ridge.solve_direct(A64, p.b.astype(np.float64), p.nu2)
    return p, xs, ridge.hessian(A64, p.nu2)


@pytest.mark.parametrize("kind", ["srht", "gaussian"])
@pytest.mark.parametrize("dt", ["bf16", "fp8"])
def test_precision_form_reaches_oracle_solution(rs, problem, kind, dt):
    p, xs, H = problem
    x, info = rs.rs_adaptive_solve(dev_padded(p.A, rs), torch.from_numpy(p.b).cuda(), p.nu2,
                                   kind=kind, sketch_dtype=dt)
    assert info["status"] == "ok", info
    rel = ridge.relative_error(H, host(x), xs)
    assert rel <= 1e-6, rel


def test_precision_form_full_size_2p20x4096(rs):
    # the 2^20 x 4096 FP32 problem (16 GiB, sigma_i = exp(-i/400), nu^2 = 1e-3):
    # BF16 and FP8 sketches, and the learned start with BF16 sketches, each against
    # the oracle's FP64 solution from a Gram accumulated from the stored A
    from paper_2006_05874_amd import learned as L
    from synth import make_problem_torch, spectrum
    n, d = 1 << 20, 4096
    sig = spectrum("exp", d, 400.0)
    nu2 = 1e-3 * float(sig[0]) ** 2
    A0, b, _ = make_problem_torch(n, d, sig, 0.1, 3, "cuda")
    A = rs.padded(n, d, dtype=torch.float32)
    A.copy_(A0)
    del A0
    params, mu, sd, _ = L.load_model()
    sols = {dt: rs.rs_adaptive_solve(A, b, nu2, sketch_dtype=dt) for dt in ("bf16", "fp8")}
    sols["learned_bf16"] = rs.rs_learned_solve(A, b, nu2, params, mu, sd, sketch_dtype="bf16")
    G = np.zeros((d, d))
    Atb = np.zeros(d)
    for r0 in range(0, n, 65536):
        Ac = A[r0:r0 + 65536].cpu().numpy().astype(np.float64)
        G += Ac.T @ Ac
        Atb += Ac.T @ b[r0:r0 + 65536].cpu().numpy().astype(np.float64)
    xs = ridge.solve_direct_from_gram(G, Atb, nu2)
    H = G + nu2 * np.eye(d)
    for name, (x, info) in sols.items():
        assert info["status"] == "ok", name
        assert ridge.relative_error(H, x.cpu().numpy(), xs) <= 1e-6, name
