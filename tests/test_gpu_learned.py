"""GPU parity of the learned-start form: features, MLP forward/backward and Adam
against the FP64 oracle, training on the GPU, and the learned solve's fallback."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import learned, ridge  # noqa: E402
from synth import config_c1, make_problem, spectrum  # noqa: E402

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


@pytest.mark.parametrize("n,d,dt", [(1024, 64, np.float64), (3000, 200, np.float64),
                                    (5000, 300, np.float32), (100, 37, np.float64),
                                    (9000, 8192, np.float32)])
def test_features_against_oracle(rs, n, d, dt):
    if d > 4096:
        # the evaluation width: Gaussian rows with decaying column scales (a Haar
        # rotation at this d costs half a minute of host time and is not needed here)
        rng = np.random.default_rng(n + d)
        A = (rng.standard_normal((n, d)) / np.sqrt(n) * spectrum("poly", d, 1.0)).astype(dt)
        nu2 = 1e-3
    else:
        p = make_problem(n, d, spectrum("poly", d, 1.0), 1e-3, 0.1, n + d, dtype=dt)
        A, nu2 = p.A, p.nu2
    f = host(rs.rs_features(dev_padded(A, rs), nu2, seed=7)).astype(np.float64)
    want = learned.features(A.astype(np.float64), nu2, 7)
    np.testing.assert_allclose(f[:3], want[:3], rtol=1e-6)
    # probes: FP32 storage of the feature; FP32 sketch for FP32 data
    tol = 1e-5 if dt == np.float64 else 2e-3
    np.testing.assert_allclose(f[3:11], want[3:11], rtol=0, atol=tol)
    np.testing.assert_allclose(f[11:], want[11:], rtol=0, atol=1e-5)


@pytest.fixture(scope="module")
def mlp_case():
    rng = np.random.default_rng(0)
    X = (rng.standard_normal((64, 16)) * 3 + 1).astype(np.float32)
    t = (rng.standard_normal(64) * 2 + 5).astype(np.float32)
    mu = X.mean(0).astype(np.float32)
    sd = (X.std(0) + 0.1).astype(np.float32)
    th = learned.init_params(1).astype(np.float32)
    return X, t, mu, sd, th


def test_mlp_forward_backward_against_oracle(rs, mlp_case):
    X, t, mu, sd, th = mlp_case
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    y, C = rs.rs_mlp_forward(d(th), d(X), d(mu), d(sd), cache=True)
    G, loss = rs.rs_mlp_backward(d(th), C, d(t))
    y_o, _ = learned.forward(th.astype(np.float64), X, mu.astype(np.float64), sd.astype(np.float64))
    l_o, g_o = learned.loss_and_grad(th.astype(np.float64), X, t, mu.astype(np.float64),
                                     sd.astype(np.float64))
    np.testing.assert_allclose(host(y), y_o, rtol=2e-5, atol=2e-5 * np.abs(y_o).max())
    assert abs(host(loss)[0] - l_o) <= 2e-5 * l_o
    np.testing.assert_allclose(host(G), g_o, rtol=0, atol=1e-5 * np.abs(g_o).max())


def test_mlp_gradient_central_differences_on_gpu(rs, mlp_case):
    X, t, mu, sd, th = mlp_case
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    _, C = rs.rs_mlp_forward(d(th), d(X), d(mu), d(sd), cache=True)
    G = host(rs.rs_mlp_backward(d(th), C, d(t))[0])
    th64 = th.astype(np.float64)
    for idx in np.random.default_rng(2).choice(th.size, 12, replace=False):
        e = np.zeros_like(th64)
        e[idx] = 1e-4
        lp, _ = learned.loss_and_grad(th64 + e, X, t, mu.astype(np.float64), sd.astype(np.float64))
        lm, _ = learned.loss_and_grad(th64 - e, X, t, mu.astype(np.float64), sd.astype(np.float64))
        assert abs((lp - lm) / 2e-4 - G[idx]) <= 1e-3 * max(1.0, abs(G[idx]))


def test_adam_against_oracle(rs, mlp_case):
    _, _, _, _, th = mlp_case
    rng = np.random.default_rng(3)
    P = torch.from_numpy(th.copy()).cuda()
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    cur, m, v = th.astype(np.float64), np.zeros(th.size), np.zeros(th.size)
    for step in range(1, 4):
        g = rng.standard_normal(th.size).astype(np.float32)
        rs.rs_mlp_adam_step(P, torch.from_numpy(g).cuda(), M, V, step)
        cur, m, v = learned.adam_step(cur, g.astype(np.float64), m, v, step)
    np.testing.assert_allclose(host(P), cur, rtol=0, atol=1e-6)


def test_training_on_gpu_lowers_the_loss(rs, mlp_case):
    X, t, mu, sd, th = mlp_case
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    P, Xd, td, mud, sdd = d(th.copy()), d(X), d(t), d(mu), d(sd)
    M, V = torch.zeros_like(P), torch.zeros_like(P)
    losses = []
    for step in range(1, 301):
        _, C = rs.rs_mlp_forward(P, Xd, mud, sdd, cache=True)
        G, loss = rs.rs_mlp_backward(P, C, td)
        rs.rs_mlp_adam_step(P, G, M, V, step, lr=3e-3)
        losses.append(float(host(loss)[0]))
    assert losses[-1] < 0.05 * losses[0]


@pytest.mark.parametrize("bias", [-5.0, 3.0, 30.0])
def test_learned_solve_falls_back_to_the_adaptive_rule(rs, bias):
    # any starting m converges (Theorems 5 and 6 hold for every m_initial): a
    # predictor forced to 2^-5, 2^3 or 2^30 (clamped) must still reach x*
    p = config_c1()
    th = np.zeros(18817, dtype=np.float32)
    th[-1] = bias
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x, info = rs.rs_learned_solve(dev_padded(p.A, rs), d(p.b), p.nu2, d(th),
                                  d(np.zeros(16, np.float32)), d(np.ones(16, np.float32)))
    expect = 1 if bias < 0 else min(2 ** int(math.floor(bias)), 1024)
    assert info["m_init"] == expect and info["status"] == "ok"
    xs = ridge.solve_direct(p.A, p.b, p.nu2)
    assert ridge.relative_error(ridge.hessian(p.A, p.nu2), host(x), xs) <= 1e-6


@pytest.mark.parametrize("bias", [3.0, 6.0])
def test_learned_start_at_origin_reuses_the_features_pass(rs, bias):
    # started at 0, a learned solve takes g_1 = -A^T b from the features pass
    # (eq. (1) at x = 0) instead of a gradient pass of its own: in FP64 it follows
    # the event trajectory of the plain solve started at the same m and lands on
    # the same x; a nonzero start still runs its own gradient pass and converges
    p = config_c1()
    th = np.zeros(18817, dtype=np.float32)
    th[-1] = bias
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    A, b = dev_padded(p.A, rs), d(p.b)
    mu, sd = d(np.zeros(16, np.float32)), d(np.ones(16, np.float32))
    x, il = rs.rs_learned_solve(A, b, p.nu2, d(th), mu, sd, seed=3)
    xp, ip = rs.rs_adaptive_solve(A, b, p.nu2, seed=3, m_init=il["m_init"])
    assert il["events"] == ip["events"] and il["steps"] == ip["steps"]
    np.testing.assert_allclose(host(x), host(xp), rtol=1e-9, atol=1e-12)
    xs = ridge.solve_direct(p.A, p.b, p.nu2)
    x0 = np.full(p.A.shape[1], 0.01)
    xw, iw = rs.rs_learned_solve(A, b, p.nu2, d(th), mu, sd, seed=3, x0=d(x0))
    xpw, ipw = rs.rs_adaptive_solve(A, b, p.nu2, seed=3, m_init=iw["m_init"], x0=d(x0))
    assert iw["events"] == ipw["events"]
    np.testing.assert_allclose(host(xw), host(xpw), rtol=1e-9, atol=1e-12)
    for xx in (x, xw):
        assert ridge.relative_error(ridge.hessian(p.A, p.nu2), host(xx), xs) <= 1e-6


def test_trained_model_gains_over_plain(rs):
    # held-out problems of the training distribution (indices never generated for
    # training): the committed predictor must skip most of the doubling ladder and
    # cut the total solve time, while every solve still meets its stopping rule;
    # the three smallest problems are checked against the oracle's solution
    from paper_2006_05874_amd import learned as L
    params, mu, sd, meta = L.load_model()
    assert meta["problems"] >= 20000
    plain_t = learned_t = 0.0
    plain_dbl, learned_dbl = [], []
    specs = [L.problem_spec(p) for p in range(2 * 10 ** 5, 2 * 10 ** 5 + 40)]
    small = sorted(range(len(specs)), key=lambda i: specs[i]["n"] * specs[i]["d"])[:3]
    import time
    for i, spec in enumerate(specs):
        A, b = L.make_device_problem(spec)
        rs.rs_adaptive_solve(A, b, spec["nu2"], seed=spec["seed"])      # warm allocations
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, ip = rs.rs_adaptive_solve(A, b, spec["nu2"], seed=spec["seed"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, il = rs.rs_learned_solve(A, b, spec["nu2"], params, mu, sd, seed=spec["seed"])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        plain_t += t1 - t0
        learned_t += t2 - t1
        assert ip["status"] == "ok" and il["status"] == "ok"
        plain_dbl.append(ip["doublings"])
        learned_dbl.append(il["doublings"])
        if i in small:
            A64 = host(A).astype(np.float64)
            b64 = host(b).astype(np.float64)
            xs = ridge.solve_direct(A64, b64, spec["nu2"])
            assert ridge.relative_error(ridge.hessian(A64, spec["nu2"]), host(x), xs) <= 1e-6
    assert np.mean(learned_dbl) <= 0.25 * np.mean(plain_dbl)
    assert learned_t < 0.8 * plain_t


def test_learned_batch_equals_single_learned_solves(rs):
    # uneven problems through the batched learned form: every job gives exactly
    # what rs_learned_solve gives alone (same prediction, same trajectory, same x)
    from paper_2006_05874_amd import learned as L
    params, mu, sd, _ = L.load_model()
    probs = []
    for i in range(6):
        n, d = [(4096, 100), (3000, 37), (8192, 300), (5000, 64), (2048, 250), (6000, 129)][i]
        p = make_problem(n, d, spectrum("poly", d, 1.0), 10.0 ** (-1 - i % 4), 0.1, 300 + i)
        probs.append((dev_padded(p.A, rs), torch.from_numpy(p.b).cuda(), p.nu2, p))
    res = rs.rs_learned_solve_batch([(A, b, nu2) for A, b, nu2, _ in probs], params, mu, sd,
                                    sketch_dtype="bf16", workers=3)
    for (A, b, nu2, p), (x, info) in zip(probs, res):
        x1, i1 = rs.rs_learned_solve(A, b, nu2, params, mu, sd, sketch_dtype="bf16")
        assert info["m_init"] == i1["m_init"] and info["events"] == i1["events"]
        assert info["status"] == "ok" and torch.equal(x, x1)
        A64 = p.A.astype(np.float64)
        xs = ridge.solve_direct(A64, p.b.astype(np.float64), nu2)
        assert ridge.relative_error(ridge.hessian(A64, nu2), host(x), xs) <= 1e-6


def test_full_size_65536x1024_learned_bf16_batched_and_plain(rs):
    # the benchmark's problem and launch configuration: both nu^2 solved as one
    # learned + BF16 batch over two streams, and by the plain FP32 method; every
    # solution against the oracle's FP64 solution of the stored problem
    from paper_2006_05874_amd import learned as L
    from synth import config_c2
    p = config_c2(nu2=1e-2, seed=0)
    A = dev_padded(p.A, rs)
    b = torch.from_numpy(p.b).cuda()
    params, mu, sd, _ = L.load_model()
    nus = (1e-2, 1e-4)
    res = rs.rs_learned_solve_batch([(A, b, nu) for nu in nus], params, mu, sd,
                                    sketch_dtype="bf16", workers=2)
    A64 = p.A.astype(np.float64)
    G = A64.T @ A64
    Atb = A64.T @ p.b.astype(np.float64)
    for nu, (x, info) in zip(nus, res):
        assert info["status"] == "ok"
        xs = ridge.solve_direct_from_gram(G, Atb, nu)
        assert ridge.relative_error(G + nu * np.eye(1024), host(x), xs) <= 1e-6
        xp, ip = rs.rs_adaptive_solve(A, b, nu, sketch_dtype="f32")
        assert ip["status"] == "ok"
        assert ridge.relative_error(G + nu * np.eye(1024), host(xp), xs) <= 1e-6
