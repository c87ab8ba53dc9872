"""Pins for the oracle's learned-form pieces: MLP gradients against torch
autograd (a library routine) and central differences, Adam against torch.optim,
GELU against torch, and the Hutchinson probe's expectation."""
import math

import numpy as np
import pytest
import torch

from oracle import ihs, learned, ridge, sketch
from synth import make_problem, spectrum


@pytest.fixture(scope="module")
def batch():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((32, learned.N_FEAT)) * 3 + 1
    t = rng.standard_normal(32) * 2 + 5
    mu = X.mean(0)
    sd = X.std(0) + 0.1
    return X, t, mu, sd, learned.init_params(1)


def test_gelu_against_torch():
    z = np.linspace(-6, 6, 1001)
    want = torch.nn.functional.gelu(torch.from_numpy(z), approximate="none").numpy()
    np.testing.assert_allclose(learned.gelu(z), want, rtol=1e-14, atol=1e-15)
    zt = torch.from_numpy(z).requires_grad_(True)
    torch.nn.functional.gelu(zt, approximate="none").sum().backward()
    np.testing.assert_allclose(learned.gelu_grad(z), zt.grad.numpy(), rtol=1e-12, atol=1e-14)


def test_mlp_gradient_against_torch_autograd(batch):
    X, t, mu, sd, th = batch
    loss, g = learned.loss_and_grad(th, X, t, mu, sd)
    T = torch.from_numpy(th.copy()).requires_grad_(True)
    W1 = T[learned.OFF_W1:learned.OFF_B1].view(learned.N_FEAT, learned.H)
    b1 = T[learned.OFF_B1:learned.OFF_W2]
    W2 = T[learned.OFF_W2:learned.OFF_B2].view(learned.H, learned.H)
    b2 = T[learned.OFF_B2:learned.OFF_W3]
    W3 = T[learned.OFF_W3:learned.OFF_B3]
    b3 = T[learned.OFF_B3]
    Xn = (torch.from_numpy(X) - torch.from_numpy(mu)) / torch.from_numpy(sd)
    gelu = lambda z: torch.nn.functional.gelu(z, approximate="none")
    y = gelu(gelu(Xn @ W1 + b1) @ W2 + b2) @ W3 + b3
    L = torch.mean((y - torch.from_numpy(t)) ** 2)
    L.backward()
    assert abs(L.item() - loss) < 1e-12 * max(1, loss)
    np.testing.assert_allclose(g, T.grad.numpy(), rtol=1e-9, atol=1e-12)


def test_mlp_gradient_central_differences(batch):
    X, t, mu, sd, th = batch
    _, g = learned.loss_and_grad(th, X, t, mu, sd)
    rng = np.random.default_rng(3)
    for idx in rng.choice(learned.N_PARAMS, 40, replace=False):
        e = np.zeros_like(th)
        e[idx] = 1e-6
        lp, _ = learned.loss_and_grad(th + e, X, t, mu, sd)
        lm, _ = learned.loss_and_grad(th - e, X, t, mu, sd)
        assert abs((lp - lm) / 2e-6 - g[idx]) <= 1e-5 * max(1.0, abs(g[idx]))


def test_adam_against_torch(batch):
    X, t, mu, sd, th = batch
    T = torch.from_numpy(th.copy()).requires_grad_(True)
    opt = torch.optim.Adam([T], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    cur = th.copy()
    rng = np.random.default_rng(4)
    for step in range(1, 6):
        g = rng.standard_normal(th.size)
        T.grad = torch.from_numpy(g.copy())
        opt.step()
        cur, m, v = learned.adam_step(cur, g, m, v, step)
    np.testing.assert_allclose(cur, T.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_training_decreases_loss(batch):
    X, t, mu, sd, th = batch
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    l0, _ = learned.loss_and_grad(th, X, t, mu, sd)
    for step in range(1, 200):
        _, g = learned.loss_and_grad(th, X, t, mu, sd)
        th, m, v = learned.adam_step(th, g, m, v, step, lr=3e-3)
    l1, _ = learned.loss_and_grad(th, X, t, mu, sd)
    assert l1 < 0.05 * l0


def test_probe_is_a_trace_estimate():
    # E_w[(A^T w)^T P (A^T w)] = tr(A P A^T); with the full sketch P = H^-1 and the
    # trace is d_e (Section 1's definition)
    p = make_problem(512, 24, spectrum("geom", 24, 0.8), 1e-2, 0.1, 5, dtype=np.float64)
    P = ihs.SketchedHessian(sketch.srht_sketch(p.A, 1, learned.PROBE_SKETCH_ID, 512)[0], p.nu2)
    vals = []
    for k in range(400):
        u = p.A.T @ learned.probe_signs(1, k, 512)
        vals.append(u @ P.solve(u))
    de = ridge.effective_dimension_trace(p.A, p.nu2)
    assert abs(np.mean(vals) - de) < 4 * np.std(vals) / math.sqrt(len(vals))


def test_features_shape_and_order():
    p = make_problem(1000, 40, spectrum("poly", 40, 1.0), 1e-3, 0.1, 2, dtype=np.float64)
    f = learned.features(p.A, p.nu2, 3)
    assert f.shape == (16,)
    assert f[0] == math.log2(1000) and f[1] == math.log2(40) and abs(f[2] + 3) < 1e-12
    assert np.all(np.diff(f[11:16]) >= 0)
    lcn = 0.5 * np.log(np.sum(p.A ** 2, 0))
    assert f[11] == lcn.min() and f[15] == lcn.max()
