"""Learned starting sketch size (oracle side, FP64).

Test infrastructure: see the package docstring.

The paper's guarantees for Algorithm 1 hold for any initial sketch size
m_initial >= 1 (Theorems 5 and 6), and it mentions a Hutchinson-type trace
estimate of d_e as a heuristic (Section 1).  The learned form predicts log2 of
the final sketch size of a plain run from cheap features and starts the
doubling ladder there; the adaptive rule stays in place as the fallback.

Features (16, in this order):
  0  log2 n            1  log2 d            2  log10 nu^2
  3..10  log of the 8 Hutchinson probes q_k = (A^T w_k)^T H_S0^-1 (A^T w_k),
         w_k Rademacher (Philox stream 7, sketch_id k, index = row), H_S0 the
         sketched Hessian of a min(256, padded n)-row SRHT (seed, sketch_id
         0x7fff0000) -- an estimate of tr(A H^-1 A^T) = d_e
  11..15 quantiles (0, 1/4, 1/2, 3/4, 1) of the log column norms ln ||A e_j||,
         each the order statistic at index round(q (d - 1)).
MLP: 16 -> 128 -> 128 -> 1, exact GELU (x Phi(x)) on both hidden layers, inputs
standardised as (f - mu) / sd.  Loss: mean squared error.  Adam.

Parity unpinned: the trained predictor's quality (it is measured, not pinned).
"""
import math

import numpy as np

from . import ihs, philox, sketch

N_FEAT = 16
H = 128
PROBE_SKETCH_ID = 0x7FFF0000
PROBE_ROWS = 256
QUANTILES = (0.0, 0.25, 0.5, 0.75, 1.0)

# flat parameter layout
OFF_W1 = 0
OFF_B1 = OFF_W1 + N_FEAT * H
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + H
N_PARAMS = OFF_B3 + 1


def probe_signs(seed, k, n):
    w0, _, _, _ = philox.draw(seed, philox.STREAM_PROBE, k, np.arange(n, dtype=np.uint64))
    return 1.0 - 2.0 * (w0 & np.uint64(1)).astype(np.float64)


def features(A, nu2, seed):
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    m0 = min(PROBE_ROWS, sketch.next_pow2(n))
    SA, _ = sketch.srht_sketch(A, seed, PROBE_SKETCH_ID, m0)
    P = ihs.SketchedHessian(SA, nu2)
    f = np.empty(N_FEAT)
    f[0] = math.log2(n)
    f[1] = math.log2(d)
    f[2] = math.log10(nu2)
    for k in range(8):
        u = A.T @ probe_signs(seed, k, n)
        f[3 + k] = math.log(max(float(u @ P.solve(u)), 1e-30))
    lcn = np.sort(0.5 * np.log(np.maximum(np.sum(A * A, axis=0), 1e-300)))
    for i, q in enumerate(QUANTILES):
        f[11 + i] = lcn[int(round(q * (d - 1)))]
    return f


def unpack(theta):
    th = np.asarray(theta, dtype=np.float64)
    W1 = th[OFF_W1:OFF_B1].reshape(N_FEAT, H)
    b1 = th[OFF_B1:OFF_W2]
    W2 = th[OFF_W2:OFF_B2].reshape(H, H)
    b2 = th[OFF_B2:OFF_W3]
    W3 = th[OFF_W3:OFF_B3]
    b3 = th[OFF_B3]
    return W1, b1, W2, b2, W3, b3


def gelu(z):
    """Exact GELU: z * Phi(z) = z (1 + erf(z / sqrt 2)) / 2."""
    from scipy.special import erf
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    from scipy.special import erf
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def forward(theta, X, mu, sd):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    Xn = (np.asarray(X, dtype=np.float64) - mu) / sd
    Z1 = Xn @ W1 + b1
    H1 = gelu(Z1)
    Z2 = H1 @ W2 + b2
    H2 = gelu(Z2)
    y = H2 @ W3 + b3
    return y, (Xn, Z1, H1, Z2, H2)


def loss_and_grad(theta, X, t, mu, sd):
    """MSE loss mean((y - t)^2) and its gradient w.r.t. the flat parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    y, (Xn, Z1, H1, Z2, H2) = forward(theta, X, mu, sd)
    B = len(t)
    r = y - np.asarray(t, dtype=np.float64)
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B
    g = np.zeros(N_PARAMS)
    g[OFF_W3:OFF_B3] = H2.T @ dy
    g[OFF_B3] = dy.sum()
    dZ2 = np.outer(dy, W3) * gelu_grad(Z2)
    g[OFF_W2:OFF_B2] = (H1.T @ dZ2).ravel()
    g[OFF_B2:OFF_W3] = dZ2.sum(0)
    dZ1 = (dZ2 @ W2.T) * gelu_grad(Z1)
    g[OFF_W1:OFF_B1] = (Xn.T @ dZ1).ravel()
    g[OFF_B1:OFF_W2] = dZ1.sum(0)
    return loss, g


def adam_step(theta, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; returns new arrays."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """He-style initialisation: W ~ N(0, 2 / fan_in), biases 0."""
    rng = np.random.default_rng(seed)
    th = np.zeros(N_PARAMS)
    th[OFF_W1:OFF_B1] = rng.standard_normal(N_FEAT * H) * math.sqrt(2.0 / N_FEAT)
    th[OFF_W2:OFF_B2] = rng.standard_normal(H * H) * math.sqrt(2.0 / H)
    th[OFF_W3:OFF_B3] = rng.standard_normal(H) * math.sqrt(1.0 / H)
    return th
