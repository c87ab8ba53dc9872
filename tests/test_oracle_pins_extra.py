"""Pins for the oracle helpers that the full-size GPU checks lean on (CPU only).

* ``sketch.srht_sketch_rows`` (a few rows of SA, used at large n where the whole
  sketch is out of reach) against the pinned dense ``sketch.srht_sketch`` and
  against an SRHT built from ``scipy.linalg.hadamard`` (Appendix C.2: S = R H
  diag(eps), scaled by 1/sqrt(m) with the +-1 Hadamard matrix).
* ``ridge.solve_direct_from_gram`` (x* from a Gram accumulated elsewhere, used for
  every full-size check) against the SVD closed form of eq. (1) and against a
  vanishing gradient.
* Algorithm 1's Polyak test (r_p / r_1)^(1/t) <= cbar_p with t the step index,
  pinned without replaying the oracle's own record: with the full SRHT (m = padded
  n) S^T S = I, so C_S = I and the error recursion of the proof of Theorems 1-2
  reduces to the scalar heavy-ball recursion e_{t+1} = (1 + beta - mu) e_t -
  beta e_{t-1} along x*.  From x_0 = x_1 = 0 every decrement is c_t^2 r_1 with
  c_t from that recursion, so the accept/reject sequence follows in closed form.
"""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import ihs, philox, ridge, sketch
from synth import make_problem, spectrum


# ------------------------------------------------------------ srht_sketch_rows
@pytest.mark.parametrize("n,m", [(64, 8), (100, 16), (257, 40), (128, 128)])
def test_srht_rows_equal_dense_sketch(n, m):
    rng = np.random.default_rng(n + m)
    A = rng.standard_normal((n, 5))
    full, _ = sketch.srht_sketch(A, 7, 3, m)
    which = sorted(set([0, m - 1, m // 2] + list(rng.integers(0, m, 4))))
    part = sketch.srht_sketch_rows(A, 7, 3, m, which)
    np.testing.assert_allclose(part, full[which], rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,m", [(64, 8), (100, 16)])
def test_srht_rows_equal_library_hadamard(n, m):
    """Independent construction: S = (1/sqrt(m)) R H_pm diag(eps) with H_pm from
    scipy (Sylvester order), zero-padded rows of A beyond n."""
    rng = np.random.default_rng(11)
    A = rng.standard_normal((n, 3))
    npad = sketch.next_pow2(n)
    H = scipy.linalg.hadamard(npad).astype(np.float64)
    eps = philox.rademacher_signs(5, 2, npad)
    keys = philox.row_keys(5, 2, npad)
    order = np.lexsort((np.arange(npad), keys))
    rows = np.sort(order[:m])
    Apad = np.zeros((npad, 3))
    Apad[:n] = A
    want = (H[rows] * eps[None, :]) @ Apad / math.sqrt(m)
    got = sketch.srht_sketch_rows(A, 5, 2, m, list(range(m)))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_srht_rows_planted_sign_error_is_caught():
    """A sign slice off by one row (the plausible slip) changes the rows."""
    rng = np.random.default_rng(2)
    A = rng.standard_normal((64, 4))
    full, rows = sketch.srht_sketch(A, 1, 0, 8)
    eps = sketch.srht_signs(1, 0, 64)
    shifted = np.roll(eps, 1)
    h = sketch.hadamard_entries(rows[[0]], np.arange(64))[0]
    wrong = (h * shifted) @ A / math.sqrt(8)
    assert np.max(np.abs(wrong - full[0])) > 1e-3


# ------------------------------------------------------- solve_direct_from_gram
@pytest.mark.parametrize("nu2", [1.0, 1e-2, 1e-6])
def test_direct_from_gram_equals_svd_closed_form(nu2):
    p = make_problem(300, 24, spectrum("geom", 24, 0.7), nu2, 0.05, 4, dtype=np.float64)
    G = p.A.T @ p.A
    Atb = p.A.T @ p.b
    x = ridge.solve_direct_from_gram(G, Atb, nu2)
    xs = ridge.solve_svd(p.A, p.b, nu2)
    np.testing.assert_allclose(x, xs, rtol=1e-9, atol=1e-12 * np.linalg.norm(xs))
    g = ridge.gradient(p.A, p.b, nu2, x)
    assert np.linalg.norm(g) <= 1e-10 * np.linalg.norm(Atb)


def test_direct_from_gram_chunked_sum_equals_whole():
    """The full-size checks accumulate the Gram in row blocks; the sum of block
    Grams gives the same solution."""
    p = make_problem(512, 16, spectrum("poly", 16, 1.0), 1e-3, 0.1, 6, dtype=np.float64)
    G = np.zeros((16, 16))
    Atb = np.zeros(16)
    for r0 in range(0, 512, 96):
        Ac, bc = p.A[r0:r0 + 96], p.b[r0:r0 + 96]
        G += Ac.T @ Ac
        Atb += Ac.T @ bc
    x = ridge.solve_direct_from_gram(G, Atb, 1e-3)
    np.testing.assert_allclose(x, ridge.solve_svd(p.A, p.b, 1e-3), rtol=1e-9, atol=1e-12)


def test_direct_from_gram_planted_shift_error_is_caught():
    p = make_problem(200, 10, spectrum("geom", 10, 0.8), 1e-2, 0.05, 1, dtype=np.float64)
    G, Atb = p.A.T @ p.A, p.A.T @ p.b
    wrong = ridge.solve_direct_from_gram(G, Atb, 2e-2)   # nu instead of nu^2, say
    xs = ridge.solve_svd(p.A, p.b, 1e-2)
    assert np.linalg.norm(wrong - xs) > 1e-4 * np.linalg.norm(xs)


# ------------------------------------------------ Polyak test at C_S = I
def _scalar_algorithm1(prm, polyak, tol, max_steps=60):
    """Algorithm 1 on the scalar error model e_t = c_t x* (C_S = I, x_0 = x_1 = 0):
    the decrement at an iterate with coefficient c is c^2 r_1.  Returns the
    accepted kinds and the decrement ratios r_t / r_1 after each step."""
    c_prev, c = -1.0, -1.0          # e_0 = e_1 = -x*
    kinds, ratios = [], [1.0]
    t = 1
    while c * c > tol and t <= max_steps:
        acc = None
        if polyak:
            cp = (1.0 + prm.beta_p - prm.mu_p) * c - prm.beta_p * c_prev
            if (cp * cp) ** (1.0 / t) <= prm.cbar_p:     # (r_p / r_1)^(1/t)
                acc = ("polyak", cp)
        if acc is None:
            cg = (1.0 - prm.mu_gd) * c
            assert (cg * cg) / (c * c) <= prm.cbar_gd    # C_S = I: always accepted
            acc = ("gd", cg)
        kinds.append(acc[0])
        c_prev, c = c, acc[1]
        ratios.append(c * c)
        t += 1
    return kinds, ratios


@pytest.mark.parametrize("variant", ["polyak", "gd"])
@pytest.mark.parametrize("rho", [0.1, 0.3])
def test_polyak_test_follows_closed_form_at_full_sketch(variant, rho):
    n, d = 64, 6
    p = make_problem(n, d, spectrum("geom", d, 0.8), 1e-2, 0.05, 9, dtype=np.float64)
    tol = 1e-14
    opts = ihs.Options(kind="srht", rho=rho, variant=variant, m_init=n, tol=tol, max_iter=80)
    _, info = ihs.adaptive_solve(p.A, p.b, p.nu2, opts)
    prm = ihs.params_for("srht", rho)
    kinds, ratios = _scalar_algorithm1(prm, variant == "polyak", tol)
    got = [ev for (_, ev, _) in info.events if ev in ("polyak", "gd")]
    assert info.doublings == 0
    assert got == kinds
    r1 = info.r_history[0]
    np.testing.assert_allclose(np.array(info.r_history) / r1, ratios, rtol=1e-6, atol=1e-15)


def test_polyak_closed_form_first_steps():
    """The first two Polyak steps by hand: c_2 = mu_p - 1 and
    c_3 = (1 + beta_p - mu_p)(mu_p - 1) + beta_p; both pass (c^2)^(1/t) <= beta_p
    at rho = 0.1 (t = 1, then t = 2), while the same values fail if the exponent
    were 1/(t+1) at t = 1 -- the slip this pin is there to catch."""
    prm = ihs.params_for("srht", 0.1)
    a, bt = prm.mu_p, prm.beta_p
    c2 = a - 1.0
    c3 = (1.0 + bt - a) * c2 + bt
    assert (c2 * c2) ** (1.0 / 1) <= prm.cbar_p
    assert (c3 * c3) ** (1.0 / 2) <= prm.cbar_p
    assert (c2 * c2) ** (1.0 / 2) > prm.cbar_p
    kinds, _ = _scalar_algorithm1(prm, True, 1e-30, max_steps=2)
    assert kinds[:2] == ["polyak", "polyak"]
