"""Iterative Hessian sketch and the adaptive method (oracle side, FP64).

Test infrastructure: see the package docstring.

* Step sizes and rates: Theorem 1 (gradient-IHS) and Theorem 2 (Polyak-IHS),
  evaluated at the bounds of Definition 3.1 (Gaussian) or 3.2 (SRHT).
* Sketched Hessian H_S = A^T S^T S A + nu^2 I (eq. (3)),
  inverted through the Woodbury identity with an m x m Cholesky factor as in the
  proof of Theorem 7; when m >= d the d x d matrix is factored instead (it is
  the same H_S).
* Sketched Newton decrement r = 1/2 g^T H_S^-1 g (Lemma 1).
* Algorithm 1 ("Adaptive Polyak-IHS") and its gradient-only variant (Section
  4, numerical experiments).

Readings where the paper is silent:
  - x_0 = x_1 = the initial point.
  - After doubling m, g~_t is recomputed (as written) and so is r_t, which is
    defined as 1/2 g_t^T H_S^-1 g_t under the current sketch; r_1 and t keep
    their values; the retry starts again from the Polyak candidate.
  - Ties in the two ratio tests accept.
  - m is capped at m_max; a double rejection at the cap accepts the gradient
    candidate if it lowers r, and otherwise ends with "no convergence".
  - Stopping: the paper runs a fixed number of steps and measures precision
    against x*.  Here the run stops when r_t <= tol * r_ref, with
    r_ref = 1/2 g_1^T H_S^-1 g_1 re-evaluated under the current sketch, or after
    max_iter accepted steps.  With ref_at_zero the reference gradient is the one
    at the origin, g(0) = -A^T b, whatever the starting point: a warm-started
    solve then stops at the accuracy delta(x) / delta(0) a cold one would (a start
    at the origin is its own reference, so nothing extra is evaluated).
* Sparse A (the remark on sparse data matrices): the CountSketch, whose cost is
  O(nnz); the paper leaves its analysis open, so the step sizes are the SRHT's for
  the same rho, and a doubling refines each bucket into two (nested) or re-hashes
  (fresh).
* Underdetermined case (appendix, the dual problem): Algorithm 1 unchanged on the
  data matrix A^T with gradient A A^T z - b + nu^2 z; the primal solution is A^T z.
* Regularization path (Section 4, warm starts): nu^2 decreasing, each solve
  starting from the previous solution and at the previous final sketch size,
  with nested sketches so that one sketch family serves the whole path.
* IHS with refreshed embeddings (Section 1, the other IHS versions it cites): a
  new sketch of fixed size m at every step, the fixed-embedding step sizes, no
  tests and no doubling; an ablation of the fixed sketch.
"""
import math
from dataclasses import dataclass, field

import numpy as np

from . import ridge, sketch


# ---------------------------------------------------------------- parameters
def mu_gd(lam, Lam):
    """Theorem 1: mu_gd = 2 / (1/lambda + 1/Lambda)."""
    return 2.0 / (1.0 / lam + 1.0 / Lam)


def c_gd(lam, Lam):
    """Theorem 1: c_gd = ((Lambda - lambda) / (Lambda + lambda))^2."""
    return ((Lam - lam) / (Lam + lam)) ** 2


def mu_p(lam, Lam):
    """Theorem 2: mu_p = 4 / (1/sqrt(lambda) + 1/sqrt(Lambda))^2."""
    return 4.0 / (1.0 / math.sqrt(lam) + 1.0 / math.sqrt(Lam)) ** 2


def beta_p(lam, Lam):
    """Theorem 2: beta_p = ((sqrt(Lambda) - sqrt(lambda)) / (sqrt(Lambda) + sqrt(lambda)))^2."""
    return ((math.sqrt(Lam) - math.sqrt(lam)) / (math.sqrt(Lam) + math.sqrt(lam))) ** 2


def c_p(lam, Lam):
    """Theorem 2: c_p has the same expression as beta_p."""
    return ((math.sqrt(Lam) - math.sqrt(lam)) / (math.sqrt(Lam) + math.sqrt(lam))) ** 2


def srht_bounds(rho):
    """Definition 3.2: lambda = 1 - sqrt(rho), Lambda = 1 + sqrt(rho)."""
    if not 0.0 < rho < 1.0:
        raise ValueError("SRHT needs rho in (0, 1)")
    return 1.0 - math.sqrt(rho), 1.0 + math.sqrt(rho)


def gaussian_bounds(rho, eta):
    """Definition 3.1: (1 -+ sqrt(c_eta rho))^2 with c_eta = (1 + 3 sqrt(eta))^2."""
    if not (0.0 < rho <= 0.18 and 0.0 < eta <= 0.01):
        raise ValueError("Gaussian bounds need rho in (0, 0.18], eta in (0, 0.01]")
    c_eta = (1.0 + 3.0 * math.sqrt(eta)) ** 2
    s = math.sqrt(c_eta * rho)
    return (1.0 - s) ** 2, (1.0 + s) ** 2


@dataclass
class Params:
    mu_gd: float
    mu_p: float
    beta_p: float
    cbar_gd: float
    cbar_p: float


def params_for(kind, rho=0.1, eta=0.01):
    # the CountSketch takes the SRHT's bounds (a reading: the paper gives none)
    lam, Lam = srht_bounds(rho) if kind in ("srht", "count") else gaussian_bounds(rho, eta)
    return Params(mu_gd=mu_gd(lam, Lam), mu_p=mu_p(lam, Lam), beta_p=beta_p(lam, Lam),
                  cbar_gd=c_gd(lam, Lam), cbar_p=c_p(lam, Lam))


# ---------------------------------------------------------- sketched Hessian
class SketchedHessian:
    """H_S = (SA)^T SA + nu^2 I and its inverse.

    m < d : Woodbury, H_S^-1 = nu^-2 (I - (SA)^T (nu^2 I_m + SA SA^T)^-1 SA),
            with the m x m matrix factored by Cholesky (proof of Theorem 7).
    m >= d: Cholesky of the d x d matrix (SA)^T SA + nu^2 I_d.
    """

    def __init__(self, SA, nu2):
        self.SA = np.asarray(SA, dtype=np.float64)
        self.nu2 = float(nu2)
        m, d = self.SA.shape
        self.woodbury = m < d
        if self.woodbury:
            M = nu2 * np.eye(m) + self.SA @ self.SA.T
        else:
            M = self.SA.T @ self.SA + nu2 * np.eye(d)
        self.L = np.linalg.cholesky(M)

    def _chol_solve(self, y):
        return np.linalg.solve(self.L.T, np.linalg.solve(self.L, y))

    def solve(self, g):
        g = np.asarray(g, dtype=np.float64)
        if self.woodbury:
            z = self._chol_solve(self.SA @ g)
            return (g - self.SA.T @ z) / self.nu2
        return self._chol_solve(g)

    def decrement(self, g):
        """(H_S^-1 g, r) with r = 1/2 g^T H_S^-1 g (Lemma 1)."""
        gt = self.solve(g)
        return gt, 0.5 * float(np.dot(g, gt))


def make_sketch(A, kind, seed, sketch_id, m, gauss_precision="f64"):
    if kind == "count":
        return sketch.count_sketch(A, seed, sketch_id, m)
    if kind == "srht":
        SA, _ = sketch.srht_sketch(A, seed, sketch_id, m)
        return SA
    return sketch.gaussian_sketch(A, seed, sketch_id, m, precision=gauss_precision)


# ---------------------------------------------------------------- updates
def polyak_candidate(x, x_prev, gt, mu, beta):
    """Polyak-IHS update (eq. (2)): x - mu H_S^-1 g + beta (x - x_prev)."""
    return x - mu * gt + beta * (x - x_prev)


def gd_candidate(x, gt, mu):
    """Gradient-IHS update: eq. (2) with beta = 0."""
    return x - mu * gt


# ---------------------------------------------------------------- Algorithm 1
@dataclass
class Options:
    kind: str = "srht"           # "srht" | "gaussian"
    rho: float = 0.1
    eta: float = 0.01
    variant: str = "polyak"      # "polyak" (Algorithm 1) | "gd" (gradient-only variant)
    resample: str = "fresh"      # "fresh" (new sketch_id) | "nested"
    m_init: int = 1
    m_max: int = 0               # 0 -> padded n (SRHT) or n (Gaussian)
    tol: float = 1e-7
    max_iter: int = 200
    seed: int = 0
    gauss_precision: str = "f64"
    ref_at_zero: bool = False    # stop-test reference gradient at x = 0 (warm starts)


@dataclass
class Info:
    status: str = "ok"           # "ok" | "no_convergence"
    events: list = field(default_factory=list)   # (t, kind, m): kind in polyak|gd|double|stop
    m_final: int = 0
    doublings: int = 0
    grad_evals: int = 0
    applies: int = 0
    accepted_polyak: int = 0
    accepted_gd: int = 0
    t_final: int = 0
    r_history: list = field(default_factory=list)
    m_history: list = field(default_factory=list)


def adaptive_solve(A, b, nu2, opts=None, x_init=None):
    """Algorithm 1 (Polyak variant) or its gradient-only variant.

    Returns (x, info).  The structure follows the algorithm: sample S, form SA;
    g_1, g~_1, r_1; then per step a Polyak candidate with the test
    (r_p / r_1)^(1/t) <= cbar_p, else a gradient candidate with the test
    r_gd / r_t <= cbar_gd, else double m, resample, recompute g~_t and retry.
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return _algorithm1(A, lambda x: ridge.gradient(A, b, nu2, x), nu2, opts, x_init)


def adaptive_solve_dual(A, b, nu2, opts=None, z_init=None):
    """The underdetermined case (appendix, dual problem): Algorithm 1 on
    min_z 1/2 |A^T z - b^|^2 + nu^2/2 |z|^2, whose data matrix is A^T (d x n, the
    sketch acts on its d rows) and whose gradient A A^T z - b + nu^2 z needs no
    b^ = A^+ b.  Returns (x, z, info) with x = A^T z the primal solution."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    z, info = _algorithm1(A.T, lambda z: ridge.dual_gradient(A, b, nu2, z), nu2, opts, z_init)
    return A.T @ z, z, info


def adaptive_solve_sparse(A, b, nu2, opts=None, x_init=None):
    """Algorithm 1 for a sparse A (scipy.sparse, n x d) with the CountSketch
    (opts.kind "count"): the sketch and the gradient cost O(nnz).  Returns (x, info)."""
    b = np.asarray(b, dtype=np.float64)
    return _algorithm1(A, lambda x: ridge.sparse_gradient(A, b, nu2, x), nu2, opts, x_init)


def _algorithm1(A, gradient, nu2, opts, x_init):
    """Algorithm 1 for the ridge problem with data matrix A (n x d, sketched along
    its n rows) and gradient function `gradient`."""
    opts = opts or Options()
    n, d = A.shape
    prm = params_for(opts.kind, opts.rho, opts.eta)
    m_cap = sketch.next_pow2(n) if opts.kind == "srht" else n
    if opts.m_max:
        m_cap = min(m_cap, opts.m_max)
    m = min(opts.m_init, m_cap)
    sketch_id = 0

    def grad(x):
        info.grad_evals += 1
        return gradient(x)

    info = Info()
    x = np.zeros(d) if x_init is None else np.asarray(x_init, dtype=np.float64).copy()
    x_prev = x.copy()
    P = SketchedHessian(make_sketch(A, opts.kind, opts.seed, sketch_id, m, opts.gauss_precision), nu2)
    g = grad(x)
    gt, r = P.decrement(g)
    info.applies += 1
    r1 = r
    if opts.ref_at_zero and np.any(x != 0):
        g_ref = grad(np.zeros(d))
        _, r_ref = P.decrement(g_ref)
        info.applies += 1
    else:
        g_ref = g.copy()
        r_ref = r
    t = 1
    while True:
        info.r_history.append(r)
        info.m_history.append(m)
        if r <= opts.tol * r_ref:
            info.events.append((t, "stop", m))
            break
        if t >= opts.max_iter:
            info.status = "no_convergence"
            break
        accepted = None
        if opts.variant == "polyak":
            xp = polyak_candidate(x, x_prev, gt, prm.mu_p, prm.beta_p)
            gp = grad(xp)
            gtp, rp = P.decrement(gp)
            info.applies += 1
            if (rp / r1) ** (1.0 / t) <= prm.cbar_p:
                accepted = ("polyak", xp, gp, gtp, rp)
        if accepted is None:
            xg = gd_candidate(x, gt, prm.mu_gd)
            gg = grad(xg)
            gtg, rg = P.decrement(gg)
            info.applies += 1
            if rg / r <= prm.cbar_gd:
                accepted = ("gd", xg, gg, gtg, rg)
            elif m >= m_cap:
                if rg < r:
                    accepted = ("gd", xg, gg, gtg, rg)
                else:
                    info.status = "no_convergence"
                    break
        if accepted is None:
            m = min(2 * m, m_cap)
            if opts.resample == "fresh":
                sketch_id += 1
            P = SketchedHessian(make_sketch(A, opts.kind, opts.seed, sketch_id, m,
                                            opts.gauss_precision), nu2)
            gt, r = P.decrement(g)
            _, r_ref = P.decrement(g_ref)
            info.applies += 2
            info.doublings += 1
            info.events.append((t, "double", m))
            continue
        kind_acc, x_new, g, gt, r = accepted
        info.events.append((t, kind_acc, m))
        if kind_acc == "polyak":
            info.accepted_polyak += 1
        else:
            info.accepted_gd += 1
        x_prev, x = x, x_new
        t += 1
    info.m_final = m
    info.t_final = t
    return x, info


def solve_path(A, b, nu2s, opts=None):
    """Regularization path: nu^2 in the given (non-increasing) order, each solve
    warm-started at the previous solution, starting at the previous final m, with
    nested sketches and the stop test referred to x = 0.  Returns (X, infos) with
    X[j] the solution at nu2s[j]."""
    opts = opts or Options()
    A = np.asarray(A, dtype=np.float64)
    d = A.shape[1]
    X = np.zeros((len(nu2s), d))
    infos = []
    x = np.zeros(d)
    m = opts.m_init
    for j, nu2 in enumerate(nu2s):
        if j and nu2 > nu2s[j - 1]:
            raise ValueError("solve_path: nu^2 must not increase along the path")
        o = Options(**{**opts.__dict__, "m_init": m, "resample": "nested", "ref_at_zero": True})
        x, info = adaptive_solve(A, b, nu2, o, x_init=x)
        X[j] = x
        infos.append(info)
        m = info.m_final
    return X, infos


@dataclass
class RefreshInfo:
    status: str = "ok"
    steps: int = 0            # updates taken
    r_history: list = field(default_factory=list)


def refreshed_ihs(A, b, nu2, m, opts=None, x_init=None):
    """IHS with refreshed embeddings (Section 1, other versions of the IHS): the
    update of eq. (2) (beta = 0 for the gradient variant) with a new sketch
    S_t of fixed size m drawn at every step (sketch_id = t - 1) and H_{S_t}
    re-formed; no acceptance tests and no doubling.  The parameters are the
    fixed-embedding ones for (kind, rho, eta).  Stops once
    r_t = 1/2 g_t^T H_{S_t}^-1 g_t <= tol * r_1 or after max_iter updates.
    Returns (x, RefreshInfo)."""
    opts = opts or Options()
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n, d = A.shape
    prm = params_for(opts.kind, opts.rho, opts.eta)
    mu, beta = (prm.mu_p, prm.beta_p) if opts.variant == "polyak" else (prm.mu_gd, 0.0)
    x = np.zeros(d) if x_init is None else np.asarray(x_init, dtype=np.float64).copy()
    x_prev = x.copy()
    info = RefreshInfo()
    r1 = None
    t = 1
    while True:
        P = SketchedHessian(make_sketch(A, opts.kind, opts.seed, t - 1, m, opts.gauss_precision),
                            nu2)
        gt, r = P.decrement(ridge.gradient(A, b, nu2, x))
        info.r_history.append(r)
        if r1 is None:
            r1 = r
        if r <= opts.tol * r1:
            break
        if info.steps >= opts.max_iter:
            info.status = "no_convergence"
            break
        x_prev, x = x, polyak_candidate(x, x_prev, gt, mu, beta)
        info.steps += 1
        t += 1
    return x, info
