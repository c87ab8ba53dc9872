"""A bound on the relative prediction error for problems too large for the FP64 Gram.

Test infrastructure: see the package docstring.

The error metric of Section 1.1 is delta(x) / delta(0) with
delta(x) = 1/2 (x - x*)^T H (x - x*), H = A^T A + nu^2 I.  Since the gradient of
eq. (1) is g(x) = A^T (A x - b) + nu^2 x = H (x - x*), delta(x) = 1/2 g^T H^-1 g and
delta(0) = 1/2 c^T H^-1 c with c = A^T b.  Neither needs x*, only H^-1 applied to
a known vector, which the two bounds below replace by quantities that one pass
over the rows of A provides (no d x d Gram, no factorisation of H):

* upper bound on delta(x): for any M with 0 < M <= H (Loewner order),
  H^-1 <= M^-1, so delta(x) <= 1/2 g^T M^-1 g.  M = nu^2 I + K_N with K_N the
  Nystrom approximation Y (Omega^T Y)^-1 Y^T of K = A^T A from a Gaussian test
  matrix Omega (d x k) and Y = K Omega; K_N <= K holds for every PSD K
  (K - K_N = K^1/2 (I - P) K^1/2 with P the orthogonal projector onto the
  range of K^1/2 Omega).  The bound is tight up to (lambda_{k+1}(K) + nu^2) / nu^2
  on the part of g outside the top-k eigenspace, and exact when k = d.
* lower bound on delta(0): the concave quadratic 2 v^T c - v^T H v is at most
  c^T H^-1 c for every v, with equality at v = H^-1 c = x*; v is the point being
  judged (close to x*), so the bound is close to exact, and a poor point can only
  weaken it.  Also c^T H^-1 c >= |c|^2 / (|A|_F^2 + nu^2) (H <= (|A|_F^2 + nu^2) I);
  the larger of the two is used.

Everything is FP64 (A and b are the stored values, upcast).  The pass over A is
fed row blocks in any order and any split; sums are plain FP64 products.
"""
import numpy as np


class StreamedCertificate:
    """Accumulate, over row blocks of (A, b), what the bounds need for a set of
    points X (d x s, one column per point): A^T (A X - b), |A X|^2 per column,
    A^T b, |A|_F^2 and Y = A^T A Omega for a seeded Gaussian Omega (d x k)."""

    def __init__(self, d, X, k=256, seed=12345):
        self.d = int(d)
        self.X = np.asarray(X, dtype=np.float64).reshape(self.d, -1)
        k = int(min(k, self.d))
        rng = np.random.default_rng(seed)
        self.Omega = rng.standard_normal((self.d, k))
        self.Y = np.zeros((self.d, k))
        self.R = np.zeros_like(self.X)           # A^T (A X - b)
        self.ax2 = np.zeros(self.X.shape[1])     # |A x|^2 per point
        self.c = np.zeros(self.d)                # A^T b
        self.fro = 0.0
        self.rows = 0

    def add(self, Ab, bb):
        """One row block: Ab (r x d) and bb (r), any float type."""
        Ab = np.asarray(Ab, dtype=np.float64)
        bb = np.asarray(bb, dtype=np.float64)
        AX = Ab @ self.X
        self.R += Ab.T @ (AX - bb[:, None])
        self.ax2 += np.einsum("ij,ij->j", AX, AX)
        self.c += Ab.T @ bb
        self.fro += float(np.einsum("ij,ij->", Ab, Ab))
        self.Y += Ab.T @ (Ab @ self.Omega)
        self.rows += Ab.shape[0]

    def _nystrom(self):
        """U (d x k'), lam (k'): K_N = U diag(lam) U^T, from W = Omega^T Y = L L^T
        and the SVD of B = Y L^-T (K_N = B B^T)."""
        Y, Om = self.Y, self.Omega
        k = Y.shape[1]
        while k > 0:
            W = Om[:, :k].T @ Y[:, :k]
            W = 0.5 * (W + W.T)
            try:
                L = np.linalg.cholesky(W)
                break
            except np.linalg.LinAlgError:
                k //= 2   # a numerically singular W: keep a leading subset
        if k == 0:
            return np.zeros((self.d, 0)), np.zeros(0)
        B = np.linalg.solve(L, Y[:, :k].T).T   # Y L^-T
        U, s, _ = np.linalg.svd(B, full_matrices=False)
        return U, s * s

    def bounds(self, nu2, cols=None):
        """Per point j (or the listed columns): (upper bound on delta(x_j),
        lower bound on delta(0), their ratio).  nu2 may differ per column
        (a scalar or one value per listed column)."""
        cols = list(range(self.X.shape[1])) if cols is None else list(cols)
        nu2s = np.broadcast_to(np.asarray(nu2, dtype=np.float64), (len(cols),))
        U, lam = self._nystrom()
        out = []
        for j, nu in zip(cols, nu2s):
            x = self.X[:, j]
            g = self.R[:, j] + nu * x
            ug = U.T @ g
            rest = g - U @ ug
            up = 0.5 * (float(rest @ rest) / nu + float(np.sum(ug * ug / (lam + nu))))
            dual = float(x @ self.c) - 0.5 * (self.ax2[j] + nu * float(x @ x))
            spec = 0.5 * float(self.c @ self.c) / (self.fro + nu)
            lo = max(dual, spec)
            out.append((up, lo, up / lo))
        return out
