"""The regularised least-squares problem (oracle side, FP64).

Test infrastructure: see the package docstring.

Problem (eq. (1)): x* = argmin_x f(x) = 1/2 ||Ax - b||^2 + nu^2/2 ||x||^2,
with A (n x d), n >= d.  Section 1.1 ("Notations") defines the stacked matrix
Abar = [A; nu I], the error delta(x) = 1/2 ||Abar (x - x*)||^2, the diagonal
D = diag(sigma_i / sqrt(sigma_i^2 + nu^2)) and the effective dimension.

The method converges to x* for any sketch: the fixed point of the update
(eq. (2)) is grad f = 0 (error recursion in the proof of Theorems 1-2),
so the final-answer oracle is the plain definition written out below.
"""
import numpy as np


def gradient(A, b, nu2, x):
    """grad f(x) = A^T (A x - b) + nu^2 x (from eq. (1))."""
    A = np.asarray(A, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    return A.T @ (A @ x - np.asarray(b, dtype=np.float64)) + nu2 * x


def sparse_gradient(A, b, nu2, x):
    """grad f(x) = A^T (A x - b) + nu^2 x for a scipy.sparse A (two products)."""
    x = np.asarray(x, dtype=np.float64)
    return A.T @ (A @ x - np.asarray(b, dtype=np.float64)) + nu2 * x


def dual_gradient(A, b, nu2, z):
    """grad g(z) = A A^T z - b + nu^2 z: the gradient of the dual problem of the
    underdetermined case (appendix), min_z 1/2 |A^T z|^2 + nu^2/2 |z|^2 - b^T z."""
    A = np.asarray(A, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    return A @ (A.T @ z) - np.asarray(b, dtype=np.float64) + nu2 * z


def solve_dual_direct(A, b, nu2):
    """z* = (A A^T + nu^2 I)^-1 b by Cholesky: the dual optimum (appendix)."""
    A = np.asarray(A, dtype=np.float64)
    L = np.linalg.cholesky(A @ A.T + nu2 * np.eye(A.shape[0]))
    return np.linalg.solve(L.T, np.linalg.solve(L, np.asarray(b, dtype=np.float64)))


def hessian(A, nu2):
    """H = Abar^T Abar = A^T A + nu^2 I."""
    A = np.asarray(A, dtype=np.float64)
    return A.T @ A + nu2 * np.eye(A.shape[1])


def solve_direct(A, b, nu2):
    """x* from the normal equations (A^T A + nu^2 I) x = A^T b by Cholesky."""
    A = np.asarray(A, dtype=np.float64)
    H = hessian(A, nu2)
    L = np.linalg.cholesky(H)
    rhs = A.T @ np.asarray(b, dtype=np.float64)
    y = np.linalg.solve(L, rhs)
    return np.linalg.solve(L.T, y)


def solve_direct_from_gram(G, Atb, nu2):
    """Same as solve_direct from a precomputed Gram A^T A and A^T b."""
    H = np.asarray(G, dtype=np.float64) + nu2 * np.eye(G.shape[0])
    L = np.linalg.cholesky(H)
    return np.linalg.solve(L.T, np.linalg.solve(L, np.asarray(Atb, dtype=np.float64)))


def solve_svd(A, b, nu2):
    """x* = V diag(sigma / (sigma^2 + nu^2)) U^T b, from A = U Sigma V^T."""
    U, s, Vt = np.linalg.svd(np.asarray(A, dtype=np.float64), full_matrices=False)
    return Vt.T @ ((s / (s * s + nu2)) * (U.T @ np.asarray(b, dtype=np.float64)))


def delta(H, x, xstar):
    """delta(x) = 1/2 (x - x*)^T H (x - x*) = 1/2 ||Abar (x - x*)||^2."""
    e = np.asarray(x, dtype=np.float64) - np.asarray(xstar, dtype=np.float64)
    return 0.5 * float(e @ (H @ e))


def relative_error(H, x, xstar):
    """delta(x) / delta(0): the squared relative prediction error."""
    return delta(H, x, xstar) / delta(H, np.zeros_like(xstar), xstar)


def effective_dimension_trace(A, nu2):
    """d_e = trace(A (A^T A + nu^2 I)^-1 A^T), computed without an SVD."""
    A = np.asarray(A, dtype=np.float64)
    H = hessian(A, nu2)
    return float(np.trace(A @ np.linalg.solve(H, A.T)))


def effective_dimension_svd(A, nu2):
    """sum_i sigma_i^2 / (sigma_i^2 + nu^2) = ||D||_F^2."""
    s = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    return float(np.sum(s * s / (s * s + nu2)))


def effective_dimension_ratio(A, nu2):
    """d_e = ||D||_F^2 / ||D||_2^2 (the definition in Section 1.1)."""
    s = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    dd = s * s / (s * s + nu2)
    return float(np.sum(dd) / np.max(dd))


def stacked_svd(A, nu2):
    """Ubar, Sigmabar, V of Abar = [A; nu I] as built in the proof of Theorems 1-2."""
    A = np.asarray(A, dtype=np.float64)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    nu = np.sqrt(nu2)
    den = np.sqrt(s * s + nu2)
    Ubar = np.vstack([U * (s / den), Vt.T * (nu / den)])
    return Ubar, den, Vt.T


def c_matrix(A, nu2, S):
    """C_S = D (U^T S^T S U - I) D + I (Section 1.1)."""
    A = np.asarray(A, dtype=np.float64)
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    D = np.diag(s / np.sqrt(s * s + nu2))
    SU = np.asarray(S, dtype=np.float64) @ U
    return D @ (SU.T @ SU - np.eye(A.shape[1])) @ D + np.eye(A.shape[1])
