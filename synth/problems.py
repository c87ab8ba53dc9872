"""Generators for A = G diag(sigma) V^T and b = A x_pl + c xi.

numpy (PCG64) on the host for problems that fit comfortably in host memory;
torch on a device for the multi-GiB ones.  V is Haar: the Q factor of a Gaussian
matrix with the signs of diag(R) folded in (F. Mezzadri, "How to generate random
matrices from the classical compact groups", Notices AMS 2007).
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class Problem:
    A: np.ndarray          # (n, d), row-major
    b: np.ndarray          # (n,)
    x_pl: np.ndarray       # planted vector
    sigma: np.ndarray      # nominal singular values
    nu2: float
    name: str = ""


def spectrum(kind, d, rate=None):
    """Nominal singular values.

    kind: "geom"  sigma_i = rate^i,        i = 0..d-1
          "poly"  sigma_i = i^-rate,       i = 1..d
          "exp"   sigma_i = exp(-i/rate),  i = 1..d
    """
    if kind == "geom":
        return rate ** np.arange(d, dtype=np.float64)
    if kind == "poly":
        return np.arange(1, d + 1, dtype=np.float64) ** (-rate)
    if kind == "exp":
        return np.exp(-np.arange(1, d + 1, dtype=np.float64) / rate)
    raise ValueError(kind)


def haar_orthogonal(rng, d):
    Z = rng.standard_normal((d, d))
    Q, R = np.linalg.qr(Z)
    return Q * np.sign(np.diag(R))[None, :]


def make_problem(n, d, sigma, nu2, noise, seed, dtype=np.float32, name="",
                 planted_scale=1.0):
    """A = G diag(sigma) V^T, G ~ N(0, 1/n); b = A x_pl + noise * xi."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, d)) / np.sqrt(n)
    V = haar_orthogonal(rng, d)
    A64 = (G * sigma[None, :]) @ V.T
    x_pl = rng.standard_normal(d) * planted_scale
    xi = rng.standard_normal(n)
    A = np.ascontiguousarray(A64.astype(dtype))
    b64 = A.astype(np.float64) @ x_pl + noise * xi
    b = b64.astype(dtype)
    return Problem(A=A, b=b, x_pl=x_pl, sigma=sigma, nu2=float(nu2), name=name)


def config_c1(seed=0):
    """1024 x 64 FP64, sigma_i = 0.9^i (i = 0..63), nu^2 = 1e-2, noise 0.01."""
    return make_problem(1024, 64, spectrum("geom", 64, 0.9), 1e-2, 0.01, seed,
                        dtype=np.float64, name="c1_1024x64_f64")


def config_c2(nu2=1e-2, seed=0, n=65536, d=1024):
    """65536 x 1024 FP32, sigma_i = 1/i, noise 0.1; nu^2 in {1e-2, 1e-4}."""
    return make_problem(n, d, spectrum("poly", d, 1.0), nu2, 0.1, seed,
                        dtype=np.float32, name=f"c2_{n}x{d}_f32_nu2_{nu2:g}")


def make_problem_torch(n, d, sigma, noise, seed, device, dtype=None, row_block=1 << 16):
    """Device-side generator for large problems (returns torch tensors A, b).

    G is drawn in row blocks with a seeded torch generator on ``device``.
    """
    import torch
    dtype = dtype or torch.float32
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    Z = torch.randn(d, d, generator=gen, device=device, dtype=torch.float64)
    Q, R = torch.linalg.qr(Z)
    V = Q * torch.sign(torch.diagonal(R))[None, :]
    sig = torch.as_tensor(sigma, device=device, dtype=torch.float64)
    M = (sig[:, None] * V.T).to(torch.float32)            # diag(sigma) V^T
    x_pl = torch.randn(d, generator=gen, device=device, dtype=torch.float64)
    A = torch.empty(n, d, device=device, dtype=dtype)
    b = torch.empty(n, device=device, dtype=dtype)
    for r0 in range(0, n, row_block):
        r1 = min(n, r0 + row_block)
        G = torch.randn(r1 - r0, d, generator=gen, device=device, dtype=torch.float32)
        G.mul_(1.0 / np.sqrt(n))
        blk = (G @ M).to(dtype)
        A[r0:r1] = blk
        xi = torch.randn(r1 - r0, generator=gen, device=device, dtype=torch.float64)
        b[r0:r1] = (blk.to(torch.float64) @ x_pl + noise * xi).to(dtype)
    return A, b, x_pl


def config_c4b_specs(count=256, seed=4):
    """Uneven problem set: n = 2^U{12..16} (4096 to 65536), d = U{128..1024},
    sigma_i = 0.95^i, nu^2 = 1e-3 (sigma_1 = 1), noise 0.1; problem i is drawn
    with seed 4000 * seed + i.  Returns a list of dicts (n, d, seed, nu2)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = 2 ** int(rng.integers(12, 17))
        d = int(rng.integers(128, 1025))
        out.append({"n": n, "d": d, "seed": 4000 * seed + i, "nu2": 1e-3})
    return out


def make_c4b_problem(spec, device, dtype=None):
    """Device tensors (A, b) for one config_c4b_specs entry."""
    return make_problem_torch(spec["n"], spec["d"], spectrum("geom", spec["d"], 0.95), 0.1,
                              spec["seed"], device, dtype=dtype)[:2]


C4A_N, C4A_D = 1 << 18, 2048


def config_c4a_nu2(count=64):
    """nu^2 grid of the shared-A problem: log-spaced in [1e-6, 1] sigma_1^2."""
    return np.logspace(-6.0, 0.0, count)


def make_c4a_problem(device, dtype=None, n=C4A_N, d=C4A_D, seed=41):
    """Shared A for the nu grid: sigma_i = i^-0.8 (sigma_1 = 1), noise 0.1."""
    return make_problem_torch(n, d, spectrum("poly", d, 0.8), 0.1, seed, device, dtype=dtype)[:2]


PATH_N, PATH_D = 1 << 16, 1024


def config_path_nu2():
    """Regularization path of the synthetic experiments: nu = 10^0 .. 10^-4 in
    decreasing order, as nu^2 = 1, 1e-2, 1e-4, 1e-6, 1e-8."""
    return np.array([10.0 ** (-2 * j) for j in range(5)])


def make_path_problem(device, dtype=None, n=PATH_N, d=PATH_D, seed=17):
    """A for the path: 65536 x 1024, sigma_i = 1/i (sigma_1 = 1), noise 0.1."""
    return make_problem_torch(n, d, spectrum("poly", d, 1.0), 0.1, seed, device, dtype=dtype)[:2]


def make_wide_problem_torch(n, d, sigma, noise, seed, device, dtype=None):
    """An underdetermined problem (n < d) on the device: A is the transpose of a
    d x n draw of make_problem_torch (so its singular values are sigma), and
    b = A x_pl + noise * xi with x_pl ~ N(0, I_d) from the same seed."""
    import torch
    dtype = dtype or torch.float32
    T = make_problem_torch(d, n, sigma, noise, seed, device, dtype=dtype)[0]
    A = T.t().contiguous()
    del T
    gen = torch.Generator(device=device)
    gen.manual_seed(seed + 1)
    x_pl = torch.randn(d, generator=gen, device=device, dtype=torch.float64)
    xi = torch.randn(n, generator=gen, device=device, dtype=torch.float64)
    b = (A.to(torch.float64) @ x_pl + noise * xi).to(dtype)
    return A, b


DUAL_N, DUAL_D = 1024, 1 << 16


def make_dual_problem(device, dtype=None, n=DUAL_N, d=DUAL_D, seed=23):
    """The wide problem of the dual form: 1024 x 65536 (the transpose of the
    headline shape), sigma_i = 1/i, noise 0.1."""
    return make_wide_problem_torch(n, d, spectrum("poly", n, 1.0), 0.1, seed, device, dtype=dtype)


def make_sparse_problem(n, d, per_row, alpha, noise, seed, dtype=np.float32):
    """A sparse CSR problem with power-law column popularity (text-like data):
    each row draws per_row columns with P(j) proportional to (j + 1)^-alpha
    (repeats within a row dropped), values N(0, 1) / sqrt(n); b = A x_pl + noise
    * xi with x_pl ~ N(0, I_d).  Returns numpy (rowptr int64, col int32, val, b)."""
    rng = np.random.default_rng(seed)
    p = (np.arange(1, d + 1, dtype=np.float64)) ** (-alpha)
    cdf = np.cumsum(p / p.sum())
    cols = np.searchsorted(cdf, rng.random((n, per_row)), side="right").clip(0, d - 1)
    cols.sort(axis=1)
    keep = np.ones_like(cols, dtype=bool)
    keep[:, 1:] = cols[:, 1:] != cols[:, :-1]
    counts = keep.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = cols[keep].astype(np.int32)
    val = (rng.standard_normal(col.size) / np.sqrt(n)).astype(dtype)
    x_pl = rng.standard_normal(d)
    Ax = np.zeros(n)
    np.add.at(Ax, np.repeat(np.arange(n), counts), val.astype(np.float64) * x_pl[col])
    b = (Ax + noise * rng.standard_normal(n)).astype(dtype)
    return rowptr, col, val, b


SPARSE_N, SPARSE_D, SPARSE_PER_ROW = 1 << 20, 1024, 16


def config_sparse(seed=29):
    """The sparse workload: 2^20 x 1024, 16 draws per row, alpha = 0.8, noise 0.1,
    nu^2 = 0.1 (d_e about 105)."""
    return make_sparse_problem(SPARSE_N, SPARSE_D, SPARSE_PER_ROW, 0.8, 0.1, seed), 0.1
