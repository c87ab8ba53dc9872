"""Random embeddings S and the sketch SA (oracle side, FP64, dense).

Test infrastructure: see the package docstring.

SRHT (Appendix C.2, "Preliminaries"): S = R H diag(eps) with H the normalised
Walsh-Hadamard matrix of size n, eps Rademacher and R a uniform subset of m rows
drawn without replacement (the sampling rule of Theorem 10).  The proof of
Theorem 4 scales each sampled row by sqrt(n/m); with that scaling
S = (1/sqrt(m)) R H_pm diag(eps), where H_pm[i, j] = (-1)^popcount(i & j) is the
unnormalised Sylvester-ordered Hadamard matrix, and E[S^T S] = I as for the
Gaussian embedding.  A row count n that is not a power of two is zero-padded to
the next power of two (padded rows of A and b are zero, so f is unchanged).

Row subset: the m indices with the smallest (key_i, i) over the padded range,
returned in ascending index order.  Taking the 2m smallest keeps the m rows of
the previous sketch (the nested resampling option).

Gaussian (Section 1): S[k, j] = z_{k n + j} / sqrt(m) with z standard normal.

CountSketch (the O(nnz) sparse embedding the paper names for sparse A in its
complexity remark): S has one nonzero per column, S[h_i, i] = s_i, with the bucket
h_i uniform on [0, m) and the sign s_i Rademacher; S^T S has a unit diagonal and
E[S^T S] = I without scaling.

Nothing here uses a fast transform: every Hadamard entry is evaluated from its
definition.
"""
import numpy as np

from . import philox


def next_pow2(n):
    p = 1
    while p < n:
        p *= 2
    return p


def hadamard_entries(rows, cols):
    """H_pm[rows[k], cols[j]] = (-1)^popcount(rows[k] & cols[j]) as float64."""
    r = np.asarray(rows, dtype=np.uint64)[:, None]
    c = np.asarray(cols, dtype=np.uint64)[None, :]
    x = r & c
    # popcount parity by folding the bits
    parity = np.zeros(x.shape, dtype=np.uint64)
    while np.any(x):
        parity ^= x & np.uint64(1)
        x = x >> np.uint64(1)
    return 1.0 - 2.0 * parity.astype(np.float64)


def srht_rows(seed, sketch_id, n, m):
    """Sampled rows of the padded transform: m smallest (key, index), ascending."""
    npad = next_pow2(n)
    if not 1 <= m <= npad:
        raise ValueError("need 1 <= m <= padded n")
    keys = philox.row_keys(seed, sketch_id, npad)
    idx = np.arange(npad, dtype=np.int64)
    order = np.lexsort((idx, keys))          # primary key, then index
    return np.sort(order[:m]).astype(np.int64)


def srht_signs(seed, sketch_id, n):
    """Rademacher signs over the padded length."""
    return philox.rademacher_signs(seed, sketch_id, next_pow2(n))


def srht_sketch(A, seed, sketch_id, m, row_block=256):
    """SA = (1/sqrt(m)) R H_pm diag(eps) A, by dense sums over all n rows."""
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    rows = srht_rows(seed, sketch_id, n, m)
    eps = srht_signs(seed, sketch_id, n)[:n]
    DA = eps[:, None] * A
    SA = np.empty((m, d), dtype=np.float64)
    cols = np.arange(n)
    for k0 in range(0, m, row_block):
        Hk = hadamard_entries(rows[k0:k0 + row_block], cols)
        SA[k0:k0 + row_block] = Hk @ DA
    return SA / np.sqrt(m), rows


def srht_sketch_rows(A, seed, sketch_id, m, which):
    """Selected rows ``which`` (positions into the ascending row list) of SA."""
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    rows = srht_rows(seed, sketch_id, n, m)
    eps = srht_signs(seed, sketch_id, n)[:n]
    out = np.empty((len(which), d))
    cols = np.arange(n)
    for k, w in enumerate(which):
        h = hadamard_entries(rows[[w]], cols)[0]
        out[k] = (h * eps) @ A
    return out / np.sqrt(m)


def gaussian_matrix(seed, sketch_id, m, n, precision="f64"):
    """S (m x n) with S[k, j] = z_{k n + j} / sqrt(m)."""
    idx = np.arange(m * n, dtype=np.uint64)
    z = philox.gaussian_entries(seed, sketch_id, idx, precision)
    return z.reshape(m, n) / np.sqrt(m)


def gaussian_sketch(A, seed, sketch_id, m, precision="f64", row_block=64):
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    SA = np.empty((m, d))
    for k0 in range(0, m, row_block):
        k1 = min(m, k0 + row_block)
        idx = (np.arange(k0, k1, dtype=np.uint64)[:, None] * np.uint64(n)
               + np.arange(n, dtype=np.uint64)[None, :])
        z = philox.gaussian_entries(seed, sketch_id, idx.ravel(), precision).reshape(k1 - k0, n)
        SA[k0:k1] = z @ A
    return SA / np.sqrt(m)


def count_sketch(A, seed, sketch_id, m):
    """SA for the CountSketch S (m x n, S[h_i, i] = s_i), as a sparse-times-matrix
    product; A may be dense or a scipy.sparse matrix.  Returns a dense FP64 array."""
    import scipy.sparse as sp
    n = A.shape[0]
    h, s = philox.count_sketch_hash(seed, sketch_id, n, m)
    S = sp.csr_matrix((s, (h, np.arange(n))), shape=(m, n))
    SA = S @ A
    return np.asarray(SA.todense() if sp.issparse(SA) else SA, dtype=np.float64)
