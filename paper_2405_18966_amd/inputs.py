"""Seeded synthetic inputs for the truncated-SVD solver.

This module only *draws* matrices and start vectors; it contains none of the
solver's arithmetic.  The kernels and the CPU oracle are fed from here and from
nowhere else, so both sides see bit-identical inputs.

Every generator takes an explicit seed and uses ``numpy.random.default_rng``.
The order of the draws is part of each generator's definition (changing it
changes the matrix), so it is spelled out in each docstring.

Workloads (the paper's test matrices, Sec. 3.1, are either synthetic with a
prescribed singular-value decay, or public datasets that are not available
here; the synthetic families below stand in for them):

* ``sparse_uniform``     -- m x n, nnz distinct positions drawn uniformly
                             without replacement, N(0,1) values.
* ``sparse_zipf``        -- m x n, per row a fixed number of i.i.d. column draws
                             from a Zipf law truncated to n ranks (power-law
                             column degrees), duplicates dropped, U(0,1) values.
* ``dense_lowrank``      -- G1 diag(d) G2^T + noise, column-major, with BF16
                             and FP32 storage copies (the stored copy is the
                             matrix of record for low-precision runs).
* ``batch_uniform``      -- many ``sparse_uniform`` instances of uneven size.
* ``prescribed_sparse`` / ``prescribed_dense`` / ``diag_matrix`` -- matrices
                             whose singular values are known exactly, built
                             with the decay laws of Sec. 3.1 (Decay1/2/3).
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np

__all__ = [
    "CSR", "Dense", "start_vector", "sparse_uniform", "sparse_zipf",
    "dense_lowrank", "batch_uniform", "round_values_f32", "decay1", "decay2",
    "decay3", "haar_orthogonal", "prescribed_sparse", "prescribed_dense",
    "prescribed_dense_dct", "diag_matrix", "config_matrix", "CONFIG_SEEDS", "paper_suite", "PAPER_SUITE_SEEDS", "PAPER_SUITE_SOLVE",
]

# Seed of workload c (1-based) is 2405000 + c; the start vector uses seed + 1.
CONFIG_SEEDS = {c: 2405000 + c for c in range(1, 6)}


@dataclass
class CSR:
    """0-based three-array CSR, rows half-open [row_ptr[i], row_ptr[i+1]),
    column indices strictly increasing within a row."""
    m: int
    n: int
    row_ptr: np.ndarray  # int32, m+1
    col_idx: np.ndarray  # int32, nnz
    val: np.ndarray      # float64 (or float32 for FP32-stored values)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self, dtype=np.float64):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val.astype(dtype), self.col_idx, self.row_ptr),
                             shape=(self.m, self.n))


@dataclass
class Dense:
    """Column-major m x n matrix.  ``a`` is the storage array (Fortran order);
    for BF16 storage it is a uint16 array holding the bit patterns."""
    m: int
    n: int
    a: np.ndarray
    dtype: str  # "f64" | "f32" | "bf16"


def _csr_from_sorted(m, n, rows, cols, vals) -> CSR:
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 range")
    return CSR(m, n, row_ptr.astype(np.int32), cols.astype(np.int32),
               np.ascontiguousarray(vals))


def start_vector(n: int, seed: int) -> np.ndarray:
    """v0 ~ N(0,1)^n from ``default_rng(seed)`` (one ``standard_normal`` call)."""
    return np.random.default_rng(seed).standard_normal(n)


def sparse_uniform(m: int, n: int, nnz: int, seed: int, values: str = "normal") -> CSR:
    """nnz distinct positions uniform without replacement over the m*n grid.

    Draw order: ``rng.choice(m*n, nnz, replace=False)`` (row-major linear
    position), then ``nnz`` values (``standard_normal`` for "normal",
    ``random`` for "uniform") assigned in sorted-position order.
    """
    rng = np.random.default_rng(seed)
    pos = rng.choice(m * n, size=nnz, replace=False)
    pos.sort()
    if values == "normal":
        v = rng.standard_normal(nnz)
    elif values == "uniform":
        v = rng.random(nnz)
    else:
        raise ValueError(values)
    rows = pos // n
    cols = pos % n
    return _csr_from_sorted(m, n, rows, cols, v)


def sparse_zipf(m: int, n: int, draws_per_row: int, a: float, seed: int) -> CSR:
    """Power-law column degrees.

    Per row, ``draws_per_row`` i.i.d. column ranks r in 1..n with
    P(r) proportional to r^-a (inverse-CDF sampling: one ``rng.random`` array of
    shape (m, draws_per_row)), column index = r - 1 (unpermuted, so column 0 is
    the heaviest).  Duplicates within a row are dropped.  Then one
    ``rng.random(nnz)`` array of U(0,1) values in CSR order.
    """
    rng = np.random.default_rng(seed)
    w = np.arange(1, n + 1, dtype=np.float64) ** (-a)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random((m, draws_per_row))
    cols = np.searchsorted(cdf, u, side="right")
    np.minimum(cols, n - 1, out=cols)
    cols.sort(axis=1)
    keep = np.ones_like(cols, dtype=bool)
    keep[:, 1:] = cols[:, 1:] != cols[:, :-1]
    counts = keep.sum(axis=1)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cols[keep].astype(np.int32)
    vals = rng.random(int(row_ptr[-1]))
    return CSR(m, n, row_ptr.astype(np.int32), col_idx, vals)


def round_values_f32(A: CSR) -> CSR:
    """Same pattern, values rounded to FP32 (round-to-nearest-even)."""
    return CSR(A.m, A.n, A.row_ptr, A.col_idx, A.val.astype(np.float32))


def _f32_to_bf16_bits(x32: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 bit patterns with round-to-nearest-even (finite inputs)."""
    b = x32.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return b.astype(np.uint16)


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    """Exact widening of BF16 bit patterns to float64."""
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def dense_lowrank(m: int, n: int, r: int, decay: float, noise: float, seed: int):
    """A = G1 diag(decay^i, i<r) G2^T + noise * N(0,1), generated in FP64.

    Draw order: G1 (m x r), G2 (n x r), then the m x n noise (row-major draw).
    Returns a dict with the FP64 matrix, the FP32 and BF16 storage copies
    (FP64 -> FP32 RNE -> BF16 RNE), all column-major, and the exact FP64
    widening of each stored copy (the matrix of record of a low-precision run).
    """
    rng = np.random.default_rng(seed)
    g1 = rng.standard_normal((m, r))
    g2 = rng.standard_normal((n, r))
    d = decay ** np.arange(r, dtype=np.float64)
    A = (g1 * d) @ g2.T
    A += noise * rng.standard_normal((m, n))
    A = np.asfortranarray(A)
    a32 = np.asfortranarray(A.astype(np.float32))
    b16 = np.asfortranarray(_f32_to_bf16_bits(a32))
    return {
        "f64": Dense(m, n, A, "f64"),
        "f32": Dense(m, n, a32, "f32"),
        "bf16": Dense(m, n, b16, "bf16"),
        "record_f32": np.asfortranarray(a32.astype(np.float64)),
        "record_bf16": np.asfortranarray(bf16_bits_to_f64(b16)),
    }


def batch_uniform(count: int, mmin: int, mmax: int, density: float, seed: int):
    """``count`` instances: m ~ U{mmin..mmax}, n ~ U{ceil(m/2)..m},
    nnz = round(density*m*n) uniform distinct positions, N(0,1) values.

    Draw order: one ``rng.integers`` pair per instance from the batch rng, and
    an instance seed ``rng.integers(2**62)``; instance i is then
    ``sparse_uniform(m, n, nnz, instance_seed)``.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        m = int(rng.integers(mmin, mmax + 1))
        n = int(rng.integers(math.ceil(m / 2), m + 1))
        s = int(rng.integers(2**62))
        nnz = int(round(density * m * n))
        out.append(sparse_uniform(m, n, nnz, s))
    return out


# --- prescribed spectra (Sec. 3.1 decay laws) --------------------------------

def decay1(N: int) -> np.ndarray:
    """Decay1: 10^(-4(i-1)/19) for i <= 20, then 1e-4 / (i-20)^0.1."""
    i = np.arange(1, N + 1, dtype=np.float64)
    return np.where(i <= 20, 10.0 ** (-4.0 * (i - 1) / 19.0),
                    1e-4 / np.maximum(i - 20, 1) ** 0.1)


def decay2(N: int) -> np.ndarray:
    """Decay2: i^-2."""
    return np.arange(1, N + 1, dtype=np.float64) ** -2.0


def decay3(N: int) -> np.ndarray:
    """Decay3: i^-3."""
    return np.arange(1, N + 1, dtype=np.float64) ** -3.0


def haar_orthogonal(rng, m: int, n: int) -> np.ndarray:
    """m x n (m >= n) matrix with orthonormal columns: QR of a Gaussian draw with
    the signs of R's diagonal folded into Q (Haar distributed)."""
    q, r = np.linalg.qr(rng.standard_normal((m, n)))
    return q * np.sign(np.where(np.diag(r) == 0, 1.0, np.diag(r)))


def prescribed_sparse(nblocks: int, bs: int, sigma: np.ndarray, seed: int) -> CSR:
    """Square (nblocks*bs)^2 sparse matrix with exactly the singular values
    ``sigma`` (length nblocks*bs) and ``bs`` nonzeros per row and column:
    P_r . blockdiag(Q_b diag(s_b) W_b^T) . P_c with Haar bs x bs blocks.

    Draw order: permutation assigning sigma to blocks, then per block Q_b, W_b,
    then the row permutation and the column permutation.
    """
    N = nblocks * bs
    sigma = np.asarray(sigma, dtype=np.float64)
    assert sigma.shape == (N,)
    rng = np.random.default_rng(seed)
    s = sigma[rng.permutation(N)].reshape(nblocks, bs)
    rows, cols, vals = [], [], []
    for b in range(nblocks):
        Q = haar_orthogonal(rng, bs, bs)
        W = haar_orthogonal(rng, bs, bs)
        blk = (Q * s[b]) @ W.T
        ii, jj = np.meshgrid(np.arange(bs), np.arange(bs), indexing="ij")
        rows.append((b * bs + ii).ravel())
        cols.append((b * bs + jj).ravel())
        vals.append(blk.ravel())
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    pr = rng.permutation(N)
    pc = rng.permutation(N)
    rows = pr[rows]
    cols = pc[cols]
    order = np.lexsort((cols, rows))
    return _csr_from_sorted(N, N, rows[order], cols[order], vals[order])


def prescribed_dense(m: int, n: int, sigma: np.ndarray, seed: int) -> np.ndarray:
    """Column-major m x n matrix P diag(sigma) Q^T with Haar P (m x r),
    Q (n x r), r = len(sigma) <= min(m, n).  Draw order: P, then Q."""
    rng = np.random.default_rng(seed)
    r = len(sigma)
    P = haar_orthogonal(rng, m, r)
    Q = haar_orthogonal(rng, n, r)
    return np.asfortranarray((P * np.asarray(sigma, dtype=np.float64)) @ Q.T)


def prescribed_dense_dct(m: int, n: int, sigma: np.ndarray, seed: int) -> np.ndarray:
    """Column-major m x n matrix P diag(sigma) Q^T with exactly the singular
    values ``sigma`` (r = len(sigma) <= min(m, n)), built in O(mn log(mn))
    instead of the O(n^3) of Haar factors.  The orthonormal columns are
    P(:, j) = d1 * C_m(:, pi1(j)) and Q(:, j) = d2 * C_n(:, pi2(j)): C_L is
    the orthonormal DCT-II matrix of order L, d1, d2 are random sign vectors
    and pi1, pi2 random injections of the r indices, so every singular vector
    is a dense, randomly signed cosine.

    Draw order: d1 (m signs), d2 (n signs), pi1 = the first r entries of a
    permutation of m, pi2 = the first r entries of a permutation of n.
    A is formed as d1 * (C_m B C_n^T) * d2^T with B[pi1(j), pi2(j)] = sigma_j,
    two passes of a fast DCT.
    """
    import scipy.fft as sfft
    sigma = np.asarray(sigma, dtype=np.float64)
    r = len(sigma)
    assert r <= min(m, n)
    rng = np.random.default_rng(seed)
    d1 = np.where(rng.random(m) < 0.5, -1.0, 1.0)
    d2 = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    pi1 = rng.permutation(m)[:r]
    pi2 = rng.permutation(n)[:r]
    B = np.zeros((m, n), order="F")
    B[pi1, pi2] = sigma
    B = sfft.dct(B, type=2, norm="ortho", axis=0, overwrite_x=True)
    B = sfft.dct(B, type=2, norm="ortho", axis=1, overwrite_x=True)
    B *= d1[:, None]
    B *= d2[None, :]
    return np.asfortranarray(B)


def diag_matrix(m: int, n: int, d: np.ndarray) -> CSR:
    """Rectangular diagonal m x n with A[i,i] = d[i] (zeros kept out of the
    pattern).  Its singular values are sorted |d| padded with zeros."""
    d = np.asarray(d, dtype=np.float64)
    r = min(m, n)
    assert d.shape == (r,)
    idx = np.nonzero(d)[0]
    return _csr_from_sorted(m, n, idx, idx, d[idx])


def dense_to_csr(A: np.ndarray) -> CSR:
    """Exact conversion of a dense array (zeros dropped) to CSR."""
    rows, cols = np.nonzero(A)
    return _csr_from_sorted(A.shape[0], A.shape[1], rows, cols, A[rows, cols])


def config_matrix(c: int):
    """The five benchmark workloads.

    1: 2000 x 1000, nnz 20,000 uniform, N(0,1); k=10, p=30, tol=1e-10.
    2: 1,000,000 x 500,000, 10 Zipf(1.1) draws per row, U(0,1); k=50, p=150, tol=1e-8.
    3: 20000 x 10000 dense, G1 diag(0.95^i, i<200) G2^T + 1e-3 N(0,1);
       k=100, p=250, tol=1e-8 (returns the ``dense_lowrank`` dict).
    4: workload 1 with FP32 values; k=50, p=150, tol=1e-8.
    5: 256 instances, m ~ U{500..20000}, n ~ U{m/2..m}, 0.5% density; k=8, p=24.
    """
    s = CONFIG_SEEDS[c]
    if c == 1:
        return sparse_uniform(2000, 1000, 20000, s)
    if c == 2:
        return sparse_zipf(1_000_000, 500_000, 10, 1.1, s)
    if c == 3:
        return dense_lowrank(20000, 10000, 200, 0.95, 1e-3, s)
    if c == 4:
        return round_values_f32(sparse_uniform(2000, 1000, 20000, CONFIG_SEEDS[1]))
    if c == 5:
        return batch_uniform(256, 500, 20000, 0.005, s)
    raise ValueError(c)


# --- the paper's synthetic suite (Sec. 3.1) -----------------------------------
# Sparse1-3: 40,000 x 40,000 with 5 nonzeros per row, Dense1-3: 10,000 x
# 10,000, singular values from Decay1/2/3; every case is solved for k = 100
# (so t = max(15, 3k) = 300), tol = 1e-10, at most 10 cycles (Sec. 3).  The
# paper does not state its generator; here the sparse ones are the 5 x 5
# block construction of prescribed_sparse and the dense ones the signed,
# permuted DCT factors of prescribed_dense_dct (seconds at 10,000 x 10,000,
# where Haar factors take minutes).
PAPER_SUITE_SEEDS = {name: 2405100 + i for i, name in
                     enumerate(("sparse1", "sparse2", "sparse3", "dense1", "dense2", "dense3"))}
PAPER_SUITE_SOLVE = dict(k=100, p=300, tol=1e-10, maxit=10)


def paper_suite(name: str, n: int | None = None):
    """(A, sigma): the named case and its exact singular values (descending).
    ``n`` overrides the order (40,000 sparse, 10,000 dense) for smaller runs;
    sparse orders are rounded down to a multiple of 5.  A is a CSR for the
    sparse cases and a column-major ndarray for the dense ones."""
    law = {"1": decay1, "2": decay2, "3": decay3}[name[-1]]
    seed = PAPER_SUITE_SEEDS[name]
    if name.startswith("sparse"):
        N = (n or 40000) // 5 * 5
        sig = law(N)
        return prescribed_sparse(N // 5, 5, sig, seed), sig
    N = n or 10000
    sig = law(N)
    return prescribed_dense_dct(N, N, sig, seed), sig


CONFIG_SOLVE = {
    1: dict(k=10, p=30, tol=1e-10),
    2: dict(k=50, p=150, tol=1e-8),
    3: dict(k=100, p=250, tol=1e-8),
    4: dict(k=50, p=150, tol=1e-8),
    5: dict(k=8, p=24, tol=1e-8),
}
