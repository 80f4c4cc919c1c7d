"""Hand-written one-sided Jacobi SVD (Hestenes, 1958) -- brute-force checker.

TEST INFRASTRUCTURE: part of the CPU oracle package.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may use it.

It computes the full SVD of a small dense matrix without LAPACK, so that the
Lanczos oracle (which uses LAPACK's gesvd for the small SVD of T, as the paper
does with LAPACKE_dgesvd, Sec. 2.2.2) can be checked against an independent
algorithm: the k largest singular triplets of A from the restarted Lanczos
process must agree with the leading triplets returned here (eq. (1)).

Method: columns of W (initially A, m >= n) are orthogonalised pairwise by plane
rotations applied from the right, W <- W J, V <- V J, sweeping all pairs in
round-robin (tournament) order so that n/2 disjoint pairs rotate together.  For
a pair with a = |w_i|^2, b = |w_j|^2, c = w_i.w_j the rotation that zeroes the
new inner product is t = sign(z)/(|z| + sqrt(1+z^2)), z = (b-a)/(2c),
cs = 1/sqrt(1+t^2), sn = cs t, w_i' = cs w_i - sn w_j, w_j' = sn w_i + cs w_j
(Rutishauser's stable formulas).  A pair is skipped when
|c| <= tol sqrt(a b); the sweep loop ends after a sweep with no rotation.
Then sigma_i = |w_i|, u_i = w_i / sigma_i, sorted descending.
"""
from __future__ import annotations

import numpy as np


def _round_robin(n_even: int):
    """Pairs of each step of one tournament sweep over n_even players."""
    others = list(range(1, n_even))
    steps = []
    for s in range(n_even - 1):
        ring = others[s:] + others[:s]
        I = [0] + ring[1:n_even // 2]
        J = [ring[0]] + ring[::-1][:n_even // 2 - 1]
        steps.append((np.array(I), np.array(J)))
    return steps


def jacobi_svd(A: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """Full SVD A = U diag(s) V^T of a dense FP64 matrix.

    Returns (U, s, V, sweeps) with U m x r, s (r,), V n x r, r = min(m, n),
    s descending.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        U, s, V, sw = jacobi_svd(A.T, tol, max_sweeps)
        return V, s, U, sw
    ne = n + (n & 1)
    W = np.zeros((m, ne))
    W[:, :n] = A
    V = np.eye(ne)
    steps = _round_robin(ne) if ne >= 2 else []
    sweeps = 0
    for sweeps in range(1, max_sweeps + 1):
        rotated = 0
        for I, J in steps:
            wi, wj = W[:, I], W[:, J]
            a = np.einsum("ij,ij->j", wi, wi)
            b = np.einsum("ij,ij->j", wj, wj)
            c = np.einsum("ij,ij->j", wi, wj)
            act = np.abs(c) > tol * np.sqrt(a * b)
            if not act.any():
                continue
            rotated += int(act.sum())
            I, J, a, b, c = I[act], J[act], a[act], b[act], c[act]
            z = (b - a) / (2.0 * c)
            t = np.where(z >= 0, 1.0, -1.0) / (np.abs(z) + np.sqrt(1.0 + z * z))
            cs = 1.0 / np.sqrt(1.0 + t * t)
            sn = cs * t
            wi, wj = W[:, I], W[:, J]
            W[:, I], W[:, J] = cs * wi - sn * wj, sn * wi + cs * wj
            vi, vj = V[:, I], V[:, J]
            V[:, I], V[:, J] = cs * vi - sn * vj, sn * vi + cs * vj
        if rotated == 0:
            break
    s = np.sqrt(np.einsum("ij,ij->j", W, W))[:n]
    order = np.argsort(-s, kind="stable")
    s = s[order]
    W = W[:, order]
    V = V[:n, order]
    U = np.zeros((m, n))
    nz = s > 0
    U[:, nz] = W[:, nz] / s[nz]
    return U, s, V, sweeps
