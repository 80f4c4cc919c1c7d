"""Pins of the CPU oracle against facts fixed outside it (no GPU needed).

Each test checks the oracle against something other than itself: published
known-answer vectors, closed-form spectra, textbook special cases, an
independent hand-written Jacobi SVD, LAPACK on the dense matrix, and the
identities of Proposition 1 / eqs. (2)-(7).
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2405_18966_amd import inputs
from oracle import jacobi, philox, svds_ref
from oracle.svds_ref import svds, lbp, explicit_residuals, as_operator, harmonic_restart_basis

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --- Philox4x32-10 -----------------------------------------------------------

def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(x, 16) for x in line.split()])
    return rows


def test_philox_known_answers():
    rows = _kat_rows()
    assert len(rows) == 3
    for r in rows:
        out = philox.philox4x32_10(*[np.array([x], dtype=np.uint64) for x in r[:6]])
        assert [int(o[0]) for o in out] == r[6:]


def test_philox_normal_statistics_and_layout():
    z = philox.normal_vector(400001, seed=12345, stream=3)
    assert z.shape == (400001,)
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 0.02
    # prefix property: a shorter vector is the prefix of a longer one
    np.testing.assert_array_equal(philox.normal_vector(7, 12345, 3), z[:7])
    # streams and seeds give different vectors
    assert not np.allclose(philox.normal_vector(8, 12345, 4), z[:8])
    assert not np.allclose(philox.normal_vector(8, 12346, 3), z[:8])
    # Box-Muller pair from block 0, recomputed from the raw words
    x = philox.philox4x32_10(0, 0, 3, 0, 12345, 0)
    u1 = ((((int(x[1][()]) << 32) | int(x[0][()])) >> 11) + 1) * 2.0**-53
    u2 = ((((int(x[3][()]) << 32) | int(x[2][()])) >> 11)) * 2.0**-53
    rad = np.sqrt(-2 * np.log(u1))
    np.testing.assert_allclose(z[:2], [rad * np.cos(2 * np.pi * u2), rad * np.sin(2 * np.pi * u2)],
                               rtol=1e-15)


# --- the hand-written Jacobi checker ------------------------------------------

@pytest.mark.parametrize("n", [2, 5, 8, 13])
def test_round_robin_covers_every_pair_once(n):
    ne = n + (n & 1)
    seen = []
    for I, J in jacobi._round_robin(ne):
        step = set(I.tolist()) | set(J.tolist())
        assert len(step) == ne  # disjoint pairs cover every column
        seen += [tuple(sorted(x)) for x in zip(I.tolist(), J.tolist())]
    assert sorted(seen) == sorted((i, j) for i in range(ne) for j in range(i + 1, ne))


def test_jacobi_diagonal_closed_form():
    d = np.array([3.0, -7.0, 0.5, 0.0, 2.0, -2.0])
    U, s, V, _ = jacobi.jacobi_svd(np.diag(d))
    np.testing.assert_array_equal(s, np.sort(np.abs(d))[::-1])


def test_jacobi_2x2_closed_form():
    # [[a, b], [0, c]]: sigma1*sigma2 = |a c|, sigma1^2 + sigma2^2 = a^2+b^2+c^2
    a, b, c = 3.0, 4.0, 2.0
    _, s, _, _ = jacobi.jacobi_svd(np.array([[a, b], [0.0, c]]))
    assert abs(s[0] * s[1] - abs(a * c)) < 1e-14 * s[0] ** 2
    assert abs(s[0] ** 2 + s[1] ** 2 - (a * a + b * b + c * c)) < 1e-13 * s[0] ** 2


@pytest.mark.parametrize("shape", [(60, 40), (40, 60), (31, 31)])
def test_jacobi_prescribed_spectrum_and_factorisation(shape):
    m, n = shape
    r = min(m, n)
    sig = np.sort(np.random.default_rng(5).uniform(0.1, 10, r))[::-1]
    A = inputs.prescribed_dense(m, n, sig, seed=11)
    U, s, V, sweeps = jacobi.jacobi_svd(A)
    np.testing.assert_allclose(s, sig, rtol=1e-13)
    np.testing.assert_allclose((U * s) @ V.T, A, atol=1e-13 * sig[0])
    assert np.abs(U.T @ U - np.eye(r)).max() < 1e-13
    assert np.abs(V.T @ V - np.eye(r)).max() < 1e-13
    assert sweeps < 20


def test_jacobi_matches_lapack():
    A = np.random.default_rng(3).standard_normal((50, 35))
    _, s, _, _ = jacobi.jacobi_svd(A)
    np.testing.assert_allclose(s, np.linalg.svd(A, compute_uv=False), rtol=1e-13)


# --- helpers -------------------------------------------------------------------

def _subspace_err(X, Y):
    """sin of the largest principal angle between span(X) and span(Y)."""
    qx, _ = np.linalg.qr(X)
    qy, _ = np.linalg.qr(Y)
    return np.linalg.norm(qx - qy @ (qy.T @ qx), 2)


def _check_vectors(U, S, V, Ur, Vr, Sr_all, tol, k):
    """Vectors agree column-wise up to sign, within the Davis-Kahan style bound
    10 * tol * sigma_j / gap_j (floor 1e-12); multiple values are compared as
    subspaces."""
    for j in range(k):
        gap = min(abs(Sr_all[j] - Sr_all[i]) for i in range(len(Sr_all)) if i != j)
        bound = max(10 * tol * Sr_all[j] / max(gap, 1e-300), 1e-12)
        if gap < 1e-12 * Sr_all[0]:
            continue
        for X, Y in ((U, Ur), (V, Vr)):
            err = min(np.linalg.norm(X[:, j] - Y[:, j]), np.linalg.norm(X[:, j] + Y[:, j]))
            assert err <= bound, (j, err, bound)


# --- P1: brute force, tiny -----------------------------------------------------

@pytest.mark.parametrize("shape,k,p", [((120, 80), 5, 15), ((80, 120), 4, 12), ((60, 60), 1, 2)])
def test_oracle_against_jacobi_bruteforce(shape, k, p):
    m, n = shape
    A = inputs.sparse_uniform(m, n, m * n // 5, seed=17)
    Asp = as_operator(A)
    v0 = inputs.start_vector(n, 18)
    U, S, V, info = svds(Asp, k, p, 1e-12, 2000, v0=v0)
    assert info.converged
    Uj, Sj, Vj, _ = jacobi.jacobi_svd(Asp.toarray())
    np.testing.assert_allclose(S, Sj[:k], rtol=1e-12)
    _check_vectors(U, S, V, Uj, Vj, Sj, 1e-12, k)
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-12
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-12


# --- P2: complete bidiagonalisation (Golub-Kahan) -----------------------------

@pytest.mark.parametrize("shape", [(50, 30), (40, 40)])
def test_complete_bidiagonalisation_reproduces_spectrum(shape):
    m, n = shape
    A = np.random.default_rng(2).standard_normal(shape)
    v0 = inputs.start_vector(n, 3)
    U, T, V, beta, info = lbp(A, n, v0)
    # T is upper bidiagonal, its singular values are those of A
    assert np.all(np.tril(T, -1) == 0) and np.all(np.triu(T, 2) == 0)
    np.testing.assert_allclose(np.linalg.svd(T, compute_uv=False),
                               np.linalg.svd(A, compute_uv=False), rtol=1e-12)
    # v_{n+1} cannot exist in R^n: the last beta is a breakdown
    assert beta == 0.0 and info.breakdowns == 1
    # Lanczos relation A V = U T (Alg. 1 output)
    assert np.abs(A @ V - U @ T).max() < 1e-13 * np.abs(T).max()


# --- P3: prescribed spectra (decay laws of Sec. 3.1) ---------------------------

@pytest.mark.parametrize("law", ["decay1", "decay2", "decay3"])
def test_prescribed_sparse_spectrum(law):
    nb, bs = 120, 5
    sig = getattr(inputs, law)(nb * bs)
    A = inputs.prescribed_sparse(nb, bs, sig, seed=7)
    assert np.all(np.diff(A.row_ptr) == bs)
    k = 8
    U, S, V, info = svds(as_operator(A), k, 0, 1e-10, 500, v0=inputs.start_vector(A.n, 8))
    assert info.converged
    np.testing.assert_allclose(S, np.sort(sig)[::-1][:k], rtol=1e-10)


def test_prescribed_dense_spectrum():
    sig = inputs.decay1(300)
    A = inputs.prescribed_dense(400, 300, sig, seed=9)
    U, S, V, info = svds(A, 20, 0, 1e-10, 500, v0=inputs.start_vector(300, 10))
    assert info.converged
    np.testing.assert_allclose(S, sig[:20], rtol=1e-10)
    r1, r2 = explicit_residuals(A, U, S, V)
    assert r1.max() < 1e-10 * S[0] and (r2 / S).max() < 1e-10


# --- P4: library routine (LAPACK on the dense matrix), workload 1 ---------------

def test_workload1_against_lapack():
    A = inputs.config_matrix(1)
    Asp = as_operator(A)
    cfg = inputs.CONFIG_SOLVE[1]
    U, S, V, info = svds(Asp, cfg["k"], cfg["p"], cfg["tol"], 2000,
                         v0=inputs.start_vector(A.n, inputs.CONFIG_SEEDS[1] + 1))
    assert info.converged
    Ur, Sr, Vrt = np.linalg.svd(Asp.toarray(), full_matrices=False)
    np.testing.assert_allclose(S, Sr[:cfg["k"]], rtol=1e-12)
    _check_vectors(U, S, V, Ur, Vrt.T, Sr, cfg["tol"], cfg["k"])


# --- P5: diagonal with repeated values (breakdowns, multiple sigma) ------------

def test_diagonal_with_repeats_breaks_down_and_stays_exact():
    d = np.repeat([5.0, 4.0, 3.0, 2.0, 1.0, 0.5], [4, 3, 3, 2, 3, 35])
    A = inputs.diag_matrix(60, 50, d)
    k = 8
    U, S, V, info = svds(as_operator(A), k, 20, 1e-10, 200, v0=inputs.start_vector(50, 4))
    assert info.breakdowns > 0
    np.testing.assert_allclose(S, np.sort(d)[::-1][:k], rtol=1e-12)
    # multiple singular values: compare subspaces of each cluster
    D = as_operator(A).toarray()
    for val in (5.0, 4.0):
        cols = np.nonzero(np.abs(S - val) < 1e-9)[0]
        exact = np.eye(50)[:, np.nonzero(np.abs(np.abs(np.diag(D[:50, :50])) - val) < 1e-12)[0]]
        assert len(cols) == exact.shape[1]
        assert _subspace_err(V[:, cols], exact) < 1e-9
    r1, r2 = explicit_residuals(as_operator(A), U, S, V)
    assert r1.max() < 1e-10 * S[0] and r2.max() < 1e-10 * S[0]


def test_zero_matrix():
    A = inputs.CSR(30, 20, np.zeros(31, np.int32), np.zeros(0, np.int32), np.zeros(0))
    U, S, V, info = svds(as_operator(A), 2, 5, 1e-10, 3, v0=inputs.start_vector(20, 1))
    assert np.all(S == 0) and info.converged and info.breakdowns >= 1


# --- P6: invariants of Proposition 1 and eqs. (2)-(7) ---------------------------

def test_lanczos_invariants_every_cycle():
    A = inputs.sparse_uniform(300, 200, 3000, seed=21)
    Asp = as_operator(A)
    k, p = 6, 18
    checked = {"lbp": 0, "svd": 0, "restart": 0}

    def cb(stage, st, ex):
        U, V, T = st.U, st.V, st.T
        scale = max(abs(T).max(), 1.0)
        if stage in ("lbp", "svd"):
            # A V_p = U_p T_p ;  A^T U_p = V_p T_p^T + beta_p v_{p+1} e_p^T
            assert np.abs(Asp @ V[:, :p] - U @ T[:p, :p]).max() < 1e-13 * scale
            E = np.zeros((p, p)); E[p - 1, p - 1] = 1
            lhs = Asp.T @ U - V[:, :p] @ T[:p, :p].T - T[p - 1, p] * np.outer(V[:, p], E[p - 1])
            assert np.abs(lhs).max() < 1e-13 * scale
            assert np.abs(U.T @ U - np.eye(p)).max() < 1e-12
            assert np.abs(V.T @ V - np.eye(p + 1)).max() < 1e-12
        if stage == "svd":
            # eq. (4): estimate equals the explicit residual of A^T u~ - s v~
            Ut = U @ ex["Uh"][:, :k]
            Vt = V[:, :p] @ ex["Vh"][:, :k]
            expl = np.linalg.norm(Asp.T @ Ut - Vt * ex["s"][:k], axis=0) / ex["s"][:k]
            np.testing.assert_allclose(expl, ex["res"], atol=1e-12)
            # eq. (2) first identity: A v~ = s u~
            assert np.abs(Asp @ Vt - Ut * ex["s"][:k]).max() < 1e-12 * scale
        if stage == "restart":
            # eq. (6): u~_j^T A v_{t+1} = beta_t Uh(t, j) = rho_j
            np.testing.assert_allclose(ex["Uk"].T @ (Asp @ V[:, k]), ex["rho"], atol=1e-12 * scale)
            # restarted T: diag(Sigma_k) with the arrow column rho
            np.testing.assert_array_equal(T[:k, k], ex["rho"])
        checked[stage] += 1

    U, S, V, info = svds(Asp, k, p, 1e-12, 50, v0=inputs.start_vector(200, 22), callback=cb)
    assert checked["svd"] == info.cycles and checked["restart"] == info.restarts >= 1


# --- P7: mat-vec counts ---------------------------------------------------------

@pytest.mark.parametrize("maxit", [1, 2, 5])
def test_matvec_counts(maxit):
    A = inputs.sparse_uniform(200, 150, 2000, seed=31)
    k, p = 5, 15
    _, _, _, info = svds(as_operator(A), k, p, 1e-14, maxit, v0=inputs.start_vector(150, 32))
    R = info.restarts
    assert info.cycles == R + 1 <= maxit
    assert info.n_spmv == p + R * (p - k)
    assert info.n_spmvT == p + R * (p - k)


def test_not_converged_reports_partial():
    A = inputs.config_matrix(1)
    _, S, _, info = svds(as_operator(A), 10, 30, 1e-10, 1,
                         v0=inputs.start_vector(1000, inputs.CONFIG_SEEDS[1] + 1))
    assert not info.converged and info.cycles == 1 and 0 <= info.nconv < 10


def test_validation_errors():
    A = as_operator(inputs.sparse_uniform(20, 10, 50, seed=1))
    for k, p in [(0, 5), (5, 5), (3, 10), (3, 21)]:
        with pytest.raises(ValueError):
            svds(A, k, p)


def test_default_start_vector_is_philox_stream0():
    A = as_operator(inputs.sparse_uniform(100, 80, 800, seed=41))
    seen = {}

    def cb(stage, st, ex):
        if stage == "lbp":
            seen["v1"] = st.V[:, 0].copy()
    svds(A, 3, 10, 1e-10, 30, seed=99, callback=cb)
    z = philox.normal_vector(80, 99, 0)
    np.testing.assert_allclose(seen["v1"], z / np.linalg.norm(z), rtol=1e-15)


def test_sign_normalisation():
    U = np.array([[1.0, 2.0], [3.0, -1.0]])
    V = np.array([[0.2, -0.9], [-0.8, 0.9], [0.1, 0.1]])
    Un, Vn = svds_ref.sign_normalize(U, V)
    np.testing.assert_array_equal(Vn[:, 0], -V[:, 0])  # largest |.| is -0.8
    np.testing.assert_array_equal(Vn[:, 1], -V[:, 1])  # tie -0.9 / 0.9: lowest index
    np.testing.assert_array_equal(Un, U * [-1, -1])


# --- planted mistakes: the pins above must catch them ----------------------------

def test_planted_wrong_arrow_column_is_caught(monkeypatch):
    """A sign error in rho (eq. (6)) leaves u_{k+1} unchanged (CGS2 removes the
    Uk components anyway) but corrupts T; the Lanczos relation pin fails."""
    orig = svds_ref.svds
    A = inputs.sparse_uniform(300, 200, 3000, seed=21)
    Asp = as_operator(A)
    k, p = 6, 18

    def bad_cb(stage, st, ex):
        if stage == "restart":
            st.T[:k, k] = -st.T[:k, k]

    failures = []

    def check(stage, st, ex):
        if stage == "svd":
            err = np.abs(Asp.T @ st.U - st.V[:, :p] @ st.T[:p, :p].T
                         - st.T[p - 1, p] * np.outer(st.V[:, p], np.eye(p)[p - 1])).max()
            failures.append(err)

    def both(stage, st, ex):
        bad_cb(stage, st, ex)
        check(stage, st, ex)

    orig(Asp, k, p, 1e-12, 3, v0=inputs.start_vector(200, 22), callback=both)
    assert failures[0] < 1e-12 and max(failures[1:]) > 1e-6


def test_planted_single_pass_without_reorth_is_caught(monkeypatch):
    """Without re-orthogonalisation the bases lose orthogonality (the reason
    the paper gives for full re-orthogonalisation, Sec. 2.1)."""
    monkeypatch.setattr(svds_ref, "cgs2", lambda w, Q: w)
    A = inputs.prescribed_dense(200, 150, inputs.decay2(150), seed=3)
    U, T, V, beta, info = svds_ref.lbp(A, 60, inputs.start_vector(150, 4))
    assert np.abs(V.T @ V - np.eye(60)).max() > 1e-6


def test_planted_transposed_operand_is_caught(monkeypatch):
    """A^T u computed with A itself (square, non-symmetric A): the complete
    bidiagonalization pin (sigma(T) = sigma(A), P2) fails."""
    orig_init = svds_ref._Op.__init__

    def bad_init(self, A, info):
        orig_init(self, A, info)
        self.AT = A  # the planted mistake: the transpose is dropped

    monkeypatch.setattr(svds_ref._Op, "__init__", bad_init)
    A = np.random.default_rng(2).standard_normal((40, 40))
    U, T, V, beta, info = lbp(A, 40, inputs.start_vector(40, 3))
    s_T = np.linalg.svd(T, compute_uv=False)
    s_A = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(s_T - s_A) / s_A[0]) > 1e-3


# --- the paper's synthetic suite at reduced order (Sec. 3.1, Sec. 3 settings) ---

@pytest.mark.parametrize("name,n", [("sparse1", 500), ("sparse3", 500), ("dense1", 300), ("dense2", 200),
                                    ("dense3", 300)])
def test_paper_suite_generator_spectrum(name, n):
    """The generator's matrices have exactly the decay law's singular values
    (dense LAPACK SVD of the whole matrix), 5 nonzeros per row when sparse."""
    A, sig = inputs.paper_suite(name, n)
    if name.startswith("sparse"):
        assert np.all(np.diff(A.row_ptr) == 5)
        D = np.zeros((A.m, A.n))
        for i in range(A.m):
            D[i, A.col_idx[A.row_ptr[i]:A.row_ptr[i + 1]]] = A.val[A.row_ptr[i]:A.row_ptr[i + 1]]
    else:
        D = A
    s = np.linalg.svd(D, compute_uv=False)
    np.testing.assert_allclose(s, sig, rtol=1e-9, atol=1e-15 * sig[0])


def test_paper_suite_settings_oracle():
    """k = 100, t = 300, tol = 1e-10, at most 10 cycles, on Sparse2 at order
    2000: the oracle reaches the closed-form values."""
    A, sig = inputs.paper_suite("sparse2", 2000)
    c = inputs.PAPER_SUITE_SOLVE
    U, S, V, info = svds(as_operator(A), c["k"], c["p"], c["tol"], c["maxit"],
                         v0=inputs.start_vector(A.n, 5))
    assert info.converged
    np.testing.assert_allclose(S, sig[:c["k"]], rtol=1e-10)


# --- smallest triplets (Ritz augmentation with the k smallest Ritz values) ---

def _small_cluster_spectrum(N):
    """Five small values well apart from the rest: [0.01 .. 0.08] then [1, 2]."""
    return np.concatenate([[0.01, 0.02, 0.035, 0.05, 0.08], np.linspace(1.0, 2.0, N - 5)])


@pytest.mark.parametrize("kind", ["sparse", "dense"])
def test_smallest_triplets_against_lapack(kind):
    """The k smallest singular values (ascending) equal LAPACK's, the
    vectors are singular vectors (residuals), and the pairs are orthonormal."""
    if kind == "sparse":
        sig = _small_cluster_spectrum(600)
        A = inputs.prescribed_sparse(120, 5, sig, seed=21)
        op = as_operator(A)
        D = op.toarray()
    else:
        sig = _small_cluster_spectrum(200)
        D = inputs.prescribed_dense(260, 200, sig, seed=22)
        op = D
    k = 4
    U, S, V, info = svds(op, k, 20, 1e-10, 3000, v0=inputs.start_vector(D.shape[1], 23), which="smallest")
    assert info.converged
    exact = np.sort(np.linalg.svd(D, compute_uv=False))[:k]
    np.testing.assert_allclose(S, exact, rtol=1e-10)
    assert np.all(np.diff(S) > 0)
    r1, r2 = explicit_residuals(op, U, S, V)
    assert r1.max() <= 1e-12 * sig.max() and (r2 / S).max() <= 2e-10
    assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-12
    assert np.abs(V.T @ V - np.eye(k)).max() <= 1e-12


def test_smallest_on_diagonal_matrix():
    """Rectangular diagonal: the smallest nonzero |d| values, exactly."""
    d = np.concatenate([[0.5, 0.25, 0.125], np.linspace(3.0, 4.0, 147)])
    A = inputs.diag_matrix(150, 150, d)
    U, S, V, info = svds(as_operator(A), 3, 12, 1e-10, 5000, v0=inputs.start_vector(150, 24), which="smallest")
    np.testing.assert_allclose(S, [0.125, 0.25, 0.5], rtol=1e-10)


# --- selective second pass (DGKS test) ----------------------------------------

def test_selective_pass_decision_and_orthogonality():
    """A vector mostly inside span(Q) needs the second pass; a random one
    against a few columns does not.  Either way the result is orthogonal to
    Q to working precision and the component outside span(Q) is kept."""
    rng = np.random.default_rng(31)
    Q = svds_ref.np.linalg.qr(rng.standard_normal((4000, 30)))[0]
    z = rng.standard_normal(4000)
    zp = z - Q @ (Q.T @ z)
    w_in = Q @ rng.standard_normal(30) * 1e6 + zp  # |w1| / |w| ~ 1e-5
    x, second = svds_ref.cgs_selective(w_in, Q)
    assert second
    assert np.abs(Q.T @ x).max() <= 1e-13 * np.linalg.norm(x)
    np.testing.assert_allclose(x, zp, rtol=0, atol=1e-8 * np.linalg.norm(zp))
    x, second = svds_ref.cgs_selective(z, Q)
    assert not second
    assert np.abs(Q.T @ x).max() <= 1e-13 * np.linalg.norm(x)


def test_selective_solve_matches_lapack_and_stays_orthogonal():
    A = inputs.config_matrix(1)
    op = as_operator(A)
    v0 = inputs.start_vector(A.n, inputs.CONFIG_SEEDS[1] + 1)
    U, S, V, info = svds(op, 10, 30, 1e-10, 3000, v0=v0, selective=True)
    assert info.converged and info.reorth_tests > 0
    assert info.reorth_second_passes < info.reorth_tests
    exact = np.linalg.svd(op.toarray(), compute_uv=False)[:10]
    np.testing.assert_allclose(S, exact, rtol=1e-10)
    assert np.abs(U.T @ U - np.eye(10)).max() <= 1e-12
    assert np.abs(V.T @ V - np.eye(10)).max() <= 1e-12


# --- partial re-orthogonalisation (omega recurrences, PROPACK style) ----------

def _snapshots(op, k, p, maxit, v0, **kw):
    snaps = []

    def cb(stage, st, extra):
        if stage == "svd":
            snaps.append((st.U.copy(), st.V.copy(), st.T.copy()))
    out = svds(op, k, p, 1e-14, maxit, v0=v0, callback=cb, **kw)
    return snaps, out


def test_omega_recurrences_reproduce_true_inner_products(monkeypatch):
    """With re-orthogonalisation switched off the bases lose orthogonality
    to O(1).  Fed with the TRUE inner products of the newest vectors, the
    recurrences must give the true inner products of the next vector (up to
    rounding), on the bidiagonal T of the first cycle and on the arrow-shaped
    T after a restart: a dropped term, a wrong index or a wrong sign in
    either recurrence fails this."""
    monkeypatch.setattr(svds_ref, "cgs2", lambda w, Q: w)
    A = inputs.sparse_uniform(300, 200, 6000, seed=71)
    op = as_operator(A)
    k, p = 4, 40
    snaps, _ = _snapshots(op, k, p, 2, inputs.start_vector(200, 72))
    assert len(snaps) == 2
    smax = np.linalg.norm(op.toarray(), 2)
    worst_true = 0.0
    for cyc, (U, V, T) in enumerate(snaps):
        i0 = 0 if cyc == 0 else k
        for i in range(i0, p):
            mu = U[:, :i + 1].T @ U[:, i]
            nu = V[:, :i + 1].T @ V[:, i]
            x = svds_ref.omega_v_inner(T, mu, nu, i)
            true = V[:, :i + 1].T @ (T[i, i + 1] * V[:, i + 1])
            worst_true = max(worst_true, float(np.abs(true[:max(i - 1, 0)]).max(initial=0)) / T[i, i + 1])
            assert np.abs(x - true).max() <= 1e-10 * smax, (cyc, "v", i)
        for i in range(i0 + 1, p):
            nu = V[:, :i + 1].T @ V[:, i]
            mu = U[:, :i].T @ U[:, i - 1]
            x = svds_ref.omega_u_inner(T, mu, nu, i)
            true = U[:, :i].T @ (T[i, i] * U[:, i])
            assert np.abs(x - true).max() <= 1e-10 * smax, (cyc, "u", i)
    assert worst_true > 1e-3  # orthogonality really was lost: the check had something to see


@pytest.mark.parametrize("case", ["workload1", "decay1", "decay2", "decay3", "repeated_diagonal"])
def test_partial_reorth_matches_exact_singular_values(case):
    """Partial re-orthogonalisation: singular values as exact as the full
    mode's (LAPACK, closed-form spectra, and a diagonal with repeated values,
    the property that the paper reports PROPACK's lansvd getting wrong);
    every basis stays semi-orthogonal (at most ~sqrt(eps) off) at every
    cycle; fewer columns are projected out than full re-orthogonalisation
    projects."""
    if case == "workload1":
        A = inputs.config_matrix(1)
        op = as_operator(A)
        exact = np.linalg.svd(op.toarray(), compute_uv=False)
        k, p, v0 = 10, 30, inputs.start_vector(A.n, inputs.CONFIG_SEEDS[1] + 1)
    elif case == "repeated_diagonal":
        d = np.zeros(400)
        d[:40] = np.repeat(np.arange(10, 0, -1), 4)
        op = as_operator(inputs.diag_matrix(500, 400, d))
        exact = np.sort(d)[::-1]
        k, p, v0 = 8, 24, inputs.start_vector(400, 73)
    else:
        sig = getattr(inputs, case)(3000)
        op = as_operator(inputs.prescribed_sparse(600, 5, sig, 11))
        exact = np.sort(sig)[::-1]
        k, p, v0 = 20, 60, inputs.start_vector(3000, 74)
    orth = []

    def cb(stage, st, extra):
        if stage == "svd":
            j = st.p
            orth.append(max(np.abs(st.U[:, :j].T @ st.U[:, :j] - np.eye(j)).max(),
                            np.abs(st.V[:, :j + 1].T @ st.V[:, :j + 1] - np.eye(j + 1)).max()))
    U, S, V, info = svds(op, k, p, 1e-10, 3000, v0=v0, partial=True, callback=cb)
    assert info.converged
    np.testing.assert_allclose(S, exact[:k], rtol=1e-12)
    assert max(orth) <= 10 * np.sqrt(svds_ref.EPS)
    assert np.abs(U.T @ U - np.eye(k)).max() <= 10 * np.sqrt(svds_ref.EPS)
    assert np.abs(V.T @ V - np.eye(k)).max() <= 10 * np.sqrt(svds_ref.EPS)
    assert 0 < info.partial_columns < 0.6 * info.partial_possible


def test_partial_reorth_mode_exclusive_with_selective():
    A = inputs.sparse_uniform(100, 80, 800, seed=75)
    with pytest.raises(ValueError):
        svds(as_operator(A), 3, 10, 1e-10, 10, selective=True, partial=True)


# --- harmonic-Ritz augmentation (smallest triplets) ---------------------------

def _harmonic_case():
    sig = _small_cluster_spectrum(600)
    A = inputs.prescribed_sparse(120, 5, sig, seed=21)
    return as_operator(A), sig


def test_harmonic_residuals_share_one_direction():
    """The textbook property the augmentation rests on: the residuals
    A^T A V_t s_j - theta_j V_t s_j of all harmonic Ritz pairs (theta_j the
    squared singular values of [T, beta_t e_t], s_j = T^{-1} x_j) are
    parallel to f = v_{t+1} - beta_t V_t T^{-1} e_t."""
    op, sig = _harmonic_case()
    D = op.toarray()
    p = 20
    U, Tp, V, beta, _ = lbp(op, p, inputs.start_vector(600, 81))
    Vfull = np.zeros((600, p + 1))
    Vfull[:, :p] = V
    # v_{t+1} from the relation A^T u_t = alpha_t v_t + beta_t v_{t+1}
    Vfull[:, p] = (D.T @ U[:, p - 1] - Tp[p - 1, p - 1] * V[:, p - 1]) / beta
    B = np.hstack([Tp, np.zeros((p, 1))])
    B[p - 1, p] = beta
    X, sb, _ = np.linalg.svd(B, full_matrices=False)
    z = np.linalg.solve(Tp, np.eye(p)[:, p - 1])
    f = Vfull[:, p] - beta * V @ z
    f /= np.linalg.norm(f)
    for j in range(p):
        s_j = np.linalg.solve(Tp, X[:, j])
        x = V @ s_j
        r = D.T @ (D @ x) - sb[j] ** 2 * x
        rn = np.linalg.norm(r)
        if rn > 1e-10 * np.linalg.norm(x) * sb[0] ** 2:
            assert abs(abs(r @ f) / rn - 1.0) <= 1e-8, j


def test_harmonic_restart_keeps_the_lanczos_relations():
    """After harmonic restarts, A V_t = U_t T and A^T U_t = V_t T^T +
    beta_t v_{t+1} e_t^T still hold to rounding and the bases stay
    orthonormal (T starts with the full k x k block R_M)."""
    op, sig = _harmonic_case()
    D = op.toarray()
    k, p = 4, 12
    checks = []

    def cb(stage, st, extra):
        if stage == "svd" and st.info.harmonic_restarts > 0:
            U, V, T = st.U, st.V, st.T
            e1 = np.abs(D @ V[:, :p] - U @ T[:p, :p]).max()
            R = D.T @ U - V[:, :p] @ T[:p, :p].T
            R[:, p - 1] -= T[p - 1, p] * V[:, p]
            checks.append((e1, np.abs(R).max(), np.abs(U.T @ U - np.eye(p)).max(),
                           np.abs(V.T @ V - np.eye(p + 1)).max()))
    U, S, V, info = svds(op, k, p, 1e-10, 5000, v0=inputs.start_vector(600, 23), which="smallest", harmonic=True,
                         callback=cb)
    assert info.converged and info.harmonic_restarts > 0 and checks
    for e1, e2, ou, ov in checks:
        assert e1 <= 1e-13 and e2 <= 1e-13
        assert ou <= 1e-13 and ov <= 1e-13
    exact = np.sort(sig)[:k]
    np.testing.assert_allclose(S, exact, rtol=1e-10)
    r1, r2 = explicit_residuals(op, U, S, V)
    assert (r2 / S).max() <= 2e-10


def test_harmonic_restart_basis_spans_the_harmonic_ritz_vectors():
    """The restart coefficients against their textbook definition, built
    here through the solve with T: span(Q_C) = span{[g_j; 0], [-beta z; 1]}
    with g_j = y_j(1:t) + beta y_j(t+1) z, z = T^{-1} e_t; the first k
    columns of Q_C lie in span(V_t); Q_C and Q_M are orthonormal;
    B Q_C(:, 1:k) = Q_M R_M and B^T Q_M lies in span(Q_C) to rounding."""
    op, sig = _harmonic_case()
    p, k = 20, 4
    _, Tp, _, beta, _ = lbp(op, p, inputs.start_vector(600, 84))
    T = np.zeros((p + 1, p + 1))
    T[:p, :p] = Tp
    T[p - 1, p] = beta
    QC, QM, RM = harmonic_restart_basis(T, p, k)
    B = T[:p, :p + 1]
    _, sb, Yt = np.linalg.svd(B)
    idx = np.argsort(sb)[:k]
    z = np.linalg.solve(Tp, np.eye(p)[:, p - 1])
    C = np.zeros((p + 1, k + 1))
    C[:p, :k] = Yt.T[:p, idx] + beta * np.outer(z, Yt.T[p, idx])
    C[:p, k] = -beta * z
    C[p, k] = 1.0
    Qc, _ = np.linalg.qr(C)
    assert np.abs(Qc @ Qc.T - QC @ QC.T).max() <= 1e-10
    assert np.all(QC[p, :k] == 0.0) and QC[p, k] > 0
    assert np.abs(QC.T @ QC - np.eye(k + 1)).max() <= 1e-14
    assert np.abs(QM.T @ QM - np.eye(k)).max() <= 1e-14
    assert np.abs(B @ QC[:, :k] - QM @ RM).max() <= 1e-14 * sb[0]
    G = B.T @ QM
    assert np.abs(G - QC @ (QC.T @ G)).max() <= 1e-14 * sb[0]
    # B restricted to the kept spans, Q_M^T B Q_C = [R_M, coupling], has
    # exactly the k harmonic values as its singular values
    assert np.allclose(np.sort(np.linalg.svd(QM.T @ B @ QC, compute_uv=False)), np.sort(sb[idx]), rtol=1e-12)


def test_harmonic_fewer_cycles_on_clustered_small_values():
    """Six clustered small values 1e-4 (1 + 0.01 i) below a bulk in [0.5, 1]
    (1000 x 1000, five nonzeros per row): the harmonic restart converges in
    far fewer cycles than plain Ritz augmentation, to the prescribed values
    within 1e-10 relative."""
    N = 1000
    sig = np.concatenate([1e-4 * (1 + 0.01 * np.arange(6)), np.linspace(0.5, 1.0, N - 6)])
    op = as_operator(inputs.prescribed_sparse(N // 5, 5, sig, seed=1))
    exact = np.sort(sig)[:4]
    res = {}
    for h in (False, True):
        U, S, V, info = svds(op, 4, 20, 1e-10, 3000, v0=inputs.start_vector(N, 23), which="smallest", harmonic=h)
        assert info.converged
        np.testing.assert_allclose(S, exact, rtol=1e-10)
        r1, r2 = explicit_residuals(op, U, S, V)
        assert (r1 / S).max() <= 1e-9 and (r2 / S).max() <= 1e-9
        res[h] = info
    assert res[True].harmonic_restarts == res[True].cycles - 1
    assert res[True].cycles * 5 < res[False].cycles


def test_harmonic_needs_smallest_and_full_reorth():
    A = as_operator(inputs.sparse_uniform(100, 80, 800, seed=82))
    for kw in (dict(harmonic=True), dict(harmonic=True, which="smallest", partial=True)):
        with pytest.raises(ValueError):
            svds(A, 3, 10, 1e-10, 10, **kw)


# --- eq. (4) inside a cycle (the reading behind the early stop) -----------------

def test_proposition1_holds_at_every_lanczos_dimension():
    """Proposition 1 for the leading block: after j Lanczos steps (first
    cycle or after a restart), the Ritz triplets of T(1:j,1:j) with the first
    j basis vectors have |A^T u_i - s_i v_i| = |beta_j Uh(j, i)| and
    A v_i = s_i u_i, so testing eq. (4) at any j is testing the triplets that
    would be output at j."""
    A = inputs.config_matrix(1)
    op = as_operator(A)
    D = op.toarray()
    k, p = 10, 30
    states = []

    def cb(stage, st, extra):
        if stage in ("lbp", "svd"):
            states.append((st.U.copy(), st.V.copy(), st.T.copy(), stage))
    svds(op, k, p, 1e-14, 3, v0=inputs.start_vector(A.n, inputs.CONFIG_SEEDS[1] + 1), callback=cb)
    # the first LBP and the second cycle (arrow T after a restart)
    for U, V, T, stage in (states[0], states[2]):
        for j in range(k + 2, p + 1, 3):
            Uh, s, Vht = np.linalg.svd(T[:j, :j])
            beta = T[j - 1, j]
            Ut = U[:, :j] @ Uh[:, :k]
            Vt = V[:, :j] @ Vht.T[:, :k]
            est = np.abs(beta * Uh[j - 1, :k])
            true = np.linalg.norm(D.T @ Ut - Vt * s[:k], axis=0)
            np.testing.assert_allclose(true, est, rtol=0, atol=1e-12 * s[0])
            assert np.abs(D @ Vt - Ut * s[:k]).max() <= 1e-12 * s[0]
