"""Per-step parity of the HIP kernels (through the C ABI) against the CPU
oracle / plain definitions, on the same seeded inputs.

Rows covered: SpMV A x and A^T y with the fused Lanczos terms, the device
transpose (bit-exact), CGS2 re-orthogonalization, the small SVD + eq. (4)
test + restart set-up, the restart rotation, the Philox start vector, the
dense mat-vecs.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.linalg as sla

from paper_2405_18966_amd import inputs
from oracle import svds_ref, philox

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_18966_amd import svds
    return svds


def _t(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _scalar(v):
    return _t(np.array([v], dtype=np.float64))


# --- Philox start vector -------------------------------------------------------

@pytest.mark.parametrize("L,seed,stream", [(1, 0, 0), (7, 2405001, 0), (100001, 99, 5), (4096, 2**63 + 5, 1)])
def test_philox_normal_matches_oracle(S, L, seed, stream):
    g = S.svds_op_philox_normal(L, seed, stream).cpu().numpy()
    ref = philox.normal_vector(L, seed, stream)
    np.testing.assert_allclose(g, ref, rtol=1e-13, atol=1e-15)


# --- SpMV ---------------------------------------------------------------------

def _spmv_case(A, S, dtype_basis, x_scale, coef, use_prev, seed):
    import torch
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(A.n)
    yp = rng.standard_normal(A.m)
    tb = torch.float64 if dtype_basis == "f64" else torch.float32
    Ad, keep = S.csr_to_device(A)
    xd = _t(x, tb)
    y = S.svds_op_spmv_csr(Ad, xd, _scalar(x_scale), _scalar(coef) if use_prev else None,
                           _t(yp, tb) if use_prev else None).cpu().numpy().astype(np.float64)
    xr = x if dtype_basis == "f64" else x.astype(np.float32).astype(np.float64)
    ypr = yp if dtype_basis == "f64" else yp.astype(np.float32).astype(np.float64)
    Asp = A.to_scipy()
    ref = x_scale * (Asp @ xr) - (coef * ypr if use_prev else 0.0)
    scale = np.abs(Asp) @ np.abs(xr) * abs(x_scale) + (abs(coef) * np.abs(ypr) if use_prev else 0.0)
    # forward error bound of a length-l sum with one extra scale/subtract:
    # (l + 3) u |terms|, u the unit roundoff of the basis type
    u = 2.0**-53 if dtype_basis == "f64" else 2.0**-24
    lens = np.diff(A.row_ptr).astype(np.float64)
    return y, ref, (lens + 3) * u * scale + 1e-300


@pytest.mark.parametrize("shape,nnz", [((2000, 1000), 20000), ((1, 5), 3), ((700, 3), 1500), ((5000, 4000), 0)])
def test_spmv_uniform_matches_scipy(S, shape, nnz):
    A = inputs.sparse_uniform(shape[0], shape[1], nnz, seed=5)
    for basis in ("f64", "f32"):
        y, ref, bound = _spmv_case(A, S, basis, 0.37, -1.25, True, 6)
        assert np.all(np.abs(y - ref) <= bound), basis


def test_spmv_power_law_long_rows(S):
    """Transposed Zipf matrix: rows with tens of thousands of entries go through
    the piece path with its ordered last-piece reduction."""
    A = inputs.sparse_zipf(60000, 20000, 10, 1.1, seed=7)
    At = A.to_scipy().T.tocsr()
    At.sort_indices()
    T = inputs.CSR(A.n, A.m, At.indptr.astype(np.int32), At.indices.astype(np.int32), At.data)
    assert np.diff(T.row_ptr).max() > 20000  # long rows present
    assert (np.diff(T.row_ptr) == 0).any()   # empty rows present
    y, ref, bound = _spmv_case(T, S, "f64", 1.0, 0.5, True, 8)
    assert np.all(np.abs(y - ref) <= bound)


def test_spmv_fp32_values_widened(S):
    A = inputs.round_values_f32(inputs.sparse_uniform(300, 200, 3000, seed=9))
    y, ref, bound = _spmv_case(A, S, "f64", 1.0, 0.0, False, 10)
    assert np.all(np.abs(y - ref) <= bound)


def test_spmv_deterministic(S):
    A = inputs.sparse_zipf(30000, 10000, 10, 1.1, seed=11)
    At = A.to_scipy().T.tocsr()
    T = inputs.CSR(A.n, A.m, At.indptr.astype(np.int32), At.indices.astype(np.int32), At.data)
    y1, _, _ = _spmv_case(T, S, "f64", 1.0, 0.5, True, 12)
    y2, _, _ = _spmv_case(T, S, "f64", 1.0, 0.5, True, 12)
    assert np.array_equal(y1, y2)


@pytest.mark.parametrize("m,panels", [(300_001, 2), (600_003, 4), (1_100_005, 8)])
def test_transposed_product_column_panels(S, m, panels):
    """A^T x as the solver runs it, with x long enough to be cut into column
    panels (2, 4, 8 slices of at most 2 MiB of FP64 gathers; the last panel
    ragged).  Power-law rows of A^T are split into pieces inside each panel.
    Against scipy to the forward error bound of a sum of the row's terms
    (any order) plus the panel partials, in both basis types; repeat calls are
    bit-identical; the forward product through the same plan too."""
    import torch
    A = inputs.sparse_zipf(m, 20_000, 10, 1.1, seed=17)
    Asp = A.to_scipy()
    At = Asp.T.tocsr()
    Ad, keep = S.csr_to_device(A)
    rng = np.random.default_rng(18)
    x = rng.standard_normal(A.m)
    yp = rng.standard_normal(A.n)
    lens = np.diff(At.indptr).astype(np.float64)
    assert lens.max() > 4 * 4096  # pieces in every panel
    for tb, u in ((torch.float64, 2.0**-53), (torch.float32, 2.0**-24)):
        xr = x if tb == torch.float64 else x.astype(np.float32).astype(np.float64)
        ypr = yp if tb == torch.float64 else yp.astype(np.float32).astype(np.float64)
        y, npan = S.svds_op_csr_matvec(Ad, True, _t(x, tb), _scalar(0.37), _scalar(-1.25), _t(yp, tb))
        assert npan == panels
        y = y.cpu().numpy().astype(np.float64)
        ref = 0.37 * (At @ xr) + 1.25 * ypr
        scale = 0.37 * (np.abs(At) @ np.abs(xr)) + 1.25 * np.abs(ypr)
        assert np.all(np.abs(y - ref) <= (lens + panels + 3) * u * scale + 1e-300)
        y2, _ = S.svds_op_csr_matvec(Ad, True, _t(x, tb), _scalar(0.37), _scalar(-1.25), _t(yp, tb))
        assert np.array_equal(y, y2.cpu().numpy().astype(np.float64))
    # no yprev term, and the forward product through the same entry point
    y, _ = S.svds_op_csr_matvec(Ad, True, _t(x), None, None, None)
    np.testing.assert_allclose(y.cpu().numpy(), At @ x, rtol=1e-12, atol=1e-12 * np.abs(At @ x).max())
    v = rng.standard_normal(A.n)
    y, npan = S.svds_op_csr_matvec(Ad, False, _t(v), None, None, None)
    assert npan == 1
    np.testing.assert_allclose(y.cpu().numpy(), Asp @ v, rtol=1e-12, atol=1e-12 * np.abs(Asp @ v).max())


@pytest.mark.parametrize("maker", [
    lambda: inputs.sparse_zipf(60000, 20000, 10, 1.1, seed=23),
    lambda: inputs.sparse_uniform(9000, 7000, 300000, seed=24),
    lambda: inputs.round_values_f32(inputs.sparse_uniform(3000, 2000, 60000, seed=25)),
])
def test_column_sorted_items_bit_identical(S, maker):
    """A plan stores every work item's nonzeros sorted by column and puts the
    products back at their row-order positions: A x and A^T x through a plan
    equal, bit for bit, the row-ordered product over the same items.  With
    FP32 bases a plan of FP64 values reads its FP32 copies (the FP32 phase of
    a mixed solve), so the row-ordered reference then takes the values
    rounded to FP32."""
    import torch
    A = maker()
    Ad, keep = S.csr_to_device(A)
    A32 = inputs.round_values_f32(A)
    Ad32, keep32 = S.csr_to_device(A32)
    rng = np.random.default_rng(26)
    for tb in (torch.float64, torch.float32):
        R, Rd = (A, Ad) if tb == torch.float64 else (A32, Ad32)
        x = _t(rng.standard_normal(A.n), tb)
        yp = _t(rng.standard_normal(A.m), tb)
        y_plan, _ = S.svds_op_csr_matvec(Ad, False, x, _scalar(0.5), _scalar(2.0), yp)
        y_rows = S.svds_op_spmv_csr(Rd, x, _scalar(0.5), _scalar(2.0), yp)
        assert torch.equal(y_plan, y_rows)
        vdt = torch.float64 if R.val.dtype == np.float64 else torch.float32
        trp, tci, tv = S.svds_op_csc_build(Rd, vdt)
        T = S.make_csr(trp, tci, tv, A.n, A.m)
        u = _t(rng.standard_normal(A.m), tb)
        z_plan, npan = S.svds_op_csr_matvec(Ad, True, u)
        assert npan == 1
        z_rows = S.svds_op_spmv_csr(T, u)
        assert torch.equal(z_plan, z_rows)


def test_transposed_product_column_panels_fp32_values(S):
    """Column panels over a matrix stored with FP32 values (widened exactly),
    FP64 and FP32 bases."""
    import torch
    A = inputs.round_values_f32(inputs.sparse_zipf(600_003, 30_000, 10, 1.1, seed=27))
    Ad, keep = S.csr_to_device(A)
    At = sp.csr_matrix((A.val.astype(np.float64), A.col_idx, A.row_ptr), shape=(A.m, A.n)).T.tocsr()
    lens = np.diff(At.indptr).astype(np.float64)
    x = np.random.default_rng(28).standard_normal(A.m)
    for tb, u in ((torch.float64, 2.0**-53), (torch.float32, 2.0**-24)):
        xr = x if tb == torch.float64 else x.astype(np.float32).astype(np.float64)
        y, npan = S.svds_op_csr_matvec(Ad, True, _t(x, tb))
        assert npan == 4
        ref = At @ xr
        bound = (lens + 4 + 3) * u * (np.abs(At) @ np.abs(xr)) + 1e-300
        assert np.all(np.abs(y.cpu().numpy().astype(np.float64) - ref) <= bound)


def test_transposed_product_no_panels_for_short_or_sparse(S):
    """Short x, or too few entries per row of A^T: the plain product."""
    for A in (inputs.sparse_zipf(200_000, 20_000, 10, 1.1, seed=19),
              inputs.sparse_uniform(400_000, 300_000, 1_000_000, seed=20)):
        Ad, keep = S.csr_to_device(A)
        x = np.random.default_rng(21).standard_normal(A.m)
        y, npan = S.svds_op_csr_matvec(Ad, True, _t(x), None, None, None)
        assert npan == 1
        ref = A.to_scipy().T @ x
        np.testing.assert_allclose(y.cpu().numpy(), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


# --- device transpose (bit-exact) ----------------------------------------------

@pytest.mark.parametrize("maker", [
    lambda: inputs.sparse_uniform(2000, 1000, 20000, seed=1),
    lambda: inputs.sparse_zipf(50000, 30000, 10, 1.1, seed=2),
    lambda: inputs.sparse_uniform(3, 300, 7, seed=3),
    lambda: inputs.sparse_uniform(400, 5, 0, seed=4),
    lambda: inputs.round_values_f32(inputs.sparse_uniform(100, 70000, 5000, seed=5)),
])
def test_transpose_bit_exact(S, maker):
    import torch
    A = maker()
    Ad, keep = S.csr_to_device(A)
    vdt = torch.float64 if A.val.dtype == np.float64 else torch.float32
    trp, tci, tv = S.svds_op_csc_build(Ad, vdt)
    At = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.m, A.n)).T.tocsr()
    At.sort_indices()  # canonical: increasing row of A within each column
    assert np.array_equal(trp.cpu().numpy(), At.indptr.astype(np.int32))
    assert np.array_equal(tci.cpu().numpy(), At.indices.astype(np.int32))
    assert np.array_equal(tv.cpu().numpy().view(np.uint8), np.asarray(At.data, dtype=A.val.dtype).view(np.uint8))


# --- CGS2 ------------------------------------------------------------------------

# short vectors (<= 2048 row tiles, j <= 256) take the tile-per-block update,
# longer ones or wider bases the row-per-thread update: both, at the limits
@pytest.mark.parametrize("L,j", [(1000, 0), (1000, 1), (1000, 16), (1000, 17), (2049, 100),
                                 (100003, 150), (5000, 161), (5000, 256), (6000, 300), (70, 60),
                                 (262144, 200), (400000, 60), (4000, 320), (5000, 321), (3000, 700)])
def test_cgs2_matches_oracle(S, L, j):
    import torch
    rng = np.random.default_rng(L + j)
    Q = np.linalg.qr(rng.standard_normal((L, max(j, 1))))[0][:, :j]
    w = rng.standard_normal(L) + (Q @ rng.standard_normal(j) * 10 if j else 0)
    ref = svds_ref.cgs2(w, Q)
    Qd = _t(np.asfortranarray(Q).T.copy()) if j else None  # (j, L) rows = columns
    out, nrm = S.svds_op_cgs2(Qd, j, _t(w), ldq=L)
    out = out.cpu().numpy()
    assert np.linalg.norm(out - ref) <= 1e-14 * np.linalg.norm(w) * max(1, np.sqrt(j))
    assert abs(nrm - np.linalg.norm(ref)) <= 1e-13 * np.linalg.norm(w)
    if j:
        assert np.abs(Q.T @ out).max() <= 1e-14 * np.linalg.norm(w)


@pytest.mark.parametrize("L,ld,j", [(2049, 2050, 100), (100003, 100004, 150), (999, 1000, 20)])
def test_cgs2_ragged_tail_padded_ld(S, L, ld, j):
    """Odd length with an even leading dimension: the 16-byte row accesses
    run with a one-row tail in the last tile."""
    rng = np.random.default_rng(L + 7 * j)
    Q = np.linalg.qr(rng.standard_normal((L, j)))[0]
    w = rng.standard_normal(L) + Q @ rng.standard_normal(j) * 10
    ref = svds_ref.cgs2(w, Q)
    Qp = np.zeros((j, ld))
    Qp[:, :L] = Q.T
    out, nrm = S.svds_op_cgs2(_t(Qp), j, _t(w), ldq=ld)
    out = out.cpu().numpy()
    assert np.linalg.norm(out - ref) <= 1e-14 * np.linalg.norm(w) * np.sqrt(j)
    assert abs(nrm - np.linalg.norm(ref)) <= 1e-13 * np.linalg.norm(w)
    assert np.abs(Q.T @ out).max() <= 1e-14 * np.linalg.norm(w)


def test_cgs2_fp32(S):
    import torch
    rng = np.random.default_rng(3)
    L, j = 20000, 77
    Q = np.linalg.qr(rng.standard_normal((L, j)))[0].astype(np.float32)
    w = rng.standard_normal(L).astype(np.float32)
    ref = svds_ref.cgs2(w.astype(np.float64), Q.astype(np.float64))
    out, nrm = S.svds_op_cgs2(_t(np.ascontiguousarray(Q.T)), j, _t(w), ldq=L)
    assert np.linalg.norm(out.cpu().numpy() - ref) <= 5e-6 * np.linalg.norm(w)


# --- small SVD + test + restart set-up ----------------------------------------------

def _lanczos_T(m, n, p, seed, restarted_k=0):
    """A real T from the oracle: bidiagonal (first LBP) or arrow-shaped (the
    T of the second cycle, after one restart with k kept vectors)."""
    A = svds_ref.as_operator(inputs.sparse_uniform(m, n, m * n // 10, seed=seed))
    v0 = inputs.start_vector(n, seed + 1)
    seen = []

    def cb(stage, st, ex):
        if stage == "svd":
            seen.append(st.T.copy())
    svds_ref.svds(A, restarted_k or 1, p, 1e-15, 2, v0=v0, callback=cb)
    return seen[1] if restarted_k else seen[0]


@pytest.mark.parametrize("p,k,restarted", [(2, 1, 0), (3, 1, 0), (15, 5, 0), (30, 10, 0), (30, 10, 1),
                                           (63, 20, 1), (64, 20, 0), (150, 50, 1), (250, 100, 1)])
def test_small_svd_matches_lapack(S, p, k, restarted):
    import torch
    Tfull = _lanczos_T(max(3 * p, 40), max(2 * p + 2, 30), p, 100 + p, k if restarted else 0)
    Tp = Tfull[:p, :p]
    beta = Tfull[p - 1, p]
    Uh, s, Vh = svds_ref.small_svd(Tp)
    Td = _t(Tfull.copy())
    tol = 1e-6
    Uk, Vext, sig, res, rho, flags = S.svds_op_small_svd(Td, p, k, tol)
    sig = sig.cpu().numpy()
    np.testing.assert_allclose(sig, s[:k], rtol=1e-13, atol=1e-14 * s[0])
    Uk = Uk.cpu().numpy().T
    Vx = Vext.cpu().numpy().T
    for j in range(k):
        gap = min([abs(s[j] - s[i]) for i in range(p) if i != j])
        if gap < 1e-8 * s[0]:
            continue
        bound = 1e-12 * s[0] / gap + 1e-13
        sgn = np.sign(Uk[:, j] @ Uh[:, j])
        assert np.abs(Uk[:, j] - sgn * Uh[:, j]).max() < bound
        assert np.abs(Vx[:p, j] - sgn * Vh[:, j]).max() < bound
    assert np.all(Vx[p, :k] == 0) and np.array_equal(Vx[:, k], np.eye(p + 1)[p])
    # eq. (4) estimates and eq. (6) arrow from the device's own vectors
    ref_res = np.abs(beta * Uk[p - 1, :]) / np.maximum(sig, max(2.0**-52 * sig[0], np.finfo(float).tiny))
    np.testing.assert_array_equal(res.cpu().numpy(), ref_res)
    np.testing.assert_array_equal(rho.cpu().numpy(), beta * Uk[p - 1, :])
    assert flags[0] == int(np.all(ref_res < tol))
    lead = 0
    while lead < k and ref_res[lead] < tol:
        lead += 1
    assert flags[1] == lead and 1 <= flags[2] <= 30
    # restarted T (Alg. 2 step 9)
    Tn = Td.cpu().numpy()
    ref_T = np.zeros_like(Tn)
    ref_T[np.arange(k), np.arange(k)] = sig
    ref_T[:k, k] = beta * Uk[p - 1, :]
    np.testing.assert_array_equal(Tn, ref_T)


def test_small_svd_repeated_and_zero_values(S):
    """Diagonal T with repeated and zero entries: exact values, no NaN."""
    p, k = 12, 6
    d = np.array([3, 3, 3, 2, 0, 1, 1, 0.5, 0, 0, 2, 3], dtype=np.float64)
    T = np.zeros((p + 1, p + 1))
    T[np.arange(p), np.arange(p)] = d
    T[p - 1, p] = 0.25
    Uk, Vext, sig, res, rho, flags = S.svds_op_small_svd(_t(T), p, k, 1e-10)
    np.testing.assert_array_equal(sig.cpu().numpy(), np.sort(d)[::-1][:k])
    assert np.all(np.isfinite(res.cpu().numpy()))


# --- restart rotation ---------------------------------------------------------------

@pytest.mark.parametrize("L,pc,kc", [(1000, 30, 10), (1000, 31, 11), (65537, 150, 50), (3001, 251, 101),
                                     (100, 600, 3), (64, 1, 1)])
@pytest.mark.parametrize("vector", [False, True])
def test_rotate_matches_numpy(S, L, pc, kc, vector):
    """Matrix-core (FP64 / FP32 MFMA) and vector-FMA kernels against numpy."""
    import torch
    rng = np.random.default_rng(L + pc)
    B = rng.standard_normal((L, pc))
    Y = rng.standard_normal((pc, kc))
    out = S.svds_op_rotate(_t(np.ascontiguousarray(B.T)), pc, _t(np.ascontiguousarray(Y.T)), kc, vector=vector)
    ref = B @ Y
    scale = np.abs(B) @ np.abs(Y)
    assert np.all(np.abs(out.cpu().numpy().T - ref) <= 4e-16 * pc * scale)
    out32 = S.svds_op_rotate(_t(np.ascontiguousarray(B.T), torch.float32), pc,
                             _t(np.ascontiguousarray(Y.T)), kc, vector=vector)
    # FP32 arithmetic: B in FP32, Y rounded to FP32, FP32 accumulation
    B32 = B.astype(np.float32).astype(np.float64)
    Y32 = Y.astype(np.float32).astype(np.float64)
    assert np.all(np.abs(out32.cpu().numpy().T - B32 @ Y32) <= 3e-7 * pc * (np.abs(B32) @ np.abs(Y32)))


# --- dense mat-vecs -------------------------------------------------------------------

@pytest.mark.parametrize("m,n", [(1000, 700), (513, 257), (64, 3000), (20000, 300), (1002, 300), (1004, 33)])
@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
def test_dense_matvec_matches_numpy(S, m, n, store):
    import torch
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n))
    if store == "f64":
        a = np.asfortranarray(A)
        rec = A
        at = _t(a.ravel(order="F"))
    elif store == "f32":
        a = np.asfortranarray(A.astype(np.float32))
        rec = a.astype(np.float64)
        at = _t(a.ravel(order="F"))
    else:
        bits = inputs._f32_to_bf16_bits(np.asfortranarray(A.astype(np.float32)))
        rec = inputs.bf16_bits_to_f64(bits)
        at = _t(np.asfortranarray(bits).ravel(order="F").view(np.int16)).view(torch.bfloat16)
    Ad = S.make_dense(at, m, n)
    x = rng.standard_normal(n)
    u = rng.standard_normal(m)
    yp_m = rng.standard_normal(m)
    yp_n = rng.standard_normal(n)
    y = S.svds_op_dense_matvec(Ad, False, _t(x), _scalar(0.5), _scalar(2.0), _t(yp_m)).cpu().numpy()
    ref = 0.5 * (rec @ x) - 2.0 * yp_m
    sc = 0.5 * (np.abs(rec) @ np.abs(x)) + 2 * np.abs(yp_m)
    assert np.all(np.abs(y - ref) <= (n + 3) * 2.0**-53 * sc)
    z = S.svds_op_dense_matvec(Ad, True, _t(u), _scalar(1.0), _scalar(-1.0), _t(yp_n)).cpu().numpy()
    ref = rec.T @ u + yp_n
    sc = np.abs(rec.T) @ np.abs(u) + np.abs(yp_n)
    assert np.all(np.abs(z - ref) <= (m + 3) * 2.0**-53 * sc)


def test_small_svd_near_degenerate_pair(S):
    """Decay1 has sigma_20 = sigma_21 exactly; T of the first Lanczos cycle has
    a pair of Ritz values 1e-13 apart whose inner product sits at the rounding
    floor.  Every lane of a wave must take the same rotation decision and
    angle, or the accumulated right vectors lose orthogonality."""
    sig = inputs.decay1(300)
    A = inputs.prescribed_dense(500, 300, sig, seed=61)
    seen = []
    svds_ref.svds(A, 20, 60, 1e-10, 1, v0=inputs.start_vector(300, 62),
                  callback=lambda st, s, ex: seen.append(s.T.copy()) if st == "svd" else None)
    T = seen[0]
    p, k = 60, 20
    s_ref = sla.svd(T[:p, :p], compute_uv=False, lapack_driver="gesvd")
    Uk, Vext, sg, res, rho, flags = S.svds_op_small_svd(_t(T.copy()), p, k, 1e-10)
    Uk = Uk.cpu().numpy().T
    Vk = Vext.cpu().numpy().T[:p, :k]
    np.testing.assert_allclose(sg.cpu().numpy(), s_ref[:k], rtol=1e-13)
    assert np.abs(Vk.T @ Vk - np.eye(k)).max() < 1e-13
    assert np.abs(Uk.T @ Uk - np.eye(k)).max() < 1e-13


# --- explicit residuals (block products over 8 triplets at a time) ---------------------

@pytest.mark.parametrize("k", [1, 5, 8, 13])
@pytest.mark.parametrize("vdt", ["f64", "f32"])
def test_block_residuals_match_numpy(S, k, vdt):
    """|A v_j - s_j u_j| and |A^T u_j - s_j v_j| for arbitrary (not singular)
    triplets, on a Zipf matrix whose heaviest columns are long rows of A^T
    (pieces + long-row fix-up)."""
    A = inputs.sparse_zipf(30000, 9000, 12, 1.3, seed=k + 3)
    if vdt == "f32":
        A = inputs.round_values_f32(A)
    rng = np.random.default_rng(k)
    U = rng.standard_normal((A.m, k))
    V = rng.standard_normal((A.n, k))
    s = rng.uniform(1, 2, k)
    Ad, keep = S.csr_to_device(A)
    r1, r2 = S.svds_residuals_csr(Ad, _t(U), _t(s), _t(V))
    Asp = svds_ref.as_operator(inputs.CSR(A.m, A.n, A.row_ptr, A.col_idx, A.val.astype(np.float64)))
    e1 = np.linalg.norm(Asp @ V - U * s, axis=0)
    e2 = np.linalg.norm(Asp.T @ U - V * s, axis=0)
    np.testing.assert_allclose(r1.cpu().numpy(), e1, rtol=1e-12)
    np.testing.assert_allclose(r2.cpu().numpy(), e2, rtol=1e-12)


@pytest.mark.parametrize("m,n,k", [(1000, 700, 20), (513, 257, 7), (300, 2000, 150), (1001, 333, 9), (4100, 97, 1)])
@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
def test_dense_block_residuals_match_numpy(S, m, n, k, store):
    """|A v_j - s_j u_j| and |A^T u_j - s_j v_j| of the dense form for arbitrary
    (not singular) triplets: FP64 matrix-core block products over the stored
    matrix.  Ragged row blocks and K chunks, two column groups (k = 150), an
    odd leading dimension (element-wise loads) and k = 1."""
    import torch
    rng = np.random.default_rng(m * 7 + n + k)
    A = rng.standard_normal((m, n))
    if store == "f64":
        rec = np.asfortranarray(A)
        at = _t(rec.ravel(order="F"))
    elif store == "f32":
        a = np.asfortranarray(A.astype(np.float32))
        rec = a.astype(np.float64)
        at = _t(a.ravel(order="F"))
    else:
        bits = inputs._f32_to_bf16_bits(np.asfortranarray(A.astype(np.float32)))
        rec = inputs.bf16_bits_to_f64(bits)
        at = _t(np.asfortranarray(bits).ravel(order="F").view(np.int16)).view(torch.bfloat16)
    Ad = S.make_dense(at, m, n)
    U = rng.standard_normal((m, k))
    V = rng.standard_normal((n, k))
    s = rng.uniform(1, 2, k)
    r1, r2 = S.svds_residuals_dense(Ad, _t(U), _t(s), _t(V))
    e1 = np.linalg.norm(rec @ V - U * s, axis=0)
    e2 = np.linalg.norm(rec.T @ U - V * s, axis=0)
    np.testing.assert_allclose(r1.cpu().numpy(), e1, rtol=1e-12)
    np.testing.assert_allclose(r2.cpu().numpy(), e2, rtol=1e-12)


def test_dense_block_residuals_of_exact_triplets(S):
    """Exact singular triplets of a prescribed-spectrum matrix: the residuals
    are at rounding level (no cancellation left uncovered)."""
    import torch
    sig = inputs.decay2(200)
    A = inputs.prescribed_dense_dct(700, 500, sig, seed=5)
    Uf, sf, Vtf = np.linalg.svd(A, full_matrices=False)
    k = 40
    Ad = S.make_dense(_t(np.asfortranarray(A).ravel(order="F")), 700, 500)
    r1, r2 = S.svds_residuals_dense(Ad, _t(Uf[:, :k]), _t(sf[:k]), _t(Vtf[:k].T))
    e1 = np.linalg.norm(A @ Vtf[:k].T - Uf[:, :k] * sf[:k], axis=0)
    e2 = np.linalg.norm(A.T @ Uf[:, :k] - Vtf[:k].T * sf[:k], axis=0)
    assert np.abs(r1.cpu().numpy() - e1).max() <= 1e-13 * sf[0]
    assert np.abs(r2.cpu().numpy() - e2).max() <= 1e-13 * sf[0]


@pytest.mark.parametrize("L,nseg,uneven", [(1, 1, False), (5000, 1, False), (123457, 8, True), (40000, 3, False)])
def test_gather_copy_matches_indexing(S, L, nseg, uneven):
    """The gather-rate reference: out[i] = x[idx[i]] bit for bit, over
    segments that are uneven, empty or shorter than a chunk."""
    import torch
    print(f"gather copy L={L} nseg={nseg}", flush=True)
    rng = np.random.default_rng(L)
    x = torch.from_numpy(rng.standard_normal(7001)).cuda()
    idx = torch.from_numpy(rng.integers(0, 7001, L).astype(np.int32)).cuda()
    seg = None
    if uneven:
        cuts = np.sort(rng.integers(0, L, nseg - 1))
        cuts[1] = cuts[0]  # an empty segment
        seg = [0] + [int(c) for c in cuts] + [L]
    out, ms = S.svds_op_gather_copy(idx, x, nseg, seg, reps=2)
    torch.cuda.synchronize()
    assert torch.equal(out, x[idx.long()]) and ms > 0
