"""End-to-end parity of the HIP solver (C ABI) against the FP64 CPU oracle on
the same seeded inputs and start vector: singular values to a relative
error, vectors up to sign (and as subspaces for multiple values), residuals,
orthogonality, mat-vec counts, edge cases and determinism."""
import numpy as np
import pytest

from paper_2405_18966_amd import inputs
from oracle import svds_ref
from oracle.svds_ref import as_operator

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_18966_amd import svds
    return svds


def _gpu_solve(S, A, k, p, tol, maxit, v0=None, seed=0, precision=0, flags=0):
    import torch
    Ad, keep = S.csr_to_device(A)
    v0d = None if v0 is None else torch.from_numpy(v0).cuda()
    r = S.svds_csr_solve(Ad, S.make_opts(k, p, tol, maxit, precision=precision, seed=seed, v0=v0d,
                                         flags=flags))
    torch.cuda.synchronize()
    return r.U.cpu().numpy(), r.S.cpu().numpy(), r.V.cpu().numpy(), r.info, r.status


def _compare(Ug, Sg, Vg, Ur, Sr, Vr, s_all, tol_sigma, vec_tol_scale):
    np.testing.assert_allclose(Sg, Sr, rtol=tol_sigma)
    k = len(Sr)
    for j in range(k):
        gap = min(abs(s_all[j] - s_all[i]) for i in range(len(s_all)) if i != j)
        if gap < 1e-9 * s_all[0]:
            continue
        bound = max(vec_tol_scale * s_all[j] / gap, 1e-10)
        for X, Y in ((Ug, Ur), (Vg, Vr)):
            d = np.linalg.norm(X[:, j] - Y[:, j])  # both sign-normalized
            assert d <= bound, (j, d, bound)


def _invariants(A, Ug, Sg, Vg, tol):
    Asp = as_operator(A)
    k = len(Sg)
    assert np.abs(Ug.T @ Ug - np.eye(k)).max() <= 1e-12
    assert np.abs(Vg.T @ Vg - np.eye(k)).max() <= 1e-12
    r1, r2 = svds_ref.explicit_residuals(Asp, Ug, Sg, Vg)
    assert r1.max() <= 1e-12 * Sg[0]
    assert (r2 / np.maximum(Sg, 1e-300 + 2**-52 * Sg[0])).max() <= 2 * tol


def _counts_ok(info, p, k):
    R = info["cycles"] - 1
    assert info["n_spmv"] == p + R * (p - k)
    assert info["n_spmvT"] == p + R * (p - k)


@pytest.mark.parametrize("case", ["w1", "tall", "wide", "square_small", "lds_max"])
def test_parity_with_oracle(S, case):
    """w1, tall and wide take the step-by-step launches, square_small and
    lds_max the one-workgroup cycles (lds_max: the longest vector those hold
    in LDS, 6144 entries, with 8000 nonzeros and 496 KB of bases)."""
    if case == "w1":
        A = inputs.config_matrix(1)
        k, p, tol = 10, 30, 1e-10
        v0 = inputs.start_vector(A.n, inputs.CONFIG_SEEDS[1] + 1)
    elif case == "tall":
        A = inputs.sparse_uniform(5000, 800, 40000, seed=3)
        k, p, tol = 8, 24, 1e-10
        v0 = inputs.start_vector(A.n, 4)
    elif case == "wide":
        A = inputs.sparse_uniform(700, 3000, 30000, seed=5)
        k, p, tol = 5, 15, 1e-10
        v0 = inputs.start_vector(A.n, 6)
    elif case == "lds_max":
        A = inputs.sparse_uniform(6144, 200, 8000, seed=9)
        k, p, tol = 3, 9, 1e-10
        v0 = inputs.start_vector(A.n, 10)
    else:
        A = inputs.sparse_uniform(60, 60, 900, seed=7)
        k, p, tol = 3, 9, 1e-12
        v0 = inputs.start_vector(A.n, 8)
    Ur, Sr, Vr, info_r = svds_ref.svds(as_operator(A), k, p, tol, 3000, v0=v0)
    Ug, Sg, Vg, info, st = _gpu_solve(S, A, k, p, tol, 3000, v0=v0)
    assert st == 0 and info["converged"] == 1 and info_r.converged
    s_all = np.linalg.svd(as_operator(A).toarray(), compute_uv=False)
    _compare(Ug, Sg, Vg, Ur, Sr, Vr, s_all, 1e-10, 10 * tol)
    _invariants(A, Ug, Sg, Vg, tol)
    _counts_ok(info, p, k)
    assert abs(info["cycles"] - info_r.cycles) <= 1
    assert info["max_res_true"] <= 2 * tol and info["max_res_est"] < tol


@pytest.mark.parametrize("case", ["ragged", "g21", "breakdowns", "zero"])
def test_mid_size_cycles(S, case):
    """Mid-size sparse problems past the one-workgroup limits (bases of 0.7
    to 10.5 MB), in the step-by-step launches.  ragged: row counts that 64
    does not divide; g21: 20,011 x 12,003 (10.5 MB of bases); breakdowns: a
    diagonal matrix with six distinct values, whose Krylov space ends after a
    few steps, so replacement vectors enter the basis; zero: every step breaks
    down.  Same bar as the oracle parity cases."""
    if case == "ragged":
        A = inputs.sparse_uniform(2003, 997, 20000, seed=61)
        k, p, tol, maxit = 10, 30, 1e-10, 3000
    elif case == "g21":
        A = inputs.sparse_uniform(20011, 12003, 200000, seed=63)
        k, p, tol, maxit = 5, 40, 1e-10, 3000
    elif case == "breakdowns":
        d = np.repeat([6.0, 5.0, 4.0, 3.0, 2.0, 1.0], [3, 2, 2, 2, 2, 2988])
        A = inputs.diag_matrix(3001, 2999, d)
        k, p, tol, maxit = 8, 20, 1e-10, 200
    else:
        A = inputs.CSR(3000, 2000, np.zeros(3001, np.int32), np.zeros(0, np.int32), np.zeros(0))
        k, p, tol, maxit = 2, 20, 1e-10, 3
    v0 = inputs.start_vector(A.n, 62)
    Ug, Sg, Vg, info, st = _gpu_solve(S, A, k, p, tol, maxit, v0=v0)
    if case == "zero":
        assert np.all(Sg == 0) and st == 0 and info["breakdowns"] >= p
        assert np.all(np.isfinite(Ug)) and np.all(np.isfinite(Vg))
        return
    Ur, Sr, Vr, info_r = svds_ref.svds(as_operator(A), k, p, tol, maxit, v0=v0)
    assert st == 0 and info["converged"] == 1 and info_r.converged
    if case == "breakdowns":
        assert info["breakdowns"] > 0 and info_r.breakdowns > 0
        np.testing.assert_allclose(Sg, np.sort(d)[::-1][:k], rtol=1e-12)
        # values wholly inside the k: the same invariant subspaces
        for val in (6.0, 5.0, 4.0):
            cols = np.nonzero(np.abs(Sg - val) < 1e-9)[0]
            colsr = np.nonzero(np.abs(Sr - val) < 1e-9)[0]
            qg, _ = np.linalg.qr(Vg[:, cols])
            qr, _ = np.linalg.qr(Vr[:, colsr])
            assert np.linalg.norm(qg - qr @ (qr.T @ qg), 2) < 1e-9
        # one of the two copies of 3: any unit vector of its subspace
        assert np.linalg.norm(Vg[d != 3.0, k - 1]) < 1e-9
    elif case == "g21":
        np.testing.assert_allclose(Sg, Sr, rtol=1e-10)
    else:
        s_all = np.linalg.svd(as_operator(A).toarray(), compute_uv=False)
        _compare(Ug, Sg, Vg, Ur, Sr, Vr, s_all, 1e-10, 10 * tol)
    _invariants(A, Ug, Sg, Vg, tol)
    _counts_ok(info, p, k)
    assert abs(info["cycles"] - info_r.cycles) <= 1


def test_parity_with_column_panel_transpose(S):
    """A long u (300,001 rows of A): the transposed products run in the
    column-panel form (two panels, power-law rows split into pieces).  Same
    bar as the other parity cases."""
    A = inputs.sparse_zipf(300_001, 30_000, 10, 1.1, seed=51)
    Ad, keep = S.csr_to_device(A)
    import torch
    _, npan = S.svds_op_csr_matvec(Ad, True, torch.zeros(A.m, dtype=torch.float64, device="cuda"))
    assert npan == 2
    k, p, tol = 8, 24, 1e-10
    v0 = inputs.start_vector(A.n, 52)
    Ur, Sr, Vr, info_r = svds_ref.svds(as_operator(A), k, p, tol, 3000, v0=v0)
    Ug, Sg, Vg, info, st = _gpu_solve(S, A, k, p, tol, 3000, v0=v0)
    assert st == 0 and info["converged"] == 1 and info_r.converged
    np.testing.assert_allclose(Sg, Sr, rtol=1e-10)
    _invariants(A, Ug, Sg, Vg, tol)
    _counts_ok(info, p, k)
    assert abs(info["cycles"] - info_r.cycles) <= 1
    assert info["max_res_true"] <= 2 * tol and info["max_res_est"] < tol


@pytest.mark.parametrize("mode,draws", [("arena", 10), ("panel_items", 10), ("panel_items", 1)])
def test_panel_fallbacks(S, mode, draws):
    """The two out-of-memory fallbacks of plan creation, forced through the
    SVDS_TEST_NO_ROOM hook on 300,001-row matrices that take two column
    panels: 'arena' (no room for the arena with the panel copy: the plan is
    carved without panels) and 'panel_items' (no room for the panel work
    items: the panels are dropped after the arena was carved; their region
    takes the column-sorted copy of A^T where it fits, as with one Zipf draw
    per row, 5 nonzeros per stacked row, and not with ten draws).  Either
    way the transposed product runs without panels and the solve is
    bit-identical to a plan made without panels (SVDS_FLAG_NO_PANELS), with
    oracle parity."""
    import os
    import torch
    A = inputs.sparse_zipf(300_001, 30_000, draws, 1.1, seed=51 if draws == 10 else 53)
    Ad, keep = S.csr_to_device(A)
    k, p, tol = 8, 24, 1e-10
    v0 = inputs.start_vector(A.n, 52 if draws == 10 else 54)
    Ur, Sr, Vr, info_r = svds_ref.svds(as_operator(A), k, p, tol, 3000, v0=v0)
    Un, Sn, Vn, info_n, st_n = _gpu_solve(S, A, k, p, tol, 3000, v0=v0, flags=S.SVDS_FLAG_NO_PANELS)
    os.environ["SVDS_TEST_NO_ROOM"] = mode
    try:
        _, npan = S.svds_op_csr_matvec(Ad, True, torch.zeros(A.m, dtype=torch.float64, device="cuda"))
        Ug, Sg, Vg, info, st = _gpu_solve(S, A, k, p, tol, 3000, v0=v0)
    finally:
        del os.environ["SVDS_TEST_NO_ROOM"]
    assert npan == 1
    assert st == 0 and st_n == 0 and info["converged"] == 1
    assert np.array_equal(Sg, Sn) and np.array_equal(Ug, Un) and np.array_equal(Vg, Vn)
    np.testing.assert_allclose(Sg, Sr, rtol=1e-10)
    _invariants(A, Ug, Sg, Vg, tol)
    if mode == "arena":
        assert info["workspace_bytes"] == info_n["workspace_bytes"]


@pytest.mark.parametrize("law", ["decay1", "decay2", "decay3"])
def test_prescribed_spectrum(S, law):
    nb, bs = 400, 5
    sig = getattr(inputs, law)(nb * bs)
    A = inputs.prescribed_sparse(nb, bs, sig, seed=17)
    k, p = 12, 36
    Ug, Sg, Vg, info, st = _gpu_solve(S, A, k, p, 1e-10, 2000, v0=inputs.start_vector(A.n, 18))
    assert st == 0
    np.testing.assert_allclose(Sg, np.sort(sig)[::-1][:k], rtol=1e-10)
    _invariants(A, Ug, Sg, Vg, 1e-10)


def test_repeated_values_and_breakdowns(S):
    d = np.repeat([5.0, 4.0, 3.0, 2.0, 1.0, 0.5], [4, 3, 3, 2, 3, 35])
    A = inputs.diag_matrix(60, 50, d)
    k, p = 8, 20
    v0 = inputs.start_vector(50, 4)
    Ur, Sr, Vr, info_r = svds_ref.svds(as_operator(A), k, p, 1e-10, 200, v0=v0)
    Ug, Sg, Vg, info, st = _gpu_solve(S, A, k, p, 1e-10, 200, v0=v0)
    assert info["breakdowns"] > 0 and info_r.breakdowns > 0
    np.testing.assert_allclose(Sg, np.sort(d)[::-1][:k], rtol=1e-12)
    # multiple singular values: compare invariant subspaces
    for val in (5.0, 4.0):
        cols = np.nonzero(np.abs(Sg - val) < 1e-9)[0]
        colsr = np.nonzero(np.abs(Sr - val) < 1e-9)[0]
        qg, _ = np.linalg.qr(Vg[:, cols])
        qr, _ = np.linalg.qr(Vr[:, colsr])
        assert np.linalg.norm(qg - qr @ (qr.T @ qg), 2) < 1e-9
    _invariants(A, Ug, Sg, Vg, 1e-10)


def test_default_start_vector_matches_oracle_philox(S):
    A = inputs.sparse_uniform(400, 300, 4000, seed=21)
    k, p = 4, 14
    Ur, Sr, Vr, info_r = svds_ref.svds(as_operator(A), k, p, 1e-10, 500, seed=2405)
    Ug, Sg, Vg, info, st = _gpu_solve(S, A, k, p, 1e-10, 500, v0=None, seed=2405)
    np.testing.assert_allclose(Sg, Sr, rtol=1e-10)
    assert abs(info["cycles"] - info_r.cycles) <= 1


def test_not_converged_status(S):
    A = inputs.config_matrix(1)
    v0 = inputs.start_vector(A.n, inputs.CONFIG_SEEDS[1] + 1)
    Ug, Sg, Vg, info, st = _gpu_solve(S, A, 10, 30, 1e-10, 1, v0=v0)
    Ur, Sr, Vr, info_r = svds_ref.svds(as_operator(A), 10, 30, 1e-10, 1, v0=v0)
    assert st == 1 and info["converged"] == 0 and info["cycles"] == 1
    assert info["nconv"] == info_r.nconv
    # one cycle, same Krylov space: the Ritz values agree to rounding
    np.testing.assert_allclose(Sg, Sr, rtol=1e-12)
    assert info["n_spmv"] == 30 and info["n_spmvT"] == 30


@pytest.mark.parametrize("m,n,k,p", [(40, 31, 1, 2), (40, 31, 29, 30), (30, 50, 10, 30), (31, 32, 2, 31)])
def test_extreme_dimensions(S, m, n, k, p):
    """p = k+1, p = m, p + 1 = n, k = 1: the boundaries of the validation."""
    A = inputs.sparse_uniform(m, n, m * n // 3, seed=m * n)
    v0 = inputs.start_vector(n, 1)
    Ur, Sr, Vr, info_r = svds_ref.svds(as_operator(A), k, p, 1e-10, 3000, v0=v0)
    Ug, Sg, Vg, info, st = _gpu_solve(S, A, k, p, 1e-10, 3000, v0=v0)
    assert st == 0 and info_r.converged
    s_all = np.linalg.svd(as_operator(A).toarray(), compute_uv=False)
    np.testing.assert_allclose(Sg, s_all[:k], rtol=1e-10)
    _invariants(A, Ug, Sg, Vg, 1e-10)


def test_empty_rows_and_columns(S):
    A = inputs.sparse_uniform(500, 400, 800, seed=31)  # many empty rows and columns
    assert (np.diff(A.row_ptr) == 0).sum() > 50
    k, p = 5, 16
    v0 = inputs.start_vector(400, 32)
    Ug, Sg, Vg, info, st = _gpu_solve(S, A, k, p, 1e-10, 3000, v0=v0)
    s_all = np.linalg.svd(as_operator(A).toarray(), compute_uv=False)
    np.testing.assert_allclose(Sg, s_all[:k], rtol=1e-10)
    _invariants(A, Ug, Sg, Vg, 1e-10)


def test_zero_matrix(S):
    A = inputs.CSR(30, 20, np.zeros(31, np.int32), np.zeros(0, np.int32), np.zeros(0))
    Ug, Sg, Vg, info, st = _gpu_solve(S, A, 2, 5, 1e-10, 3, v0=inputs.start_vector(20, 1))
    assert np.all(Sg == 0) and st == 0 and info["breakdowns"] >= 1
    assert np.all(np.isfinite(Ug)) and np.all(np.isfinite(Vg))


def test_bitwise_deterministic(S):
    A = inputs.sparse_zipf(20000, 8000, 10, 1.1, seed=41)
    v0 = inputs.start_vector(A.n, 42)
    a = _gpu_solve(S, A, 6, 18, 1e-10, 300, v0=v0)
    b = _gpu_solve(S, A, 6, 18, 1e-10, 300, v0=v0)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)


def test_plan_reuse(S):
    import torch
    A = inputs.config_matrix(1)
    v0 = torch.from_numpy(inputs.start_vector(A.n, inputs.CONFIG_SEEDS[1] + 1)).cuda()
    Ad, keep = S.csr_to_device(A)
    plan = S.Plan(Ad, S.make_opts(10, 30, 1e-10, 3000, v0=v0))
    r1 = plan.execute()
    r2 = plan.execute()
    torch.cuda.synchronize()
    assert torch.equal(r1.S, r2.S) and torch.equal(r1.U, r2.U) and torch.equal(r1.V, r2.V)
    plan.destroy()


def test_fp32_stored_values_fp64_path(S):
    """FP32-stored CSR values widen exactly: the matrix of record is the
    widened one, and the FP64 path matches the oracle on it."""
    A = inputs.round_values_f32(inputs.sparse_uniform(1500, 900, 15000, seed=51))
    A64 = inputs.CSR(A.m, A.n, A.row_ptr, A.col_idx, A.val.astype(np.float64))
    v0 = inputs.start_vector(A.n, 52)
    Ur, Sr, Vr, _ = svds_ref.svds(as_operator(A64), 6, 18, 1e-10, 2000, v0=v0)
    Ug, Sg, Vg, info, st = _gpu_solve(S, A, 6, 18, 1e-10, 2000, v0=v0)
    np.testing.assert_allclose(Sg, Sr, rtol=1e-10)


def test_dense_fp64_matches_oracle(S):
    import torch
    sig = inputs.decay1(300)
    A = inputs.prescribed_dense(500, 300, sig, seed=61)
    v0 = inputs.start_vector(300, 62)
    k, p = 20, 60
    Ur, Sr, Vr, info_r = svds_ref.svds(A, k, p, 1e-10, 500, v0=v0)
    Ad = S.make_dense(torch.from_numpy(A.ravel(order="F")).cuda(), 500, 300)
    r = S.svds_dense_solve(Ad, S.make_opts(k, p, 1e-10, 500, v0=torch.from_numpy(v0).cuda()))
    np.testing.assert_allclose(r.S.cpu().numpy(), sig[:k], rtol=1e-10)
    np.testing.assert_allclose(r.S.cpu().numpy(), Sr, rtol=1e-10)
    assert r.status == 0


def test_full_size_zipf_workload_against_stored_oracle(S):
    """The 1,000,000 x 500,000 Zipf workload (k=50, p=150, tol=1e-8) in the
    configuration the benchmark times: singular values against the stored
    oracle values, outputs orthonormal, and residuals recomputed with torch's
    own sparse product (independent of the library's kernels)."""
    import os
    import torch
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "workload2_sigma.txt")
    gold = np.array([float(x) for x in open(path) if x.strip() and not x.startswith("#")])
    A = inputs.config_matrix(2)
    v0 = inputs.start_vector(A.n, inputs.CONFIG_SEEDS[2] + 1)
    Ad, keep = S.csr_to_device(A)
    r = S.svds_csr_solve(Ad, S.make_opts(50, 150, 1e-8, 2000, v0=torch.from_numpy(v0).cuda()))
    torch.cuda.synchronize()
    assert r.status == 0 and r.info["converged"] == 1
    np.testing.assert_allclose(r.S.cpu().numpy(), gold[:50], rtol=1e-10)
    eye = torch.eye(50, dtype=torch.float64, device="cuda")
    assert float((r.U.T @ r.U - eye).abs().max()) <= 1e-12
    assert float((r.V.T @ r.V - eye).abs().max()) <= 1e-12
    At = torch.sparse_csr_tensor(torch.from_numpy(A.row_ptr.astype(np.int64)), torch.from_numpy(A.col_idx.astype(np.int64)),
                                 torch.from_numpy(A.val), size=(A.m, A.n)).cuda()
    AV = At @ r.V.contiguous()
    res_av = torch.linalg.norm(AV - r.U * r.S, dim=0) / r.S[0]
    assert float(res_av.max()) <= 1e-8
    assert abs(r.info["max_res_av"] - float(res_av.max())) <= 1e-12


@pytest.mark.parametrize("form", ["plain", "wide", "graph_wide", "mixed_auto"])
def test_breakdowns_at_scale(S, form):
    """A 1,000,000 x 500,000 matrix of rank 30 (diagonal, distinct values):
    the Krylov space is exhausted after 31 steps, so the rest of the cycle
    runs on breakdown replacement vectors, each re-orthogonalized against the
    whole basis in the finish step.  plain: one workgroup per repair; wide:
    SVDS_FLAG_EXPECT_BREAKDOWNS, up to 128 workgroups of a cooperative launch;
    graph_wide: the same with captured cycles (the first cycle runs before
    any capture); mixed_auto: no flag, an FP32 cycle with one-workgroup
    repairs, then an FP64 cycle with wide ones (switched on by the FP32
    cycle's breakdowns).  Values against the exact ones and the oracle's; the
    replacement vectors are the oracle's (same Philox streams), so the FP64
    solves also match its breakdown count."""
    import time
    import torch
    print(f"breakdowns at 1e6 rows, {form}", flush=True)
    d = np.zeros(500000)
    d[:30] = np.arange(30, 0, -1, dtype=np.float64)
    A = inputs.diag_matrix(1_000_000, 500_000, d)
    k, p = 5, 40
    v0 = inputs.start_vector(500_000, 31)
    Ur, Sr, Vr, info_r = svds_ref.svds(as_operator(A), k, p, 1e-10, 50, v0=v0)
    precision = S.SVDS_PREC_MIXED if form == "mixed_auto" else 0
    flags = {"plain": 0, "wide": S.SVDS_FLAG_EXPECT_BREAKDOWNS, "mixed_auto": 0,
             "graph_wide": S.SVDS_FLAG_EXPECT_BREAKDOWNS | S.SVDS_FLAG_GRAPH}[form]
    t0 = time.perf_counter()
    Ug, Sg, Vg, info, st = _gpu_solve(S, A, k, p, 1e-10, 50, v0=v0, precision=precision, flags=flags)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert st == 0 and info["breakdowns"] > 0 and info_r.breakdowns > 0
    if form == "mixed_auto":
        assert info["cycles_fp32"] >= 1 and info["cycles_fp64"] >= 1
    else:
        assert info["breakdowns"] == info_r.breakdowns
    np.testing.assert_allclose(Sg, [30, 29, 28, 27, 26], rtol=1e-12)
    np.testing.assert_allclose(Sg, Sr, rtol=1e-12)
    _invariants(A, Ug, Sg, Vg, 1e-10)
    print(f"breakdowns gpu {info['breakdowns']} oracle {info_r.breakdowns}, {dt * 1e3:.1f} ms", flush=True)


def test_wide_repair_few_workgroups(S):
    """SVDS_FLAG_EXPECT_BREAKDOWNS on a 100,003 x 50,001 matrix of rank 30:
    the u-side repairs run over two to three workgroups (100,003 rows do not
    divide evenly), the v-side ones below the size limit in one workgroup.
    Same values, breakdown count and invariants as the oracle."""
    d = np.zeros(50_001)
    d[:30] = np.linspace(3.0, 1.0, 30)
    A = inputs.diag_matrix(100_003, 50_001, d)
    k, p = 5, 40
    v0 = inputs.start_vector(50_001, 33)
    Ur, Sr, Vr, info_r = svds_ref.svds(as_operator(A), k, p, 1e-10, 50, v0=v0)
    Ug, Sg, Vg, info, st = _gpu_solve(S, A, k, p, 1e-10, 50, v0=v0, flags=S.SVDS_FLAG_EXPECT_BREAKDOWNS)
    assert st == 0 and info["breakdowns"] == info_r.breakdowns > 0
    np.testing.assert_allclose(Sg, np.sort(d)[::-1][:k], rtol=1e-12)
    np.testing.assert_allclose(Sg, Sr, rtol=1e-12)
    _invariants(A, Ug, Sg, Vg, 1e-10)


@pytest.mark.parametrize("p", [40, 70])
def test_rank_deficient_small_svd_stays_finite(S, p):
    """Rank 30 with p = 40 (one-workgroup Jacobi) and p = 70 (block Jacobi):
    T holds exact zeros from the breakdowns, so Jacobi meets pairs whose
    columns have converged to (sub)normal nothing; such pairs must not be
    rotated (a subnormal inner product made the reciprocal infinite and the
    whole SVD NaN).  Values exact, as the oracle's."""
    d = np.zeros(1000)
    d[:30] = np.arange(30, 0, -1, dtype=np.float64)
    A = inputs.diag_matrix(2000, 1000, d)
    v0 = inputs.start_vector(1000, 32)
    Ur, Sr, Vr, info_r = svds_ref.svds(as_operator(A), 5, p, 1e-10, 50, v0=v0)
    Ug, Sg, Vg, info, st = _gpu_solve(S, A, 5, p, 1e-10, 50, v0=v0)
    assert st == 0 and info["breakdowns"] > 0
    assert np.all(np.isfinite(Ug)) and np.all(np.isfinite(Vg))
    np.testing.assert_allclose(Sg, [30, 29, 28, 27, 26], rtol=1e-12)
    np.testing.assert_allclose(Sg, Sr, rtol=1e-12)
