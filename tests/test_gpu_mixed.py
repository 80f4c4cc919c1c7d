"""Mixed-precision path: FP32 Lanczos cycles (FP32 bases, mat-vecs and CGS2),
then FP64 cycles started from the FP32 Ritz vectors, against the FP64 CPU
oracle on the matrix of record (the stored FP32/BF16 matrix widened exactly).

The paper has no mixed-precision form, so this path is pinned only by the
FP64 oracle: singular values to 1e-8 relative, explicit FP64 residuals to
tol, orthonormal outputs."""
import os

import numpy as np
import pytest

from paper_2405_18966_amd import inputs
from oracle import svds_ref
from oracle.svds_ref import as_operator

pytestmark = pytest.mark.gpu
MIXED = 1
GOLDEN_W3 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "workload3_sigma_bf16.txt")


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_18966_amd import svds
    return svds


def _csr_solve(S, A, k, p, tol, v0, precision):
    import torch
    Ad, keep = S.csr_to_device(A)
    r = S.svds_csr_solve(Ad, S.make_opts(k, p, tol, 2000, precision=precision,
                                         v0=torch.from_numpy(v0).cuda()))
    torch.cuda.synchronize()
    return r.U.cpu().numpy(), r.S.cpu().numpy(), r.V.cpu().numpy(), r.info, r.status


def _dense_solve(S, stored, k, p, tol, v0, precision):
    import torch
    a = stored.a
    if a.dtype == np.uint16:
        t = torch.from_numpy(a.ravel(order="F").view(np.int16)).view(torch.uint16).cuda()
    else:
        t = torch.from_numpy(a.ravel(order="F")).cuda()
    Ad = S.make_dense(t, stored.m, stored.n)
    r = S.svds_dense_solve(Ad, S.make_opts(k, p, tol, 2000, precision=precision,
                                           v0=torch.from_numpy(v0).cuda()))
    torch.cuda.synchronize()
    return r.U.cpu().numpy(), r.S.cpu().numpy(), r.V.cpu().numpy(), r.info, r.status


def _check_outputs(A_record, Ug, Sg, Vg, tol):
    k = len(Sg)
    assert np.abs(Ug.T @ Ug - np.eye(k)).max() <= 1e-12
    assert np.abs(Vg.T @ Vg - np.eye(k)).max() <= 1e-12
    r1, r2 = svds_ref.explicit_residuals(A_record, Ug, Sg, Vg)
    assert (r2 / Sg).max() <= 2 * tol
    assert r1.max() <= 2 * tol * Sg[0]


def test_mixed_sparse_fp32_values(S):
    """Workload 4: the 2000 x 1000 sparse matrix with FP32 values, k=50,
    p=150, tol=1e-8; its spectrum is clustered (sigma_51/sigma_50 ~ 0.9992)."""
    A = inputs.config_matrix(4)
    A64 = inputs.CSR(A.m, A.n, A.row_ptr, A.col_idx, A.val.astype(np.float64))
    v0 = inputs.start_vector(A.n, inputs.CONFIG_SEEDS[4] + 1)
    k, p, tol = 50, 150, 1e-8
    Ur, Sr, Vr, info_r = svds_ref.svds(as_operator(A64), k, p, tol, 2000, v0=v0)
    Ug, Sg, Vg, info, st = _csr_solve(S, A, k, p, tol, v0, MIXED)
    assert st == 0 and info["converged"] == 1
    assert info["cycles_fp32"] >= 1 and info["cycles_fp64"] >= 1
    np.testing.assert_allclose(Sg, Sr, rtol=1e-8)
    _check_outputs(as_operator(A64), Ug, Sg, Vg, tol)


def test_mixed_and_fp64_paths_agree_on_workload1(S):
    A = inputs.config_matrix(1)
    v0 = inputs.start_vector(A.n, inputs.CONFIG_SEEDS[1] + 1)
    k, p, tol = 10, 30, 1e-10
    Ur, Sr, Vr, _ = svds_ref.svds(as_operator(A), k, p, tol, 2000, v0=v0)
    Um, Sm, Vm, info_m, st_m = _csr_solve(S, A, k, p, tol, v0, MIXED)
    Ud, Sd, Vd, info_d, st_d = _csr_solve(S, A, k, p, tol, v0, 0)
    assert st_m == 0 and st_d == 0
    np.testing.assert_allclose(Sd, Sr, rtol=1e-10)
    np.testing.assert_allclose(Sm, Sr, rtol=1e-8)
    _check_outputs(as_operator(A), Um, Sm, Vm, tol)


@pytest.mark.parametrize("storage", ["bf16", "f32"])
def test_mixed_dense_low_precision_storage(S, storage):
    """Dense G1 diag(0.95^i) G2^T + noise, stored BF16 or FP32; the matrix of
    record is the stored copy widened exactly (rounding to BF16 moves the
    singular values far more than 1e-8, so the widened copy is what is solved)."""
    d = inputs.dense_lowrank(3000, 1500, 80, 0.95, 1e-3, 31)
    rec = d["record_" + storage]
    v0 = inputs.start_vector(1500, 32)
    k, p, tol = 30, 90, 1e-8
    Ur, Sr, Vr, _ = svds_ref.svds(rec, k, p, tol, 2000, v0=v0)
    Ug, Sg, Vg, info, st = _dense_solve(S, d[storage], k, p, tol, v0, MIXED)
    assert st == 0 and info["converged"] == 1
    np.testing.assert_allclose(Sg, Sr, rtol=1e-8)
    _check_outputs(rec, Ug, Sg, Vg, tol)
    # and the FP64 path on the same stored matrix
    Ud, Sd, Vd, info_d, st_d = _dense_solve(S, d[storage], k, p, tol, v0, 0)
    np.testing.assert_allclose(Sd, Sr, rtol=1e-10)


def _golden(path):
    return np.array([float(x) for x in open(path) if x.strip() and not x.startswith("#")])


def _full_size_w3(S, precision, rtol):
    """Workload 3 at full size: 20000 x 10000 dense BF16, k=100, p=250,
    tol=1e-8; singular values against the stored FP64 oracle values of the
    widened BF16 matrix, outputs orthonormal, and residuals checked on the
    device in FP64 by an independent torch computation."""
    import torch
    print(f"workload 3 full size, precision {precision}", flush=True)
    d = inputs.config_matrix(3)
    v0 = inputs.start_vector(10000, inputs.CONFIG_SEEDS[3] + 1)
    gold = _golden(GOLDEN_W3)
    Ug, Sg, Vg, info, st = _dense_solve(S, d["bf16"], 100, 250, 1e-8, v0, precision)
    assert st == 0 and info["converged"] == 1
    np.testing.assert_allclose(Sg, gold[:100], rtol=rtol)
    k = 100
    assert np.abs(Ug.T @ Ug - np.eye(k)).max() <= 1e-12
    assert np.abs(Vg.T @ Vg - np.eye(k)).max() <= 1e-12
    A = torch.from_numpy(d["record_bf16"]).cuda()
    U = torch.from_numpy(Ug).cuda()
    V = torch.from_numpy(Vg).cuda()
    s = torch.from_numpy(Sg).cuda()
    r2 = torch.linalg.norm(A.T @ U - V * s, dim=0) / s
    assert float(r2.max()) <= 2e-8
    # the library's FP64 residuals (block products over the stored BF16
    # matrix) agree with the independent ones; both are at rounding level
    # here, so the agreement is absolute
    assert abs(info["max_res_true"] - float(r2.max())) <= 1e-12
    r1 = torch.linalg.norm(A @ V - U * s, dim=0) / s[0]
    assert abs(info["max_res_av"] - float(r1.max())) <= 1e-12
    assert info["max_res_true"] <= 2e-8 and info["max_res_av"] <= 2e-8
    # the residuals read the stored BF16 matrix: no widened m x n FP64 copy
    # is part of the plan
    assert info["workspace_bytes"] < 8 * 20000 * 10000
    return info


@pytest.mark.skipif(not os.path.exists(GOLDEN_W3), reason="stored oracle values not generated")
def test_mixed_dense_bf16_full_size_against_stored_oracle(S):
    _full_size_w3(S, MIXED, 1e-8)


@pytest.mark.skipif(not os.path.exists(GOLDEN_W3), reason="stored oracle values not generated")
def test_fp64_dense_bf16_full_size_against_stored_oracle(S):
    """The plain FP64 path on the same stored matrix, to the FP64 bound."""
    _full_size_w3(S, 0, 1e-10)


def test_mixed_fp64_values_every_product_layout(S):
    """FP64-stored values read in FP32 by the FP32 cycles: the plan's FP32
    copies of A, A^T, the column-sorted copies and the column-panel copy.
    300000 x 150000 Zipf(1.1), 10 draws per row: long rows (pieces) in A^T
    and two column panels; each layout switch selects a different set of
    copies, and the tuner may turn the sorted copies off."""
    import torch
    print("mixed fp64 values, layouts", flush=True)
    A = inputs.sparse_zipf(300000, 150000, 10, 1.1, seed=331)
    v0 = inputs.start_vector(A.n, 332)
    Ur, Sr, Vr, _ = svds_ref.svds(as_operator(A), 6, 18, 1e-10, 2000, v0=v0)
    Ad, keep = S.csr_to_device(A)
    F = S
    ws = {}
    for name, fl in (("default", 0), ("unsorted", F.SVDS_FLAG_UNSORTED), ("nopanels", F.SVDS_FLAG_NO_PANELS),
                     ("plain", F.SVDS_FLAG_UNSORTED | F.SVDS_FLAG_NO_PANELS), ("autotune", F.SVDS_FLAG_AUTOTUNE)):
        print(f"layout {name}", flush=True)
        r = S.svds_csr_solve(Ad, S.make_opts(6, 18, 1e-10, 2000, precision=MIXED, v0=torch.from_numpy(v0).cuda(),
                                             flags=fl))
        torch.cuda.synchronize()
        assert r.status == 0, name
        assert r.info["cycles_fp32"] >= 1 and r.info["cycles_fp64"] >= 1, name
        np.testing.assert_allclose(r.S.cpu().numpy(), Sr, rtol=1e-10, err_msg=name)
        assert r.info["max_res_true"] <= 2e-10, name
        ws[name] = r.info["workspace_bytes"]
    # four FP32 copies of the values (A, A^T and their sorted copies) plus the
    # panel copy with panels, two without any sorted copy or panels
    per = (A.nnz * 4 + 255) // 256 * 256
    r64 = S.svds_csr_solve(Ad, S.make_opts(6, 18, 1e-10, 2000, v0=torch.from_numpy(v0).cuda(),
                                           flags=F.SVDS_FLAG_UNSORTED | F.SVDS_FLAG_NO_PANELS))
    torch.cuda.synchronize()
    assert ws["plain"] - r64.info["workspace_bytes"] >= 2 * per
    assert ws["default"] > ws["plain"]
