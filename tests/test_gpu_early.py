"""Early stop inside a cycle (SVDS_FLAG_EARLY_STOP): the eq. (4) test of
Proposition 1 on the leading block T(1:j,1:j) while the cycle goes on.  The
GPU solve against the CPU oracle (which always runs whole cycles), with the
explicit FP64 residuals within tol, fewer products than whole cycles where
the test passes early, and the combinations with the other options."""
import os

import numpy as np
import pytest

from paper_2405_18966_amd import inputs
from oracle import svds_ref
from oracle.svds_ref import as_operator

pytestmark = pytest.mark.gpu

GOLDEN_W2 = os.path.join(os.path.dirname(__file__), "golden", "workload2_sigma.txt")


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_18966_amd import svds
    return svds


def _solve(S, A, k, p, tol, v0, flags, precision=0):
    import torch
    Ad, keep = S.csr_to_device(A)
    r = S.svds_csr_solve(Ad, S.make_opts(k, p, tol, 3000, precision=precision, v0=torch.from_numpy(v0).cuda(),
                                         flags=flags))
    torch.cuda.synchronize()
    return r


@pytest.mark.parametrize("name,k,p,tol,prec", [("w1", 10, 30, 1e-10, 0), ("w4", 50, 150, 1e-8, 0),
                                                ("w4", 50, 150, 1e-8, 1), ("zipf", 8, 24, 1e-10, 0),
                                                ("uniform", 20, 120, 1e-10, 0)])
def test_early_stop_matches_oracle(S, name, k, p, tol, prec):
    print(f"early {name} k={k} p={p} precision {prec}", flush=True)
    if name == "w1":
        A = inputs.config_matrix(1)
    elif name == "w4":
        A = inputs.config_matrix(4)
    elif name == "zipf":
        A = inputs.sparse_zipf(200000, 100000, 10, 1.1, seed=701)
    else:
        A = inputs.sparse_uniform(20000, 12000, 400000, seed=702)
    A64 = inputs.CSR(A.m, A.n, A.row_ptr, A.col_idx, A.val.astype(np.float64))
    v0 = inputs.start_vector(A.n, 703)
    Ur, Sr, Vr, info_r = svds_ref.svds(as_operator(A64), k, p, tol, 3000, v0=v0)
    full = _solve(S, A, k, p, tol, v0, 0, prec)
    r = _solve(S, A, k, p, tol, v0, S.SVDS_FLAG_EARLY_STOP, prec)
    assert r.status == 0 and r.info["converged"] == 1
    s = r.S.cpu().numpy()
    np.testing.assert_allclose(s, Sr, rtol=1e-10 if prec == 0 else 1e-8)
    U, V = r.U.cpu().numpy(), r.V.cpu().numpy()
    assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-12 and np.abs(V.T @ V - np.eye(k)).max() <= 1e-12
    r1, r2 = svds_ref.explicit_residuals(as_operator(A64), U, s, V)
    assert r1.max() <= 1e-12 * s[0] and (r2 / s).max() <= 2 * tol
    assert r.info["early_checks"] > 0
    assert k < r.info["lanczos_dim_last"] <= p
    products = r.info["n_spmv"] + r.info["n_spmvT"]
    full_products = full.info["n_spmv"] + full.info["n_spmvT"]
    assert products <= full_products
    print(name, "stopped at j =", r.info["lanczos_dim_last"], "of", p, "after", r.info["early_checks"], "checks;",
          "products", products, "vs", full_products, "; cycles", r.info["cycles"], "vs", full.info["cycles"],
          flush=True)


def test_early_stop_with_partial_and_smallest(S):
    A = inputs.sparse_uniform(4000, 3000, 60000, seed=704)
    v0 = inputs.start_vector(A.n, 705)
    exact = np.linalg.svd(as_operator(A).toarray(), compute_uv=False)
    r = _solve(S, A, 10, 40, 1e-10, v0, S.SVDS_FLAG_EARLY_STOP | S.SVDS_FLAG_PARTIAL_REORTH)
    assert r.status == 0
    np.testing.assert_allclose(r.S.cpu().numpy(), exact[:10], rtol=1e-10)
    sig = np.concatenate([[0.01, 0.02, 0.035, 0.05, 0.08], np.linspace(1.0, 2.0, 595)])
    B = inputs.prescribed_sparse(120, 5, sig, seed=21)
    rs = _solve(S, B, 4, 20, 1e-10, inputs.start_vector(600, 23), S.SVDS_FLAG_EARLY_STOP | S.SVDS_FLAG_SMALLEST)
    assert rs.status == 0
    np.testing.assert_allclose(rs.S.cpu().numpy(), np.sort(sig)[:4], rtol=1e-10)


def test_early_stop_ignored_with_graph(S):
    A = inputs.sparse_uniform(3000, 2000, 60000, seed=706)
    v0 = inputs.start_vector(A.n, 707)
    r = _solve(S, A, 10, 30, 1e-10, v0, S.SVDS_FLAG_EARLY_STOP | S.SVDS_FLAG_GRAPH)
    assert r.info["early_checks"] == 0 and r.info["lanczos_dim_last"] == 30


@pytest.mark.skipif(not os.path.exists(GOLDEN_W2), reason="stored oracle values not generated")
def test_early_stop_full_size_zipf(S):
    """1,000,000 x 500,000 Zipf, k=50, p=150, tol=1e-8: the stored FP64 oracle
    values (whole cycles) at 1e-10, the explicit residuals within tol."""
    print("early full-size zipf", flush=True)
    A = inputs.config_matrix(2)
    gold = np.array([float(x) for x in open(GOLDEN_W2) if x.strip() and not x.startswith("#")])
    v0 = inputs.start_vector(A.n, inputs.CONFIG_SEEDS[2] + 1)
    r = _solve(S, A, 50, 150, 1e-8, v0, S.SVDS_FLAG_EARLY_STOP)
    assert r.status == 0 and r.info["max_res_true"] <= 2e-8
    np.testing.assert_allclose(r.S.cpu().numpy(), gold[:50], rtol=1e-10)
    assert r.info["lanczos_dim_last"] < 150
    print("full size: stopped at j =", r.info["lanczos_dim_last"], "after", r.info["early_checks"], "checks,",
          r.info["ms_total"], "ms", flush=True)
