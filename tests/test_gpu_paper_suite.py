"""The paper's synthetic suite (Sec. 3.1) at the paper's shape: Sparse1-3
(40,000 x 40,000, 5 nonzeros per row) and Dense1-3 (10,000 x 10,000), with
Decay1/2/3 spectra, solved as in Sec. 3 (k = 100, t = 300, tol = 1e-10, at
most 10 cycles).  The singular values are known in closed form, so the GPU
result is checked against them directly, and against the a-posteriori bound
|s_j - sigma_j| <= max(|A v_j - s_j u_j|, |A^T u_j - s_j v_j|)."""
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


@pytest.mark.parametrize("name,n", [("sparse1", None), ("sparse2", None), ("sparse3", None),
                                    ("dense1", None), ("dense2", None), ("dense3", None), ("dense2", 3000)])
def test_paper_suite_exact_spectrum(S, name, n):
    import torch
    print(f"paper suite {name} n={n}", flush=True)
    A, sig = inputs.paper_suite(name, n)
    N = len(sig)
    cfg = inputs.PAPER_SUITE_SOLVE
    k = cfg["k"]
    v0 = torch.from_numpy(inputs.start_vector(N, inputs.PAPER_SUITE_SEEDS[name] + 1)).cuda()
    opts = S.make_opts(k, cfg["p"], cfg["tol"], cfg["maxit"], v0=v0)
    if name.startswith("sparse"):
        Ad, keep = S.csr_to_device(A)
        r = S.svds_csr_solve(Ad, opts)
        op = as_operator(A)
    else:
        Ad = S.make_dense(torch.from_numpy(A.ravel(order="F")).cuda(), N, N)
        r = S.svds_dense_solve(Ad, opts)
        op = A
    torch.cuda.synchronize()
    assert r.status == 0 and r.info["nconv"] == k
    s = r.S.cpu().numpy()
    U, V = r.U.cpu().numpy(), r.V.cpu().numpy()
    np.testing.assert_allclose(s, sig[:k], rtol=1e-10)
    r1, r2 = svds_ref.explicit_residuals(op, U, s, V)
    assert np.all(np.abs(s - sig[:k]) <= np.maximum(r1, r2) + 4e-16 * sig[0])
    assert r1.max() <= 1e-12 * sig[0]
    # the library's own FP64 residuals (block products on the device) agree
    # with the CPU ones; both sit at rounding level, so the agreement is absolute
    assert abs(r.info["max_res_av"] - r1.max() / s.max()) <= 1e-13
    assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-12
    assert np.abs(V.T @ V - np.eye(k)).max() <= 1e-12
