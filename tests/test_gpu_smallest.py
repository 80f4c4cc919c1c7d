"""The k smallest singular triplets (SVDS_FLAG_SMALLEST): Ritz augmentation
with the k smallest Ritz triplets, against the FP64 oracle run in the same
mode and against LAPACK's full SVD."""
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


def _spectrum(N, nsmall):
    """nsmall small values in [0.01, 0.1], well apart from the rest in [1, 2]."""
    return np.concatenate([np.linspace(0.01, 0.1, nsmall), np.linspace(1.0, 2.0, N - nsmall)])


@pytest.mark.parametrize("k,p", [(4, 20), (10, 72)])
def test_smallest_sparse_matches_oracle_and_lapack(S, k, p):
    import torch
    print(f"smallest sparse k={k} p={p}", flush=True)
    sig = _spectrum(3000, 12)
    A = inputs.prescribed_sparse(600, 5, sig, seed=401)
    v0 = inputs.start_vector(A.n, 402)
    Ur, Sr, Vr, info_r = svds_ref.svds(as_operator(A), k, p, 1e-10, 3000, v0=v0, which="smallest")
    assert info_r.converged
    Ad, keep = S.csr_to_device(A)
    r = S.svds_csr_solve(Ad, S.make_opts(k, p, 1e-10, 3000, v0=torch.from_numpy(v0).cuda(),
                                         flags=S.SVDS_FLAG_SMALLEST))
    torch.cuda.synchronize()
    assert r.status == 0 and r.info["nconv"] == k
    s = r.S.cpu().numpy()
    exact = np.sort(sig)[:k]
    np.testing.assert_allclose(s, exact, rtol=1e-10)
    np.testing.assert_allclose(s, Sr, rtol=1e-10)
    assert np.all(np.diff(s) > 0)  # ascending
    U, V = r.U.cpu().numpy(), r.V.cpu().numpy()
    # vectors: distinct, well separated values -> sign-normalized vectors agree
    for X, Y in ((U, Ur), (V, Vr)):
        assert np.abs(X - Y).max() <= 1e-8
    r1, r2 = svds_ref.explicit_residuals(as_operator(A), U, s, V)
    assert r1.max() <= 1e-12 * sig.max() and (r2 / s).max() <= 2e-10
    assert r.info["max_res_true"] <= 2e-10
    assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-12 and np.abs(V.T @ V - np.eye(k)).max() <= 1e-12
    assert r.info["cycles"] == info_r.cycles or abs(r.info["cycles"] - info_r.cycles) <= 1


def test_smallest_dense(S):
    import torch
    print("smallest dense", flush=True)
    sig = _spectrum(300, 8)
    A = inputs.prescribed_dense(500, 300, sig, seed=411)
    v0 = inputs.start_vector(300, 412)
    Ad = S.make_dense(torch.from_numpy(A.ravel(order="F")).cuda(), 500, 300)
    r = S.svds_dense_solve(Ad, S.make_opts(5, 24, 1e-10, 3000, v0=torch.from_numpy(v0).cuda(),
                                           flags=S.SVDS_FLAG_SMALLEST))
    torch.cuda.synchronize()
    assert r.status == 0
    np.testing.assert_allclose(r.S.cpu().numpy(), np.sort(sig)[:5], rtol=1e-10)
    Ur, Sr, Vr, _ = svds_ref.svds(A, 5, 24, 1e-10, 3000, v0=v0, which="smallest")
    np.testing.assert_allclose(r.S.cpu().numpy(), Sr, rtol=1e-10)
