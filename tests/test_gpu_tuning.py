"""Launch shapes of the products and of CGS2: every fixed shape the plan-time
tuner chooses from (SVDS_FLAG_ITEMS_1K, SVDS_FLAG_UNSORTED,
SVDS_FLAG_NO_PANELS) against the FP64 oracle, and the tuner itself
(SVDS_FLAG_AUTOTUNE) on single, dense and batched solves."""
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


@pytest.fixture(scope="module")
def zipf():
    """300000 x 150000, 10 Zipf(1.1) column draws per row: A^T has rows of
    every length (pieces, 1024 < len <= 2048, short rows) and u is large
    enough for two column panels."""
    A = inputs.sparse_zipf(300000, 150000, 10, 1.1, seed=301)
    v0 = inputs.start_vector(A.n, 302)
    Ur, Sr, Vr, info = svds_ref.svds(as_operator(A), 6, 18, 1e-10, 2000, v0=v0)
    return A, v0, Sr


def _solve(S, A, v0, flags, k=6, p=18):
    import torch
    Ad, keep = S.csr_to_device(A)
    r = S.svds_csr_solve(Ad, S.make_opts(k, p, 1e-10, 2000, v0=torch.from_numpy(v0).cuda(), flags=flags))
    torch.cuda.synchronize()
    return r


def test_fixed_shapes_match_oracle(S, zipf):
    import torch
    A, v0, Sr = zipf
    F = S
    runs = {}
    for name, fl in (("default", 0), ("items1k", F.SVDS_FLAG_ITEMS_1K), ("unsorted", F.SVDS_FLAG_UNSORTED),
                     ("nopanels", F.SVDS_FLAG_NO_PANELS),
                     ("all", F.SVDS_FLAG_ITEMS_1K | F.SVDS_FLAG_UNSORTED | F.SVDS_FLAG_NO_PANELS)):
        print(f"shape {name}", flush=True)
        r = _solve(S, A, v0, fl)
        assert r.status == 0, name
        np.testing.assert_allclose(r.S.cpu().numpy(), Sr, rtol=1e-10, err_msg=name)
        assert r.info["max_res_true"] <= 2e-10, name
        runs[name] = r
    # the column-sorted layout puts every product back in row order: the
    # solve is bit-identical with and without it
    assert torch.equal(runs["default"].S, runs["unsorted"].S)
    assert torch.equal(runs["default"].U, runs["unsorted"].U)
    # the default plan really had panels to switch off: its workspace holds the
    # panel copy in place of a column-sorted copy of A^T
    assert runs["default"].info["workspace_bytes"] != runs["nopanels"].info["workspace_bytes"]


def test_autotune_single(S, zipf):
    A, v0, Sr = zipf
    print("autotune single", flush=True)
    r = _solve(S, A, v0, S.SVDS_FLAG_AUTOTUNE)
    t = r.info["tuning"]
    assert t["tuned"] == 1
    assert t["fwd_nnz_cap"] in (1024, 2048) and t["bwd_nnz_cap"] in (1024, 2048)
    assert t["fwd_sorted"] in (0, 1) and t["bwd_sorted"] in (0, 1)
    assert t["bwd_panels"] in (1, 2)
    assert t["cgs_slab_shift"] in (-1, 0, 1) and t["cgs_cpw"] in (0, 8, 10)
    # the built-in shape is one of the timed candidates
    for a, b in (("fwd_us", "fwd_default_us"), ("bwd_us", "bwd_default_us"), ("cgs_us", "cgs_default_us")):
        assert 0 < t[a] <= t[b], (a, t)
    assert t["ms_tune"] > 0
    np.testing.assert_allclose(r.S.cpu().numpy(), Sr, rtol=1e-10)
    assert r.info["max_res_true"] <= 2e-10
    plain = _solve(S, A, v0, 0)
    assert plain.info["tuning"]["tuned"] == 0


def test_autotune_dense(S):
    import torch
    print("autotune dense", flush=True)
    sig = inputs.decay1(300)
    A = inputs.prescribed_dense(2000, 300, sig, seed=311)
    v0 = torch.from_numpy(inputs.start_vector(300, 312)).cuda()
    Ad = S.make_dense(torch.from_numpy(A.ravel(order="F")).cuda(), 2000, 300)
    r = S.svds_dense_solve(Ad, S.make_opts(20, 120, 1e-10, 500, v0=v0, flags=S.SVDS_FLAG_AUTOTUNE))
    torch.cuda.synchronize()
    t = r.info["tuning"]
    assert t["tuned"] == 1 and 0 < t["cgs_us"] <= t["cgs_default_us"]
    assert t["cgs_slab_shift"] in (-1, 0, 1) and t["cgs_cpw"] in (0, 8, 10)
    np.testing.assert_allclose(r.S.cpu().numpy(), sig[:20], rtol=1e-10)


def test_autotune_batched(S):
    import torch
    print("autotune batched", flush=True)
    rng = np.random.default_rng(321)
    As = []
    for _ in range(6):
        m = int(rng.integers(500, 4000))
        n = int(rng.integers(m // 2 + 20, m + 1))
        As.append(inputs.sparse_uniform(m, n, int(0.01 * m * n), int(rng.integers(2**62))))
    dev = [S.csr_to_device(A) for A in As]
    out = []
    for fl in (0, S.SVDS_FLAG_AUTOTUNE):
        r, rc = S.svds_csr_solve_batched([d[0] for d in dev], S.make_opts(5, 15, 1e-10, 2000, seed=9, flags=fl))
        torch.cuda.synchronize()
        assert rc == 0
        out.append(r)
    t = out[1][0].info["tuning"]
    assert t["tuned"] == 1 and t["bwd_panels"] == 1 and t["cgs_us"] == 0  # no CGS tuning for the batch
    assert 0 < t["fwd_us"] <= t["fwd_default_us"]
    for b, A in enumerate(As):
        Ur, Sr, Vr, _ = svds_ref.svds(as_operator(A), 5, 15, 1e-10, 2000, seed=9 + b)
        np.testing.assert_allclose(out[1][b].S.cpu().numpy(), Sr, rtol=1e-10)
        np.testing.assert_allclose(out[1][b].S.cpu().numpy(), out[0][b].S.cpu().numpy(), rtol=1e-11)
