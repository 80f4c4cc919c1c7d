"""Host runtime of the library around the kernels: the process-wide caches of
timing events and pinned read-back buffers, shared by every plan.  Plans made
one after another and plans made at once from several host threads must give
the same bits as a lone plan (every kernel is deterministic)."""
import threading

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


def _solve(S, Ad, n, k, p, seed, flags=0, stream=None):
    import torch
    v0 = torch.from_numpy(inputs.start_vector(n, seed)).cuda()
    r = S.svds_csr_solve(Ad, S.make_opts(k, p, 1e-10, 2000, v0=v0, flags=flags, stream=stream))
    if stream is not None:
        stream.synchronize()
    torch.cuda.synchronize()
    return r


def test_timed_plans_in_sequence(S):
    """Each timed plan takes its events from the cache the previous plans
    returned them to: every solve still samples launches and times them,
    and the timing does not change the results."""
    import torch
    print("timed plans in sequence", flush=True)
    A = inputs.sparse_uniform(3000, 2000, 30000, seed=501)
    Ad, keep = S.csr_to_device(A)
    plain = _solve(S, Ad, A.n, 8, 24, 502)
    for it in range(6):
        r = _solve(S, Ad, A.n, 8, 24, 502, flags=S.SVDS_FLAG_TIMING)
        assert r.status == 0, it
        assert r.info["kc_sampled_launches"]["spmv"] > 0, it
        assert r.info["kc_ms"]["spmv"] > 0, it
        assert torch.equal(r.S, plain.S) and torch.equal(r.U, plain.U) and torch.equal(r.V, plain.V), it


def test_plans_from_threads(S):
    """Four host threads create and run plans at once, each on its own
    stream; two of the matrices are large enough for column panels (three
    row-pointer read-backs through the pinned cache).  Every result equals
    the same solve made alone."""
    import torch
    print("plans from threads", flush=True)
    cases = [
        (inputs.sparse_uniform(400000, 150000, 1600000, seed=511), 6, 18, 512),
        (inputs.sparse_zipf(300000, 150000, 6, 1.1, seed=513), 6, 18, 514),
        (inputs.sparse_uniform(5000, 3000, 50000, seed=515), 8, 24, 516),
        (inputs.sparse_uniform(2000, 1500, 20000, seed=517), 5, 15, 518),
    ]
    dev = [S.csr_to_device(A) for A, _, _, _ in cases]
    alone = [_solve(S, d[0], A.n, k, p, seed) for (A, k, p, seed), d in zip(cases, dev)]
    assert alone[0].info["workspace_bytes"] > 0
    out = [None] * len(cases)
    errs = []

    def work(i):
        try:
            A, k, p, seed = cases[i]
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                out[i] = _solve(S, dev[i][0], A.n, k, p, seed, stream=st)
        except Exception as e:  # reported in the main thread
            errs.append((i, repr(e)))

    th = [threading.Thread(target=work, args=(i,)) for i in range(len(cases))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs, errs
    for i, (a, b) in enumerate(zip(alone, out)):
        assert b.status == 0, i
        assert torch.equal(a.S, b.S) and torch.equal(a.U, b.U) and torch.equal(a.V, b.V), i
    # and the lone solves agree with the oracle
    A, k, p, seed = cases[2]
    Ur, Sr, Vr, _ = svds_ref.svds(as_operator(A), k, p, 1e-10, 2000, v0=inputs.start_vector(A.n, seed))
    np.testing.assert_allclose(alone[2].S.cpu().numpy(), Sr, rtol=1e-10)
