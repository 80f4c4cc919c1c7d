#!/usr/bin/env python3
"""Benchmark: k-triplet truncated-SVD solves per second on one MI355X.

Workload (one "step" = one complete solve through the C ABI: device transpose,
Lanczos cycles with CGS2, small SVDs, restarts, outputs, residuals):
  sparse CSR A 1,000,000 x 500,000, 10 Zipf(1.1) column draws per row
  (~9.15 nnz/row, power-law column degrees), U(0,1) values, FP64;
  k = 50, p = 150, tol = 1e-8.  Inputs are seeded and synthetic and are
  resident in HBM before the timed region.

Prints ONE JSON line.  Besides solves/s it reports the roofline of the
dominant kernel (device time from HIP events recorded by the library on the
stream the kernels run on), the headline SpMV+CGS2 GB/s, parity of the
singular values against stored oracle values, and the CPU oracle timed on a
complete solve of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-paper-dense]

It also times the paper's synthetic Sparse1-3 and Dense1-3 suite (Sec. 3.1)
against the closed-form singular values, with the paper's own CPU times as
context, the other workloads (2000 x 1000 sparse; 20000 x 10000 dense BF16
and 2000 x 1000 FP32-valued, FP64 and mixed; the 256-problem batch), and the
CPU oracle on each of them.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "k-triplet solves/s at rel.err≤1e-8; SpMV+CGS2 HBM GB/s; mixed vs FP64 x"
HBM_PEAK_GBS = 8000.0
GOLDEN_W2 = os.path.join(ROOT, "tests", "golden", "workload2_sigma.txt")
GOLDEN_W3 = os.path.join(ROOT, "tests", "golden", "workload3_sigma_bf16.txt")
GOLDEN_W4 = os.path.join(ROOT, "tests", "golden", "workload4_sigma.txt")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_workload2.json")
WORKLOAD = dict(workload="zipf-sparse-svds", m=1_000_000, n=500_000, draws_per_row=10, zipf_a=1.1,
                values="U(0,1)", k=50, p=150, tol=1e-8, storage="fp64 CSR")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_golden(path=GOLDEN_W2):
    if not os.path.exists(path):
        return None
    import numpy as np
    vals = [float(x) for x in open(path) if x.strip() and not x.startswith("#")]
    return np.array(vals)


def kernel_source_hash():
    """Hash of the code (comments and whitespace removed) of the kernel
    sources the stored PMC traffic figures were measured on."""
    import re
    h = hashlib.sha256()
    for f in ("kernels_cgs.hpp", "kernels_spmv.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2405_18966_amd", "csrc", f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def cpu_baseline(A, v0, k, p, tol):
    """Times the CPU oracle (FP64 NumPy/SciPy) on the workload: complete solves
    from the same start vector, tolerance and Lanczos dimension, repeated until
    10 s have passed (at most 3; one solve takes 5-20 s depending on the host).
    Returns solves/s."""
    from oracle import svds_ref

    Asp = svds_ref.as_operator(A)
    n, dt = 0, 0.0
    while n < 3 and (n == 0 or dt < 10.0):
        t0 = time.perf_counter()
        U, S, V, info = svds_ref.svds(Asp, k, p, tol, 2000, v0=v0)
        dt += time.perf_counter() - t0
        n += 1
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    log(f"cpu oracle: {n} solve(s) in {dt:.1f} s, cycles {info.cycles}")
    return {"value": round(n / dt, 6), "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": (f"{n} complete oracle solve(s) of the workload ({dt:.1f} s, {info.cycles} cycle(s) "
                       f"each); sparse products single-threaded (scipy), dense BLAS on {threads} threads"),
            "sigma": S.tolist()}


def host_cpu():
    """The bench host's CPU as lscpu reports it (model, sockets, cores,
    threads), and the threads the oracle's BLAS may use."""
    import subprocess
    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)",
                     "CPU max MHz", "NUMA node(s)"):
                info[k] = v
    except (OSError, subprocess.SubprocessError):
        pass
    info["blas_threads"] = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return info


def oracle_rate(A, k, p, tol, v0=None, seed=0, reps=3, budget_s=20.0):
    """Complete CPU-oracle solves of one matrix (same start vector or seed,
    k, p, tol as the GPU run), repeated up to ``reps`` times while under
    ``budget_s``; returns (median solves/s, cycles, singular values)."""
    from oracle import svds_ref

    op = svds_ref.as_operator(A)
    ts, S_, info = [], None, None
    while len(ts) < reps and (not ts or sum(ts) < budget_s):
        t0 = time.perf_counter()
        U, S_, V, info = svds_ref.svds(op, k, p, tol, 2000, v0=v0, seed=seed)
        ts.append(time.perf_counter() - t0)
    return 1.0 / sorted(ts)[len(ts) // 2], info.cycles, S_, len(ts)


def config1(S, inputs, np, torch, cpu: bool):
    """The 2000 x 1000 sparse workload (20,000 uniform positions, N(0,1)),
    FP64, k=10, p=30, tol=1e-10: median of 5 GPU solves after one warm-up,
    and the CPU oracle on the same matrix and start vector."""
    A = inputs.config_matrix(1)
    c = inputs.CONFIG_SOLVE[1]
    v0 = inputs.start_vector(A.n, inputs.CONFIG_SEEDS[1] + 1)
    Ad, keep = S.csr_to_device(A)
    v0d = torch.from_numpy(v0).cuda()
    run = lambda: S.svds_csr_solve(Ad, S.make_opts(c["k"], c["p"], c["tol"], 2000, v0=v0d))
    r = run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        r = run()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t = sorted(ts)[2]
    out = {"workload": "sparse 2000x1000, nnz 20000 uniform, N(0,1), fp64, k=10 p=30 tol=1e-10",
           "gpu_ms": round(t * 1e3, 3), "gpu_solves_per_s": round(1 / t, 2), "cycles": r.info["cycles"],
           "status": r.status}
    if cpu:
        rate, cyc, s_or, n = oracle_rate(A, c["k"], c["p"], c["tol"], v0=v0)
        s = r.S.cpu().numpy()
        out["cpu_oracle"] = {"solves_per_s": round(rate, 3), "cycles": cyc, "runs": n,
                             "sample": f"median of {n} complete oracle solves"}
        out["sigma_rel_err_vs_oracle"] = float(np.max(np.abs(s - s_or) / s_or))
        out["x_vs_cpu_oracle"] = round(out["gpu_solves_per_s"] / rate, 1)
    return out


def mixed_vs_fp64(S, inputs, np, torch, cpu: bool = False):
    """Mixed (FP32 cycles + FP64 refinement) against the plain FP64 GPU path,
    same stored matrix, same start vector, tol=1e-8: median solve time of 3
    after one warm-up each.  The dense 20000 x 10000 BF16 workload and the
    2000 x 1000 sparse workload with FP32 values (k=50, p=150)."""
    out = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts, r = [], None
        for _ in range(3):
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[1] * 1e3, r

    d = inputs.config_matrix(3)
    t = torch.from_numpy(d["bf16"].a.ravel(order="F").view(np.int16)).view(torch.uint16).cuda()
    Ad = S.make_dense(t, 20000, 10000)
    v0 = torch.from_numpy(inputs.start_vector(10000, inputs.CONFIG_SEEDS[3] + 1)).cuda()
    gold = load_golden(GOLDEN_W3)
    res = {}
    E = S.SVDS_FLAG_EARLY_STOP
    for name, prec, fl in (("fp64", 0, 0), ("mixed", 1, 0), ("fp64_early", 0, E), ("mixed_early", 1, E)):
        ms, r = timed(lambda: S.svds_dense_solve(Ad, S.make_opts(100, 250, 1e-8, 2000, precision=prec, v0=v0,
                                                                 flags=fl)))
        s = r.S.cpu().numpy()
        res[name] = {"ms": round(ms, 2), "cycles_fp32": r.info["cycles_fp32"], "cycles_fp64": r.info["cycles_fp64"],
                     "lanczos_dim_last": r.info["lanczos_dim_last"],
                     "sigma_rel_err_vs_oracle": float(np.max(np.abs(s - gold[:100]) / gold[:100]))
                     if gold is not None else None, "status": r.status}
    out["dense_20000x10000_bf16_k100_p250"] = dict(res, x=round(res["fp64"]["ms"] / res["mixed"]["ms"], 3),
                                                   x_early=round(res["fp64_early"]["ms"] / res["mixed_early"]["ms"], 3))
    if cpu:
        # the CPU oracle on the stored matrix widened to FP64 (the matrix of
        # record), same start vector, FP64, tol=1e-8: one complete solve
        rate, cyc, s_or, n = oracle_rate(d["record_bf16"], 100, 250, 1e-8, v0=v0.cpu().numpy(), reps=1)
        out["dense_20000x10000_bf16_k100_p250"]["cpu_oracle"] = {
            "solves_per_s": round(rate, 4), "cycles": cyc, "runs": n,
            "sample": "one complete FP64 oracle solve (dense BLAS mat-vecs)",
            "x_fp64_gpu_vs_cpu": round(rate and (1e3 / res["fp64"]["ms"]) / rate, 1)}
    del d, t, Ad
    A = inputs.config_matrix(4)
    Ad4, keep = S.csr_to_device(A)
    v0 = torch.from_numpy(inputs.start_vector(A.n, inputs.CONFIG_SEEDS[4] + 1)).cuda()
    gold = load_golden(GOLDEN_W4)
    res = {}
    for name, prec, fl in (("fp64", 0, 0), ("mixed", 1, 0), ("fp64_early", 0, E), ("mixed_early", 1, E)):
        ms, r = timed(lambda: S.svds_csr_solve(Ad4, S.make_opts(50, 150, 1e-8, 2000, precision=prec, v0=v0,
                                                               flags=fl)))
        s = r.S.cpu().numpy()
        res[name] = {"ms": round(ms, 2), "cycles_fp32": r.info["cycles_fp32"], "cycles_fp64": r.info["cycles_fp64"],
                     "lanczos_dim_last": r.info["lanczos_dim_last"],
                     "sigma_rel_err_vs_oracle": float(np.max(np.abs(s - gold[:50]) / gold[:50]))
                     if gold is not None else None, "status": r.status}
    out["sparse_2000x1000_fp32_k50_p150"] = dict(res, x=round(res["fp64"]["ms"] / res["mixed"]["ms"], 3),
                                                 x_early=round(res["fp64_early"]["ms"] / res["mixed_early"]["ms"], 3))
    if cpu:
        rate, cyc, s_or, n = oracle_rate(A, 50, 150, 1e-8, v0=v0.cpu().numpy())
        out["sparse_2000x1000_fp32_k50_p150"]["cpu_oracle"] = {
            "solves_per_s": round(rate, 3), "cycles": cyc, "runs": n,
            "sample": f"median of {n} complete FP64 oracle solves of the FP32-valued matrix",
            "x_fp64_gpu_vs_cpu": round((1e3 / res["fp64"]["ms"]) / rate, 1)}
    return out


def batched_vs_loop(S, inputs, np, torch, cpu: bool = False):
    """The 256-problem workload (m ~ U{500..20000}, n ~ U{m/2..m}, 0.5%
    density, N(0,1), k=8, p=24, tol=1e-8): one lockstep batched call against
    a loop of single-problem solves, mixed and FP64; median of 3 after one
    warm-up each (the loop: one timed pass).  Problems/s = 256 / wall time."""
    As = inputs.config_matrix(5)
    dev = [S.csr_to_device(A) for A in As]
    seed = inputs.CONFIG_SEEDS[5]
    out = {"problems": len(As), "nnz_total": int(sum(A.nnz for A in As))}
    for name, prec in (("fp64", 0), ("mixed", 1)):
        opts = S.make_opts(8, 24, 1e-8, 2000, precision=prec, seed=seed)
        res, rc = S.svds_csr_solve_batched([d[0] for d in dev], opts)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            res, rc = S.svds_csr_solve_batched([d[0] for d in dev], opts)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        tb = sorted(ts)[1]
        sig_b = [r.S.cpu().numpy() for r in res]
        ok = rc == 0 and all(r.info["converged"] == 1 and r.info["max_res_true"] <= 2e-8 for r in res)
        t0 = time.perf_counter()
        worst = 0.0
        for b, d in enumerate(dev):
            one = S.svds_csr_solve(d[0], S.make_opts(8, 24, 1e-8, 2000, precision=prec, seed=seed + b))
            torch.cuda.synchronize()
            s1 = one.S.cpu().numpy()
            worst = max(worst, float(np.max(np.abs(s1 - sig_b[b]) / s1)))
        tl = time.perf_counter() - t0
        # the same batched call with each cycle replayed as a captured HIP graph,
        # and with the plan-time autotuner (median of 3 after one warm-up)
        variants = {}
        for vname, vflag in (("graph", S.SVDS_FLAG_GRAPH), ("autotune", S.SVDS_FLAG_AUTOTUNE)):
            vopts = S.make_opts(8, 24, 1e-8, 2000, precision=prec, seed=seed, flags=vflag)
            vres, vrc = S.svds_csr_solve_batched([d[0] for d in dev], vopts)
            torch.cuda.synchronize()
            vts = []
            for _ in range(3):
                t0 = time.perf_counter()
                vres, vrc = S.svds_csr_solve_batched([d[0] for d in dev], vopts)
                torch.cuda.synchronize()
                vts.append(time.perf_counter() - t0)
            vdiff = max(float(np.max(np.abs(r.S.cpu().numpy() - sig_b[b]) / sig_b[b])) for b, r in enumerate(vres))
            variants[vname] = {"ms": round(sorted(vts)[1] * 1e3, 2), "status": vrc,
                               "sigma_rel_diff_vs_plain": vdiff,
                               "graph_captures": vres[0].info["graph_captures"],
                               "graph_replays": vres[0].info["graph_replays"],
                               "tuning_ms": round(vres[0].info["tuning"]["ms_tune"], 2)}
        out[name] = {"batched_ms": round(tb * 1e3, 2), "looped_ms": round(tl * 1e3, 2), "variants": variants,
                     "batched_problems_per_s": round(len(As) / tb, 2),
                     "looped_problems_per_s": round(len(As) / tl, 2), "x": round(tl / tb, 2),
                     "cycles": res[0].info["cycles"], "all_converged": bool(ok),
                     "sigma_rel_diff_batched_vs_looped": worst}
    if cpu:
        # CPU oracle: problems solved alone, in order, until 15 s have passed
        from oracle import svds_ref
        t0, nb = time.perf_counter(), 0
        while nb < len(As) and time.perf_counter() - t0 < 15.0:
            svds_ref.svds(svds_ref.as_operator(As[nb]), 8, 24, 1e-8, 2000, seed=seed + nb)
            nb += 1
        dt = time.perf_counter() - t0
        share = sum(A.nnz for A in As[:nb]) / out["nnz_total"]
        out["cpu_oracle"] = {
            "problems_per_s": round(nb / dt, 3),
            "problems_per_s_nnz_weighted": round(len(As) * share / dt, 4),
            "sample": f"problems 0..{nb - 1} solved alone by the FP64 oracle in {dt:.1f} s "
                      f"({100 * share:.1f}% of the batch's nonzeros); nnz-weighted rate = 256 / (time / share)"}
    return out


# The paper's own times for its synthetic suite: svds-C with MKL on 16
# threads of 2x 8-core Intel Xeon @ 2.10 GHz, seconds (Table 2; FP64,
# k = 100, t = 300, tol = 1e-10, r = 10).  Context only: another machine.
PAPER_TABLE2_MKL16_S = {"sparse1": 2.14, "sparse2": 1.24, "sparse3": 1.33,
                        "dense1": 16.5, "dense2": 10.7, "dense3": 10.2}


def smallest_harmonic(S, inputs, np, torch):
    """The k = 4 smallest triplets (p = 20, tol = 1e-10, at most 3000 cycles)
    of square matrices with six clustered small values 1e-4 (1 + 0.01 i) below
    a bulk in [0.5, 1], five nonzeros per row: plain Ritz restarts
    (SVDS_FLAG_SMALLEST) against harmonic-Ritz restarts (+ SVDS_FLAG_HARMONIC),
    one timed solve each after a warm-up of the harmonic one."""
    out = {}
    for N, seed in ((1000, 1), (2000, 3)):
        sig = np.concatenate([1e-4 * (1 + 0.01 * np.arange(6)), np.linspace(0.5, 1.0, N - 6)])
        A = inputs.prescribed_sparse(N // 5, 5, sig, seed=seed)
        exact = np.sort(sig)[:4]
        Ad, keep = S.csr_to_device(A)
        v0d = torch.from_numpy(inputs.start_vector(N, 23)).cuda()
        res = {}
        for name, f in (("harmonic", S.SVDS_FLAG_SMALLEST | S.SVDS_FLAG_HARMONIC), ("plain", S.SVDS_FLAG_SMALLEST)):
            if name == "harmonic":
                S.svds_csr_solve(Ad, S.make_opts(4, 20, 1e-10, 3000, v0=v0d, flags=f))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = S.svds_csr_solve(Ad, S.make_opts(4, 20, 1e-10, 3000, v0=v0d, flags=f))
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            s = r.S.cpu().numpy()
            res[name] = {"ms": round(t * 1e3, 2), "cycles": r.info["cycles"], "converged": r.info["nconv"] == 4,
                         "sigma_rel_err_vs_exact": float(np.max(np.abs(s - exact) / exact))}
        out[f"sparse_{N}x{N}_k4_p20"] = dict(res, cycles_ratio=round(res["plain"]["cycles"] /
                                                                     res["harmonic"]["cycles"], 2))
        log(f"smallest {N}: {out[f'sparse_{N}x{N}_k4_p20']}")
    return out


def paper_suite(S, inputs, np, torch, dense: bool):
    """Sparse1-3 (40,000 x 40,000, 5 nnz/row) and, with ``dense``, Dense1-3
    (10,000 x 10,000) of Sec. 3.1 at the paper's shape and settings; best of
    2 solves after one warm-up, singular values against the closed-form
    Decay1/2/3 values."""
    out = {}
    c = inputs.PAPER_SUITE_SOLVE
    names = ["sparse1", "sparse2", "sparse3"] + (["dense1", "dense2", "dense3"] if dense else [])
    for name in names:
        log(f"paper suite {name} ...")
        A, sig = inputs.paper_suite(name)
        N = len(sig)
        v0 = torch.from_numpy(inputs.start_vector(N, inputs.PAPER_SUITE_SEEDS[name] + 1)).cuda()
        opts = S.make_opts(c["k"], c["p"], c["tol"], c["maxit"], v0=v0)
        if name.startswith("sparse"):
            Ad, keep = S.csr_to_device(A)
            run = lambda: S.svds_csr_solve(Ad, opts)
        else:
            Ad = S.make_dense(torch.from_numpy(A.ravel(order="F")).cuda(), N, N)
            run = lambda: S.svds_dense_solve(Ad, opts)
        r = run()
        torch.cuda.synchronize()
        ts = []
        for _ in range(2):
            t0 = time.perf_counter()
            r = run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        sv = r.S.cpu().numpy()
        t = min(ts)
        # the same case with the eq. (4) test checked inside the cycle
        opts_e = S.make_opts(c["k"], c["p"], c["tol"], c["maxit"], v0=v0, flags=S.SVDS_FLAG_EARLY_STOP)
        if name.startswith("sparse"):
            run_e = lambda: S.svds_csr_solve(Ad, opts_e)
        else:
            run_e = lambda: S.svds_dense_solve(Ad, opts_e)
        re_ = run_e()
        torch.cuda.synchronize()
        tes = []
        for _ in range(2):
            t0 = time.perf_counter()
            re_ = run_e()
            torch.cuda.synchronize()
            tes.append(time.perf_counter() - t0)
        se = re_.S.cpu().numpy()
        out[name] = {"n": N, "ms": round(t * 1e3, 2), "solves_per_s": round(1 / t, 2), "cycles": r.info["cycles"],
                     "status": r.status, "nconv": r.info["nconv"],
                     "sigma_rel_err_vs_exact": float(np.max(np.abs(sv - sig[:c["k"]]) / sig[:c["k"]])),
                     "paper_mkl16_s": PAPER_TABLE2_MKL16_S[name],
                     "x_vs_paper_mkl16": round(PAPER_TABLE2_MKL16_S[name] / t, 1),
                     "early_stop": {"ms": round(min(tes) * 1e3, 2), "lanczos_dim_last": re_.info["lanczos_dim_last"],
                                    "cycles": re_.info["cycles"], "status": re_.status,
                                    "sigma_rel_err_vs_exact": float(np.max(np.abs(se - sig[:c["k"]]) / sig[:c["k"]]))}}
        del A, Ad
    return out


def gather_ceiling(S, inputs, np, torch):
    """The sparse products of the Zipf workload against the gather-copy
    reference over the same index streams (svds_op_gather_copy): A v gathers
    v through A's column indices; A^T u, in the column-panel form the solver
    runs, gathers u through the row indices of each of 8 row panels of A,
    panel g on XCD g.  Each stream also in a chunk-sorted order (the indices
    of every 2048-entry chunk sorted: the same entries, gathered in address
    order).  Two plain solves run first, so a kernel trace of this section
    holds the products' own durations (per-dispatch timing events are left
    off: they change the caches the products find).  Prints one line per
    reference (no JSON)."""
    import scipy.sparse as sp
    A = inputs.config_matrix(2)
    m, n = A.m, A.n
    Ad, keep = S.csr_to_device(A)
    v0 = torch.from_numpy(inputs.start_vector(n, inputs.CONFIG_SEEDS[2] + 1)).cuda()
    for _ in range(2):
        r = S.svds_csr_solve(Ad, S.make_opts(WORKLOAD["k"], WORKLOAD["p"], WORKLOAD["tol"], 2000, v0=v0))
        torch.cuda.synchronize()
        print(f"solve: {r.info['ms_total']:.1f} ms, {r.info['n_spmv']} + {r.info['n_spmvT']} products", flush=True)
    nnz = A.nnz
    print(f"{nnz} nonzeros", flush=True)
    csr = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(m, n))
    rpp = -(-m // 8)
    parts, seg = [], [0]
    for g in range(8):
        t = csr[g * rpp:min(m, (g + 1) * rpp)].T.tocsr()
        parts.append(t.indices.astype(np.int32) + g * rpp)
        seg.append(seg[-1] + t.nnz)
    panel_idx = np.concatenate(parts)

    def chunk_sorted(ix, seg_):
        out = ix.copy()
        for a, b in zip(seg_[:-1], seg_[1:]):
            for c0 in range(a, b, 2048):
                out[c0:min(b, c0 + 2048)].sort()
        return out

    xv = torch.rand(n, dtype=torch.float64, device="cuda")
    xu = torch.rand(m, dtype=torch.float64, device="cuda")
    cases = [("A v, column indices of A", A.col_idx.astype(np.int32), xv, 1, None),
             ("A v, chunk-sorted", chunk_sorted(A.col_idx.astype(np.int32), [0, nnz]), xv, 1, None),
             ("A^T u, 8 row panels (XCD g: panel g)", panel_idx, xu, 8, seg),
             ("A^T u, 8 row panels, chunk-sorted", chunk_sorted(panel_idx, seg), xu, 8, seg)]
    for name, ix, x, nseg, sg in cases:
        it = torch.from_numpy(np.ascontiguousarray(ix)).cuda()
        out, _ = S.svds_op_gather_copy(it, x, nseg, sg, reps=3)
        assert torch.equal(out, x[it.long()])
        _, t = S.svds_op_gather_copy(it, x, nseg, sg, out=out, reps=50)
        us = t * 1e3
        print(f"gather copy  : {name}: {us:.2f} us per launch, {nnz / us / 1e3:.1f} G entries/s", flush=True)


def profile_section(which, S, inputs, np, torch):
    """Two solves of one workload for a kernel trace (see --profile-section)."""
    if which == "dense":
        d = inputs.config_matrix(3)
        t = torch.from_numpy(d["bf16"].a.ravel(order="F").view(np.int16)).view(torch.uint16).cuda()
        Ad = S.make_dense(t, 20000, 10000)
        v0 = torch.from_numpy(inputs.start_vector(10000, inputs.CONFIG_SEEDS[3] + 1)).cuda()
        for prec in (0, 1):
            for _ in range(2):
                r = S.svds_dense_solve(Ad, S.make_opts(100, 250, 1e-8, 2000, precision=prec, v0=v0))
                torch.cuda.synchronize()
                log(f"dense precision {prec}: {r.info['ms_total']:.1f} ms, cycles {r.info['cycles']}")
    elif which == "sparse2":
        A, sig = inputs.paper_suite("sparse2")
        Ad, keep = S.csr_to_device(A)
        v0 = torch.from_numpy(inputs.start_vector(A.n, inputs.PAPER_SUITE_SEEDS["sparse2"] + 1)).cuda()
        c = inputs.PAPER_SUITE_SOLVE
        for _ in range(2):
            r = S.svds_csr_solve(Ad, S.make_opts(c["k"], c["p"], c["tol"], c["maxit"], v0=v0))
            torch.cuda.synchronize()
            log(f"sparse2: {r.info['ms_total']:.1f} ms, cycles {r.info['cycles']}")
    elif which == "gather":
        gather_ceiling(S, inputs, np, torch)
    elif which == "stream":
        # attainable streaming rates on this GPU, beside which the CGS passes
        # are judged: the library's FP64 copy (read + write) and a plain FP64
        # read reduction (torch sum), both over 1.2 GB
        n = 150 * 1_000_000
        src = torch.rand(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            S.svds_op_copy_f64(src, dst)
            s_ = src.sum()
        torch.cuda.synchronize()
        log(f"stream: {n * 8 / 1e9:.2f} GB copied and summed 5 times, sum {s_.item():.6e}")
    elif which == "breakdowns":
        d = np.zeros(500000)
        d[:30] = np.arange(30, 0, -1, dtype=np.float64)
        A = inputs.diag_matrix(1_000_000, 500_000, d)
        Ad, keep = S.csr_to_device(A)
        v0 = torch.from_numpy(inputs.start_vector(500_000, 31)).cuda()
        for flags, name in ((0, "one-workgroup repairs"), (S.SVDS_FLAG_EXPECT_BREAKDOWNS, "wide repairs")):
            for _ in range(2):
                r = S.svds_csr_solve(Ad, S.make_opts(5, 40, 1e-10, 50, v0=v0, flags=flags))
                torch.cuda.synchronize()
                log(f"rank-30 1,000,000 x 500,000, {name}: {r.info['ms_total']:.1f} ms, "
                    f"breakdowns {r.info['breakdowns']}")
    elif which == "config1":
        A = inputs.config_matrix(1)
        c = inputs.CONFIG_SOLVE[1]
        Ad, keep = S.csr_to_device(A)
        v0 = torch.from_numpy(inputs.start_vector(A.n, inputs.CONFIG_SEEDS[1] + 1)).cuda()
        for _ in range(3):
            r = S.svds_csr_solve(Ad, S.make_opts(c["k"], c["p"], c["tol"], 2000, v0=v0))
            torch.cuda.synchronize()
            log(f"2000 x 1000: {r.info['ms_total']:.2f} ms, cycles {r.info['cycles']}")
    else:
        As = inputs.config_matrix(5)
        dev = [S.csr_to_device(A) for A in As]
        opts = S.make_opts(8, 24, 1e-8, 2000, seed=inputs.CONFIG_SEEDS[5])
        for _ in range(2):
            res, rc = S.svds_csr_solve_batched([d[0] for d in dev], opts)
            torch.cuda.synchronize()
            log(f"batched: {res[0].info['ms_total']:.1f} ms, rc {rc}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed vs FP64 comparison")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched vs looped comparison")
    ap.add_argument("--no-suite", action="store_true", help="skip the paper's Sparse1-3 suite")
    ap.add_argument("--no-selective", action="store_true", help="skip the selective re-orthogonalization run")
    ap.add_argument("--no-paper-dense", action="store_true",
                    help="leave Dense1-3 (10,000 x 10,000) out of the paper suite")
    ap.add_argument("--no-harmonic", action="store_true",
                    help="skip the smallest-triplet runs (plain vs harmonic-Ritz restarts)")
    ap.add_argument("--no-config1", action="store_true",
                    help="skip the 2000 x 1000 sparse workload (k=10, p=30, tol=1e-10)")
    ap.add_argument("--profile-run", action="store_true",
                    help="one solve + one plain copy (for rocprofv3 counter runs); no JSON")
    ap.add_argument("--profile-section", choices=["dense", "batched", "sparse2", "gather", "config1", "breakdowns",
                                                  "stream"],
                    help="only two solves of one other workload, for a rocprofv3 kernel trace: the "
                         "20000 x 10000 BF16 dense matrix (FP64 then mixed), the 256-problem batch (FP64), "
                         "or the paper's Sparse2 (40,000 x 40,000, k=100, p=300); 'gather': the Zipf "
                         "workload's products against the gather-copy reference; 'config1': three solves "
                         "of the 2000 x 1000 workload; 'breakdowns': a rank-30 1,000,000 x 500,000 matrix "
                         "with one-workgroup and with wide breakdown repairs; 'stream': the FP64 copy and "
                         "read-reduction rates over 1.2 GB; no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the solver does not "
              "shard a problem across GPUs.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2405_18966_amd import inputs
    from paper_2405_18966_amd import svds as S

    rank = int(os.environ.get("RANK", "0"))
    torch.cuda.set_device(0)
    if args.profile_section:
        profile_section(args.profile_section, S, inputs, np, torch)
        return
    log("generating workload ...")
    A = inputs.config_matrix(2)
    v0 = inputs.start_vector(A.n, inputs.CONFIG_SEEDS[2] + 1)
    k, p, tol = WORKLOAD["k"], WORKLOAD["p"], WORKLOAD["tol"]
    Ad, keep = S.csr_to_device(A)
    v0d = torch.from_numpy(v0).cuda()
    stream = torch.cuda.current_stream()
    maxit = 2000
    log(f"nnz = {A.nnz}")

    def solve(flags=0):
        return S.svds_csr_solve(Ad, S.make_opts(k, p, tol, maxit, v0=v0d, flags=flags, stream=stream))

    if args.profile_run:
        r = solve()
        torch.cuda.synchronize()
        src = torch.empty(64 << 20, dtype=torch.float64, device="cuda").uniform_()
        dst = torch.empty_like(src)
        S.svds_op_copy_f64(src, dst)
        torch.cuda.synchronize()
        log(f"profile run done: cycles {r.info['cycles']} status {r.status}")
        return

    for i in range(args.warmup):
        r = solve()
        torch.cuda.synchronize()
        log(f"warmup {i}: {r.info['ms_total']:.1f} ms, cycles {r.info['cycles']}, status {r.status}")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        r = solve(S.SVDS_FLAG_TIMING)
        results.append(r)
        log(f"step {i}: {r.info['ms_total']:.1f} ms, cycles {r.info['cycles']}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = args.steps / elapsed
    last = results[-1]
    info = last.info

    # parity of the singular values against stored oracle values
    golden = load_golden()
    s = last.S.cpu().numpy()
    parity = {"status": last.status, "converged": info["converged"], "cycles": info["cycles"],
              "max_res_true": info["max_res_true"], "max_res_av": info["max_res_av"]}
    if golden is not None and len(golden) >= k:
        parity["sigma_rel_err_vs_oracle"] = float(np.max(np.abs(s - golden[:k]) / golden[:k]))
    valid = info["converged"] == 1 and info["max_res_true"] <= 2 * tol
    if "sigma_rel_err_vs_oracle" in parity:
        valid = valid and parity["sigma_rel_err_vs_oracle"] <= 1e-8
    parity["valid"] = bool(valid)

    # roofline of the dominant kernel (summed over the timed steps)
    # (device time of one launch in four of each class, with the algorithmic
    # bytes of exactly those launches)
    kc_ms = {c: sum(r.info["kc_ms"][c] for r in results) for c in S.KERNEL_CLASSES}
    kc_b = {c: sum(r.info["kc_sampled_bytes"][c] for r in results) for c in S.KERNEL_CLASSES}
    kc_n = {c: sum(r.info["kc_sampled_launches"][c] for r in results) for c in S.KERNEL_CLASSES}
    kc_all = {c: sum(r.info["kc_launches"][c] for r in results) for c in S.KERNEL_CLASSES}
    # estimated time per class = sampled time scaled to all launches
    kc_est = {c: kc_ms[c] * kc_all[c] / kc_n[c] if kc_n[c] else 0.0 for c in S.KERNEL_CLASSES}
    dom = max(kc_est, key=lambda c: kc_est[c])
    achieved = kc_b[dom] / (kc_ms[dom] * 1e-3) / 1e9 if kc_ms[dom] > 0 else 0.0
    traffic = None
    if os.path.exists(TRAFFIC):
        tr = json.load(open(TRAFFIC))
        if tr.get("source_hash") == kernel_source_hash() and dom in tr.get("kernels", {}):
            traffic = tr["kernels"][dom]["bytes_per_launch"] / 1e9  # GB per launch, PMC-scaled
    hot = ["spmv", "spmvT", "cgs_proj", "cgs_updproj", "cgs_updnorm"]
    hot_gbs = sum(kc_b[c] for c in hot) / (sum(kc_ms[c] for c in hot) * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_unit": "GB per launch",
                "traffic_note": "rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-kernel calibrated, averaged over all "
                                "launches of the class in one solve; null when the kernel sources changed",
                "kernel": dom,
                "avg_launch_us": round(kc_ms[dom] * 1e3 / max(kc_n[dom], 1), 2),
                "alg_bytes_per_launch": round(kc_b[dom] / max(kc_n[dom], 1)),
                "spmv_cgs2_gbs": round(hot_gbs, 1),
                "timing_sample": "1 launch in 16 per class, rotating offset; events carried by the "
                                 "dispatches of the products and CGS2 passes",
                "per_class": {c: {"est_ms": round(kc_est[c] / args.steps, 3),
                                  "gbs": round(kc_b[c] / (kc_ms[c] * 1e-3) / 1e9, 1) if kc_ms[c] else None,
                                  "launches": kc_all[c] // args.steps} for c in S.KERNEL_CLASSES}}

    # the same workload with the selective second pass (one projection per
    # vector unless the DGKS test asks for a second): best of 3 solves
    sel = None
    if not args.no_selective:
        log("selective re-orthogonalization ...")
        ts, rs = [], None
        for _ in range(3):
            t1 = time.perf_counter()
            rs = solve(S.SVDS_FLAG_SELECTIVE_REORTH)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        ss = rs.S.cpu().numpy()
        sel = {"ms": round(min(ts) * 1e3, 2), "solves_per_s": round(1 / min(ts), 3),
               "x_vs_cgs2": round((elapsed / args.steps) / min(ts), 3),
               "second_passes": rs.info["reorth_second_passes"], "tests": rs.info["reorth_tests"],
               "cycles": rs.info["cycles"], "status": rs.status, "max_res_true": rs.info["max_res_true"],
               "sigma_rel_err_vs_oracle": float(np.max(np.abs(ss - golden[:k]) / golden[:k]))
               if golden is not None else None}

    # the same workload with partial re-orthogonalization (omega recurrences):
    # best of 3 solves
    part = None
    if not args.no_selective:
        log("partial re-orthogonalization ...")
        ts, rp = [], None
        for _ in range(3):
            t1 = time.perf_counter()
            rp = solve(S.SVDS_FLAG_PARTIAL_REORTH)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        sp_ = rp.S.cpu().numpy()
        eye = torch.eye(k, dtype=torch.float64, device="cuda")
        part = {"ms": round(min(ts) * 1e3, 2), "solves_per_s": round(1 / min(ts), 3),
                "x_vs_cgs2": round((elapsed / args.steps) / min(ts), 3),
                "columns_taken_frac": round(rp.info["partial_columns"] / max(1, rp.info["partial_possible"]), 4),
                "vectors_reorthogonalized": rp.info["partial_steps"], "cycles": rp.info["cycles"],
                "status": rp.status, "max_res_true": rp.info["max_res_true"],
                "orthogonality": max(float((rp.U.T @ rp.U - eye).abs().max()),
                                     float((rp.V.T @ rp.V - eye).abs().max())),
                "sigma_rel_err_vs_oracle": float(np.max(np.abs(sp_ - golden[:k]) / golden[:k]))
                if golden is not None else None}

    # the same workload with the eq. (4) test checked inside the cycle
    # (SVDS_FLAG_EARLY_STOP), alone and with partial re-orthogonalization:
    # best of 3 solves each
    early = None
    if not args.no_selective:
        log("early stop ...")
        early = {}
        for ename, efl in (("early_stop", S.SVDS_FLAG_EARLY_STOP),
                           ("early_stop_partial_reorth", S.SVDS_FLAG_EARLY_STOP | S.SVDS_FLAG_PARTIAL_REORTH)):
            ts, re_ = [], None
            for _ in range(3):
                t1 = time.perf_counter()
                re_ = solve(efl)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t1)
            se = re_.S.cpu().numpy()
            eye = torch.eye(k, dtype=torch.float64, device="cuda")
            early[ename] = {
                "ms": round(min(ts) * 1e3, 2), "solves_per_s": round(1 / min(ts), 3),
                "x_vs_cgs2": round((elapsed / args.steps) / min(ts), 3),
                "lanczos_dim_last": re_.info["lanczos_dim_last"], "early_checks": re_.info["early_checks"],
                "cycles": re_.info["cycles"], "status": re_.status, "max_res_true": re_.info["max_res_true"],
                "orthogonality": max(float((re_.U.T @ re_.U - eye).abs().max()),
                                     float((re_.V.T @ re_.V - eye).abs().max())),
                "sigma_rel_err_vs_oracle": float(np.max(np.abs(se - golden[:k]) / golden[:k]))
                if golden is not None else None}

    mixed = None
    if not args.no_mixed:
        log("mixed vs FP64 ...")
        mixed = mixed_vs_fp64(S, inputs, np, torch, cpu=not args.no_cpu and rank == 0)

    batched = None
    if not args.no_batched:
        log("batched vs looped ...")
        batched = batched_vs_loop(S, inputs, np, torch, cpu=not args.no_cpu and rank == 0)

    c1 = None
    if not args.no_config1:
        log("2000 x 1000 sparse workload ...")
        c1 = config1(S, inputs, np, torch, cpu=not args.no_cpu and rank == 0)

    harm = None
    if not args.no_harmonic:
        log("smallest triplets, plain vs harmonic restarts ...")
        harm = smallest_harmonic(S, inputs, np, torch)

    suite = None
    if not args.no_suite:
        suite = paper_suite(S, inputs, np, torch, not args.no_paper_dense)

    cpu = None
    if not args.no_cpu and rank == 0:
        cpu = cpu_baseline(A, v0, k, p, tol)
        s_or = np.array(cpu.pop("sigma"))
        parity["sigma_rel_err_vs_oracle_live"] = float(np.max(np.abs(s - s_or) / s_or))

    # a step is one svds_csr_solve: plan creation, the execute call (timed by
    # the library on the host), plan destruction
    ms_step = elapsed * 1e3 / args.steps
    ms_exec = float(np.mean([r.info["ms_total"] for r in results]))
    out = {"metric": METRIC, "value": round(value, 5), "unit": "solves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 2),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", "config": dict(WORKLOAD, parallelism="single GPU"),
           "roofline": roofline, "cpu_baseline": cpu, "parity": parity, "mixed_vs_fp64": mixed,
           "batched_vs_looped": batched, "paper_suite": suite, "selective_reorth": sel,
           "partial_reorth": part, "early_stop": early,
           "config_2000x1000": c1, "smallest_harmonic": harm, "host_cpu": host_cpu(),
           "step_ms": {"execute": round(ms_exec, 2), "create_and_destroy": round(ms_step - ms_exec, 2)}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
