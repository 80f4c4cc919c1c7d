"""Writes workload5_sigma.txt: the CPU oracle's 8 largest singular values of
each of the 256 sparse problems of the batched workload (m ~ U{500..20000},
n ~ U{ceil(m/2)..m}, 0.5% density, N(0,1) values), each solved alone from
the start vector the batched solver draws for it (Philox4x32-10 stream 0 of
seed 2405005 + problem index), k = 8, p = 24, tol = 1e-12.  Calls only the
oracle and the input generators.

    python tests/golden/make_workload5_sigma.py [--jobs N]

One line per problem: index, m, n, nnz, cycles, then the 8 values.
"""
import argparse
import concurrent.futures as cf
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2405_18966_amd import inputs  # noqa: E402
from oracle import svds_ref  # noqa: E402

SEED = inputs.CONFIG_SEEDS[5]
TOL = 1e-12


def _solve_chunk(bs):
    # one generator call per worker chunk (the batch is drawn in sequence)
    As = inputs.config_matrix(5)
    cfg = inputs.CONFIG_SOLVE[5]
    out = []
    for b in bs:
        A = As[b]
        U, S, V, info = svds_ref.svds(svds_ref.as_operator(A), cfg["k"], cfg["p"], TOL, 5000, seed=SEED + b)
        out.append((b, A.m, A.n, A.nnz, info.cycles, bool(info.converged), [float(s) for s in S]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    t0 = time.perf_counter()
    chunks = [list(range(i, 256, args.jobs)) for i in range(args.jobs)]
    rows = []
    with cf.ProcessPoolExecutor(max_workers=args.jobs) as ex:
        for part in ex.map(_solve_chunk, chunks):
            rows.extend(part)
    rows.sort()
    dt = time.perf_counter() - t0
    assert all(r[5] for r in rows), "an oracle solve did not converge"
    with open(os.path.join(HERE, "workload5_sigma.txt"), "w") as f:
        f.write("# CPU FP64 oracle, 256 sparse problems: m ~ U{500..20000}, n ~ U{ceil(m/2)..m},\n")
        f.write("# 0.5% density, N(0,1) values (inputs.config_matrix(5)); each solved alone,\n")
        f.write(f"# start vector Philox4x32-10 stream 0 of seed {SEED} + index, k=8 p=24 tol={TOL:g}\n")
        f.write(f"# written by tests/golden/make_workload5_sigma.py in {dt:.0f} s\n")
        f.write("# index m n nnz cycles sigma_1 .. sigma_8\n")
        for b, m, n, nnz, cyc, _, s in rows:
            f.write(f"{b} {m} {n} {nnz} {cyc} " + " ".join(repr(x) for x in s) + "\n")
    print(f"done in {dt:.1f} s")


if __name__ == "__main__":
    main()
