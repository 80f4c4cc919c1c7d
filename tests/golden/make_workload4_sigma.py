"""Writes workload4_sigma.txt: the CPU oracle's 50 largest singular values of
the 2000 x 1000 sparse workload with its values rounded to FP32 and widened
exactly to FP64 (the matrix of record of an FP32-valued run), from its seeded
start vector, k = 50, p = 150, tol = 1e-10.  Calls only the oracle and the
input generators.

    python tests/golden/make_workload4_sigma.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from paper_2405_18966_amd import inputs  # noqa: E402
from oracle import svds_ref  # noqa: E402


def main():
    A = inputs.config_matrix(4)
    A64 = svds_ref.as_operator(inputs.CSR(A.m, A.n, A.row_ptr, A.col_idx, A.val.astype(np.float64)))
    v0 = inputs.start_vector(A.n, inputs.CONFIG_SEEDS[4] + 1)
    cfg = inputs.CONFIG_SOLVE[4]
    t0 = time.perf_counter()
    U, S, V, info = svds_ref.svds(A64, cfg["k"], cfg["p"], 1e-10, 2000, v0=v0)
    dt = time.perf_counter() - t0
    r1, r2 = svds_ref.explicit_residuals(A64, U, S, V)
    with open(os.path.join(HERE, "workload4_sigma.txt"), "w") as f:
        f.write("# CPU FP64 oracle, sparse 2000 x 1000, 20,000 uniform positions, N(0,1) values rounded to\n")
        f.write("# FP32 and widened exactly (matrix of record)\n")
        f.write(f"# seed {inputs.CONFIG_SEEDS[1]}, start vector seed {inputs.CONFIG_SEEDS[4] + 1}, "
                f"k={cfg['k']} p={cfg['p']} tol=1e-10\n")
        f.write(f"# cycles {info.cycles}, converged {info.converged}, max |A^T u - s v|/s "
                f"{(r2 / S).max():.3e}, oracle time {dt:.1f} s\n")
        f.write("# written by tests/golden/make_workload4_sigma.py\n")
        for s in S:
            f.write(f"{float(s)!r}\n")
    print(f"done in {dt:.1f} s, cycles {info.cycles}, res {(r2 / S).max():.3e}")


if __name__ == "__main__":
    main()
