"""Writes workload2_sigma.txt: the CPU oracle's singular values for the
1,000,000 x 500,000 Zipf(1.1) workload (k = 50, p = 150, tol = 1e-8) from its
seeded start vector.  Calls only the oracle and the input generators.

    python tests/golden/make_workload2_sigma.py
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
    A = inputs.config_matrix(2)
    v0 = inputs.start_vector(A.n, inputs.CONFIG_SEEDS[2] + 1)
    cfg = inputs.CONFIG_SOLVE[2]
    t0 = time.perf_counter()
    U, S, V, info = svds_ref.svds(svds_ref.as_operator(A), cfg["k"], cfg["p"], cfg["tol"], 2000, v0=v0)
    dt = time.perf_counter() - t0
    r1, r2 = svds_ref.explicit_residuals(svds_ref.as_operator(A), U, S, V)
    with open(os.path.join(HERE, "workload2_sigma.txt"), "w") as f:
        f.write("# CPU FP64 oracle, workload 1,000,000 x 500,000, 10 Zipf(1.1) draws/row, U(0,1) values,\n")
        f.write(f"# seed {inputs.CONFIG_SEEDS[2]}, start vector seed {inputs.CONFIG_SEEDS[2] + 1}, "
                f"k={cfg['k']} p={cfg['p']} tol={cfg['tol']}\n")
        f.write(f"# cycles {info.cycles}, converged {info.converged}, max |A^T u - s v|/s "
                f"{(r2 / S).max():.3e}, oracle time {dt:.1f} s\n")
        f.write("# written by tests/golden/make_workload2_sigma.py\n")
        for s in S:
            f.write(f"{float(s)!r}\n")
    print(f"done in {dt:.1f} s, cycles {info.cycles}, res {(r2 / S).max():.3e}")


if __name__ == "__main__":
    main()
