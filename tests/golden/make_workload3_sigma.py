"""Writes workload3_sigma_bf16.txt: the CPU oracle's 100 largest singular
values of the dense 20000 x 10000 workload G1 diag(0.95^i, i<200) G2^T +
1e-3 N(0,1) as stored in BF16 and widened exactly to FP64 (the matrix of
record of a BF16 run), from its seeded start vector, k = 100, p = 250,
tol = 1e-10.  Calls only the oracle and the input generators.

    python tests/golden/make_workload3_sigma.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2405_18966_amd import inputs  # noqa: E402
from oracle import svds_ref  # noqa: E402


def main():
    d = inputs.config_matrix(3)
    A = d["record_bf16"]
    del d
    v0 = inputs.start_vector(A.shape[1], inputs.CONFIG_SEEDS[3] + 1)
    cfg = inputs.CONFIG_SOLVE[3]
    t0 = time.perf_counter()
    U, S, V, info = svds_ref.svds(A, cfg["k"], cfg["p"], 1e-10, 2000, v0=v0)
    dt = time.perf_counter() - t0
    r1, r2 = svds_ref.explicit_residuals(A, U, S, V)
    with open(os.path.join(HERE, "workload3_sigma_bf16.txt"), "w") as f:
        f.write("# CPU FP64 oracle, dense 20000 x 10000, G1 diag(0.95^i, i<200) G2^T + 1e-3 N(0,1),\n")
        f.write("# stored BF16 (FP64 -> FP32 RNE -> BF16 RNE) and widened exactly (matrix of record)\n")
        f.write(f"# seed {inputs.CONFIG_SEEDS[3]}, start vector seed {inputs.CONFIG_SEEDS[3] + 1}, "
                f"k={cfg['k']} p={cfg['p']} tol=1e-10\n")
        f.write(f"# cycles {info.cycles}, converged {info.converged}, max |A^T u - s v|/s "
                f"{(r2 / S).max():.3e}, oracle time {dt:.1f} s\n")
        f.write("# written by tests/golden/make_workload3_sigma.py\n")
        for s in S:
            f.write(f"{float(s)!r}\n")
    print(f"done in {dt:.1f} s, cycles {info.cycles}, res {(r2 / S).max():.3e}")


if __name__ == "__main__":
    main()
