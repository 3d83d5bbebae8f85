"""Writes the stored expected values for the full-size GPU parity tests of the
12 x 36 workload and the 4096-matrix batch.  It calls only the oracle
(``oracle/``: the FP64 enumerator, the exact subset dynamic program and the
Pfaffian minor-summation formula) and the seeded input generators; nothing
here touches the GPU library.

    python tests/golden/make_golden.py [--threads T] [--only 4|5]

workload4_12x36.txt
    The exact Radic value (Definition 3, eq. (1)) of the 12 x 36 matrix, as a
    reduced fraction and rounded to double, from the subset dynamic program
    (checked equal to the Pfaffian formula), and the FP64 oracle's value and
    sum |det(A_J)| over all C(36,12) = 1,251,677,700 minors.
workload5_batch4096.txt
    One line per matrix of the batch: index, kind, m, n, then for float64
    matrices the FP64 oracle's value and sum |det(A_J)|, for int32 matrices the
    exact value from the subset dynamic program.
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import exact  # noqa: E402
import workloads  # noqa: E402

W4 = os.path.join(HERE, "workload4_12x36.txt")
W5 = os.path.join(HERE, "workload5_batch4096.txt")


def make_w4(threads):
    A = workloads.single_matrix(4)
    ex = exact.radic_subset_dp(A)
    pf = exact.radic_pfaffian(A)
    if ex != pf:
        raise SystemExit("subset DP and Pfaffian formula disagree")
    t0 = time.time()
    r = oracle.radic_f64(A, nthreads=threads)
    dt = time.time() - t0
    with open(W4, "w") as f:
        f.write("# Radic determinant of the 12 x 36 workload: float64 N(0,1) entries times a per-row\n"
                "# lognormal(0, 2) scale, seed 150801330 (workloads.single_matrix(4)).\n"
                "# Written by tests/golden/make_golden.py from the oracle only.\n"
                "# exact_*: subset dynamic program over rows, equal to the Pfaffian minor-summation value.\n"
                f"# oracle_*: FP64 enumeration of all 1251677700 minors ({threads} threads, {dt:.0f} s).\n")
        f.write(f"exact_num {ex.numerator}\n")
        f.write(f"exact_den {ex.denominator}\n")
        f.write(f"exact_float {float(ex)!r}\n")
        f.write(f"oracle_value {r['value']!r}\n")
        f.write(f"oracle_abs_sum {r['abs_sum']!r}\n")
    print(f"wrote {W4} ({dt:.0f} s oracle)")


def make_w5(threads):
    mats = workloads.batch_matrices()
    t0 = time.time()
    with open(W5, "w") as f:
        f.write("# Radic determinants of the 4096-matrix batch (workloads.batch_matrices(), seed 150801331).\n"
                "# Written by tests/golden/make_golden.py from the oracle only.\n"
                "# f64 lines: index f64 m n oracle_value oracle_abs_sum (FP64 enumeration)\n"
                "# i32 lines: index i32 m n exact_value (subset dynamic program)\n")
        for b, (kind, M) in enumerate(mats):
            m, n = M.shape
            if kind == "f64":
                r = oracle.radic_f64(M, nthreads=threads)
                f.write(f"{b} f64 {m} {n} {r['value']!r} {r['abs_sum']!r}\n")
            else:
                f.write(f"{b} i32 {m} {n} {exact.radic_subset_dp(M)}\n")
    print(f"wrote {W5} ({time.time() - t0:.0f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=min(os.cpu_count() or 1, 16))
    ap.add_argument("--only", type=int, choices=[4, 5])
    args = ap.parse_args()
    if args.only in (None, 5):
        make_w5(args.threads)
    if args.only in (None, 4):
        make_w4(args.threads)


if __name__ == "__main__":
    main()
