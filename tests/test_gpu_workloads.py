"""Full-size GPU parity on the 12 x 36 precision-stress matrix and on every
matrix of the 4096-matrix batch, against stored values that the oracle wrote
(``tests/golden/make_golden.py``): the exact Radic value of eq. (1) and the
oracle's sum |det(A_J)| for the 12 x 36 matrix, the oracle's value and sum for
each float64 matrix of the batch, the exact value for each int32 matrix.

Every case prints its identity before the GPU call so a failing run names it."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads
from tests.parity import TOL

pytestmark = pytest.mark.gpu

radic = pytest.importorskip("paper_1508_01326_amd")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_kv(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                out[k] = v
    return out


def read_batch():
    rows = {}
    with open(os.path.join(GOLDEN, "workload5_batch4096.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            p = line.split()
            b, kind, m, n = int(p[0]), p[1], int(p[2]), int(p[3])
            if kind == "f64":
                rows[b] = (kind, m, n, float(p[4]), float(p[5]))
            else:
                rows[b] = (kind, m, n, int(p[4]), None)
    return rows


@pytest.fixture(autouse=True)
def _defaults():
    radic.set_launch(0, 0)
    radic.set_fallback_tau(1.0 / 1024)
    radic.set_enumeration("auto")
    radic.set_prime_set([])
    yield
    radic.set_enumeration("auto")


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_workload4_full(precision):
    # all C(36,12) = 1,251,677,700 minors of the 12 x 36 matrix with rows scaled
    # by lognormal(0, 2) factors, through the default path of radic_det
    import torch
    g = read_kv("workload4_12x36.txt")
    exact = float(Fraction(int(g["exact_num"]), int(g["exact_den"])))
    assert exact == float(g["exact_float"])
    S = float(g["oracle_abs_sum"])
    A = workloads.single_matrix(4)
    print(f"[case] workload4 12x36 full {precision}", flush=True)
    got = radic.radic_det(torch.from_numpy(A).to("cuda"), precision=precision)
    assert got["status"] == 0
    assert got["n_subsets"] == math.comb(36, 12)
    err = abs(got["value"] - exact)
    print(f"workload4 {precision}: value {got['value']!r} exact {exact!r} err/S {err / S:.3e} "
          f"n_fallback {got['n_fallback']} ({got['n_fallback'] / got['n_subsets']:.2e} of the minors)")
    assert err <= TOL[precision] * S
    assert abs(got["abs_sum"] - S) <= 10 * TOL[precision] * S
    if precision == "fp64":
        assert got["n_fallback"] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_workload5_every_matrix(precision):
    # every one of the 4096 matrices: int32 bit-exact, float64 within tol * sum|det|
    from oracle import exact
    batch = workloads.batch_matrices()
    gold = read_batch()
    assert len(gold) == len(batch) == 4096
    mats = [A for _, A in batch]
    print(f"[case] workload5 4096 {precision}", flush=True)
    res = radic.radic_det_batched(radic.Batch(mats), precision)
    assert sum(r["n_subsets"] for r in res) == 342865835
    bad = []
    for b, (kind, A) in enumerate(batch):
        gk, m, n, val, S = gold[b]
        assert (gk, m, n) == (kind, A.shape[0], A.shape[1])
        r = res[b]
        if r["status"] != 0:
            bad.append((b, "status", r["status"]))
        elif kind == "i32":
            if r["exact"] != val:
                bad.append((b, "exact", r["exact"], val))
        else:
            if S <= 1e-9 * exact.hadamard_sum(A):
                S = exact.hadamard_sum(A)
            if not abs(r["value"] - val) <= TOL[precision] * S:
                bad.append((b, "value", r["value"], val, S))
    assert not bad, bad[:10]
