"""GPU parity of the O(n) two-row Radic determinant (radic_det_2xn) against the
oracle: enumeration for small n, the exact Pfaffian minor-summation value for
large n, and identities of eq. (1) at sizes no enumeration reaches."""
import math

import numpy as np
import pytest

import oracle
from oracle import exact
from tests.parity import to_device

pytestmark = pytest.mark.gpu

radic = pytest.importorskip("paper_1508_01326_amd")


def run(A, what):
    print(f"[case] 2xn {what} n={np.shape(A)[1]}", flush=True)
    return radic.radic_det_2xn(to_device(A))


def cpu_bound(A):
    # sum_{j<k} (|u_j||v_k| + |u_k||v_j|) with |u| = |a_1|, |v| = |a_2|, by prefix sums
    ua, va = np.abs(A[0]), np.abs(A[1])
    Ua = np.concatenate([[0.0], np.cumsum(ua)[:-1]])
    Va = np.concatenate([[0.0], np.cumsum(va)[:-1]])
    return float(math.fsum(Ua * va) + math.fsum(Va * ua))


@pytest.mark.parametrize("n", [2, 3, 4, 17, 200, 1001])
def test_small_against_enumeration(n):
    A = np.random.default_rng(500 + n).standard_normal((2, n))
    ref = oracle.radic_f64(A)
    got = run(A, "random")
    assert got["status"] == 0 and got["n_subsets"] == math.comb(n, 2)
    assert abs(got["value"] - ref["value"]) <= 1e-12 * ref["abs_sum"]
    assert got["abs_sum"] >= ref["abs_sum"] * (1 - 1e-12)      # an upper bound on sum |det|


def test_large_against_exact_pfaffian():
    A = np.random.default_rng(501).standard_normal((2, 50000))
    ex = exact.to_float(exact.radic_pfaffian(A))
    got = run(A, "exact")
    assert abs(got["value"] - ex) <= 1e-12 * cpu_bound(A)


def test_identities_at_large_n():
    rng = np.random.default_rng(502)
    n = 3_000_000
    A = rng.standard_normal((2, n))
    base = run(A, "base")["value"]
    # rows exchanged: the sign flips
    assert abs(run(A[::-1].copy(), "rows exchanged")["value"] + base) <= 1e-14 * cpu_bound(A)
    # both rows times 2: every minor times 4, exactly
    assert run(2.0 * A, "scaled")["value"] == 4.0 * base
    # equal rows: zero (up to the double-double rounding of the cross products)
    assert abs(run(np.vstack([A[0], A[0]]), "equal rows")["value"]) <= 1e-14 * cpu_bound(np.vstack([A[0], A[0]]))
    # linear in the first row
    B = rng.standard_normal(n)
    s = run(np.vstack([A[0] + B, A[1]]), "sum row")["value"]
    t = run(np.vstack([B, A[1]]), "second term")["value"]
    assert abs(s - (base + t)) <= 1e-12 * (cpu_bound(A) + cpu_bound(np.vstack([B, A[1]])))


def test_degenerate_and_strided():
    got = run(np.ones((2, 1)), "n=1")
    assert got["value"] == 0.0 and got["status"] == 0
    base = np.random.default_rng(503).standard_normal((2, 40))
    ref = oracle.radic_f64(base[:, 5:31])
    print("[case] 2xn strided", flush=True)
    got = radic.radic_det_2xn(to_device(base)[:, 5:31])
    assert abs(got["value"] - ref["value"]) <= 1e-12 * ref["abs_sum"]
    A = np.random.default_rng(504).standard_normal((2, 9))
    A[1, 4] = np.nan
    got = run(A, "nan")
    assert got["status"] == radic.RADIC_ENONFINITE and math.isnan(got["value"])
