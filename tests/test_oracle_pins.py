"""Pins for the oracle's Radic determinant values (Definition 3, eq. (1)).

The oracle is checked against things other than itself: permutation-expansion
brute force, two independent exact evaluators (column-by-column subset DP and the
Pfaffian minor-summation formula), closed forms of special cases (m = n, m = 1,
m = 2, m = n - 1), and identities that follow from the definition (equal rows,
multilinearity, left multiplication, row exchange, zero columns).  A dropped
term, a wrong sign convention (e.g. 0-based s), a transposed operand or a wrong
pivot fails at least one of these."""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle
from oracle import exact
import workloads


def rel_close(a, b, scale, tol=1e-13):
    return abs(float(a) - float(b)) <= tol * scale


# ----------------------------------------------------------------- exact evaluators
@pytest.mark.parametrize("seed", range(12))
def test_exact_evaluators_agree_int(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 5))
    n = int(rng.integers(m, 8))
    A = rng.integers(-5, 6, size=(m, n))
    bf = exact.radic_bruteforce(A)
    assert exact.radic_subset_dp(A) == bf
    assert exact.radic_pfaffian(A) == bf


def test_pfaffian_definitions_agree():
    rng = np.random.default_rng(7)
    for k in (2, 4, 6):
        X = rng.integers(-4, 5, size=(k, k))
        S = (X - X.T).tolist()
        assert exact.pfaffian(S) == exact.pfaffian_expansion(S)
        # Pf^2 = det
        assert exact.pfaffian(S) ** 2 == exact.leibniz_det(S)


# ----------------------------------------------------------------- oracle vs exact
@pytest.mark.parametrize("seed", range(10))
def test_oracle_f64_vs_bruteforce(seed):
    rng = np.random.default_rng(100 + seed)
    m = int(rng.integers(1, 5))
    n = int(rng.integers(m, 9))
    A = rng.uniform(-1, 1, size=(m, n))
    res = oracle.radic_f64(A, nthreads=2)
    ex = exact.radic_bruteforce(A)
    assert rel_close(res["value"], ex, max(res["abs_sum"], 1e-300), 1e-13)


@pytest.mark.parametrize("shape", [(5, 14), (6, 12), (7, 15), (3, 20)])
def test_oracle_f64_vs_subset_dp(shape):
    m, n = shape
    A = workloads.random_float(m, n, seed=m * 100 + n)
    res = oracle.radic_f64(A)
    ex = exact.radic_subset_dp(A)
    assert rel_close(res["value"], ex, res["abs_sum"], 1e-13)
    assert rel_close(res["value"], exact.radic_pfaffian(A), res["abs_sum"], 1e-13)


def test_workload1_exact():
    A = workloads.single_matrix(1)
    res = oracle.radic_f64(A)
    ex = exact.radic_subset_dp(A)
    assert rel_close(res["value"], ex, res["abs_sum"], 1e-14)
    assert res["abs_sum"] <= exact.hadamard_sum(A) * (1 + 1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_oracle_int_vs_exact(seed):
    rng = np.random.default_rng(200 + seed)
    m = int(rng.integers(1, 7))
    n = int(rng.integers(m, 12))
    A = rng.integers(-50, 51, size=(m, n)).astype(np.int32)
    assert oracle.radic_int(A, nthreads=3) == exact.radic_subset_dp(A)


def test_oracle_int_large_entries():
    # int32 extremes push Bareiss intermediates far beyond 64 bits
    rng = np.random.default_rng(5)
    A = rng.integers(-2 ** 31, 2 ** 31, size=(6, 9), dtype=np.int64).astype(np.int32)
    assert oracle.radic_int(A) == exact.radic_subset_dp(A)
    A[2] = A[0]
    assert oracle.radic_int(A) == 0


def test_oracle_int_zero_pivots():
    # leading zeros force Bareiss row exchanges
    A = np.array([[0, 0, 1, 2, 3], [0, 1, 0, 4, 5], [1, 0, 0, 6, 7]], dtype=np.int32)
    assert oracle.radic_int(A) == exact.radic_bruteforce(A)


# ----------------------------------------------------------------- special cases
def test_m_equals_n_is_ordinary_det():
    rng = np.random.default_rng(11)
    for k in range(1, 9):
        A = rng.standard_normal((k, k))
        res = oracle.radic_f64(A)
        assert abs(res["value"] - np.linalg.det(A)) <= 1e-12 * max(1.0, abs(np.linalg.det(A)) * 10)


def test_one_row_alternating_sum():
    rng = np.random.default_rng(12)
    for n in (1, 2, 5, 17, 40):
        a = rng.standard_normal(n)
        expect = sum(((-1) ** j) * a[j] for j in range(n))  # a1 - a2 + a3 - ...
        assert abs(oracle.radic_f64(a[None, :])["value"] - expect) <= 1e-13 * np.abs(a).sum()
        ai = rng.integers(-9, 10, size=n)
        assert oracle.radic_int(ai[None, :].astype(np.int32)) == sum(((-1) ** j) * int(ai[j]) for j in range(n))


def test_two_rows_prefix_form():
    # m = 2: det = -sum_k (U_{k-1} v_k - V_{k-1} u_k), u_j = (-1)^j a_1j, v_j = (-1)^j a_2j (1-based)
    rng = np.random.default_rng(13)
    for n in (2, 3, 9, 30):
        A = rng.integers(-20, 21, size=(2, n))
        u = [(-1) ** j * int(A[0, j - 1]) for j in range(1, n + 1)]
        v = [(-1) ** j * int(A[1, j - 1]) for j in range(1, n + 1)]
        U = V = 0
        tot = 0
        for k in range(n):
            tot += U * v[k] - V * u[k]
            U += u[k]
            V += v[k]
        assert oracle.radic_int(A.astype(np.int32)) == -tot
        Af = A.astype(float) / 7.0
        assert abs(oracle.radic_f64(Af)["value"] - (-tot / 49.0)) <= 1e-12 * (1 + abs(tot) / 49.0)


def test_m_equals_n_minus_1_bordered():
    # Laplace along an appended row of ones: Radic(A) = det([A; 1 ... 1])
    rng = np.random.default_rng(14)
    for n in (2, 4, 7, 9):
        A = rng.integers(-9, 10, size=(n - 1, n))
        bordered = np.vstack([A, np.ones((1, n), dtype=A.dtype)])
        r = oracle.radic_int(A.astype(np.int32))
        if n <= 7:
            assert r == exact.leibniz_det(bordered.tolist())
        assert r == round(np.linalg.det(bordered))


def test_m_greater_than_n_is_zero():
    A = np.ones((4, 3))
    assert oracle.radic_f64(A)["value"] == 0.0
    assert oracle.radic_int(np.ones((4, 3), dtype=np.int32)) == 0


# ----------------------------------------------------------------- identities
def test_equal_rows_give_zero():
    rng = np.random.default_rng(15)
    A = rng.standard_normal((5, 11))
    A[3] = A[1]
    res = oracle.radic_f64(A)
    # true division makes the duplicate row exactly zero after elimination
    assert abs(res["value"]) <= 1e-14 * res["abs_sum"] + 1e-300
    Ai = rng.integers(-9, 10, size=(5, 11)).astype(np.int32)
    Ai[4] = Ai[0]
    assert oracle.radic_int(Ai) == 0


def test_multilinear_in_each_row():
    rng = np.random.default_rng(16)
    m, n = 4, 9
    base = rng.integers(-9, 10, size=(m, n))
    x = rng.integers(-9, 10, size=n)
    y = rng.integers(-9, 10, size=n)
    for i in range(m):
        Ax, Ay, Axy = base.copy(), base.copy(), base.copy()
        Ax[i], Ay[i], Axy[i] = x, y, 3 * x - 2 * y
        rx, ry, rxy = (oracle.radic_int(M.astype(np.int32)) for M in (Ax, Ay, Axy))
        assert rxy == 3 * rx - 2 * ry


def test_left_multiplication():
    # (GA)_J = G A_J, so Radic(GA) = det(G) Radic(A)
    rng = np.random.default_rng(17)
    m, n = 4, 10
    A = rng.integers(-9, 10, size=(m, n))
    G = rng.integers(-3, 4, size=(m, m))
    assert oracle.radic_int((G @ A).astype(np.int32)) == exact.leibniz_det(G.tolist()) * oracle.radic_int(A.astype(np.int32))


def test_row_exchange_flips_sign():
    rng = np.random.default_rng(18)
    A = rng.integers(-9, 10, size=(5, 10)).astype(np.int32)
    B = A[[0, 3, 2, 1, 4]]
    assert oracle.radic_int(B) == -oracle.radic_int(A)


def test_zero_columns():
    rng = np.random.default_rng(19)
    m, n = 3, 7
    A = rng.integers(-9, 10, size=(m, n)).astype(np.int32)
    z = np.zeros((m, 1), dtype=np.int32)
    r = oracle.radic_int(A)
    assert oracle.radic_int(np.hstack([A, z])) == r            # [A | 0]
    assert oracle.radic_int(np.hstack([z, A])) == (-1) ** m * r  # [0 | A]: s grows by m


def test_column_reversal():
    # reversing the columns maps j -> n+1-j and reverses each minor's columns
    rng = np.random.default_rng(20)
    for m, n in [(2, 5), (3, 7), (4, 8)]:
        A = rng.integers(-9, 10, size=(m, n)).astype(np.int32)
        expect = (-1) ** (m * (n + 1) + m * (m - 1) // 2) * oracle.radic_int(A)
        assert oracle.radic_int(np.ascontiguousarray(A[:, ::-1])) == expect


def test_power_of_two_row_scaling_exact():
    rng = np.random.default_rng(21)
    A = rng.standard_normal((5, 12))
    r = oracle.radic_f64(A)
    # every row scaled alike: pivot choices unchanged, every minor scales by 2^(5*7) exactly
    r_all = oracle.radic_f64(A * 2.0 ** 7)
    assert r_all["value"] == r["value"] * 2.0 ** 35
    assert r_all["abs_sum"] == r["abs_sum"] * 2.0 ** 35
    # one row scaled: exact in value (multilinearity) but pivots move, so within rounding
    A2 = A.copy()
    A2[2] *= 2.0 ** 40
    r2 = oracle.radic_f64(A2)
    assert abs(r2["value"] - r["value"] * 2.0 ** 40) <= 1e-13 * r2["abs_sum"]


# ----------------------------------------------------------------- ranges / threads
def test_range_partition_adds_up():
    A = workloads.random_float(6, 14, seed=3)
    total = math.comb(14, 6)
    full = oracle.radic_f64(A, nthreads=1)
    parts = [oracle.radic_f64(A, q0=a, count=b - a, nthreads=1)
             for a, b in [(0, 1000), (1000, 1001), (1001, total)]]
    s = math.fsum(p["value"] for p in parts)
    assert abs(s - full["value"]) <= 1e-14 * full["abs_sum"]
    for t in (1, 3, 8):
        assert abs(oracle.radic_f64(A, nthreads=t)["value"] - full["value"]) <= 1e-14 * full["abs_sum"]


def test_subset_terms_sum_to_total():
    A = workloads.random_float(4, 9, seed=4)
    total = math.comb(9, 4)
    terms = [oracle.subset_term_f64(A, q)[0] for q in range(total)]
    assert abs(math.fsum(terms) - oracle.radic_f64(A)["value"]) <= 1e-14 * sum(abs(t) for t in terms)
    Ai = workloads.random_int(4, 9, seed=4)
    assert sum(oracle.subset_term_int(Ai, q) for q in range(total)) == oracle.radic_int(Ai)


def test_int_oracle_threads_and_ranges():
    Ai = workloads.random_int(5, 13, seed=9)
    total = math.comb(13, 5)
    full = oracle.radic_int(Ai, nthreads=1)
    assert oracle.radic_int(Ai, nthreads=7) == full
    assert oracle.radic_int(Ai, q0=0, count=500) + oracle.radic_int(Ai, q0=500, count=total - 500) == full
