"""Pins for the oracle's signed accumulation and its sum of |det(A_J)|.

Definition 3, eq. (1) is a sum of C(n, m) signed minors with heavy cancellation
(Section 6 sums them by a tree).  The oracle adds the terms by Neumaier's
compensated summation (A. Neumaier, ZAMM 54, 1974; N. J. Higham, Accuracy and
Stability of Numerical Algorithms, 2nd ed., section 4.3).  These tests check that
sum against things other than itself:

* inputs whose every minor the oracle's elimination computes exactly (each
  column has a single nonzero entry, a signed power of two), with two equal
  adjacent columns of size 2^80 whose terms cancel exactly; the exact value
  comes from the subset dynamic program of ``exact.py`` and plain left-to-right
  summation of the same terms provably misses it;
* the workload-size 8 x 32 matrix: the oracle's total against ``math.fsum`` (a
  correctly rounded sum) of the very terms it adds, within the error bound of
  Neumaier's algorithm computed from the running sums;
* the sum of |det(A_J)| against the exact sum of |Leibniz minor| (Fractions).

Error bound used (derived from the algorithm, valid for any data): with t_i the
running sums, e_i the exact rounding error of step i (|e_i| <= u |t_i|, captured
exactly by the branch of the algorithm) and the compensation c the plainly
summed e_i, the returned fl(s + c) differs from the exact sum S by at most
u |S| + (1 + u) gamma_{N-1} u sum_i |t_i|, gamma_k = k u / (1 - k u).  With
several threads (contiguous rank chunks, Section 5) each chunk's pair (s, c)
carries its own compensation error, and the merge of the 2T chunk values is a
second compensated sum whose running sums are each at most sum |x_i| (1 + 2u).
"""
import math
from fractions import Fraction
from itertools import combinations

import numpy as np
import pytest

import oracle
from oracle import exact
import workloads

U = 2.0 ** -53


def gamma(k):
    return k * U / (1 - k * U)


def neumaier_bound(S, running_abs_sum, N):
    """Bound on |computed - S| for one compensated pass over N terms whose running
    sums have absolute values summing to running_abs_sum."""
    return U * abs(S) + (1 + U) * gamma(max(N - 1, 1)) * U * running_abs_sum


def running_abs(terms):
    # np.cumsum adds left to right, so it reproduces the running sums t_i exactly
    return float(np.abs(np.cumsum(terms)).sum())


def chunked_bound(terms, threads, S):
    """Bound on |computed - S| when `threads` contiguous chunks are summed each by
    one compensated pass and their (s, c) pairs merged by another."""
    N = len(terms)
    tot = U * abs(S)
    abs_x = float(np.abs(terms).sum())
    for k in range(threads):
        a, b = (N * k) // threads, (N * (k + 1)) // threads
        if b > a:
            tot += (1 + U) * gamma(max(b - a - 1, 1)) * U * running_abs(terms[a:b])
    M = 2 * threads
    tot += (1 + U) * gamma(M) * U * M * abs_x * (1 + 2 * U)
    return tot


def monomial_matrix(m, n, seed, big=80):
    """Every column has one nonzero entry, a signed power of two, in a random row;
    columns 1 and 2 hold 2^80 in the same row.  Elimination with partial pivoting
    is exact on every minor (each pivot column has one nonzero; every multiplier
    is 0/pivot = 0), so each term is the exact product of powers of two.  A minor
    with column 1 and its partner with column 2 instead (same position, s one
    larger) have exactly opposite terms, and both are far from each other in the
    dictionary order, with small terms in between."""
    rng = np.random.default_rng(workloads.SEED_BASE + 4000 + seed)
    rows = rng.integers(0, m, size=n)
    exps = rng.integers(-12, 13, size=n)
    sg = rng.choice([-1.0, 1.0], size=n)
    A = np.zeros((m, n))
    for j in range(n):
        A[rows[j], j] = sg[j] * 2.0 ** exps[j]
    r = int(rng.integers(0, m))
    A[:, 1] = 0.0
    A[:, 2] = 0.0
    A[r, 1] = A[r, 2] = 2.0 ** big
    return A


CANCEL_CASES = [(2, 30, 0), (3, 16, 3), (4, 18, 0), (5, 20, 2), (3, 12, 1)]


def check_cancellation(radic_f64, A):
    """The compensated total of an exactly-termed, heavily cancelling input."""
    m, n = A.shape
    terms = oracle.subset_terms_f64(A)
    S = exact.radic_subset_dp(A)
    # every term is exact: their exact sum is the exact Radic value
    assert sum(Fraction(float(t)) for t in terms) == S
    Sf = float(S)
    N = len(terms)
    # the input has teeth: plain left-to-right summation violates the bound
    plain = 0.0
    for t in terms:
        plain += float(t)
    one_pass = neumaier_bound(Sf, running_abs(terms), N)
    assert abs(plain - Sf) > 10 * one_pass, "input not hard enough for plain summation"
    for threads in (1, 3, 8):
        got = radic_f64(A, nthreads=threads)["value"]
        bound = one_pass if threads == 1 else chunked_bound(terms, threads, Sf)
        assert abs(got - Sf) <= bound, (A.shape, threads, got, Sf, bound)


def exact_abs_sum(A):
    """sum_J |det(A_J)| in exact rational arithmetic (Leibniz expansion per minor)."""
    rows = [[Fraction(float(x)) for x in row] for row in np.asarray(A)]
    m, n = len(rows), len(rows[0])
    tot = Fraction(0)
    for J in combinations(range(n), m):
        tot += abs(exact.leibniz_det([[rows[i][j] for j in J] for i in range(m)]))
    return tot


ABS_CASES = [(2, 9, 0), (3, 8, 1), (4, 9, 2), (3, 11, 3), (1, 12, 4)]


def check_abs_sum(radic_f64, A):
    ref = float(exact_abs_sum(A))
    got = radic_f64(A, nthreads=2)["abs_sum"]
    # each |minor| carries the elimination's relative error (a few m u for these
    # well-scaled random inputs); the positive terms then add with no cancellation
    assert abs(got - ref) <= 1e-13 * ref, (A.shape, got, ref)


def check_workload2_summation(radic_f64, A, terms, fs, run_abs):
    got = radic_f64(A, nthreads=1)
    bound = neumaier_bound(fs, run_abs, len(terms))
    assert abs(got["value"] - fs) <= bound, (got["value"], fs, bound)
    # hi + lo is the unevaluated compensated pair: rounding it gives value
    assert got["hi"] + got["lo"] == got["value"]


# ----------------------------------------------------------------- tests
@pytest.mark.parametrize("m,n,seed", CANCEL_CASES)
def test_compensated_sum_exact_terms(m, n, seed):
    check_cancellation(oracle.radic_f64, monomial_matrix(m, n, seed))


@pytest.mark.parametrize("m,n,seed", ABS_CASES)
def test_abs_sum_matches_exact(m, n, seed):
    A = workloads.random_float(m, n, seed=500 + seed)
    check_abs_sum(oracle.radic_f64, A)


def test_abs_sum_with_cancellation():
    # sum |det| keeps growing while the signed sum cancels: a signed or an
    # |total| stand-in for it would be far off
    A = monomial_matrix(3, 12, 2)
    terms = oracle.subset_terms_f64(A)
    ref = sum(abs(Fraction(float(t))) for t in terms)
    got = oracle.radic_f64(A, nthreads=2)
    assert got["abs_sum"] == float(ref)   # positive exact terms, far from cancellation
    assert got["abs_sum"] > 1e6 * abs(got["value"])


@pytest.fixture(scope="module")
def workload2_terms():
    A = workloads.single_matrix(2)
    terms = oracle.subset_terms_f64(A)
    return A, terms, math.fsum(terms), running_abs(terms)


def test_workload2_terms_sum_to_exact(workload2_terms):
    # the terms the oracle adds: their correctly rounded sum lies within the
    # elimination's per-minor error of the exact value (subset DP), and
    # their absolute values add up to the oracle's sum |det|
    A, terms, fs, _ = workload2_terms
    assert len(terms) == math.comb(32, 8)
    ex = float(exact.radic_subset_dp(A))
    S_abs = math.fsum(np.abs(terms))
    assert abs(fs - ex) <= 1e-15 * S_abs
    got = oracle.radic_f64(A)
    assert abs(got["abs_sum"] - S_abs) <= 4 * U * S_abs


def test_workload2_compensated_total(workload2_terms):
    A, terms, fs, run_abs = workload2_terms
    check_workload2_summation(oracle.radic_f64, A, terms, fs, run_abs)
    # the bound is tight enough to matter: plain summation of the same terms
    # (the running sums themselves) misses it
    plain = float(np.cumsum(terms)[-1])
    assert abs(plain - fs) > 10 * neumaier_bound(fs, run_abs, len(terms))


def test_workload2_threads_agree(workload2_terms):
    # contiguous rank chunks (Section 5) merged in rank order: every thread count
    # lands within the bound of the correctly rounded total
    A, terms, fs, _ = workload2_terms
    for t in (2, 8, 16):
        got = oracle.radic_f64(A, nthreads=t)["value"]
        assert abs(got - fs) <= chunked_bound(terms, t, fs), t
