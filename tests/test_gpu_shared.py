"""GPU parity of the shared enumerations against the oracle, and against the
per-minor enumeration on the same inputs: prefix-shared (minors with equal first
m-2 columns share the first m-2 steps of their pivoted LU, each minor ends with a
2 x 2 determinant) and group-shared (equal first m-3 columns share m-3 steps,
each minor ends with a 3 x 3 determinant as a dot with a cross product).  Every
test runs under both; group-shared falls back to prefix-shared for m = 3.

Every case prints its identity before the GPU call so a failing run names it."""
import math

import numpy as np
import pytest

import oracle
from oracle import exact
import workloads
from tests.parity import TOL, assert_close, normaliser, to_device

pytestmark = pytest.mark.gpu

radic = pytest.importorskip("paper_1508_01326_amd")


@pytest.fixture(autouse=True, params=["prefix_shared", "group_shared"])
def mode(request):
    radic.set_launch(0, 0)
    radic.set_fallback_tau(1.0 / 1024)
    radic.set_enumeration(request.param)
    yield request.param
    radic.set_launch(0, 0)
    radic.set_fallback_tau(1.0 / 1024)
    radic.set_enumeration("auto")


def run(A, precision, what, **kw):
    print(f"[case] {what} shape={np.shape(A)} precision={precision}", flush=True)
    return radic.radic_det(to_device(A), precision=precision, **kw)


SHAPES = [(3, 3), (3, 4), (3, 40), (3, 130), (4, 4), (4, 17), (4, 20), (5, 14), (5, 21), (6, 13), (6, 22), (7, 16),
          (7, 19), (8, 8), (8, 17), (8, 21), (9, 18), (10, 10), (10, 16), (11, 15), (11, 17), (12, 12), (12, 16),
          (12, 17)]


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
@pytest.mark.parametrize("shape", SHAPES)
def test_random_shapes(shape, precision):
    m, n = shape
    A = workloads.random_float(m, n, seed=7000 + m * 100 + n)
    ref = oracle.radic_f64(A)
    got = run(A, precision, f"random {shape}")
    assert got["status"] == 0
    assert got["n_subsets"] == math.comb(n, m)
    S = normaliser(ref["abs_sum"], A)
    assert_close(got["value"], ref["value"], S, TOL[precision], f"value {shape} {precision}")
    assert_close(got["abs_sum"], ref["abs_sum"], ref["abs_sum"], 10 * TOL[precision], "abs_sum")
    if precision == "fp64":
        assert got["n_fallback"] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_same_as_per_minor(precision, mode):
    # both enumerations evaluate every minor; they differ in rounding only
    A = workloads.random_float(8, 24, seed=81)
    a = run(A, precision, f"{mode} 8x24")
    radic.set_enumeration("per_minor")
    b = run(A, precision, "per-minor 8x24")
    ref = oracle.radic_f64(A)
    assert_close(a["value"], b["value"], ref["abs_sum"], 2 * TOL[precision], "shared vs per-minor")
    assert_close(a["abs_sum"], b["abs_sum"], ref["abs_sum"], 10 * TOL[precision], "abs_sum")


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_workload2_full(precision):
    A = workloads.single_matrix(2)
    ref = oracle.radic_f64(A)
    got = run(A, precision, "workload2 8x32")
    assert got["n_subsets"] == 10518300
    assert_close(got["value"], ref["value"], ref["abs_sum"], TOL[precision], "workload 2")
    assert_close(got["abs_sum"], ref["abs_sum"], ref["abs_sum"], 10 * TOL[precision], "abs_sum")


def test_workload1_against_exact():
    A = workloads.single_matrix(1)
    ex = float(exact.radic_subset_dp(A))
    ref = oracle.radic_f64(A)
    for prec in ("fp64", "fp32_bulk"):
        got = run(A, prec, "workload1 5x14")
        assert_close(got["value"], ex, ref["abs_sum"], TOL[prec], "workload 1 vs exact")


def test_rank_ranges_partition():
    # cuts inside prefixes, on prefix boundaries, single ranks, the last rank
    A = workloads.random_float(6, 19, seed=83)
    total = math.comb(19, 6)
    ref = oracle.radic_f64(A)
    first_prefix_len = math.comb(19 - 4, 2)          # pairs after the prefix (0, 1, 2, 3)
    cuts = [0, 1, 7, first_prefix_len, first_prefix_len + 1, 64 * 120 + 3, total // 2, total - 2, total - 1,
            total]
    s = 0.0
    for prec in ("fp64", "fp32_bulk"):
        s = 0.0
        for a, b in zip(cuts[:-1], cuts[1:]):
            print(f"[case] shared range [{a},{b}) {prec}", flush=True)
            r = radic.radic_det_range(to_device(A), a, b - a, precision=prec)
            assert r["n_subsets"] == b - a
            part = oracle.radic_f64(A, q0=a, count=b - a)
            assert_close(r["value"], part["value"], ref["abs_sum"], TOL[prec], f"range {a} {prec}")
            s += r["value"]
        assert_close(s, ref["value"], ref["abs_sum"], 2 * TOL[prec], f"sum of ranges {prec}")


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_bitwise_reproducible(precision):
    A = workloads.random_float(7, 26, seed=84)
    r1 = run(A, precision, "repro a")
    r2 = run(A, precision, "repro b")
    assert r1["hi"] == r2["hi"] and r1["lo"] == r2["lo"] and r1["abs_sum"] == r2["abs_sum"]


@pytest.mark.parametrize("block", [64, 128, 192, 256])
def test_workgroup_sizes(block):
    A = workloads.random_float(7, 22, seed=85)
    ref = oracle.radic_f64(A)
    radic.set_launch(0, block)
    for prec in ("fp64", "fp32_bulk"):
        got = run(A, prec, f"block {block}")
        assert_close(got["value"], ref["value"], ref["abs_sum"], TOL[prec], f"block {block}")


def test_degenerate_structure():
    rng = np.random.default_rng(86)
    # a zero column: every minor holding it is 0 (zero pivot column in the prefix or the pair)
    for zc in (0, 3, 11):
        A = rng.standard_normal((5, 12))
        A[:, zc] = 0.0
        ref = oracle.radic_f64(A)
        for prec in ("fp64", "fp32_bulk"):
            got = run(A, prec, f"zero column {zc}")
            assert np.isfinite(got["value"])
            assert_close(got["value"], ref["value"], ref["abs_sum"], TOL[prec], f"zero column {zc}")
    # two equal rows: the result is 0; normalised by the Hadamard sum
    A = rng.standard_normal((6, 14))
    A[4] = A[1]
    for prec in ("fp64", "fp32_bulk"):
        got = run(A, prec, "equal rows")
        assert_close(got["value"], 0.0, exact.hadamard_sum(A), TOL[prec], "equal rows")
    # m = n and m = n - 1 against their closed forms
    for k in (3, 6, 10):
        B = rng.standard_normal((k, k))
        got = run(B, "fp64", f"square {k}")
        d = np.linalg.det(B)
        assert abs(got["value"] - d) <= 1e-12 * max(abs(d), 1.0) * 10
        C = rng.standard_normal((k, k + 1))
        got = run(C, "fp64", f"m = n - 1, {k}")
        d = np.linalg.det(np.vstack([C, np.ones((1, k + 1))]))
        ref = oracle.radic_f64(C)
        assert_close(got["value"], d, ref["abs_sum"], 1e-12, "m = n - 1")


def test_nonfinite_reported():
    A = np.random.default_rng(87).standard_normal((4, 10))
    A[2, 7] = np.inf
    for prec in ("fp64", "fp32_bulk"):
        got = run(A, prec, "inf input")
        assert got["status"] == radic.RADIC_ENONFINITE
        assert math.isnan(got["value"])


# ------------------------------------------------------------------ FP32-bulk fallback in the shared kernel
def test_fallback_forced_everywhere():
    # every minor flagged: segments overflow and whole workgroups are redone in double
    A = workloads.random_float(6, 17, seed=88)
    ref = oracle.radic_f64(A)
    radic.set_fallback_tau(float("inf"))
    got = run(A, "fp32_bulk", "tau=inf")
    assert got["n_fallback"] == math.comb(17, 6)
    assert_close(got["value"], ref["value"], ref["abs_sum"], 1e-12, "all fallback")


@pytest.mark.parametrize("m", [3, 4, 5, 6, 7, 8])
def test_fallback_forced_each_m(m):
    # every minor refactored in double by the workgroup's tail, for each m it
    # serves (eight lanes per minor, rows beyond m idle); n is the smallest with
    # at least 4096 minors, below which FP32-bulk runs the double kernel
    n = next(k for k in range(m, 200) if math.comb(k, m) >= 4096)
    A = workloads.random_float(m, n, seed=900 + m)
    ref = oracle.radic_f64(A)
    radic.set_fallback_tau(float("inf"))
    got = run(A, "fp32_bulk", f"tau=inf m={m}")
    assert got["n_fallback"] == math.comb(n, m)
    assert_close(got["value"], ref["value"], ref["abs_sum"], 1e-12, f"all fallback m={m}")
    assert_close(got["abs_sum"], ref["abs_sum"], ref["abs_sum"], 1e-12, "abs_sum")


_REF_8X40 = {}


def ref_8x40():
    # 76.9 M minors: the oracle takes a few seconds, so both modes share it
    if not _REF_8X40:
        A = workloads.random_float(8, 40, seed=99840)
        _REF_8X40["A"] = A
        _REF_8X40["ref"] = oracle.radic_f64(A)
    return _REF_8X40["A"], _REF_8X40["ref"]


def test_fallback_round_overflow():
    # 8 x 40 over the whole rank space: about 21,000 waves share the deferral
    # entries, some 200 each.  With tau = 2^-10 some rounds flag more minors
    # than that and are done again over fewer prefixes; with tau = inf every
    # round overflows, down to single prefixes whose minors (up to C(34, 2))
    # outnumber the segment and are refactored in double by lane groups.
    A, ref = ref_8x40()
    S = normaliser(ref["abs_sum"], A)
    got = run(A, "fp64", "8x40 fp64")
    assert_close(got["value"], ref["value"], S, TOL["fp64"], "8x40 fp64")
    # tau set so that the threshold of this 76.9 M-minor sum is 2^-10
    N = math.comb(40, 8)
    radic.set_fallback_tau(2.0 ** -10 * (N / 8192) ** 0.25)
    assert abs(radic.fallback_tau_for(N) - 2.0 ** -10) < 1e-15
    got = run(A, "fp32_bulk", "8x40 tau=2^-10")
    assert_close(got["value"], ref["value"], S, TOL["fp32_bulk"], "8x40 tau=2^-10")
    assert 0 < got["n_fallback"] < N // 50
    radic.set_fallback_tau(float("inf"))
    got = run(A, "fp32_bulk", "8x40 tau=inf")
    assert got["n_fallback"] == math.comb(40, 8)
    assert_close(got["value"], ref["value"], S, TOL["fp64"], "8x40 tau=inf")
    assert_close(got["abs_sum"], ref["abs_sum"], ref["abs_sum"], 1e-12, "8x40 tau=inf abs_sum")


def test_fallback_near_parallel_columns():
    rng = np.random.default_rng(89)
    A = rng.standard_normal((6, 20))
    A[:, 1] = A[:, 0] * (1.0 + 1e-7) + 1e-7 * rng.standard_normal(6)
    ref = oracle.radic_f64(A)
    got = run(A, "fp32_bulk", "near-parallel columns 0, 1")
    assert got["n_fallback"] >= math.comb(18, 4)
    assert_close(got["value"], ref["value"], ref["abs_sum"], 1e-6, "near-parallel")
    radic.set_fallback_tau(0.0)
    bad = run(A, "fp32_bulk", "near-parallel columns, no fallback")
    assert bad["n_fallback"] == 0
    print("error without fallback / S:", abs(bad["value"] - ref["value"]) / ref["abs_sum"])


def test_fallback_columns_beyond_255(mode):
    # flagged minors whose columns exceed one byte: the deferral entries must
    # carry 10-bit column indices
    rng = np.random.default_rng(90)
    for m, n, c0, c1 in ((3, 300, 280, 290), (4, 262, 256, 260)):
        A = rng.standard_normal((m, n))
        A[:, c1] = A[:, c0] * (1.0 + 1e-7) + 1e-7 * rng.standard_normal(m)
        ref = oracle.radic_f64(A)
        for md in (mode, "per_minor"):
            radic.set_enumeration(md)
            got = run(A, "fp32_bulk", f"m={m} columns {c0}, {c1} near-parallel, {md}")
            assert got["n_fallback"] >= math.comb(n - 2, m - 2)
            assert_close(got["value"], ref["value"], ref["abs_sum"], 1e-6, f"wide fallback {md}")


def test_near_dependent_rows():
    A = workloads.near_dependent_rows(7, 18, seed=91, eps=1e-6)
    ref = oracle.radic_f64(A)
    got = run(A, "fp32_bulk", "near dependent rows")
    assert got["n_fallback"] > 0
    assert_close(got["value"], ref["value"], max(ref["abs_sum"], 1e-300), 1e-5, "near-dependent")


def test_workload4_sampled_ranges(mode):
    # the 12 x 36 precision-stress matrix (C(36,12) = 1.25e9 minors) on rank
    # windows the oracle finishes quickly: start, middle, end, in both precisions
    A = workloads.single_matrix(4)
    total = math.comb(36, 12)
    for q0 in (0, total // 3 + 12345, total - 50000):
        part = oracle.radic_f64(A, q0=q0, count=50000)
        for prec in ("fp64", "fp32_bulk"):
            print(f"[case] workload4 window {q0} {prec}", flush=True)
            r = radic.radic_det_range(to_device(A), q0, 50000, precision=prec)
            assert r["n_subsets"] == 50000
            assert_close(r["value"], part["value"], part["abs_sum"], TOL[prec], f"workload 4 window {q0} {prec}")
