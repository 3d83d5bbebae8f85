"""GPU parity of the floating-point Radic determinant against the oracle.

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


@pytest.fixture(autouse=True)
def _reset_launch():
    radic.set_launch(0, 0)
    radic.set_fallback_tau(1.0 / 1024)
    yield
    radic.set_launch(0, 0)
    radic.set_fallback_tau(1.0 / 1024)


SHAPES = [(1, 1), (1, 7), (1, 200), (2, 2), (2, 9), (2, 150), (3, 3), (3, 20), (4, 17), (5, 14), (5, 21),
          (6, 13), (6, 18), (7, 16), (7, 19), (8, 8), (8, 17), (8, 20), (9, 18), (10, 16), (11, 15), (11, 17),
          (12, 12), (12, 15), (12, 17)]

# The per-minor enumeration (every minor unranked or advanced and factored on its
# own by one lane: Sections 4-6) and the automatic choice (prefix-shared where it
# applies) are both compared with the oracle.
ENUMS = ["per_minor", "auto"]


@pytest.fixture(params=ENUMS)
def enum(request):
    radic.set_enumeration(request.param)
    yield request.param
    radic.set_enumeration("auto")


def run_case(A, precision, what):
    print(f"[case] {what} shape={A.shape} precision={precision}", flush=True)
    return radic.radic_det(to_device(A), precision=precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
@pytest.mark.parametrize("shape", SHAPES)
def test_random_shapes(shape, precision, enum):
    m, n = shape
    A = workloads.random_float(m, n, seed=m * 1000 + n)
    ref = oracle.radic_f64(A)
    got = run_case(A, precision, f"random {shape}")
    assert got["status"] == 0
    assert got["n_subsets"] == math.comb(n, m)
    S = normaliser(ref["abs_sum"], A)
    assert_close(got["value"], ref["value"], S, TOL[precision], f"value {shape} {precision}")
    assert_close(got["abs_sum"], ref["abs_sum"], ref["abs_sum"], TOL[precision] * 10, "abs_sum")
    if precision == "fp64":
        assert got["n_fallback"] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_workload1_exact(precision):
    A = workloads.single_matrix(1)
    ref = oracle.radic_f64(A)
    ex = float(exact.radic_subset_dp(A))
    got = run_case(A, precision, "workload1 5x14")
    assert_close(got["value"], ex, ref["abs_sum"], TOL[precision], "workload 1 vs exact")


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_workload2_full(precision, enum):
    A = workloads.single_matrix(2)
    ref = oracle.radic_f64(A)
    got = run_case(A, precision, f"workload2 8x32 {enum}")
    assert got["n_subsets"] == 10518300
    assert_close(got["value"], ref["value"], ref["abs_sum"], TOL[precision], "workload 2")
    assert_close(got["abs_sum"], ref["abs_sum"], ref["abs_sum"], 10 * TOL[precision], "abs_sum")


def test_subset_terms_and_columns(golden):
    # exported terms against the oracle term by term, columns against Table 2
    import torch
    A = workloads.random_float(5, 8, seed=77)
    print("[case] export 5x8", flush=True)
    terms, cols = radic.radic_det_subsets(to_device(A), 0, 56, precision="fp64", with_cols=True)
    for r in golden("table2_subsets_n8_m5.txt"):
        q = int(r[0])
        assert list(cols[q]) == [int(x) for x in r[1:]]
        t, _ = oracle.subset_term_f64(A, q)
        assert abs(terms[q] - t) <= 1e-13 * (abs(t) + 1e-300) + 1e-15
    # a ragged window of a larger space, both precisions: every exported term
    # against the oracle's, within the rounding bound of its precision relative
    # to the minor's Hadamard bound on the power-of-two row-scaled matrix
    # (prod_j ||column j||_2 of 2^-e_i A_J, times 2^(sum e_i)): m^2 u for the
    # elimination of an m x m minor with modest growth, u = 2^-53 or 2^-24
    B = workloads.random_float(8, 32, seed=5)
    total = math.comb(32, 8)
    e = np.array([math.frexp(float(np.abs(row).max()))[1] for row in B])
    Bs = B * np.ldexp(1.0, -e)[:, None]
    q0, cnt = total // 3 + 17, 1001
    for prec, u in (("fp64", 2.0 ** -53), ("fp32_bulk", 2.0 ** -24)):
        print(f"[case] export 8x32 window {prec}", flush=True)
        terms, cols = radic.radic_det_subsets(to_device(B), q0, cnt, precision=prec, with_cols=True)
        worst = 0.0
        for k in range(cnt):
            t, J = oracle.subset_term_f64(B, q0 + k)
            assert list(cols[k]) == J
            H = float(np.prod(np.linalg.norm(Bs[:, [j - 1 for j in J]], axis=0))) * 2.0 ** int(e.sum())
            err = abs(terms[k] - t)
            worst = max(worst, err / (u * H))
            assert err <= 64 * u * H, (k, terms[k], t, H)
        print(f"{prec}: largest |term error| / (u * Hadamard bound) = {worst:.2f}")


def test_rank_ranges_partition(enum):
    A = workloads.random_float(7, 19, seed=3)
    total = math.comb(19, 7)
    ref = oracle.radic_f64(A)
    cuts = [0, 1, 63, 64 * 8 + 5, total // 2, total - 1, total]
    s = 0.0
    for a, b in zip(cuts[:-1], cuts[1:]):
        print(f"[case] range [{a},{b})", flush=True)
        r = radic.radic_det_range(to_device(A), a, b - a)
        assert r["n_subsets"] == b - a
        part = oracle.radic_f64(A, q0=a, count=b - a)
        assert_close(r["value"], part["value"], ref["abs_sum"], 1e-12, f"range {a}")
        s += r["value"]
    assert_close(s, ref["value"], ref["abs_sum"], 1e-12, "sum of ranges")


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_bitwise_reproducible(precision):
    A = workloads.random_float(8, 24, seed=11)
    r1 = run_case(A, precision, "repro a")
    r2 = run_case(A, precision, "repro b")
    assert r1["hi"] == r2["hi"] and r1["lo"] == r2["lo"] and r1["abs_sum"] == r2["abs_sum"]


@pytest.mark.parametrize("spl,block", [(1, 64), (3, 128), (16, 256), (5, 192)])
def test_launch_shapes(spl, block, enum):
    # spl (ranks per lane chunk) sets the per-minor mapping; the workgroup size applies to every mapping
    A = workloads.random_float(6, 22, seed=12)
    ref = oracle.radic_f64(A)
    radic.set_launch(spl, block)
    for prec in ("fp64", "fp32_bulk"):
        got = run_case(A, prec, f"launch spl={spl} block={block}")
        assert_close(got["value"], ref["value"], ref["abs_sum"], TOL[prec], f"launch {spl},{block}")


def test_degenerate_inputs():
    import torch
    # m > n: zero by Definition 3
    got = run_case(np.ones((4, 3)), "fp64", "m>n")
    assert got["value"] == 0.0 and got["status"] == 0
    # m == n: the ordinary determinant
    rng = np.random.default_rng(3)
    for k in (1, 2, 5, 9, 12):
        A = rng.standard_normal((k, k))
        for prec in ("fp64", "fp32_bulk"):
            got = run_case(A, prec, f"square {k}")
            d = np.linalg.det(A)
            assert abs(got["value"] - d) <= TOL[prec] * max(abs(d), 1.0) * 10
    # one row: alternating sum
    a = rng.standard_normal((1, 33))
    got = run_case(a, "fp64", "one row")
    assert abs(got["value"] - sum((-1) ** j * a[0, j] for j in range(33))) <= 1e-13 * np.abs(a).sum()
    # an all-zero column and two equal rows
    A = rng.standard_normal((5, 12))
    A[:, 4] = 0.0
    ref = oracle.radic_f64(A)
    for prec in ("fp64", "fp32_bulk"):
        got = run_case(A, prec, "zero column")
        assert_close(got["value"], ref["value"], ref["abs_sum"], TOL[prec], "zero column")
    A = rng.standard_normal((5, 12))
    A[3] = A[1]
    for prec in ("fp64", "fp32_bulk"):
        got = run_case(A, prec, "equal rows")
        assert_close(got["value"], 0.0, exact.hadamard_sum(A), TOL[prec], "equal rows")


def test_nonfinite_input_reported():
    A = np.random.default_rng(4).standard_normal((3, 9))
    A[1, 5] = np.nan
    for prec in ("fp64", "fp32_bulk"):
        got = run_case(A, prec, "nan input")
        assert got["status"] == radic.RADIC_ENONFINITE
        assert math.isnan(got["value"])
    A[1, 5] = np.inf
    got = run_case(A, "fp64", "inf input")
    assert got["status"] == radic.RADIC_ENONFINITE


def test_strided_matrix():
    import torch
    base = workloads.random_float(6, 30, seed=21)
    A = to_device(base)[:, 3:20]      # lda = 30, n = 17
    ref = oracle.radic_f64(base[:, 3:20])
    print("[case] strided 6x17 lda 30", flush=True)
    got = radic.radic_det(A)
    assert_close(got["value"], ref["value"], ref["abs_sum"], 1e-12, "strided")


# ------------------------------------------------------------------ FP32-bulk fallback
def test_fallback_forced_everywhere_is_fp64_accurate():
    # tau = +inf refactors every minor in double (wave-cooperative LU)
    A = workloads.random_float(6, 15, seed=31)
    ref = oracle.radic_f64(A)
    radic.set_fallback_tau(float("inf"))
    got = run_case(A, "fp32_bulk", "tau=inf")
    assert got["n_fallback"] == math.comb(15, 6)
    assert_close(got["value"], ref["value"], ref["abs_sum"], 1e-12, "all fallback")


def test_fallback_disabled():
    A = workloads.random_float(6, 15, seed=32)
    ref = oracle.radic_f64(A)
    radic.set_fallback_tau(0.0)
    got = run_case(A, "fp32_bulk", "tau=0")
    assert got["n_fallback"] == 0
    assert_close(got["value"], ref["value"], ref["abs_sum"], 1e-5, "no fallback")


def test_fallback_near_dependent_rows():
    # rows 0 and m-1 nearly equal: every minor nearly singular, float LU loses
    # most digits; the fallback must catch them
    A = workloads.near_dependent_rows(6, 16, seed=33, eps=1e-6)
    ref = oracle.radic_f64(A)
    got = run_case(A, "fp32_bulk", "near dependent rows")
    assert got["n_fallback"] > 0
    S = max(ref["abs_sum"], 1e-300)
    assert_close(got["value"], ref["value"], S, 1e-5, "near-dependent")
    radic.set_fallback_tau(0.0)
    bad = run_case(A, "fp32_bulk", "near dependent rows, no fallback")
    print("error without fallback / S:", abs(bad["value"] - ref["value"]) / S)


@pytest.mark.parametrize("m,n,eps", [(6, 16, 1e-3), (7, 20, 3e-4), (7, 20, 1e-3), (8, 24, 1e-4), (9, 24, 3e-4),
                                     (8, 32, 1e-4)])
def test_fallback_uniformly_ill_conditioned(m, n, eps):
    # a row near another makes every minor about eps-conditioned, so the float
    # errors are not small against sum |det| as for random minors: the
    # threshold (scaled for the minor count) must still refactor enough of them
    A = workloads.near_dependent_rows(m, n, seed=40 + m + n, eps=eps)
    ref = oracle.radic_f64(A)
    got = run_case(A, "fp32_bulk", f"ill-conditioned {m}x{n} eps={eps:g}")
    S = max(ref["abs_sum"], 1e-300)
    err = abs(got["value"] - ref["value"]) / S
    print(f"error / S = {err:.2e}, refactored {got['n_fallback']} of {math.comb(n, m)}")
    assert err <= 1e-5


def test_fallback_overflow_in_some_workgroups(enum):
    # columns 1 and 2 nearly parallel: every minor holding both (the first
    # C(18, 4) ranks of the dictionary order) is flagged, so the waves that own
    # them overflow their deferral segment and their workgroups are redone in
    # double, while the rest keep the float result plus a few deferred minors
    rng = np.random.default_rng(34)
    A = rng.standard_normal((6, 20))
    A[:, 1] = A[:, 0] * (1.0 + 1e-7) + 1e-7 * rng.standard_normal(6)
    ref = oracle.radic_f64(A)
    got = run_case(A, "fp32_bulk", "partial overflow 6x20")
    assert math.comb(18, 4) <= got["n_fallback"] < math.comb(20, 6)
    assert_close(got["value"], ref["value"], ref["abs_sum"], 1e-6, "partial overflow")
    for spl, block in ((1, 64), (32, 256)):
        radic.set_launch(spl, block)
        got = run_case(A, "fp32_bulk", f"partial overflow spl={spl} block={block}")
        assert_close(got["value"], ref["value"], ref["abs_sum"], 1e-6, "partial overflow launch")


def test_row_scaling_wide_range():
    # rows spanning ~1e+-30: float would overflow without the power-of-two row scaling
    rng = np.random.default_rng(41)
    A = rng.standard_normal((10, 14)) * (10.0 ** rng.uniform(-30, 30, size=(10, 1)))
    ref = oracle.radic_f64(A)
    got = run_case(A, "fp32_bulk", "wide row scales")
    assert np.isfinite(got["value"])
    assert_close(got["value"], ref["value"], ref["abs_sum"], 1e-5, "row scaling")


def test_autotune_det_then_correct():
    radic.set_launch(0, 0)
    print("[case] autotune det 6x16", flush=True)
    spl, block = radic.autotune(radic.RADIC_WS_DET, 6, 16, "fp64")
    assert spl >= 1 and block in (64, 128, 256)
    A = workloads.random_float(6, 16, seed=90)
    ref = oracle.radic_f64(A)
    got = run_case(A, "fp64", "after autotune")
    assert_close(got["value"], ref["value"], ref["abs_sum"], 1e-12, "autotuned")


@pytest.mark.parametrize("shape", [(8, 8), (10, 10), (5, 12), (6, 13), (3, 30)])
def test_fp32_bulk_few_minors_in_double(shape, enum):
    # a sum over fewer than 4096 minors cannot absorb a float minor's error (up
    # to about u_f times its condition) within 1e-5 sum |det|: FP32-bulk
    # refactors every such minor in double, so the result has FP64 accuracy
    m, n = shape
    A = workloads.random_float(m, n, seed=9100 + m * 100 + n, dist="uniform")
    ref = oracle.radic_f64(A)
    got = run_case(A, "fp32_bulk", f"few minors {shape} {enum}")
    assert got["n_fallback"] == math.comb(n, m)
    assert_close(got["value"], ref["value"], normaliser(ref["abs_sum"], A), 1e-12, f"few minors {shape}")
