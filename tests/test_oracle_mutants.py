"""The summation pins have teeth: copies of the oracle with a planted mistake in
its signed accumulation or its sum |det(A_J)| (Definition 3, eq. (1); the tree
sum of Section 6) are built on the CPU and each fails at least one pin of
``test_oracle_summation``.  The real oracle is untouched; every mutant is a
text edit of its source compiled into a temporary directory."""
import ctypes
import os

import numpy as np
import pytest

import oracle
from oracle import build as oracle_build
from tests import test_oracle_summation as pins
import workloads

with open(oracle_build.SRC) as _f:
    SOURCE = _f.read()

# (name, original text, planted text)
MUTANTS = [
    ("compensation dropped",
     "    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;\n    else a->c += (x - t) + a->s;\n", ""),
    ("value is the running sum only", "    out[0] = val.s + val.c;", "    out[0] = val.s;"),
    ("chunk compensation not merged", "        nsum_add(&val, jobs[t].val.c);\n", ""),
    ("abs sum of signed terms", "nsum_add(&jb->abs, fabs(d));", "nsum_add(&jb->abs, radic_sign(B, jb->m) * d);"),
    ("abs sum replaced by |value|", "    out[3] = ab.s + ab.c;", "    out[3] = fabs(out[0]);"),
]


def build_mutant(tmp_path, name, old, new):
    assert SOURCE.count(old) == 1, f"mutation site for '{name}' not found exactly once"
    src = tmp_path / "mutant.c"
    src.write_text(SOURCE.replace(old, new))
    out = str(tmp_path / "libmutant.so")
    oracle_build.build(src=str(src), out=out)
    L = ctypes.CDLL(out)
    dp = ctypes.POINTER(ctypes.c_double)
    L.oracle_radic_f64_range.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                                         ctypes.c_uint64, ctypes.c_int, dp]
    L.oracle_radic_f64_range.restype = ctypes.c_int

    def radic_f64(A, nthreads=1):
        A = np.ascontiguousarray(A, dtype=np.float64)
        m, n = A.shape
        o = (ctypes.c_double * 4)()
        rc = L.oracle_radic_f64_range(A.ctypes.data_as(dp), m, n, n, 0, 0, nthreads, o)
        assert rc == 0
        return {"value": o[0], "hi": o[1], "lo": o[2], "abs_sum": o[3]}

    return radic_f64


def first_failing_pin(radic_f64):
    for m, n, seed in pins.CANCEL_CASES:
        try:
            pins.check_cancellation(radic_f64, pins.monomial_matrix(m, n, seed))
        except AssertionError:
            return f"cancellation {m}x{n} seed {seed}"
    for m, n, seed in pins.ABS_CASES:
        try:
            pins.check_abs_sum(radic_f64, workloads.random_float(m, n, seed=500 + seed))
        except AssertionError:
            return f"abs sum {m}x{n} seed {seed}"
    return None


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, old, new):
    radic_f64 = build_mutant(tmp_path, name, old, new)
    caught = first_failing_pin(radic_f64)
    assert caught is not None, f"mutant '{name}' passes every summation pin"
    print(f"mutant '{name}' caught by: {caught}")


def test_unmutated_copy_passes(tmp_path):
    # the harness itself: the unchanged source built the same way passes every pin
    radic_f64 = build_mutant(tmp_path, "none", "    out[0] = val.s + val.c;", "    out[0] = val.s + val.c;")
    assert first_failing_pin(radic_f64) is None


def test_uncompensated_fails_workload2(tmp_path):
    # at the 8 x 32 workload size the bound of the compensated sum separates the
    # oracle from plain summation of the same terms
    name, old, new = MUTANTS[0]
    radic_f64 = build_mutant(tmp_path, name, old, new)
    A = workloads.single_matrix(2)
    terms = oracle.subset_terms_f64(A)
    import math
    fs = math.fsum(terms)
    with pytest.raises(AssertionError):
        pins.check_workload2_summation(radic_f64, A, terms, fs, pins.running_abs(terms))
