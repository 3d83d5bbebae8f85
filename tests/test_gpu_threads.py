"""Synchronous calls from several host threads at once: each float call reads
its result from its thread's pinned buffer, each exact call from a pinned
buffer of the library's pool, and no call may see another's result."""
import math
import threading

import numpy as np
import pytest

import oracle
import workloads
from tests.parity import TOL, assert_close, to_device

pytestmark = pytest.mark.gpu

radic = pytest.importorskip("paper_1508_01326_amd")

ROUNDS = 12


def _run_threads(jobs):
    errors = []

    def worker(job):
        try:
            job()
        except BaseException as e:   # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(j,)) for j in jobs]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads), "a thread did not finish"
    if errors:
        raise errors[0]


def test_float_sync_calls_from_threads():
    cases = [workloads.random_float(m, n, seed=700 + m * 10 + n) for (m, n) in ((5, 14), (6, 16), (7, 17), (4, 20))]
    refs = [oracle.radic_f64(A) for A in cases]

    def job_for(k):
        A, ref = cases[k], refs[k]

        def job():
            dA = to_device(A)
            for r in range(ROUNDS):
                prec = "fp64" if (r + k) % 2 == 0 else "fp32_bulk"
                got = radic.radic_det(dA, precision=prec)
                assert_close(got["value"], ref["value"], ref["abs_sum"], TOL[prec], f"thread {k} round {r} {prec}")
                assert got["n_subsets"] == math.comb(A.shape[1], A.shape[0])
        return job

    print("[case] float sync calls from 4 threads", flush=True)
    _run_threads([job_for(k) for k in range(len(cases))])


def test_exact_calls_from_threads():
    cases = [workloads.random_int(m, n, seed=800 + m * 10 + n, lo=-40, hi=40) for (m, n) in ((5, 14), (6, 12), (4, 18))]
    refs = [oracle.radic_int(A) for A in cases]

    def job_for(k):
        A, ref = cases[k], refs[k]

        def job():
            dA = to_device(np.ascontiguousarray(A, dtype=np.int32))
            for r in range(ROUNDS):
                assert radic.radic_det_int_exact(dA) == ref, f"thread {k} round {r}"
        return job

    print("[case] exact calls from 3 threads", flush=True)
    _run_threads([job_for(k) for k in range(len(cases))])
