"""GPU tests of two pieces around the enumeration kernels: the library's timing
hook (HIP events bound to the main kernel's dispatch) and the order in which
whole-matrix prefix-shared launches take their blocks (colex order of the
prefixes, heaviest first, computed by the kernel itself).

Timing must not change what is computed; the block order must give the same
bits on every call of a shape, eager or replayed from a captured graph (even
when the capture is the shape's first call), and results that agree with the
oracle and with range calls (which keep dictionary order).

Every case prints its identity before the GPU call so a failing run names it."""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests.parity import TOL, assert_close, normaliser, to_device

pytestmark = pytest.mark.gpu

radic = pytest.importorskip("paper_1508_01326_amd")


@pytest.fixture(autouse=True)
def defaults():
    radic.set_launch(0, 0)
    radic.set_fallback_tau(1.0 / 1024)
    radic.set_enumeration("auto")
    radic.profile_enable(False)
    radic.profile_read_launches()
    yield
    radic.profile_enable(False)
    radic.profile_read_launches()


KEYS = ("value", "hi", "lo", "abs_sum", "n_subsets", "n_fallback", "status")


def bits(r):
    return tuple(r[k] for k in KEYS)


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_profile_times_each_call_and_changes_nothing(precision):
    A = to_device(workloads.single_matrix(2))   # 8 x 32: a block-ordered launch
    print(f"[case] profile 8x32 {precision} off", flush=True)
    plain = radic.radic_det(A, precision=precision)
    assert radic.profile_read_launches() == []
    radic.profile_enable(True)
    timed = []
    for i in range(3):
        print(f"[case] profile 8x32 {precision} on, call {i}", flush=True)
        timed.append(radic.radic_det(A, precision=precision))
    radic.profile_enable(False)
    ms = radic.profile_read_launches()
    assert len(ms) == 3
    assert all(0.0 < x < 50.0 for x in ms), ms
    for r in timed:
        assert bits(r) == bits(plain)


def test_profile_times_exact_call():
    A = workloads.random_int(6, 20, seed=8101)
    print("[case] profile exact 6x20", flush=True)
    radic.profile_enable(True)
    got = radic.radic_det_int_exact(to_device(np.ascontiguousarray(A, dtype=np.int32)))
    radic.profile_enable(False)
    assert got == oracle.radic_int(A)
    ms = radic.profile_read_launches()
    assert len(ms) == 1 and 0.0 < ms[0] < 50.0


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
@pytest.mark.parametrize("shape", [(7, 24), (8, 26), (5, 40)])
def test_block_order_reproducible_and_matches_oracle(shape, precision):
    m, n = shape
    A = workloads.random_float(m, n, seed=8200 + m * 100 + n)
    dA = to_device(A)
    print(f"[case] block order {shape} {precision}", flush=True)
    first = radic.radic_det(dA, precision=precision)
    second = radic.radic_det(dA, precision=precision)
    assert bits(first) == bits(second)
    ref = oracle.radic_f64(A)
    S = normaliser(ref["abs_sum"], A)
    assert_close(first["value"], ref["value"], S, TOL[precision], f"value {shape} {precision}")
    # two range calls (dictionary order) cover the same minors
    total = math.comb(n, m)
    half = total // 2
    print(f"[case] block order {shape} {precision} as two ranges", flush=True)
    a = radic.radic_det_range(dA, 0, half, precision=precision)
    b = radic.radic_det_range(dA, half, total - half, precision=precision)
    assert a["n_subsets"] + b["n_subsets"] == total
    assert_close(a["value"] + b["value"], first["value"], S, 2 * TOL[precision], f"ranges {shape} {precision}")
    assert_close(a["abs_sum"] + b["abs_sum"], first["abs_sum"], ref["abs_sum"], 10 * TOL[precision], "abs_sum")


def test_block_order_exact_reproducible():
    A = workloads.random_int(7, 22, seed=8301)
    print("[case] block order exact 7x22", flush=True)
    dA = to_device(np.ascontiguousarray(A, dtype=np.int32))
    ref = oracle.radic_int(A)
    assert radic.radic_det_int_exact(dA) == ref
    assert radic.radic_det_int_exact(dA) == ref


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_first_call_of_a_shape_captured(precision):
    # the first call of a shape goes into a HIP graph: it needs no allocation,
    # no host synchronisation and no table, and every replay gives the bits of
    # an eager call
    import torch
    from paper_1508_01326_amd import binding
    print("[case] device set-up call 3x9", flush=True)
    radic.radic_det(to_device(workloads.random_float(3, 9, seed=8400)))
    m, n = (7, 23) if precision == "fp64" else (7, 25)
    A = workloads.random_float(m, n, seed=8401 + n)
    dA = to_device(A)
    out = binding.new_f64_result()
    work = binding.workspace(radic.RADIC_WS_DET, m, n)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    print(f"[case] capture first call {m}x{n} {precision}", flush=True)
    with torch.cuda.graph(g, stream=side):
        radic.radic_det(dA, precision=precision, out=out, work=work, sync=False)
    replays = []
    for rep in range(3):
        out.zero_()
        torch.cuda.synchronize()
        print(f"[case] replay {rep}", flush=True)
        g.replay()
        torch.cuda.synchronize()
        replays.append(binding.read_f64_result(out))
        _ = (torch.ones(1000, device="cuda") * 2).sum().item()   # eager work between replays
    eager = radic.radic_det(dA, precision=precision)
    for r in replays:
        assert bits(r) == bits(eager)
    ref = oracle.radic_f64(A)
    assert_close(eager["value"], ref["value"], normaliser(ref["abs_sum"], A), TOL[precision], "captured shape")
    del g
