"""GPU parity of the exact integer path against the BigInt oracle (bit-exact)."""
import math

import numpy as np
import pytest

import oracle
from oracle import exact
import workloads
from tests.parity import to_device

pytestmark = pytest.mark.gpu

radic = pytest.importorskip("paper_1508_01326_amd")


@pytest.fixture(autouse=True)
def _defaults():
    radic.set_prime_set([])
    radic.set_launch(0, 0)
    yield
    radic.set_prime_set([])
    radic.set_launch(0, 0)


def run_int(A, what):
    print(f"[case] int {what} shape={A.shape}", flush=True)
    return radic.radic_det_int_exact(to_device(np.ascontiguousarray(A, dtype=np.int32)))


SHAPES = [(1, 1), (1, 9), (2, 2), (2, 40), (3, 11), (4, 13), (5, 14), (6, 12), (7, 15), (8, 16), (9, 14),
          (10, 13), (11, 14), (12, 14)]


@pytest.mark.parametrize("shape", SHAPES)
def test_random_int_shapes(shape):
    m, n = shape
    A = workloads.random_int(m, n, seed=m * 100 + n, lo=-50, hi=50)
    assert run_int(A, f"random {shape}") == oracle.radic_int(A)


def test_workload3_full():
    A = workloads.single_matrix(3)    # 6 x 40, entries in [-9, 9], C(40,6) = 3838380 minors
    ref = oracle.radic_int(A)
    assert ref == exact.radic_subset_dp(A)
    assert run_int(A, "workload3 6x40") == ref


def test_extreme_entries():
    rng = np.random.default_rng(7)
    A = rng.integers(-2 ** 31, 2 ** 31, size=(7, 11), dtype=np.int64).astype(np.int32)
    A[0, 0] = -2 ** 31
    A[3, 5] = 2 ** 31 - 1
    got = run_int(A, "int32 extremes")
    assert got == oracle.radic_int(A) == exact.radic_subset_dp(A)
    assert abs(got).bit_length() > 200     # needs many primes


def _sylvester(k):
    H = np.array([[1]], dtype=np.int64)
    for _ in range(k):
        H = np.block([[H, H], [H, -H]])
    return H


@pytest.mark.parametrize("exchange", [False, True])
def test_hadamard_bound_attained(exchange):
    # A Sylvester-Hadamard matrix of order 8 scaled by 2^31 - 1 attains the
    # bound the prime count is chosen from (Hadamard's inequality is an
    # equality): |det| = 8^4 (2^31 - 1)^8, about 2^260, nine 32-bit limbs; an
    # exchange of two rows flips the sign (m = n: the Radic determinant is the
    # ordinary one, Definition 3)
    H = _sylvester(3) * (2 ** 31 - 1)
    if exchange:
        H = H[[1, 0, 2, 3, 4, 5, 6, 7]]
    A = H.astype(np.int32)
    got = run_int(A, f"hadamard 8x8 exchange={exchange}")
    assert abs(got) == 8 ** 4 * (2 ** 31 - 1) ** 8
    assert got == oracle.radic_int(A)
    B = _sylvester(3) * (2 ** 31 - 1)
    assert got == (-1 if exchange else 1) * oracle.radic_int(B.astype(np.int32))


def test_hadamard_rows_wide():
    # the same rows with two more columns of extreme entries: 45 minors, most
    # near the bound, summed with both signs
    rng = np.random.default_rng(11)
    A = np.concatenate([_sylvester(3) * (2 ** 31 - 1),
                        rng.integers(-2 ** 31, 2 ** 31, size=(8, 2), dtype=np.int64)], axis=1).astype(np.int32)
    got = run_int(A, "hadamard rows 8x10")
    assert got == oracle.radic_int(A) == exact.radic_subset_dp(A)
    assert abs(got).bit_length() > 240


def test_zero_pivots_and_structure():
    # leading zero columns force exchanges; equal rows give exactly zero
    A = np.array([[0, 0, 1, 2, 3, 0], [0, 1, 0, 4, 5, 0], [1, 0, 0, 6, 7, 0]], dtype=np.int32)
    assert run_int(A, "leading zeros") == oracle.radic_int(A)
    B = workloads.random_int(5, 12, seed=3)
    B[4] = B[1]
    assert run_int(B, "equal rows") == 0
    Z = np.zeros((4, 9), dtype=np.int32)
    assert run_int(Z, "zero matrix") == 0
    assert run_int(np.ones((5, 4), dtype=np.int32), "m > n") == 0


def test_tiny_prime_set():
    # small primes make pivots vanish mod p and need many residues; the CRT must still be exact
    A = workloads.random_int(4, 10, seed=44, lo=-3, hi=3)
    ref = oracle.radic_int(A)
    radic.set_prime_set([3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61, 67, 71, 73, 79, 83, 89, 97])
    assert run_int(A, "tiny primes") == ref


def test_launch_shapes_int():
    A = workloads.random_int(5, 17, seed=5)
    ref = oracle.radic_int(A)
    for spl, block in [(1, 64), (7, 128), (32, 256)]:
        radic.set_launch(spl, block)
        assert run_int(A, f"launch {spl},{block}") == ref


def test_capacity_too_small():
    import ctypes
    A = workloads.random_int(6, 14, seed=9, lo=-1000, hi=1000)
    ref = oracle.radic_int(A)
    dA = to_device(A)
    work = radic.workspace(radic.RADIC_WS_INT, 6, 14, device=dA.device)
    mag = (ctypes.c_uint32 * 1)()
    ln, sg = ctypes.c_int(0), ctypes.c_int(0)
    import torch
    rc = radic.lib().radic_det_int_exact(ctypes.c_void_p(dA.data_ptr()), 6, 14, 14, mag, 1, ctypes.byref(ln),
                                         ctypes.byref(sg), ctypes.c_void_p(work.data_ptr()), work.numel(),
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    need = (abs(ref).bit_length() + 31) // 32
    if need > 1:
        assert rc == radic.RADIC_EOVERFLOW and ln.value == need
    else:
        assert rc == radic.RADIC_OK


@pytest.mark.parametrize("mode", ["per_minor", "prefix_shared", "group_shared"])
def test_enumerations_bit_exact(mode):
    # the prefix-shared exact kernel (minors sharing their first m-2 columns share
    # those fraction-free elimination steps mod p) and the per-minor kernel
    radic.set_enumeration(mode)
    try:
        for m, n, seed in [(3, 60, 1), (4, 9, 5), (5, 22, 2), (8, 16, 3), (10, 14, 4), (10, 10, 6)]:
            A = workloads.random_int(m, n, seed=900 + seed, lo=-1000, hi=1000)
            assert run_int(A, f"{mode} {m}x{n}") == oracle.radic_int(A)
    finally:
        radic.set_enumeration("auto")


def test_shared_exact_rank_deficient_prefixes():
    # repeated and zero columns make whole prefix blocks singular mod every prime
    rng = np.random.default_rng(77)
    A = rng.integers(-20, 21, size=(6, 18)).astype(np.int32)
    A[:, 3] = A[:, 1]
    A[:, 7] = 0
    A[:, 12] = 2 * A[:, 5]
    assert run_int(A, "singular prefixes") == oracle.radic_int(A)
