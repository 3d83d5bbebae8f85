"""Shared helpers for GPU parity tests: tolerances and device plumbing.

Tolerances are those stated for the method: |result - oracle| <= tol * S with
S = sum_J |det(A_J)| from the oracle, tol = 1e-12 for FP64 and 1e-5 for
FP32-bulk.  When S is zero or rounding noise (rank-deficient inputs) the
Hadamard-type normaliser e_m(column norms), an upper bound for S, is used."""
import numpy as np

TOL = {"fp64": 1e-12, "fp32_bulk": 1e-5}


def normaliser(oracle_abs_sum, A):
    from oracle import exact
    nh = exact.hadamard_sum(A)
    if oracle_abs_sum <= 1e-9 * nh:
        return nh
    return oracle_abs_sum


def assert_close(got, expect, scale, tol, what=""):
    err = abs(got - expect)
    assert err <= tol * scale, f"{what}: |{got} - {expect}| = {err:.3e} > {tol:.1e} * {scale:.3e}"


def to_device(A):
    import torch
    A = np.ascontiguousarray(A)
    return torch.from_numpy(A).to("cuda")
