"""Seeded synthetic inputs for the Radic determinant.

The paper reports no experiments and ships no data, so every input is synthetic:
numpy's PCG64 generator (``default_rng``) seeded with 150801326 + workload index.
This module only draws numbers; it contains none of the determinant arithmetic.
It is the one module shared by the GPU-side tests/benchmark and the oracle side.

Workloads (shape, entry distribution):
  1  one 5 x 14 float64 matrix, iid uniform[-1, 1]                  C(14,5) = 2,002
  2  one 8 x 32 float64 matrix, iid N(0, 1)                          C(32,8) = 10,518,300
  3  one 6 x 40 int32 matrix, iid uniform integers in [-9, 9]        C(40,6) = 3,838,380
  4  one 12 x 36 float64 matrix, N(0, 1) entries times a per-row
     lognormal(mean 0, sigma 2) scale (one scale per row)            C(36,12) = 1,251,677,700
  5  4096 matrices; per matrix draw m uniform in [2, 10], then n uniform in
     [m, 24], then the entries: even index float64 uniform[-1, 1], odd index
     int32 uniform integers in [0, 255]
"""
import numpy as np

SEED_BASE = 150801326

SHAPES = {1: (5, 14), 2: (8, 32), 3: (6, 40), 4: (12, 36)}


def rng_for(workload: int, salt: int = 0):
    return np.random.default_rng(SEED_BASE + workload + salt)


def single_matrix(workload: int):
    """The matrix of workloads 1-4 (float64, or int32 for workload 3)."""
    rng = rng_for(workload)
    m, n = SHAPES[workload]
    if workload == 1:
        return rng.uniform(-1.0, 1.0, size=(m, n))
    if workload == 2:
        return rng.standard_normal((m, n))
    if workload == 3:
        return rng.integers(-9, 10, size=(m, n)).astype(np.int32)
    if workload == 4:
        scale = rng.lognormal(mean=0.0, sigma=2.0, size=(m, 1))
        return rng.standard_normal((m, n)) * scale
    raise ValueError(workload)


def batch_matrices(count: int = 4096, workload: int = 5, m_range=(2, 10), n_max: int = 24):
    """Workload 5: list of (kind, matrix) with kind 'f64' (even index) or 'i32' (odd index)."""
    rng = rng_for(workload)
    out = []
    for b in range(count):
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        n = int(rng.integers(m, n_max + 1))
        if b % 2 == 0:
            out.append(("f64", rng.uniform(-1.0, 1.0, size=(m, n))))
        else:
            out.append(("i32", rng.integers(0, 256, size=(m, n)).astype(np.int32)))
    return out


def random_float(m: int, n: int, seed: int, dist: str = "normal"):
    """Small random float64 matrices for parity sweeps."""
    rng = np.random.default_rng(SEED_BASE + 1000 + seed)
    if dist == "normal":
        return rng.standard_normal((m, n))
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, size=(m, n))
    raise ValueError(dist)


def random_int(m: int, n: int, seed: int, lo: int = -9, hi: int = 9):
    rng = np.random.default_rng(SEED_BASE + 2000 + seed)
    return rng.integers(lo, hi + 1, size=(m, n)).astype(np.int32)


def near_dependent_rows(m: int, n: int, seed: int, eps: float = 1e-6):
    """Float64 matrix whose last row is the first row plus eps-sized noise, so every
    minor is nearly singular (drives the FP32-bulk fallback)."""
    rng = np.random.default_rng(SEED_BASE + 3000 + seed)
    A = rng.standard_normal((m, n))
    A[m - 1] = A[0] + eps * rng.standard_normal(n)
    return A
