"""GPU parity of the batched persistent path (and its HIP-graph launch)."""
import math

import numpy as np
import pytest

import oracle
import workloads
from tests.parity import TOL, normaliser

pytestmark = pytest.mark.gpu

radic = pytest.importorskip("paper_1508_01326_amd")


@pytest.fixture(autouse=True)
def _defaults():
    radic.set_launch(0, 0)
    radic.set_fallback_tau(1.0 / 1024)
    radic.set_prime_set([])
    yield


def mixed_batch(count, seed, m_max=8, n_max=14):
    rng = np.random.default_rng(seed)
    mats = []
    for b in range(count):
        m = int(rng.integers(1, m_max + 1))
        n = int(rng.integers(m, n_max + 1))
        if b % 2 == 0:
            mats.append(rng.standard_normal((m, n)))
        else:
            mats.append(rng.integers(-40, 41, size=(m, n)).astype(np.int32))
    return mats


def check(mats, res, precision, idx=None):
    for b in (range(len(mats)) if idx is None else idx):
        A, r = mats[b], res[b]
        m, n = A.shape
        assert r["status"] == 0, (b, r)
        assert r["n_subsets"] == (math.comb(n, m) if m <= n else 0)
        if A.dtype == np.int32:
            assert r["exact"] == oracle.radic_int(A), b
        else:
            ref = oracle.radic_f64(A)
            S = normaliser(ref["abs_sum"], A)
            assert abs(r["value"] - ref["value"]) <= TOL[precision] * S, (b, r["value"], ref["value"])


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_mixed_batch(precision):
    mats = mixed_batch(96, seed=1)
    print(f"[case] batched mixed 96 {precision}", flush=True)
    B = radic.Batch(mats)
    res = radic.radic_det_batched(B, precision)
    check(mats, res, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
@pytest.mark.parametrize("tau", [1.0 / 1024, math.inf])
def test_float_prefix_rounds(precision, tau):
    # float matrices above 4096 minors for m = 3..10 (their chunks run the
    # prefix-shared round; two wide ones, several chunks each), one with nearly
    # dependent rows (many FP32-bulk minors flagged); tau = inf flags every
    # FP32-bulk minor, which exercises the wave's queue refactorisation and the
    # rounds done again in double
    rng = np.random.default_rng(11)
    shapes = [(3, 40), (4, 60), (5, 24), (6, 20), (7, 18), (8, 18), (9, 17), (10, 18), (8, 16)]
    mats = [rng.standard_normal(s) for s in shapes]
    mats.append(workloads.near_dependent_rows(7, 16, seed=12, eps=1e-6))
    mats.append(rng.integers(-9, 10, size=(7, 15)).astype(np.int32))
    radic.set_fallback_tau(tau)
    print(f"[case] batched prefix rounds {precision} tau={tau}", flush=True)
    res = radic.radic_det_batched(radic.Batch(mats), precision)
    check(mats, res, precision)
    for A, r in zip(mats, res):
        if A.dtype == np.float64 and precision == "fp32_bulk" and tau == math.inf:
            assert r["n_fallback"] == math.comb(A.shape[1], A.shape[0])
        if precision == "fp64":
            assert r["n_fallback"] == 0


def test_every_row_count():
    # one float and one int matrix for every m = 1..12 (each has its own class kernel)
    rng = np.random.default_rng(2)
    mats = []
    for m in range(1, 13):
        n = m + int(rng.integers(0, 4))
        mats.append(rng.standard_normal((m, n)))
        mats.append(rng.integers(-9, 10, size=(m, n)).astype(np.int32))
    print("[case] batched m=1..12", flush=True)
    res = radic.radic_det_batched(radic.Batch(mats), "fp64")
    check(mats, res, "fp64")


def test_bad_descriptors_reported_per_matrix():
    good = np.random.default_rng(3).standard_normal((3, 7))
    mats = [good, np.ones((5, 4)), np.zeros((2, 70)), good.copy()]
    mats[3][1, 2] = np.nan
    B = radic.Batch(mats)
    # corrupt descriptor 0's lda below n
    d = B.desc_host.copy()
    bad = d.copy()
    bad[0]["lda"] = 2
    import torch
    B.desc = torch.from_numpy(bad.view(np.uint8).copy()).to("cuda")
    print("[case] batched bad descriptors", flush=True)
    res = radic.radic_det_batched(B, "fp64")
    assert res[0]["status"] == radic.RADIC_EINVAL
    assert res[1]["status"] == 0 and res[1]["value"] == 0.0          # m > n
    assert res[2]["status"] == radic.RADIC_ENOTSUP                   # n beyond the batched limit
    assert res[3]["status"] == radic.RADIC_ENONFINITE and math.isnan(res[3]["value"])


def test_bitwise_reproducible_batched():
    mats = mixed_batch(40, seed=4)
    B = radic.Batch(mats)
    r1 = radic.radic_det_batched(B, "fp32_bulk")
    r2 = radic.radic_det_batched(B, "fp32_bulk")
    for a, b in zip(r1, r2):
        assert a["hi"] == b["hi"] and a["lo"] == b["lo"] and a["exact"] == b["exact"]


def test_graph_replays():
    import torch
    mats = mixed_batch(50, seed=5)
    B = radic.Batch(mats)
    direct = radic.radic_det_batched(B, "fp64")
    G = radic.BatchGraph(B, "fp64")
    try:
        for rep in range(3):
            B.out.zero_()
            torch.cuda.synchronize()
            print(f"[case] graph replay {rep}", flush=True)
            G.launch()
            torch.cuda.synchronize()
            res = B.results()
            for a, b in zip(direct, res):
                assert a["hi"] == b["hi"] and a["lo"] == b["lo"] and a["exact"] == b["exact"]
            # eager work between replays
            _ = (torch.ones(1000, device="cuda") * 2).sum().item()
        # new contents, same shapes: the replay reflects them
        mats2 = [(-A if A.dtype == np.float64 else (A * 2).astype(np.int32)) for A in mats]
        B2 = radic.Batch(mats2)
        B.f64.copy_(B2.f64)
        B.i32.copy_(B2.i32)
        torch.cuda.synchronize()
        G.launch()
        torch.cuda.synchronize()
        check(mats2, B.results(), "fp64")
    finally:
        G.destroy()


def test_autotune_batched_and_int():
    print("[case] autotune batched", flush=True)
    spl, block = radic.autotune(radic.RADIC_WS_BATCHED, precision="fp32_bulk")
    assert spl >= 1 and block == 256
    spl, block = radic.autotune(radic.RADIC_WS_BATCHED, precision="exact")
    assert spl >= 1
    spl, block = radic.autotune(radic.RADIC_WS_INT, 5, 12)
    assert spl >= 1
    mats = mixed_batch(30, seed=8)
    res = radic.radic_det_batched(radic.Batch(mats), "fp32_bulk")
    check(mats, res, "fp32_bulk")


def test_autotune_on_own_batch():
    # tuning on the caller's batch records one chunk size for both kinds of
    # classes; later calls and graphs captured after it use it and stay correct
    rng = np.random.default_rng(13)
    mats = [rng.standard_normal((8, 18)), rng.integers(-9, 10, size=(9, 17)).astype(np.int32),
            rng.standard_normal((5, 24))] + mixed_batch(20, seed=14)
    B = radic.Batch(mats)
    print("[case] autotune on own batch", flush=True)
    spl, block = radic.autotune_batched(B, "fp32_bulk")
    assert spl in (8, 16, 32, 64, 128) and block == 256
    check(mats, B.results(), "fp32_bulk")        # the last tuning run's results
    res = radic.radic_det_batched(B, "fp32_bulk")
    check(mats, res, "fp32_bulk")
    # the tuned size sets the chunking: blocks of 64 * spl minors for the float
    # 8 x 18 matrix, rank windows of at least 64 * spl for an int32 9 x 17
    chunk, k = radic.host_batch_chunking(0, 8, 18, spl)
    assert (k - 1) * chunk < radic.host_split_blocks(8, 18, 64 * spl) <= k * chunk
    chunk, _ = radic.host_batch_chunking(1, 9, 17, spl)
    assert chunk >= 64 * spl
