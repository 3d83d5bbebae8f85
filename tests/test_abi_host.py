"""C-ABI boundary checks that need no GPU: the library loads, exports every
function declared in include/radic.h, and its host-side logic (binomials,
dictionary unranking, argument validation, workspace sizing) behaves."""
import ctypes
import math
import os
import re

import pytest

import paper_1508_01326_amd as radic
from paper_1508_01326_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "radic.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(radic_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    names = declared_functions()
    assert len(names) >= 20
    assert set(names) == set(binding.SIGNATURES), set(names) ^ set(binding.SIGNATURES)


def test_library_exports_every_symbol():
    L = radic.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings_and_version():
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert radic.status_string(code).startswith("RADIC_")
    assert "unknown" in radic.status_string(12345)
    assert radic.lib().radic_version() >= 100


def test_host_binomial():
    for a in range(0, 70):
        for b in range(0, min(a, 20) + 1):
            if math.comb(a, b) < 2 ** 64:
                assert radic.host_binomial(a, b) == math.comb(a, b)
    assert radic.host_binomial(67, 33) == math.comb(67, 33)
    with pytest.raises(radic.RadicError) as e:
        radic.host_binomial(68, 34)
    assert e.value.status == radic.RADIC_EOVERFLOW


def test_host_unrank_table2(golden):
    # Section 4, Table 2 (n = 8, m = 5)
    for r in golden("table2_subsets_n8_m5.txt"):
        assert radic.host_unrank(5, 8, int(r[0])) == [int(x) for x in r[1:]]
    # the worked example of Section 4
    assert radic.host_unrank(5, 8, 49) == [2, 5, 6, 7, 8]


def test_host_unrank_exhaustive():
    import itertools
    for n in range(1, 11):
        for m in range(1, n + 1):
            for q, c in enumerate(itertools.combinations(range(1, n + 1), m)):
                assert radic.host_unrank(m, n, q) == list(c)


def test_workspace_sizes():
    L = radic.lib()
    assert L.radic_workspace_bytes(radic.RADIC_WS_DET, 8, 32, 0) > 0
    assert L.radic_workspace_bytes(radic.RADIC_WS_DET, 0, 32, 0) == 0
    assert L.radic_workspace_bytes(99, 8, 32, 0) == 0


def test_argument_validation_without_device():
    L = radic.lib()
    nul = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    # null matrix / result
    assert L.radic_det(nul, 2, 3, 3, 0, fake, fake, 1 << 20, nul) == radic.RADIC_EINVAL
    assert L.radic_det(fake, 2, 3, 3, 0, nul, fake, 1 << 20, nul) == radic.RADIC_EINVAL
    # bad sizes, lda, precision
    assert L.radic_det(fake, 0, 3, 3, 0, fake, fake, 1 << 20, nul) == radic.RADIC_EINVAL
    assert L.radic_det(fake, 2, 0, 3, 0, fake, fake, 1 << 20, nul) == radic.RADIC_EINVAL
    assert L.radic_det(fake, 2, 3, 2, 0, fake, fake, 1 << 20, nul) == radic.RADIC_EINVAL
    assert L.radic_det(fake, 2, 3, 3, 7, fake, fake, 1 << 20, nul) == radic.RADIC_EINVAL
    # beyond the compiled limits
    assert L.radic_det(fake, binding.RADIC_MAX_M_WIDE + 1, 40, 40, 0, fake, fake, 1 << 20, nul) == radic.RADIC_ENOTSUP
    assert L.radic_det(fake, 2, radic.RADIC_MAX_N + 1, radic.RADIC_MAX_N + 1, 0, fake, fake, 1 << 20,
                       nul) == radic.RADIC_ENOTSUP
    # export mode needs an output
    assert L.radic_det_subsets(fake, 2, 3, 3, 0, 0, 1, nul, nul, nul) == radic.RADIC_EINVAL
    # two-row path: n >= 1, lda >= n, pointers
    assert L.radic_det_2xn(nul, 5, 5, fake, fake, 1 << 30, nul) == radic.RADIC_EINVAL
    assert L.radic_det_2xn(fake, 0, 5, fake, fake, 1 << 30, nul) == radic.RADIC_EINVAL
    assert L.radic_det_2xn(fake, 5, 4, fake, fake, 1 << 30, nul) == radic.RADIC_EINVAL
    assert L.radic_det_2xn(fake, 5, 5, fake, fake, 16, nul) == radic.RADIC_EWORKSPACE


def test_launch_and_tau_setters_validate():
    L = radic.lib()
    assert L.radic_set_launch(-1, 0) == radic.RADIC_EINVAL
    assert L.radic_set_launch(8, 96) == radic.RADIC_EINVAL
    assert L.radic_set_launch(8, 512) == radic.RADIC_EINVAL     # above the kernels' launch bounds
    assert L.radic_set_launch(8, 1024) == radic.RADIC_EINVAL
    assert L.radic_set_launch(0, 0) == radic.RADIC_OK
    assert L.radic_set_fallback_tau(float("nan")) == radic.RADIC_EINVAL
    assert L.radic_set_fallback_tau(-1.0) == radic.RADIC_EINVAL
    assert L.radic_set_fallback_tau(1.0 / 1024) == radic.RADIC_OK
    assert L.radic_set_enumeration(4) == radic.RADIC_EINVAL
    assert L.radic_set_enumeration(-1) == radic.RADIC_EINVAL
    for mode in ("per_minor", "prefix_shared", "group_shared", "auto"):
        radic.set_enumeration(mode)


def _is_prime(n):
    if n < 2:
        return False
    i = 2
    while i * i <= n:
        if n % i == 0:
            return False
        i += 1
    return True


def test_fallback_threshold_scaling():
    # tau' = tau * min(1, (8192 / N)^(1/4)); exact at powers of two of N / 8192
    L = radic.lib()
    t = 1.0 / 1024
    assert L.radic_set_fallback_tau(t) == radic.RADIC_OK
    try:
        assert radic.fallback_tau_for(1) == t
        assert radic.fallback_tau_for(8192) == t
        assert radic.fallback_tau_for(8192 * 16) == t / 2
        assert radic.fallback_tau_for(8192 * 2 ** 16) == t / 16
        assert t / 2 < radic.fallback_tau_for(8192 * 16 - 1) < t
        N = 10518300   # C(32, 8)
        assert abs(radic.fallback_tau_for(N) - t * (8192 / N) ** 0.25) <= 1e-18
        # never and always stay as set
        assert L.radic_set_fallback_tau(0.0) == radic.RADIC_OK
        assert radic.fallback_tau_for(10 ** 12) == 0.0
        assert L.radic_set_fallback_tau(float("inf")) == radic.RADIC_OK
        assert radic.fallback_tau_for(10 ** 12) == float("inf")
    finally:
        assert L.radic_set_fallback_tau(t) == radic.RADIC_OK


def test_default_prime_set():
    primes = [radic.host_prime(i) for i in range(radic.binding.RADIC_MAX_PRIMES)]
    assert primes == sorted(primes, reverse=True)
    assert len(set(primes)) == len(primes)
    assert all(p < 2 ** 31 for p in primes)
    assert all(_is_prime(p) for p in primes)      # trial division, independent of the library's test
    # they are the largest primes below 2^31: no prime is skipped in between
    lo = primes[-1]
    expect = [c for c in range(2 ** 31 - 1, lo - 1, -2) if _is_prime(c)]
    assert primes == expect
    with pytest.raises(radic.RadicError):
        radic.host_prime(radic.binding.RADIC_MAX_PRIMES)


def test_prime_set_validation():
    L = radic.lib()
    arr = (ctypes.c_uint32 * 3)(7, 11, 15)        # 15 is composite
    assert L.radic_set_prime_set(arr, 3) == radic.RADIC_EINVAL
    arr = (ctypes.c_uint32 * 2)(7, 7)             # duplicate
    assert L.radic_set_prime_set(arr, 2) == radic.RADIC_EINVAL
    arr = (ctypes.c_uint32 * 1)(2)                # even prime is not allowed
    assert L.radic_set_prime_set(arr, 1) == radic.RADIC_EINVAL
    arr = (ctypes.c_uint32 * 2)(13, 7)
    assert L.radic_set_prime_set(arr, 2) == radic.RADIC_OK
    assert radic.host_prime(0) == 13 and radic.host_prime(1) == 7
    assert L.radic_set_prime_set(arr, 0) == radic.RADIC_OK   # back to the default set
    assert radic.host_prime(0) == 2 ** 31 - 1


def test_int_validation_without_device():
    L = radic.lib()
    nul = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)
    mag = (ctypes.c_uint32 * 8)()
    ln, sg = ctypes.c_int(7), ctypes.c_int(7)
    assert L.radic_det_int_exact(nul, 2, 3, 3, mag, 8, ctypes.byref(ln), ctypes.byref(sg), fake, 1 << 24,
                                 nul) == radic.RADIC_EINVAL
    assert L.radic_det_int_exact(fake, 2, 3, 2, mag, 8, ctypes.byref(ln), ctypes.byref(sg), fake, 1 << 24,
                                 nul) == radic.RADIC_EINVAL
    # m > n is zero by Definition 3, decided on the host
    assert L.radic_det_int_exact(fake, 4, 3, 3, mag, 8, ctypes.byref(ln), ctypes.byref(sg), fake, 1 << 24,
                                 nul) == radic.RADIC_OK
    assert ln.value == 0 and sg.value == 0
    assert L.radic_det_int_exact(fake, 13, 20, 20, mag, 8, ctypes.byref(ln), ctypes.byref(sg), fake, 1 << 24,
                                 nul) == radic.RADIC_ENOTSUP
    assert L.radic_workspace_bytes(radic.RADIC_WS_INT, 6, 40, 0) > 0


def test_tune_table_roundtrip(tmp_path):
    # the table names the device architecture ("none" without a device, as here)
    # and the library version; shapes are keyed by column bucket and enumeration
    ver = binding.lib().radic_version()
    src = tmp_path / "in.txt"
    src.write_text(f"# table\narch none version {ver}\n0 0 8 32 0 4 128\n0 0 8 32 1 48 256\n0 1 8 32 0 16 256\n"
                   f"1 0 6 40 0 8 64\n2 2 0 0 0 2 256\n")
    radic.tune_load(src)
    out = tmp_path / "out.txt"
    radic.tune_save(out)
    lines = [l for l in out.read_text().splitlines() if not l.startswith("#")]
    assert lines[0] == f"arch none version {ver}"
    rows = [l.split() for l in lines[1:]]
    assert ["0", "0", "8", "32", "0", "4", "128"] in rows
    assert ["0", "0", "8", "32", "1", "48", "256"] in rows
    assert ["2", "2", "0", "0", "0", "2", "256"] in rows
    bad = tmp_path / "bad.txt"
    bad.write_text(f"arch none version {ver}\n0 0 8 32 0 4 96\n")   # block not a multiple of 64
    with pytest.raises(radic.RadicError):
        radic.tune_load(bad)
    for text in ("0 0 8 32 0 4 128\n",                               # no header
                 f"arch none version {ver + 1}\n0 0 8 32 0 4 128\n",    # another library version
                 f"arch none version {ver}\n0 0 8 32 4 128\n",          # no enumeration column
                 f"arch none version {ver}\n0 0 8 32 7 4 128\n"):       # no such enumeration
        other = tmp_path / "other.txt"
        other.write_text(text)
        with pytest.raises(radic.RadicError):
            radic.tune_load(other)
    with pytest.raises(radic.RadicError):
        radic.tune_load(tmp_path / "missing.txt")


def test_batch_chunking_bounds():
    # every chunk is a multiple of 64 ranks and at least 64 * spl; chunks cover the
    # rank space exactly once; float matrices have at most 256 chunks, int32 at
    # most 2^16, so a class queue over 2^24 matrices stays far below 2^63 and its
    # 64-bit counter cannot wrap
    # matrices taken in two-sided blocks (float m >= 7, int32 5 <= m <= 6): the
    # chunks are runs of blocks that cover the block list exactly once
    for dtype in (0, 1):
        for m, n in [(1, 1), (2, 24), (10, 24), (6, 40), (12, 64), (11, 64), (3, 64), (10, 64), (5, 24)]:
            for spl in (1, 4, 8, 64):
                chunk, k = radic.host_batch_chunking(dtype, m, n, spl)
                total = math.comb(n, m)
                blocks = m >= 7 if dtype == 0 else 5 <= m <= 6
                if blocks:
                    nb = radic.host_split_blocks(m, n, 64 * spl)
                    assert chunk >= 1 and (k - 1) * chunk < nb <= k * chunk
                else:
                    assert chunk % 64 == 0 and chunk >= 64 * spl
                    assert (k - 1) * chunk < total <= k * chunk
                assert k <= (256 if dtype == 0 else 1 << 16)
                assert k * (1 << 24) < 1 << 63
    # the worst single int32 matrix the batched path accepts (m <= 12, n <= 64)
    chunk, k = radic.host_batch_chunking(1, 12, 64, 1)
    assert k <= 1 << 16 and chunk >= math.comb(64, 12) // (1 << 16)
    with pytest.raises(radic.RadicError):
        radic.host_batch_chunking(2, 3, 5, 1)
    with pytest.raises(radic.RadicError):
        radic.host_batch_chunking(0, 6, 5, 1)


def _colex_run(r, K):
    pairs = r * (r - 1) // 2
    k = K // pairs if pairs else 64
    return max(1, min(64, k))


@pytest.mark.parametrize("m,n", [(3, 9), (4, 11), (5, 5), (5, 12), (6, 7), (6, 20), (7, 18), (8, 16), (9, 17),
                                 (10, 17), (11, 16), (12, 17)])
def test_split_blocks_partition(m, n):
    # the kernels' two-sided enumeration, run on the host: every minor lies on
    # exactly one side, under exactly one prefix of it, and a side-s prefix c
    # with last column v is taken exactly when c_2 <= n-1-v-s (m >= 5); side 1
    # reads column c as n-1-c
    seen = set()
    blocks = 0
    K = 64 * 64
    for v in range(m - 3, n - 2):
        r = n - 1 - v
        for side in (0, 1):
            cnt = radic.host_split_count(m, n, side, v)
            if m < 5 and side == 1:
                assert cnt == 0
            blocks += -(-cnt // _colex_run(r, K))
            for j in range(cnt):
                c = radic.host_split_prefix(m, n, side, v, j)
                assert c == sorted(set(c)) and c[-1] == v and c[0] >= 0
                if m >= 5:
                    assert c[2] <= r - side
                for a in range(v + 1, n):
                    for b in range(a + 1, n):
                        view = c + [a, b]
                        minor = tuple(sorted(n - 1 - x for x in view)) if side else tuple(view)
                        assert minor not in seen
                        seen.add(minor)
            with pytest.raises(radic.RadicError):
                radic.host_split_prefix(m, n, side, v, cnt)
    assert len(seen) == math.comb(n, m)
    assert radic.host_split_blocks(m, n, K) == blocks


def test_split_counts_match_the_bench_model():
    # two independent statements of the side rule: the kernels' (C++, host
    # build) and the executed-FLOP model of bench.py
    import bench
    for m, n in [(5, 14), (6, 40), (8, 32), (9, 30), (12, 36), (10, 64)]:
        for v in range(m - 3, n - 2):
            for side in (0, 1):
                assert radic.host_split_count(m, n, side, v) == bench.split_prefix_count(m - 2, n, side, v)
    with pytest.raises(radic.RadicError):
        radic.host_split_count(2, 5, 0, 0)
    with pytest.raises(radic.RadicError):
        radic.host_split_count(5, 9, 2, 3)
    with pytest.raises(radic.RadicError):
        radic.host_split_count(5, 9, 0, 7)
