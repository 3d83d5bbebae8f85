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
    assert L.radic_det(fake, radic.RADIC_MAX_M + 1, 40, 40, 0, fake, fake, 1 << 20, nul) == radic.RADIC_ENOTSUP
    assert L.radic_det(fake, 2, radic.RADIC_MAX_N + 1, radic.RADIC_MAX_N + 1, 0, fake, fake, 1 << 20,
                       nul) == radic.RADIC_ENOTSUP
    # export mode needs an output
    assert L.radic_det_subsets(fake, 2, 3, 3, 0, 0, 1, nul, nul, nul) == radic.RADIC_EINVAL


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
