"""Pins for the oracle's dictionary-order combinatorics (Sections 3-5).

Every expected value here is either printed in the paper (Table 2, Table 3b, the
q = 49 example; fixtures under tests/golden/) or fixed by elementary
combinatorics (itertools enumeration, Theorem 1's count)."""
import itertools
import math

import pytest

import oracle


def test_table2_unrank(golden):
    # Section 4, Example 1, Table 2: B_0..B_55 for n = 8, m = 5
    rows = golden("table2_subsets_n8_m5.txt")
    assert len(rows) == 56
    for r in rows:
        q, B = int(r[0]), [int(x) for x in r[1:]]
        assert oracle.unrank(q, 5, 8) == B, q


def test_table2_successor_chain(golden):
    # Section 5: stepping the successor from the First Member visits Table 2 in order
    rows = golden("table2_subsets_n8_m5.txt")
    B = [1, 2, 3, 4, 5]
    for r in rows:
        assert B == [int(x) for x in r[1:]]
        nxt = oracle.successor(B, 8)
        B = nxt
    assert B is None  # B_55 is the last member


def test_q49_trace(golden):
    # Section 4 worked example: q = 49 moves place 1 by p = 1 (q -> 14, [2,3,4,5,6])
    # then place 2 by p = 2 (q -> 0, [2,5,6,7,8]).
    rows = golden("q49_trace_n8_m5.txt")
    B, moves = oracle.unrank_trace(49, 5, 8)
    steps = [r for r in rows if r[0] != "final"]
    final = [r for r in rows if r[0] == "final"][0]
    assert len(moves) == len(steps)
    for (k, p, q, Bk), r in zip(moves, steps):
        assert (k, p, q) == (int(r[0]), int(r[1]), int(r[2]))
        assert Bk == [int(x) for x in r[3:]]
    assert B == [int(x) for x in final[1:]]


def test_table3b_pascal(golden):
    # Table 3b: entry (j, i) = C(i + j, j), m = 5 rows, n - m + 1 = 4 columns
    rows = golden("table3b_pascal_n8_m5.txt")
    for j, r in enumerate(rows):
        for i, v in enumerate(r):
            assert oracle.binomial(i + j, j) == int(v)


def test_place_weights_example():
    # the place weights quoted for the q = 49 example: C(7,4) C(6,3) C(5,2) C(4,1) C(3,0)
    assert [oracle.binomial(8 - k, 5 - k) for k in range(1, 6)] == [35, 20, 10, 4, 1]


@pytest.mark.parametrize("n", range(1, 13))
def test_exhaustive_enumeration(n):
    for m in range(1, n + 1):
        expect = [list(c) for c in itertools.combinations(range(1, n + 1), m)]
        # Theorem 1: exactly C(n, m) sequences
        assert oracle.binomial(n, m) == len(expect) == math.comb(n, m)
        for q, B in enumerate(expect):
            assert oracle.unrank(q, m, n) == B
        # first and last member (Section 3)
        assert expect[0] == list(range(1, m + 1))
        assert expect[-1] == list(range(n - m + 1, n + 1))
        B = expect[0]
        steps = 0
        while True:
            nxt = oracle.successor(B, n)
            if nxt is None:
                break
            steps += 1
            assert nxt == expect[steps]
            B = nxt
        assert steps == len(expect) - 1


def test_binomial_overflow_boundary():
    assert oracle.binomial(67, 33) == math.comb(67, 33)
    with pytest.raises(OverflowError):
        oracle.binomial(68, 34)
    assert oracle.binomial(64, 32) == math.comb(64, 32)


def test_unrank_large_sampled():
    # sampled ranks of a big space against a direct lexicographic count
    n, m = 36, 12
    total = math.comb(n, m)
    for q in [0, 1, 2, 12345, total // 3, total // 2, total - 2, total - 1]:
        B = oracle.unrank(q, m, n)
        # rank back by counting sequences that precede B
        rank, prev = 0, 0
        for k, b in enumerate(B, start=1):
            for v in range(prev + 1, b):
                rank += math.comb(n - v, m - k)
            prev = b
        assert rank == q
