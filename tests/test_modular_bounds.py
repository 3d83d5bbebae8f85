"""The exact kernels' lazy modular product, emulated on the host with every
rounding done exactly (integers and Fractions, IEEE round to nearest even):
h = fl(a b), l = fma(a, b, -h), q = floor(fl(h * fl(1/p))), r = fl(fma(-q, p, h) + l).
For integer operands |a|, |b| <= 4.1 p and primes p < 2^31 the result must keep
the residue of a b and stay below 2.01 p in magnitude, so that differences of two
results are again valid operands; a sum of up to twelve such products must
reduce to [-p, 2p) with one quotient estimate.  These are the invariants the
elimination updates, operator rows and minor sums of the exact path rely on."""
import math
import random
from fractions import Fraction


def fl(x):
    return float(Fraction(x))


def mulmod_lazy(a, b, p, pinv):
    h = fl(a * b)
    l = fl(a * b - Fraction(h))
    q = math.floor(fl(Fraction(h) * Fraction(pinv)))
    r1 = fl(-q * p + Fraction(h))
    return fl(Fraction(r1) + Fraction(l))


def reduce_lazy(x, p, pinv):
    q = math.floor(fl(Fraction(x) * Fraction(pinv)))
    return fl(-q * p + Fraction(x))


PRIMES = [2147483647, 2147483629, 1073741789, 16777259, 65521, 251, 3, 2]


def test_lazy_product_residue_and_range():
    rng = random.Random(7)
    for p in PRIMES:
        pinv = 1.0 / p
        B = int(4.1 * p)
        for it in range(1500):
            a = rng.randint(-B, B) if it % 5 else B * rng.choice((-1, 1))
            b = rng.randint(-B, B) if it % 7 else B * rng.choice((-1, 1))
            r = mulmod_lazy(a, b, p, pinv)
            assert r == int(r)
            assert (int(r) - a * b) % p == 0
            assert abs(r) < 2.01 * p


def test_lazy_sum_reduces_to_half_open_range():
    rng = random.Random(8)
    for p in PRIMES:
        pinv = 1.0 / p
        B = int(4.1 * p)
        for _ in range(300):
            terms = [mulmod_lazy(rng.randint(-B, B), rng.randint(0, p - 1), p, pinv) for _ in range(12)]
            s = sum(terms)                      # exact: below 2^36
            r = reduce_lazy(s, p, pinv)
            assert (int(r) - int(s)) % p == 0 and -p <= r < 2 * p


def test_plain_fma_product_would_break_without_the_error_term():
    # the low part l matters: without it the remainder is wrong for large operands
    p = 2147483647
    pinv = 1.0 / p
    a = b = int(4.1 * p)
    h = fl(a * b)
    q = math.floor(fl(Fraction(h) * Fraction(pinv)))
    r_no_l = fl(-q * p + Fraction(h))
    assert (int(r_no_l) - a * b) % p != 0
    assert (int(mulmod_lazy(a, b, p, pinv)) - a * b) % p == 0
