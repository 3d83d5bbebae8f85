"""Exact evaluators of the Radic determinant -- TEST INFRASTRUCTURE ONLY.

These are independent of the enumerating oracle in ``radic_oracle.c`` and of each
other; they pin it (and serve as exact references at sizes where enumeration is
too slow).  All arithmetic is exact: integers stay Python ints, floating-point
inputs are taken as the dyadic rationals they are.

* ``leibniz_det`` / ``radic_bruteforce``: Definition 3, eq. (1) with each minor
  expanded over all permutations (tiny inputs only).
* ``radic_subset_dp``: the same sum reorganised column by column.  Expanding every
  minor by permutations and walking the columns 1..n in order, a chosen column c
  that is the t-th chosen one receives a row i not used yet; that contributes
  a_ic, the factor (-1)^c of (-1)^s, and (-1)^(number of used rows above i) to the
  permutation sign.  The state is the set of used rows, so the cost is
  O(n * 2^m * m).
* ``radic_pfaffian``: the minor-summation formula of Pfaffians (Ishikawa and
  Wakayama, 1995): for an m x n matrix T with m even, the sum over all m-column
  subsets J of det(T_J) equals Pf(T K T^t) where K is the n x n skew matrix with
  K_ab = 1 for a < b.  With T = A diag((-1)^j) each det(T_J) carries (-1)^s; for odd
  m a unit row and column are bordered in front.  Cost O(m^2 n + m^3).
"""
from fractions import Fraction
from itertools import combinations, permutations
import math


def _to_rows(A):
    try:
        import numpy as np
        if isinstance(A, np.ndarray):
            if A.dtype.kind in "iu":
                return [[int(x) for x in row] for row in A.tolist()]
            return [[Fraction(float(x)) for x in row] for row in A.tolist()]
    except ImportError:  # pragma: no cover
        pass
    out = []
    for row in A:
        out.append([x if isinstance(x, (int, Fraction)) else Fraction(float(x)) for x in row])
    return out


def _perm_sign(p):
    inv = 0
    for a in range(len(p)):
        for b in range(a + 1, len(p)):
            if p[a] > p[b]:
                inv += 1
    return -1 if inv & 1 else 1


def leibniz_det(M):
    """Determinant by the permutation expansion (exact)."""
    k = len(M)
    total = 0
    for p in permutations(range(k)):
        term = _perm_sign(p)
        for i in range(k):
            term = term * M[i][p[i]]
        total += term
    return total


def radic_sign(J, m):
    """(-1)^(r+s) for a 1-based ascending sequence J."""
    r = m * (m + 1) // 2
    return -1 if (r + sum(J)) & 1 else 1


def radic_bruteforce(A):
    """Definition 3 with every minor by the permutation expansion."""
    rows = _to_rows(A)
    m = len(rows)
    n = len(rows[0]) if m else 0
    if m > n:
        return 0
    total = 0
    for J0 in combinations(range(n), m):
        J = [j + 1 for j in J0]
        M = [[rows[i][j] for j in J0] for i in range(m)]
        total += radic_sign(J, m) * leibniz_det(M)
    return total


def _integerise(rows):
    """Scale each row by a power of two so every entry is an integer.
    Returns (integer rows, total exponent E) with Radic(A) = Radic(int rows) / 2^E."""
    out, E = [], 0
    for row in rows:
        k = 0
        for x in row:
            if isinstance(x, Fraction):
                d = x.denominator
                if d & (d - 1):
                    raise ValueError("entries must be dyadic rationals")
                k = max(k, d.bit_length() - 1)
        E += k
        out.append([int(Fraction(x) * (1 << k)) for x in row])
    return out, E


def radic_subset_dp(A):
    """Exact Radic determinant in O(n 2^m m) (see module docstring)."""
    rows = _to_rows(A)
    m = len(rows)
    n = len(rows[0]) if m else 0
    if m > n:
        return 0
    irows, E = _integerise(rows)
    full = (1 << m) - 1
    f = [0] * (1 << m)
    f[0] = 1
    # above[S][i]: number of rows in S with index > i
    for c in range(1, n + 1):
        g = f[:]  # column c not chosen
        for S in range(full):
            v = f[S]
            if v == 0:
                continue
            for i in range(m):
                if S >> i & 1:
                    continue
                a = irows[i][c - 1]
                if a == 0:
                    continue
                inv = bin(S >> (i + 1)).count("1")
                term = v * a
                g[S | (1 << i)] += -term if (c + inv) & 1 else term
        f = g
    r = m * (m + 1) // 2
    val = -f[full] if r & 1 else f[full]
    return Fraction(val, 1 << E) if E else val


def pfaffian(M):
    """Pfaffian of an even-order skew-symmetric matrix by exact elimination with
    symmetric row/column exchanges."""
    k = len(M)
    if k % 2:
        return 0
    A = [[Fraction(x) for x in row] for row in M]
    val = Fraction(1)
    for c in range(0, k - 1, 2):
        piv = next((i for i in range(c + 1, k) if A[c][i] != 0), None)
        if piv is None:
            return 0
        if piv != c + 1:
            A[c + 1], A[piv] = A[piv], A[c + 1]
            for row in A:
                row[c + 1], row[piv] = row[piv], row[c + 1]
            val = -val
        d = A[c][c + 1]
        val *= d
        # eliminate row/column c and c+1 couplings from the trailing block:
        # B' = B - u v^t / d + v u^t / d with u = A[c+2:, c], v = A[c+2:, c+1]
        for i in range(c + 2, k):
            ui, vi = A[i][c], A[i][c + 1]
            if ui == 0 and vi == 0:
                continue
            for j in range(c + 2, k):
                uj, vj = A[j][c], A[j][c + 1]
                A[i][j] += (vi * uj - ui * vj) / d
    return val


def pfaffian_expansion(M):
    """Pfaffian by expansion along the first row (tiny sizes only)."""
    k = len(M)
    if k == 0:
        return 1
    if k % 2:
        return 0
    total = 0
    for j in range(1, k):
        if M[0][j] == 0:
            continue
        idx = [t for t in range(k) if t not in (0, j)]
        sub = [[M[a][b] for b in idx] for a in idx]
        s = 1 if (j - 1) % 2 == 0 else -1
        total += s * M[0][j] * pfaffian_expansion(sub)
    return total


def radic_pfaffian(A):
    """Exact Radic determinant by the minor-summation formula of Pfaffians."""
    rows = _to_rows(A)
    m = len(rows)
    n = len(rows[0]) if m else 0
    if m > n:
        return 0
    T = [[(-x if (j + 1) % 2 else x) for j, x in enumerate(row)] for row in rows]
    if m % 2:
        T = [[1] + [0] * n] + [[0] + row for row in T]
    mm, nn = len(T), len(T[0])
    # S = T K T^t with K_ab = sign(b - a):  (T K)_ib = sum_{a<b} T_ia - sum_{a>b} T_ia
    TK = []
    for row in T:
        pre, tot, out = 0, sum(row), []
        for b in range(nn):
            out.append(pre - (tot - pre - row[b]))
            pre += row[b]
        TK.append(out)
    S = [[sum(TK[i][b] * T[j][b] for b in range(nn)) for j in range(mm)] for i in range(mm)]
    r = m * (m + 1) // 2
    val = pfaffian(S)
    val = -val if r & 1 else val
    if isinstance(val, Fraction) and val.denominator == 1:
        return int(val)
    return val


def hadamard_sum(A):
    """e_m of the column 2-norms: an upper bound for sum_J |det(A_J)| (Hadamard's
    inequality per minor).  Floating point; used as a normaliser for tolerances."""
    import numpy as np
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    norms = np.sqrt((A * A).sum(axis=0))
    e = [1.0] + [0.0] * m
    for x in norms:
        for k in range(m, 0, -1):
            e[k] += x * e[k - 1]
    return e[m]


def to_float(x):
    return float(Fraction(x))


def comb(n, m):
    return math.comb(n, m)
