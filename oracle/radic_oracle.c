/*
 * Oracle for the Radic determinant -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU evaluation of the Radic determinant of an
 * m x n matrix (m <= n) exactly as Definition 3, eq. (1) states it:
 *
 *     det(A) = sum over 1 <= j1 < ... < jm <= n of (-1)^(r+s) det(A[:, {j1..jm}]),
 *     r = 1 + 2 + ... + m,  s = j1 + ... + jm  (1-based column indices),
 *     and det(A) = 0 when m > n.
 *
 * The column subsets are visited in dictionary order (Section 3, Definitions 1-2):
 * the First Member [1, 2, ..., m], then successive successors (Section 5, the
 * "dictionary sequence" procedure), which Theorem 1 says reaches every one of the
 * C(n, m) ascending sequences exactly once.  A thread that starts in the middle
 * of the order obtains its first sequence from its rank with the "combinatorial
 * addition" of Section 4.  Threads take contiguous rank ranges (the granularity
 * scheme of Section 5) and their partial results are merged in rank order, so the
 * output does not depend on the thread count beyond floating-point reassociation
 * at chunk boundaries (the compensated sum makes that negligible).
 *
 * Floating point: each m x m minor by Gaussian elimination with partial pivoting
 * in IEEE double (first row attaining the largest |a_ik| is the pivot; true
 * division), signed terms summed with Neumaier's compensated summation; the sum of
 * |minor| is reported beside the value.
 * Integers: each minor by Bareiss's fraction-free elimination in exact
 * multi-precision integers, summed exactly.
 *
 * Only tests/, the benchmark's CPU-baseline leg and the smoke check may load this
 * library.  It shares no code with the GPU library.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_M 64

/* ---------------------------------------------------------------------------
 * Binomial coefficients (Theorem 1 counts C(n, m) sequences).
 * Multiplicative formula with an exact division at every step; returns 0 and
 * sets *ovf when the value does not fit in 64 bits.
 * ------------------------------------------------------------------------- */
static uint64_t binom_u64(int a, int b, int *ovf)
{
    if (b < 0 || a < 0 || b > a) return 0;
    if (b > a - b) b = a - b;
    unsigned __int128 v = 1;
    for (int i = 1; i <= b; ++i) {
        v = v * (unsigned __int128)(a - b + i) / (unsigned __int128)i;
        if (v > (unsigned __int128)UINT64_MAX) { *ovf = 1; return 0; }
    }
    return (uint64_t)v;
}

uint64_t oracle_binomial(int a, int b, int *overflow)
{
    int ovf = 0;
    uint64_t v = binom_u64(a, b, &ovf);
    if (overflow) *overflow = ovf;
    return v;
}

/* ---------------------------------------------------------------------------
 * Section 4, combinatorial addition: the q-th (0-based) ascending sequence.
 *
 * Start from the First Member B = [1, 2, ..., m].  For place k = 1..m, the
 * sequences that keep B_1..B_{k-1} and put the value v at place k number
 * C(n - v, m - k) (the Pascal-table weight of that place).  While q is at least
 * that weight, take one step to the left in the table: subtract the weight from
 * q and add one unit to the last m - k + 1 places.  When q can no longer pay for
 * a step, move to the next place.  (The conditions printed in Section 4 are
 * inconsistent about < versus <=; this is the reading that reproduces Table 2 and
 * the q = 49 example.)
 * B is 1-based values stored in B[0..m-1].
 * ------------------------------------------------------------------------- */
void oracle_unrank(uint64_t q, int m, int n, int *B)
{
    int ovf = 0;
    for (int i = 0; i < m; ++i) B[i] = i + 1;
    for (int k = 1; k <= m; ++k) {
        for (;;) {
            uint64_t w = binom_u64(n - B[k - 1], m - k, &ovf);
            if (q < w) break;
            q -= w;
            for (int j = k - 1; j < m; ++j) B[j] += 1;
        }
    }
}

/* Trace of the combinatorial addition: for each place k that moves, the number
 * of steps p and the value of q afterwards, as in the worked example of
 * Section 4.  Returns the number of recorded moves (at most m). */
int oracle_unrank_trace(uint64_t q, int m, int n, int *B, int *trace_k, int *trace_p,
                        uint64_t *trace_q, int *trace_B)
{
    int ovf = 0, moves = 0;
    for (int i = 0; i < m; ++i) B[i] = i + 1;
    for (int k = 1; k <= m; ++k) {
        int p = 0;
        for (;;) {
            uint64_t w = binom_u64(n - B[k - 1], m - k, &ovf);
            if (q < w) break;
            q -= w;
            for (int j = k - 1; j < m; ++j) B[j] += 1;
            ++p;
        }
        if (p > 0) {
            trace_k[moves] = k;
            trace_p[moves] = p;
            trace_q[moves] = q;
            memcpy(trace_B + (size_t)moves * m, B, sizeof(int) * (size_t)m);
            ++moves;
        }
    }
    return moves;
}

/* ---------------------------------------------------------------------------
 * Section 5, dictionary sequence: the successor of B in dictionary order.
 * The rightmost place i whose value is below its largest possible value n-m+i
 * is increased by one and the places after it are refilled consecutively.
 * Returns 0 when B is already the last member [n-m+1, ..., n].
 * ------------------------------------------------------------------------- */
int oracle_successor(int *B, int m, int n)
{
    int i = m - 1;
    while (i >= 0 && B[i] == n - m + i + 1) --i;
    if (i < 0) return 0;
    B[i] += 1;
    for (int j = i + 1; j < m; ++j) B[j] = B[j - 1] + 1;
    return 1;
}

/* (-1)^(r+s) of Definition 3 for a 1-based ascending sequence. */
static int radic_sign(const int *B, int m)
{
    long r = (long)m * (m + 1) / 2, s = 0;
    for (int i = 0; i < m; ++i) s += B[i];
    return ((r + s) & 1) ? -1 : 1;
}

/* ---------------------------------------------------------------------------
 * Determinant of an m x m row-major matrix by Gaussian elimination with partial
 * pivoting (the matrix is overwritten).  An exactly zero pivot column gives 0.
 * ------------------------------------------------------------------------- */
static double det_gepp(double *M, int m)
{
    double det = 1.0;
    for (int k = 0; k < m; ++k) {
        int p = k;
        double best = fabs(M[k * m + k]);
        for (int i = k + 1; i < m; ++i) {
            double v = fabs(M[i * m + k]);
            if (v > best) { best = v; p = i; }
        }
        if (best == 0.0) return 0.0;
        if (p != k) {
            for (int j = 0; j < m; ++j) {
                double t = M[k * m + j];
                M[k * m + j] = M[p * m + j];
                M[p * m + j] = t;
            }
            det = -det;
        }
        double piv = M[k * m + k];
        det *= piv;
        for (int i = k + 1; i < m; ++i) {
            double l = M[i * m + k] / piv;
            for (int j = k + 1; j < m; ++j) M[i * m + j] -= l * M[k * m + j];
        }
    }
    return det;
}

/* Neumaier's improved Kahan summation. */
typedef struct { double s, c; } nsum;

static void nsum_add(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

static void gather_f64(const double *A, int64_t lda, int m, const int *B, double *M)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) M[i * m + j] = A[(int64_t)i * lda + (B[j] - 1)];
}

/* Signed term (-1)^(r+s) det(A_J) of the q-th sequence, and its columns. */
double oracle_subset_term_f64(const double *A, int m, int n, int64_t lda, uint64_t q, int *B_out)
{
    int B[ORACLE_MAX_M];
    double M[ORACLE_MAX_M * ORACLE_MAX_M];
    oracle_unrank(q, m, n, B);
    gather_f64(A, lda, m, B, M);
    if (B_out) memcpy(B_out, B, sizeof(int) * (size_t)m);
    return radic_sign(B, m) * det_gepp(M, m);
}

/* The signed terms (-1)^(r+s) det(A_J) of ranks q0 .. q0+count-1, in rank order,
 * each computed exactly as the summing loop below computes it (one thread, the
 * successor of Section 5 between ranks).  Lets a test check the compensated sum
 * against a correctly rounded sum of the very same terms.  Returns 0, or -1 for
 * bad arguments / a range past the end. */
int oracle_subset_terms_f64(const double *A, int m, int n, int64_t lda, uint64_t q0, uint64_t count, double *out)
{
    if (m < 1 || n < m || m > ORACLE_MAX_M || lda < n) return -1;
    int ovf = 0;
    uint64_t total = binom_u64(n, m, &ovf);
    if (ovf || q0 > total || count > total - q0) return -1;
    int B[ORACLE_MAX_M];
    double M[ORACLE_MAX_M * ORACLE_MAX_M];
    if (count == 0) return 0;
    oracle_unrank(q0, m, n, B);
    for (uint64_t t = 0; t < count; ++t) {
        gather_f64(A, lda, m, B, M);
        out[t] = radic_sign(B, m) * det_gepp(M, m);
        if (t + 1 < count) oracle_successor(B, m, n);
    }
    return 0;
}

typedef struct {
    const double *A;
    int64_t lda;
    int m, n;
    uint64_t q0, count;
    nsum val, abs;
} f64_job;

static void *f64_worker(void *arg)
{
    f64_job *jb = (f64_job *)arg;
    int B[ORACLE_MAX_M];
    double M[ORACLE_MAX_M * ORACLE_MAX_M];
    jb->val.s = jb->val.c = jb->abs.s = jb->abs.c = 0.0;
    if (jb->count == 0) return NULL;
    oracle_unrank(jb->q0, jb->m, jb->n, B);
    for (uint64_t t = 0; t < jb->count; ++t) {
        gather_f64(jb->A, jb->lda, jb->m, B, M);
        double d = det_gepp(M, jb->m);
        nsum_add(&jb->val, radic_sign(B, jb->m) * d);
        nsum_add(&jb->abs, fabs(d));
        if (t + 1 < jb->count) oracle_successor(B, jb->m, jb->n);
    }
    return NULL;
}

/*
 * Radic determinant over the rank range [q0, q0 + count) (count = 0 means all
 * ranks from q0 to the end).  out[0] = value (s + c of the compensated sum),
 * out[1] = s, out[2] = c, out[3] = sum of |det(A_J)|.
 * Returns 0 on success, -1 for bad arguments, -3 when C(n, m) overflows 64 bits.
 */
int oracle_radic_f64_range(const double *A, int m, int n, int64_t lda, uint64_t q0,
                           uint64_t count, int nthreads, double *out)
{
    out[0] = out[1] = out[2] = out[3] = 0.0;
    if (m < 1 || n < 1 || m > ORACLE_MAX_M || lda < n) return -1;
    if (m > n) return 0; /* Definition 3: det(A) = 0 when m > n */
    int ovf = 0;
    uint64_t total = binom_u64(n, m, &ovf);
    if (ovf) return -3;
    if (q0 >= total) return 0;
    if (count == 0 || count > total - q0) count = total - q0;
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > count) nthreads = (int)count;

    f64_job *jobs = (f64_job *)calloc((size_t)nthreads, sizeof(f64_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; ++t) {
        /* contiguous chunk [floor(t*count/k), floor((t+1)*count/k)) */
        uint64_t a = (uint64_t)(((unsigned __int128)count * t) / nthreads);
        uint64_t b = (uint64_t)(((unsigned __int128)count * (t + 1)) / nthreads);
        jobs[t] = (f64_job){A, lda, m, n, q0 + a, b - a, {0, 0}, {0, 0}};
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, f64_worker, &jobs[t]);
    f64_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);

    nsum val = {0, 0}, ab = {0, 0};
    for (int t = 0; t < nthreads; ++t) { /* merge in rank order */
        nsum_add(&val, jobs[t].val.s);
        nsum_add(&val, jobs[t].val.c);
        nsum_add(&ab, jobs[t].abs.s);
        nsum_add(&ab, jobs[t].abs.c);
    }
    out[0] = val.s + val.c;
    out[1] = val.s;
    out[2] = val.c;
    out[3] = ab.s + ab.c;
    free(jobs);
    free(th);
    return 0;
}

/* ===========================================================================
 * Exact integers: sign-magnitude multi-precision integers with 32-bit limbs.
 * ========================================================================= */
#define BIG_LIMBS 96 /* 3072 bits: Bareiss products for m <= 16 int32 inputs need < 1100 */

typedef struct {
    int len;  /* number of significant limbs, 0 for zero */
    int neg;  /* 1 when negative (never set for zero) */
    uint32_t d[BIG_LIMBS];
} big;

static int big_overflow = 0; /* sticky; checked by callers (benign race: only ever set to 1) */

static void big_norm(big *a)
{
    while (a->len > 0 && a->d[a->len - 1] == 0) a->len--;
    if (a->len == 0) a->neg = 0;
}

static void big_set_i64(big *a, int64_t v)
{
    uint64_t u = v < 0 ? (uint64_t)(-(v + 1)) + 1u : (uint64_t)v;
    a->neg = v < 0;
    a->d[0] = (uint32_t)u;
    a->d[1] = (uint32_t)(u >> 32);
    a->len = 2;
    big_norm(a);
}

/* |a| compared with |b| */
static int big_cmp_mag(const big *a, const big *b)
{
    if (a->len != b->len) return a->len < b->len ? -1 : 1;
    for (int i = a->len - 1; i >= 0; --i)
        if (a->d[i] != b->d[i]) return a->d[i] < b->d[i] ? -1 : 1;
    return 0;
}

/* r = |a| + |b| (magnitudes) */
static void mag_add(big *r, const big *a, const big *b)
{
    int n = a->len > b->len ? a->len : b->len;
    uint64_t carry = 0;
    for (int i = 0; i < n; ++i) {
        uint64_t s = carry + (i < a->len ? a->d[i] : 0) + (i < b->len ? b->d[i] : 0);
        r->d[i] = (uint32_t)s;
        carry = s >> 32;
    }
    if (carry) {
        if (n >= BIG_LIMBS) { big_overflow = 1; return; }
        r->d[n++] = (uint32_t)carry;
    }
    r->len = n;
}

/* r = |a| - |b|, requires |a| >= |b| */
static void mag_sub(big *r, const big *a, const big *b)
{
    int64_t borrow = 0;
    for (int i = 0; i < a->len; ++i) {
        int64_t s = (int64_t)a->d[i] - (i < b->len ? b->d[i] : 0) - borrow;
        borrow = s < 0;
        r->d[i] = (uint32_t)(s + (borrow ? ((int64_t)1 << 32) : 0));
    }
    r->len = a->len;
}

/* r = a + b (signed); r may alias a or b */
static void big_add(big *r, const big *a, const big *b)
{
    big t;
    if (a->neg == b->neg) {
        mag_add(&t, a, b);
        t.neg = a->neg;
    } else if (big_cmp_mag(a, b) >= 0) {
        mag_sub(&t, a, b);
        t.neg = a->neg;
    } else {
        mag_sub(&t, b, a);
        t.neg = b->neg;
    }
    big_norm(&t);
    *r = t;
}

static void big_sub(big *r, const big *a, const big *b)
{
    big nb = *b;
    if (nb.len) nb.neg = !nb.neg;
    big_add(r, a, &nb);
}

/* r = a * b (schoolbook) */
static void big_mul(big *r, const big *a, const big *b)
{
    big t;
    if (a->len == 0 || b->len == 0) { t.len = 0; t.neg = 0; *r = t; return; }
    int n = a->len + b->len;
    if (n > BIG_LIMBS) { big_overflow = 1; r->len = 0; r->neg = 0; return; }
    memset(t.d, 0, sizeof(uint32_t) * (size_t)n);
    for (int i = 0; i < a->len; ++i) {
        uint64_t carry = 0;
        for (int j = 0; j < b->len; ++j) {
            uint64_t cur = (uint64_t)a->d[i] * b->d[j] + t.d[i + j] + carry;
            t.d[i + j] = (uint32_t)cur;
            carry = cur >> 32;
        }
        t.d[i + b->len] = (uint32_t)carry;
    }
    t.len = n;
    t.neg = a->neg ^ b->neg;
    big_norm(&t);
    *r = t;
}

/* shift magnitude right by s bits (0 <= s) */
static void mag_shr(big *a, int s)
{
    int limbs = s / 32, bits = s % 32;
    if (limbs >= a->len) { a->len = 0; a->neg = 0; return; }
    for (int i = 0; i < a->len - limbs; ++i) {
        uint64_t lo = a->d[i + limbs];
        uint64_t hi = (i + limbs + 1 < a->len) ? a->d[i + limbs + 1] : 0;
        a->d[i] = (uint32_t)(((hi << 32) | lo) >> bits);
    }
    a->len -= limbs;
    big_norm(a);
}

/*
 * q = a / b where b divides a exactly (Jebelean's exact division, 1993): after
 * removing the common power of two, b is odd and has an inverse modulo 2^32;
 * each quotient limb is the current low limb of the dividend times that inverse,
 * and the dividend is reduced by that limb times b.  Exactness is what Bareiss's
 * algorithm guarantees; it is checked (remainder must vanish).
 */
static int big_divexact(big *q, const big *a, const big *b)
{
    if (b->len == 0) return -1;
    if (a->len == 0) { q->len = 0; q->neg = 0; return 0; }
    big x = *a, y = *b;
    int tz = 0;
    while (((y.d[tz / 32] >> (tz % 32)) & 1u) == 0) ++tz;
    mag_shr(&x, tz);
    mag_shr(&y, tz);
    uint32_t y0 = y.d[0], inv = y0; /* Newton iteration for y0^-1 mod 2^32 */
    for (int i = 0; i < 5; ++i) inv *= 2u - y0 * inv;
    int qlen = x.len - y.len + 1;
    if (qlen <= 0) return -1;
    big r;
    memset(r.d, 0, sizeof(r.d));
    for (int i = 0; i < qlen; ++i) {
        uint32_t qi = x.d[i] * inv;
        r.d[i] = qi;
        /* x -= qi * y << (32 i) */
        uint64_t borrow = 0, carry = 0;
        for (int j = 0; i + j < x.len; ++j) {
            uint64_t prod = (j < y.len ? (uint64_t)qi * y.d[j] : 0) + carry;
            carry = prod >> 32;
            uint64_t sub = (uint64_t)(uint32_t)prod + borrow;
            uint64_t cur = x.d[i + j];
            borrow = cur < sub;
            x.d[i + j] = (uint32_t)(cur - sub);
        }
    }
    for (int i = 0; i < x.len; ++i)
        if (x.d[i] != 0) return -2; /* not an exact division */
    r.len = qlen;
    r.neg = a->neg ^ b->neg;
    big_norm(&r);
    *q = r;
    return 0;
}

/* Bareiss fraction-free elimination; M is m x m row-major, overwritten.
 * Row exchange on a zero pivot: first nonzero entry below; none gives 0. */
static int det_bareiss(big *M, int m, big *det)
{
    big prev, t1, t2;
    big_set_i64(&prev, 1);
    int sign = 1;
    for (int k = 0; k < m - 1; ++k) {
        if (M[k * m + k].len == 0) {
            int p = -1;
            for (int i = k + 1; i < m; ++i)
                if (M[i * m + k].len != 0) { p = i; break; }
            if (p < 0) { big_set_i64(det, 0); return 0; }
            for (int j = 0; j < m; ++j) {
                big t = M[k * m + j];
                M[k * m + j] = M[p * m + j];
                M[p * m + j] = t;
            }
            sign = -sign;
        }
        for (int i = k + 1; i < m; ++i) {
            for (int j = k + 1; j < m; ++j) {
                /* M_ij <- (M_kk M_ij - M_ik M_kj) / prev */
                big_mul(&t1, &M[k * m + k], &M[i * m + j]);
                big_mul(&t2, &M[i * m + k], &M[k * m + j]);
                big_sub(&t1, &t1, &t2);
                if (big_divexact(&M[i * m + j], &t1, &prev) != 0) return -2;
            }
        }
        prev = M[k * m + k];
    }
    *det = M[(m - 1) * m + (m - 1)];
    if (sign < 0 && det->len) det->neg = !det->neg;
    return 0;
}

typedef struct {
    const int32_t *A;
    int64_t lda;
    int m, n;
    uint64_t q0, count;
    big sum;
    int err;
} int_job;

static void *int_worker(void *arg)
{
    int_job *jb = (int_job *)arg;
    int m = jb->m, B[ORACLE_MAX_M];
    big *M = (big *)malloc(sizeof(big) * (size_t)m * (size_t)m);
    big d;
    big_set_i64(&jb->sum, 0);
    jb->err = 0;
    if (!M) { jb->err = -4; return NULL; }
    if (jb->count) oracle_unrank(jb->q0, m, jb->n, B);
    for (uint64_t t = 0; t < jb->count; ++t) {
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) big_set_i64(&M[i * m + j], jb->A[(int64_t)i * jb->lda + (B[j] - 1)]);
        if (det_bareiss(M, m, &d) != 0) { jb->err = -2; break; }
        if (radic_sign(B, m) < 0 && d.len) d.neg = !d.neg;
        big_add(&jb->sum, &jb->sum, &d);
        if (t + 1 < jb->count) oracle_successor(B, m, jb->n);
    }
    free(M);
    return NULL;
}

/*
 * Exact Radic determinant of an int32 matrix over ranks [q0, q0 + count)
 * (count = 0: to the end).  The result is written as sign (*sign = -1, 0, +1)
 * and little-endian 32-bit magnitude limbs mag[0..*len-1].
 * Returns 0, -1 bad arguments, -2 internal arithmetic check failed,
 * -3 C(n, m) overflow or result larger than cap limbs (then *len = needed).
 */
int oracle_radic_int_range(const int32_t *A, int m, int n, int64_t lda, uint64_t q0, uint64_t count,
                           int nthreads, uint32_t *mag, int cap, int *len, int *sign)
{
    *len = 0;
    *sign = 0;
    if (m < 1 || n < 1 || m > ORACLE_MAX_M || lda < n) return -1;
    if (m > n) return 0;
    int ovf = 0;
    uint64_t total = binom_u64(n, m, &ovf);
    if (ovf) return -3;
    if (q0 >= total) return 0;
    if (count == 0 || count > total - q0) count = total - q0;
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > count) nthreads = (int)count;
    big_overflow = 0;

    int_job *jobs = (int_job *)calloc((size_t)nthreads, sizeof(int_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; ++t) {
        uint64_t a = (uint64_t)(((unsigned __int128)count * t) / nthreads);
        uint64_t b = (uint64_t)(((unsigned __int128)count * (t + 1)) / nthreads);
        jobs[t].A = A;
        jobs[t].lda = lda;
        jobs[t].m = m;
        jobs[t].n = n;
        jobs[t].q0 = q0 + a;
        jobs[t].count = b - a;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, int_worker, &jobs[t]);
    int_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);

    int rc = 0;
    big total_sum;
    big_set_i64(&total_sum, 0);
    for (int t = 0; t < nthreads; ++t) {
        if (jobs[t].err) rc = jobs[t].err;
        big_add(&total_sum, &total_sum, &jobs[t].sum);
    }
    free(jobs);
    free(th);
    if (big_overflow) return -2;
    if (rc) return rc;
    *len = total_sum.len;
    if (total_sum.len > cap) return -3;
    for (int i = 0; i < total_sum.len; ++i) mag[i] = total_sum.d[i];
    *sign = total_sum.len == 0 ? 0 : (total_sum.neg ? -1 : 1);
    return 0;
}

/* Signed exact term (-1)^(r+s) det(A_J) of the q-th sequence (for sampled checks). */
int oracle_subset_term_int(const int32_t *A, int m, int n, int64_t lda, uint64_t q, uint32_t *mag,
                           int cap, int *len, int *sign)
{
    return oracle_radic_int_range(A, m, n, lda, q, 1, 1, mag, cap, len, sign);
}
