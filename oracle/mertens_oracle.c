/*
 * Plain CPU oracle for the Mertens function M(n) = sum_{y<=n} mu(y).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU implementation: it is a slow, single-threaded, obviously
 * correct restatement of the definitions in "Computing the Mertens function
 * on a GPU" (Kuznetsov, arXiv:1108.0135).
 *
 * Three tiers:
 *
 *   O1  oracle_mu_range / oracle_mertens_table / oracle_mertens_many
 *       The exact block sieve of Section 3 (Implementation), the "naive"
 *       variant with integer products, steps 1-5: every entry starts at 1,
 *       every multiple of a prime p <= ceil(sqrt(y2)) is multiplied by -p,
 *       every multiple of p^2 is set to 0, and mu(y) is the sign of the entry
 *       when its magnitude equals y and minus that sign otherwise.  M is the
 *       running sum of mu in increasing y (Section 1 definition of M).
 *
 *   O2  oracle_mertens_identity
 *       The identity of Section 2, sum_{x=1}^{m} M(floor(m/x)) = 1, rewritten
 *       with a threshold t:
 *         M(m) = 1 - sum_{x=2}^{floor(m/t)} M(floor(m/x))
 *                  - sum_{y=1}^{t-1} (floor(m/y) - floor(m/(y+1))) M(y)
 *       and evaluated recursively (Section 2 notes the right-hand side can be
 *       computed that way), bottoming out in an O1 table M(0..T).  The
 *       printed form of this rewrite is garbled (its floor arguments are
 *       written n/(xt)); the form above is the reading used here, and it is
 *       exact for every 2 <= t <= m.
 *
 *   O3  oracle_interval
 *       Section 6: M(n) for every n in [a, b] from an exact M(a) plus the O1
 *       sieve over (a, b], and the smallest and largest M(n)/sqrt(n) there,
 *       compared exactly in integers.
 *
 * Integer conventions: hardware '/' only; products and partial sums of the
 * recursion are taken in wrapping uint64 and reinterpreted as int64 at the
 * end, which is exact because every true value of M here is far below 2^63
 * (signed overflow would be undefined behaviour in C).  M(0) = 0 (the empty
 * sum).
 *
 * Build: gcc -O2 -fPIC -shared -o liboracle.so mertens_oracle.c
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-22)
#define ORACLE_ENOMEM (-12)
#define ORACLE_ERANGE (-34)

/* floor(sqrt(v)) for any uint64, by a float estimate and exact correction. */
static uint64_t isqrt_u64(uint64_t v)
{
    uint64_t r = (uint64_t)sqrt((double)v);
    /* correct downwards while r*r > v (guarding the r*r overflow) */
    while (r > 0 && (r > 0xFFFFFFFFull || r * r > v))
        r--;
    while ((r + 1) <= 0xFFFFFFFFull && (r + 1) * (r + 1) <= v)
        r++;
    return r;
}

/* ceil(sqrt(v)) */
static uint64_t ceil_sqrt(uint64_t v)
{
    uint64_t r = isqrt_u64(v);
    if (r * r < v)
        r++;
    return r;
}

/*
 * All primes p <= limit, by the sieve of Eratosthenes on a byte array.
 * Returns a malloc'd array (caller frees) and its length; NULL on ENOMEM.
 */
static uint32_t *primes_upto(uint64_t limit, size_t *count)
{
    *count = 0;
    if (limit < 2) {
        return (uint32_t *)malloc(sizeof(uint32_t));
    }
    uint8_t *composite = (uint8_t *)calloc((size_t)limit + 1, 1);
    if (!composite)
        return NULL;
    for (uint64_t i = 2; i * i <= limit; i++)
        if (!composite[i])
            for (uint64_t j = i * i; j <= limit; j += i)
                composite[j] = 1;
    size_t n = 0;
    for (uint64_t i = 2; i <= limit; i++)
        n += !composite[i];
    uint32_t *p = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    if (!p) {
        free(composite);
        return NULL;
    }
    n = 0;
    for (uint64_t i = 2; i <= limit; i++)
        if (!composite[i])
            p[n++] = (uint32_t)i;
    free(composite);
    *count = n;
    return p;
}

/*
 * O1 core: mu(y) for y in [y1, y2], 1 <= y1 <= y2, using the sieving primes
 * `pr` (all primes <= ceil(sqrt(y2)), and possibly more).  Section 3, naive
 * block sieve, steps 1-4.  `mag`/`neg` hold |A| and sign(A) of the product.
 */
static void mu_block(uint64_t y1, uint64_t y2, const uint32_t *pr, size_t np,
                     uint64_t *mag, uint8_t *neg, int8_t *mu)
{
    size_t len = (size_t)(y2 - y1 + 1);
    /* step 1: every entry starts at 1 */
    for (size_t i = 0; i < len; i++) {
        mag[i] = 1;
        neg[i] = 0;
    }
    uint64_t plimit = ceil_sqrt(y2);
    for (size_t k = 0; k < np && pr[k] <= plimit; k++) {
        uint64_t p = pr[k];
        /* step 2: multiply the entries of multiples of p by -p */
        uint64_t r = y1 % p;
        uint64_t off = r ? p - r : 0; /* offset of the first multiple */
        for (uint64_t i = off; i < len; i += p) {
            mag[i] *= p;
            neg[i] ^= 1;
        }
        /* step 3: zero the entries of multiples of p^2 (p < 2^32) */
        uint64_t p2 = p * p;
        if (p2 > y2)
            continue;
        r = y1 % p2;
        off = r ? p2 - r : 0;
        for (uint64_t i = off; i < len; i += p2)
            mag[i] = 0;
    }
    /* step 4: classify by |A| == y and the sign of A */
    for (size_t i = 0; i < len; i++) {
        uint64_t y = y1 + i;
        if (mag[i] == 0) {
            mu[i] = 0;
        } else {
            int s = neg[i] ? -1 : 1;
            mu[i] = (int8_t)(mag[i] == y ? s : -s);
        }
    }
}

#define SUB_BLOCK ((uint64_t)1 << 20)

/*
 * mu(y) for every y in [y1, y2] written to mu[0 .. y2-y1].  y1 == 0 is
 * allowed and gives mu(0) = 0 (a convention: M(0) = 0).
 */
int oracle_mu_range(uint64_t y1, uint64_t y2, int8_t *mu)
{
    if (!mu || y2 < y1)
        return ORACLE_EINVAL;
    if (y1 == 0) {
        mu[0] = 0;
        if (y2 == 0)
            return ORACLE_OK;
        mu++;
        y1 = 1;
    }
    size_t np;
    uint32_t *pr = primes_upto(ceil_sqrt(y2), &np);
    uint64_t *mag = (uint64_t *)malloc(SUB_BLOCK * sizeof(uint64_t));
    uint8_t *neg = (uint8_t *)malloc(SUB_BLOCK);
    if (!pr || !mag || !neg) {
        free(pr); free(mag); free(neg);
        return ORACLE_ENOMEM;
    }
    for (uint64_t a = y1;; a += SUB_BLOCK) {
        uint64_t b = (y2 - a < SUB_BLOCK - 1) ? y2 : a + SUB_BLOCK - 1;
        mu_block(a, b, pr, np, mag, neg, mu + (a - y1));
        if (b == y2)
            break;
    }
    free(pr); free(mag); free(neg);
    return ORACLE_OK;
}

/*
 * M(0..N) into tab[0..N] (int32).  Section 3 step 5: add up mu in order.
 * Returns ORACLE_ERANGE if some |M| does not fit int32.
 */
int oracle_mertens_table(uint64_t N, int32_t *tab)
{
    if (!tab)
        return ORACLE_EINVAL;
    tab[0] = 0;
    if (N == 0)
        return ORACLE_OK;
    size_t np;
    uint32_t *pr = primes_upto(ceil_sqrt(N), &np);
    uint64_t *mag = (uint64_t *)malloc(SUB_BLOCK * sizeof(uint64_t));
    uint8_t *neg = (uint8_t *)malloc(SUB_BLOCK);
    int8_t *mu = (int8_t *)malloc(SUB_BLOCK);
    if (!pr || !mag || !neg || !mu) {
        free(pr); free(mag); free(neg); free(mu);
        return ORACLE_ENOMEM;
    }
    int64_t run = 0;
    int rc = ORACLE_OK;
    for (uint64_t a = 1; a <= N; a += SUB_BLOCK) {
        uint64_t b = (N - a < SUB_BLOCK - 1) ? N : a + SUB_BLOCK - 1;
        mu_block(a, b, pr, np, mag, neg, mu);
        for (uint64_t i = 0; i <= b - a; i++) {
            run += mu[i];
            if (run > INT32_MAX || run < INT32_MIN)
                rc = ORACLE_ERANGE;
            tab[a + i] = (int32_t)run;
        }
        if (b == N)
            break;
    }
    free(pr); free(mag); free(neg); free(mu);
    return rc;
}

/* insertion sort of indices by n[] (argument lists here are short) */
static void sort_idx(size_t *idx, size_t count, const uint64_t *n)
{
    for (size_t i = 1; i < count; i++) {
        size_t v = idx[i];
        size_t j = i;
        while (j > 0 && n[idx[j - 1]] > n[v]) {
            idx[j] = idx[j - 1];
            j--;
        }
        idx[j] = v;
    }
}

/*
 * O1 for a list of arguments: one sieve sweep from 1 to max(n), reading the
 * running sum M at every requested n (duplicates allowed, any order).
 */
int oracle_mertens_many(const uint64_t *n, size_t count, int64_t *out)
{
    if (count == 0)
        return ORACLE_OK;
    if (!n || !out)
        return ORACLE_EINVAL;
    size_t *idx = (size_t *)malloc(count * sizeof(size_t));
    if (!idx)
        return ORACLE_ENOMEM;
    for (size_t i = 0; i < count; i++)
        idx[i] = i;
    sort_idx(idx, count, n);
    uint64_t N = n[idx[count - 1]];
    size_t k = 0;
    while (k < count && n[idx[k]] == 0)
        out[idx[k++]] = 0;
    if (k == count) {
        free(idx);
        return ORACLE_OK;
    }
    size_t np;
    uint32_t *pr = primes_upto(ceil_sqrt(N), &np);
    uint64_t *mag = (uint64_t *)malloc(SUB_BLOCK * sizeof(uint64_t));
    uint8_t *neg = (uint8_t *)malloc(SUB_BLOCK);
    int8_t *mu = (int8_t *)malloc(SUB_BLOCK);
    if (!pr || !mag || !neg || !mu) {
        free(pr); free(mag); free(neg); free(mu); free(idx);
        return ORACLE_ENOMEM;
    }
    int64_t run = 0;
    for (uint64_t a = 1; a <= N; a += SUB_BLOCK) {
        uint64_t b = (N - a < SUB_BLOCK - 1) ? N : a + SUB_BLOCK - 1;
        mu_block(a, b, pr, np, mag, neg, mu);
        for (uint64_t i = 0; i <= b - a; i++) {
            run += mu[i];
            while (k < count && n[idx[k]] == a + i)
                out[idx[k++]] = run;
        }
        if (b == N)
            break;
    }
    free(pr); free(mag); free(neg); free(mu); free(idx);
    return ORACLE_OK;
}

/*
 * O2: M(floor(n/c)) for c = 1..L into byp[0..L-1], and M(n) into *mn, by the
 * Section 2 identity with threshold t = floor(sqrt(m)) + 1, evaluated for
 * m = floor(n/j) from the largest j with floor(n/j) > T down to j = 1, so
 * that every M(floor(m/x)) = M(floor(n/(j x))) it needs is either in the
 * table tab[0..T] or already computed (big[j x]).
 *
 * Requires T >= floor(sqrt(n)) so that every M(y), y < t, is in the table.
 * L may be 0 (then byp may be NULL).
 */
int oracle_mertens_identity(uint64_t n, const int32_t *tab, uint64_t T,
                            int64_t *mn, int64_t *byp, uint64_t L)
{
    if (!tab || !mn || (L > 0 && !byp))
        return ORACLE_EINVAL;
    if (T < isqrt_u64(n) || T < 1)
        return ORACLE_ERANGE;
    uint64_t J = n / (T + 1); /* j <= J  <=>  floor(n/j) > T */
    uint64_t *big = (uint64_t *)calloc((size_t)J + 1, sizeof(uint64_t));
    if (!big)
        return ORACLE_ENOMEM;
    for (uint64_t j = J; j >= 1; j--) {
        uint64_t m = n / j;
        uint64_t t = isqrt_u64(m) + 1; /* 2 <= t <= m because m > T >= 1 */
        uint64_t s = 1;
        /* first sum: x = 2 .. floor(m/t), arguments floor(m/x) >= t */
        uint64_t xmax = m / t;
        for (uint64_t x = 2; x <= xmax; x++) {
            uint64_t v = m / x;
            if (v <= T)
                s -= (uint64_t)(int64_t)tab[v];
            else
                s -= big[j * x]; /* floor(m/x) = floor(n/(j x)) and j x <= J */
        }
        /* second sum: y = 1 .. t-1, run-length weighted */
        for (uint64_t y = 1; y < t; y++) {
            uint64_t c = m / y - m / (y + 1);
            s -= c * (uint64_t)(int64_t)tab[y];
        }
        big[j] = s;
    }
    *mn = (n <= T) ? (int64_t)tab[n] : (int64_t)big[1];
    for (uint64_t c = 1; c <= L; c++) {
        uint64_t v = n / c;
        byp[c - 1] = (v <= T) ? (int64_t)tab[v] : (int64_t)big[c];
    }
    free(big);
    return ORACLE_OK;
}

/* floor(sqrt(v)), exported so tests can check table sizing. */
uint64_t oracle_isqrt(uint64_t v) { return isqrt_u64(v); }

/*
 * O3: Section 6, localizing an extreme between exact grid points.  Given
 * the exact value M(a) at a grid point a, every M(n) for n in [a, b] is
 * M(a) plus the sum of mu over (a, n] (the O1 sieve, Section 1 definition
 * of M), and the extremes of M(n)/sqrt(n) over the interval are read off
 * those values.
 *
 * Ratio order without rounding: for n1, n2 >= 1, M1/sqrt(n1) < M2/sqrt(n2)
 * holds when sign(M1) < sign(M2); for equal positive signs exactly when
 * M1^2 n2 < M2^2 n1; for equal negative signs exactly when M1^2 n2 > M2^2 n1;
 * never when both are zero.  Products are taken in unsigned 128-bit
 * arithmetic, which holds them while |M| < 2^32 (else ORACLE_ERANGE).  On
 * equal ratios the smaller n is kept.
 *
 * Outputs: *m_b = M(b); n_ext[0], m_ext[0] = the n in [a, b] with the
 * smallest M(n)/sqrt(n) and M there; n_ext[1], m_ext[1] the same for the
 * largest.  1 <= a <= b.
 */
static int ratio_less(int64_t m1, uint64_t n1, int64_t m2, uint64_t n2)
{
    int s1 = (m1 > 0) - (m1 < 0), s2 = (m2 > 0) - (m2 < 0);
    if (s1 != s2)
        return s1 < s2;
    if (s1 == 0)
        return 0;
    uint64_t a1 = (uint64_t)(m1 < 0 ? -m1 : m1), a2 = (uint64_t)(m2 < 0 ? -m2 : m2);
    unsigned __int128 l = (unsigned __int128)(a1 * a1) * n2;
    unsigned __int128 r = (unsigned __int128)(a2 * a2) * n1;
    return s1 > 0 ? l < r : l > r;
}

int oracle_interval(uint64_t a, uint64_t b, int64_t m_a, int64_t *m_b, uint64_t *n_ext,
                    int64_t *m_ext)
{
    if (!m_b || !n_ext || !m_ext || a == 0 || b < a)
        return ORACLE_EINVAL;
    const int64_t lim = (int64_t)1 << 32;
    int64_t m = m_a;
    uint64_t nmin = a, nmax = a;
    int64_t mmin = m_a, mmax = m_a;
    if (m >= lim || m <= -lim)
        return ORACLE_ERANGE;
    size_t np;
    uint32_t *pr = primes_upto(ceil_sqrt(b), &np);
    uint64_t *mag = (uint64_t *)malloc(SUB_BLOCK * sizeof(uint64_t));
    uint8_t *neg = (uint8_t *)malloc(SUB_BLOCK);
    int8_t *mu = (int8_t *)malloc(SUB_BLOCK);
    if (!pr || !mag || !neg || !mu) {
        free(pr); free(mag); free(neg); free(mu);
        return ORACLE_ENOMEM;
    }
    int rc = ORACLE_OK;
    for (uint64_t c = a; c < b && rc == ORACLE_OK; c += SUB_BLOCK) {
        /* mu over (c, c2] */
        uint64_t c2 = (b - c <= SUB_BLOCK) ? b : c + SUB_BLOCK;
        mu_block(c + 1, c2, pr, np, mag, neg, mu);
        for (uint64_t i = 0; i < c2 - c; i++) {
            uint64_t n = c + 1 + i;
            m += mu[i];
            if (m >= lim || m <= -lim) {
                rc = ORACLE_ERANGE;
                break;
            }
            /* n only grows, so a tie keeps the earlier n */
            if (ratio_less(m, n, mmin, nmin)) {
                nmin = n;
                mmin = m;
            }
            if (ratio_less(mmax, nmax, m, n)) {
                nmax = n;
                mmax = m;
            }
        }
        if (c2 == b)
            break;
    }
    free(pr); free(mag); free(neg); free(mu);
    if (rc != ORACLE_OK)
        return rc;
    *m_b = m;
    n_ext[0] = nmin;
    m_ext[0] = mmin;
    n_ext[1] = nmax;
    m_ext[1] = mmax;
    return ORACLE_OK;
}
