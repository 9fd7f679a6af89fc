/*
 * oracle.c -- plain CPU reference for elementwise primality of uint64 values.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's cpu_baseline leg may load this library.  The product path (the
 * HIP library under paper_2108_04791_amd/) never links, loads or calls it, and
 * this file shares no code, header or table with that path.
 *
 * Everything here is deliberately slow and obvious:
 *   O1  oracle_trial_is_prime  -- the definition of primality, written out
 *                                 (trial division, paper section 1: divide by
 *                                 candidates up to the square root).
 *   O2  oracle_sieve_odd       -- textbook Eratosthenes on odd numbers only
 *                                 (section 1 for the sieve, section 4 for the
 *                                 2-wheel), one flat unsegmented loop.
 *   O3  oracle_mulmod/powmod   -- modular product through a 128-bit integer
 *                                 and right-to-left square-and-multiply
 *                                 (sections 2.3-2.4 compute the same values
 *                                 without 128-bit products).
 *   O4  oracle_mr7             -- the strong probable-prime test of section
 *                                 2.1 (Eq. 1-3, read as the standard Miller
 *                                 and Rabin test) over the seven bases of
 *                                 Eq. 4, in the paper's order.
 *   O5  oracle_is_prime        -- dispatch: n < 2^32 by the O2 table, larger
 *                                 odd n by O4.
 *   O6  certificates           -- a nontrivial factor for composites (Pollard
 *                                 rho, Brent's cycle finding) and a Pratt
 *                                 (Lucas) certificate for primes.  Neither
 *                                 relies on the seven-base claim.
 *   O7  oracle_numdiv          -- the division count of MATLAB's isprime on
 *                                 1:N (section 6, Table NumDiv).
 *   O8  oracle_wheel_is_prime  -- trial division on the 2/3/5/7 wheel of
 *                                 section 3: 2, 3, 5, 7, then 1 plus the
 *                                 running sum of the period-210 difference
 *                                 cycle of Eq. 5 (the Eq. 6 construction),
 *                                 up to the square root.
 *
 * Readings of the paper taken here:
 *   - Eq. 1 prints "+-1"; Fermat's theorem gives 1.  Eq. 2-3 and the
 *     sentence after them are read as the strong test: n prime implies
 *     a^d = 1 or a^(2^r d) = -1 (mod n) for some 0 <= r < s.
 *   - A base that is 0 modulo n says nothing and is skipped (the paper is
 *     silent; for n >= 2^32 no base is reduced at all, since every base is
 *     below 2^31).
 *   - The input domain "0 to 2^64" is [0, 2^64 - 1]; 0 and 1 are not prime.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ O1 */

/* n is prime iff n >= 2 and no d with 2 <= d <= floor(sqrt(n)) divides n.
 * "d <= n / d" is the same test as d*d <= n, without overflow. */
int oracle_trial_is_prime(uint64_t n)
{
    if (n < 2)
        return 0;
    for (uint64_t d = 2; d <= n / d; ++d)
        if (n % d == 0)
            return 0;
    return 1;
}

/* ------------------------------------------------------------------ O2 */

/* Number of 32-bit words in the odd-only table for numbers below `limit`:
 * bit i stands for the odd number 2i+1, and floor(limit/2) odd numbers lie
 * below `limit`. */
uint64_t oracle_sieve_words(uint64_t limit)
{
    uint64_t nbits = limit / 2;
    return (nbits + 31) / 32;
}

static inline void clear_bit(uint32_t *t, uint64_t i) { t[i >> 5] &= ~(1u << (i & 31)); }
static inline int get_bit(const uint32_t *t, uint64_t i) { return (t[i >> 5] >> (i & 31)) & 1u; }

/* Sieve of Eratosthenes over odd numbers below `limit` (limit <= 2^32).
 * Bit i of the result (bit i&31 of word i>>5) is 1 iff 2i+1 is prime.
 * Start with every odd number marked, unmark 1, then for every odd p with
 * p*p < limit that is still marked, unmark p*p, p*p+2p, p*p+4p, ...
 * Bits past the last odd number below `limit` are left 0. */
void oracle_sieve_odd(uint64_t limit, uint32_t *bits)
{
    uint64_t nbits = limit / 2;
    uint64_t nwords = (nbits + 31) / 32;
    memset(bits, 0xff, nwords * sizeof(uint32_t));
    for (uint64_t i = nbits; i < nwords * 32; ++i)
        clear_bit(bits, i);
    if (nbits > 0)
        clear_bit(bits, 0); /* 1 is not prime */
    for (uint64_t p = 3; p * p < limit; p += 2) {
        if (!get_bit(bits, p >> 1))
            continue;
        for (uint64_t m = p * p; m < limit; m += 2 * p)
            clear_bit(bits, m >> 1);
    }
}

/* ------------------------------------------------------------------ O3 */

uint64_t oracle_mulmod(uint64_t a, uint64_t b, uint64_t n)
{
    return (uint64_t)(((u128)a * b) % n);
}

/* a^e mod n by right-to-left binary exponentiation (section 2.4). */
uint64_t oracle_powmod(uint64_t a, uint64_t e, uint64_t n)
{
    uint64_t result = 1 % n;
    uint64_t base = a % n;
    while (e) {
        if (e & 1)
            result = oracle_mulmod(result, base, n);
        base = oracle_mulmod(base, base, n);
        e >>= 1;
    }
    return result;
}

/* ------------------------------------------------------------------ O4 */

/* The seven bases of Eq. 4, in the order the paper lists them. */
static const uint64_t MR_BASES[7] = {2u, 325u, 9375u, 28178u, 450775u,
                                     9780504u, 1795265022u};

/* Base number k (0..6) as the oracle holds it, for the test that compares
 * the constants with Eq. 4; 0 outside that range. */
uint64_t oracle_mr_base(int k)
{
    return (k >= 0 && k < 7) ? MR_BASES[k] : 0;
}

/* One round of the strong probable-prime test: with n - 1 = 2^s d, d odd,
 * n passes for base a iff a^d = 1 or a^(2^r d) = n-1 for some 0 <= r < s. */
int oracle_strong_probable_prime(uint64_t n, uint64_t a)
{
    uint64_t d = n - 1;
    unsigned s = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        ++s;
    }
    uint64_t x = oracle_powmod(a, d, n);
    if (x == 1 || x == n - 1)
        return 1;
    for (unsigned r = 1; r < s; ++r) {
        x = oracle_mulmod(x, x, n);
        if (x == n - 1)
            return 1;
    }
    return 0;
}

/* Deterministic Miller-Rabin over the seven bases, for odd n >= 3.
 * A base that is 0 modulo n is skipped.  Returns 1 (prime) or 0. */
int oracle_mr7(uint64_t n)
{
    for (int k = 0; k < 7; ++k) {
        uint64_t a = MR_BASES[k] % n;
        if (a == 0)
            continue;
        if (!oracle_strong_probable_prime(n, a))
            return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------ O5 */

#define TABLE_BOUND ((uint64_t)1 << 32)

/* Primality of one value.  `table` is the O2 table for limit 2^32, or NULL,
 * in which case values below 2^32 go through O1. */
int oracle_is_prime(uint64_t n, const uint32_t *table)
{
    if (n < 2)
        return 0;
    if (n == 2)
        return 1;
    if ((n & 1) == 0)
        return 0;
    if (n < TABLE_BOUND)
        return table ? get_bit(table, n >> 1) : oracle_trial_is_prime(n);
    return oracle_mr7(n);
}

/* ------------------------------------------------------------------ O8 */

/* The difference cycle of the 2/3/5/7 wheel as the paper prints it (section
 * 3, Eq. 5): 48 gaps between consecutive numbers coprime to 210, starting
 * from 1, that repeat every 210. */
static const uint8_t WHEEL_DIFF[48] = {
    10, 2, 4, 2, 4, 6, 2, 6, 4, 2, 4, 6, 6, 2, 6, 4, 2, 6, 4, 6, 8, 4, 2, 4,
    2, 4, 8, 6, 4, 6, 2, 4, 6, 2, 6, 6, 4, 2, 4, 6, 2, 6, 4, 2, 4, 2, 10, 2};

/* Copies the cycle out (for the tests that pin it); returns its length. */
int oracle_wheel_cycle(uint8_t *out)
{
    memcpy(out, WHEEL_DIFF, sizeof(WHEEL_DIFF));
    return (int)sizeof(WHEEL_DIFF);
}

/* Section 3's medium-integer method: the removed primes 2, 3, 5, 7 are
 * tried first; then the divisors are 1 + the running sum of the repeated
 * cycle (11, 13, 17, ...), each tried while d <= floor(sqrt(n)). */
int oracle_wheel_is_prime(uint64_t n)
{
    static const uint64_t removed[4] = {2, 3, 5, 7};
    if (n < 2)
        return 0;
    for (int i = 0; i < 4; ++i) {
        if (n == removed[i])
            return 1;
        if (n % removed[i] == 0)
            return 0;
    }
    uint64_t d = 1;
    for (int k = 0;; k = (k + 1) % 48) {
        d += WHEEL_DIFF[k];
        if (d > n / d)  /* d*d > n: no divisor up to the root */
            return 1;
        if (n % d == 0)
            return 0;
    }
}

/* Which per-element function an array call applies. */
enum { APPLY_IS_PRIME = 0, APPLY_TRIAL = 1, APPLY_MR7 = 2, APPLY_WHEEL = 3 };

struct chunk {
    const uint64_t *n;
    uint8_t *out;
    uint64_t len;
    const uint32_t *table;
    int mode;
};

static void *chunk_worker(void *arg)
{
    struct chunk *c = (struct chunk *)arg;
    for (uint64_t i = 0; i < c->len; ++i) {
        uint64_t v = c->n[i];
        int r;
        if (c->mode == APPLY_TRIAL)
            r = oracle_trial_is_prime(v);
        else if (c->mode == APPLY_MR7)
            r = (v >= 3 && (v & 1)) ? oracle_mr7(v) : 0;
        else if (c->mode == APPLY_WHEEL)
            r = oracle_wheel_is_prime(v);
        else
            r = oracle_is_prime(v, c->table);
        c->out[i] = (uint8_t)r;
    }
    return NULL;
}

static int apply_array(const uint64_t *n, uint8_t *out, uint64_t len,
                       const uint32_t *table, int nthreads, int mode)
{
    if (nthreads < 1)
        nthreads = 1;
    if ((uint64_t)nthreads > len)
        nthreads = len ? (int)len : 1;
    struct chunk *cs = (struct chunk *)calloc((size_t)nthreads, sizeof(*cs));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(*th));
    uint64_t per = len / (uint64_t)nthreads, rem = len % (uint64_t)nthreads, off = 0;
    for (int t = 0; t < nthreads; ++t) {
        uint64_t l = per + ((uint64_t)t < rem ? 1 : 0);
        cs[t].n = n + off;
        cs[t].out = out + off;
        cs[t].len = l;
        cs[t].table = table;
        cs[t].mode = mode;
        off += l;
    }
    for (int t = 1; t < nthreads; ++t)
        pthread_create(&th[t], NULL, chunk_worker, &cs[t]);
    chunk_worker(&cs[0]);
    for (int t = 1; t < nthreads; ++t)
        pthread_join(th[t], NULL);
    free(cs);
    free(th);
    return nthreads;
}

/* out[i] = oracle_is_prime(n[i]) for i < len, split into `nthreads`
 * contiguous chunks on POSIX threads.  Returns the number of threads used. */
int oracle_isprime_array(const uint64_t *n, uint8_t *out, uint64_t len,
                         const uint32_t *table, int nthreads)
{
    return apply_array(n, out, len, table, nthreads, APPLY_IS_PRIME);
}

/* out[i] = oracle_trial_is_prime(n[i]) (O1 alone), threaded as above. */
int oracle_trial_array(const uint64_t *n, uint8_t *out, uint64_t len, int nthreads)
{
    return apply_array(n, out, len, NULL, nthreads, APPLY_TRIAL);
}

/* out[i] = oracle_mr7(n[i]) for odd n[i] >= 3, else 0 (O4 alone). */
int oracle_mr7_array(const uint64_t *n, uint8_t *out, uint64_t len, int nthreads)
{
    return apply_array(n, out, len, NULL, nthreads, APPLY_MR7);
}

/* out[i] = oracle_wheel_is_prime(n[i]) (O8 alone), threaded as above. */
int oracle_wheel_array(const uint64_t *n, uint8_t *out, uint64_t len, int nthreads)
{
    return apply_array(n, out, len, NULL, nthreads, APPLY_WHEEL);
}

/* ------------------------------------------------------------------ O6 */

static uint64_t gcd_u64(uint64_t a, uint64_t b)
{
    while (b) {
        uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

/* A nontrivial factor of composite n (1 < f < n), or 0 if none was found
 * within the iteration cap.  Small factors by trial division, then Pollard
 * rho with x -> x^2 + c and Brent's cycle detection, products of |x - y|
 * batched before each gcd. */
uint64_t oracle_find_factor(uint64_t n)
{
    if (n < 4)
        return 0;
    for (uint64_t p = 2; p < 1000 && p * p <= n; ++p)
        if (n % p == 0)
            return p;
    for (uint64_t c = 1; c < 64; ++c) {
        uint64_t y = 2, x = 2, q = 1, g = 1, ys = 2;
        uint64_t r = 1;
        const uint64_t m = 128;
        uint64_t steps = 0;
        while (g == 1 && steps < ((uint64_t)1 << 26)) {
            x = y;
            for (uint64_t i = 0; i < r; ++i)
                y = (uint64_t)(((u128)y * y + c) % n);
            uint64_t k = 0;
            while (k < r && g == 1) {
                ys = y;
                uint64_t lim = (m < r - k) ? m : r - k;
                for (uint64_t i = 0; i < lim; ++i) {
                    y = (uint64_t)(((u128)y * y + c) % n);
                    uint64_t diff = x > y ? x - y : y - x;
                    q = oracle_mulmod(q, diff, n);
                }
                g = gcd_u64(q, n);
                k += lim;
                steps += lim;
            }
            r *= 2;
        }
        if (g == n) {
            /* the batch overshot: step back one value at a time */
            do {
                ys = (uint64_t)(((u128)ys * ys + c) % n);
                uint64_t diff = x > ys ? x - ys : ys - x;
                g = gcd_u64(diff, n);
            } while (g == 1);
        }
        if (g != 1 && g != n)
            return g;
    }
    return 0;
}

#define MAX_FACTORS 128

static int pratt_depth(uint64_t n, int depth);

/* Complete factorisation of m >= 1 into primes, each certified by
 * pratt_depth (recursively) or by trial division.  Returns the number of
 * distinct primes written to qs, or -1 on failure. */
static int factor_distinct(uint64_t m, uint64_t *qs, int depth)
{
    int nq = 0;
    uint64_t stack[MAX_FACTORS];
    int sp = 0;
    for (uint64_t p = 2; p < 4096 && p * p <= m; ++p) {
        if (m % p == 0) {
            qs[nq++] = p;
            while (m % p == 0)
                m /= p;
        }
    }
    if (m > 1)
        stack[sp++] = m;
    while (sp > 0) {
        uint64_t c = stack[--sp];
        if (c == 1)
            continue;
        int r = pratt_depth(c, depth + 1);
        if (r == 1) {
            int seen = 0;
            for (int i = 0; i < nq; ++i)
                seen |= (qs[i] == c);
            if (!seen) {
                if (nq >= MAX_FACTORS)
                    return -1;
                qs[nq++] = c;
            }
        } else if (r == 0) {
            uint64_t f = oracle_find_factor(c);
            if (f == 0 || sp + 2 > MAX_FACTORS)
                return -1;
            stack[sp++] = f;
            stack[sp++] = c / f;
        } else {
            return -1;
        }
    }
    return nq;
}

/* 1: n certified prime; 0: n certified composite; -1: undecided.
 * Values below 2^32 by trial division.  Otherwise Lucas' converse of
 * Fermat (the Pratt certificate): n is prime iff some a has
 * a^(n-1) = 1 and a^((n-1)/q) != 1 mod n for every prime q dividing n-1. */
static int pratt_depth(uint64_t n, int depth)
{
    if (n < TABLE_BOUND)
        return oracle_trial_is_prime(n);
    if ((n & 1) == 0)
        return 0;
    if (depth > 16)
        return -1;
    if (oracle_powmod(2, n - 1, n) != 1)
        return 0; /* Fermat witness: composite */
    uint64_t qs[MAX_FACTORS];
    int nq = factor_distinct(n - 1, qs, depth);
    if (nq < 0)
        return -1;
    for (uint64_t a = 2; a < 2000; ++a) {
        if (oracle_powmod(a, n - 1, n) != 1)
            return 0;
        int ok = 1;
        for (int i = 0; i < nq && ok; ++i)
            ok = oracle_powmod(a, (n - 1) / qs[i], n) != 1;
        if (ok)
            return 1;
    }
    return -1;
}

int oracle_pratt_certify(uint64_t n) { return pratt_depth(n, 0); }

/* ------------------------------------------------------------------ O7 */

/* Divisions that MATLAB's isprime performs on 1:N (section 6): every element
 * n is divided by each prime p <= floor(sqrt(N)) with p < n.  Counted the
 * plain way, one element at a time, with a running count of such primes. */
uint64_t oracle_numdiv(uint64_t N)
{
    uint64_t r = 0;
    while ((r + 1) * (r + 1) <= N)
        ++r; /* r = floor(sqrt(N)) */
    uint64_t total = 0, below = 0; /* below = #{p <= r : p < n} */
    for (uint64_t n = 1; n <= N; ++n) {
        total += below;
        if (n <= r && oracle_trial_is_prime(n))
            ++below; /* p = n counts for every later element */
    }
    return total;
}
