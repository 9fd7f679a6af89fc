"""Pins for the CPU oracle: each check ties it to something other than itself
(values the paper prints, published constants, brute force, certificates,
Python's own integers), so that a dropped term, a wrong index or a wrong
constant anywhere in it fails at least one test."""
import math
import random

import numpy as np
import pytest

import oracle
import workloads
from conftest import golden

U64 = (1 << 64) - 1


def _popcount_u32(words: np.ndarray) -> int:
    return int(np.unpackbits(np.ascontiguousarray(words).view(np.uint8)).sum())


def _py_strong_test(n: int, a: int) -> bool:
    """Strong probable-prime test written with Python integers."""
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    x = pow(a, d, n)
    if x in (1, n - 1):
        return True
    for _ in range(s - 1):
        x = x * x % n
        if x == n - 1:
            return True
    return False


# ---------------------------------------------------------------- the paper


def test_worked_example_section1():
    """Section 1: isprime([1, 2, 3, 4, 5]) = 0 1 1 0 1."""
    lines = golden("worked_example.txt")
    inp = [int(x) for x in lines[0].split(":")[1].split()]
    exp = [int(x) for x in lines[1].split(":")[1].split()]
    out, _ = oracle.isprime_array(np.array(inp, dtype=np.uint64), use_table=False)
    assert out.tolist() == exp
    assert [oracle.trial_is_prime(v) for v in inp] == exp
    assert [oracle.is_prime(v) for v in inp] == exp


def test_bases_are_eq4():
    """Section 2.1, Eq. 4: the seven bases, in the printed order."""
    exp = [int(x) for x in golden("mr_bases.txt")[0].split()]
    assert oracle.mr_bases() == exp


def test_table_numdiv_section6():
    """Section 6, Table NumDiv: all eight printed rows, exactly."""
    for line in golden("table_numdiv.txt"):
        N, divs = (int(x) for x in line.split())
        assert oracle.numdiv(N) == divs, N


# ------------------------------------------------------- closed forms, counts


def test_pi_1e6_three_ways():
    """pi(10^6) = 78498 from the sieve, from trial division and from mr7."""
    t = oracle.sieve_odd(10 ** 6)
    assert _popcount_u32(t) + 1 == 78498  # + the even prime 2
    a = np.arange(10 ** 6, dtype=np.uint64)
    assert int(oracle.trial_array(a).sum()) == 78498
    assert int(oracle.mr7_array(a).sum()) + 1 == 78498


def test_sieve_first_word_and_small_limits():
    t = oracle.sieve_odd(1 << 20)
    # bit i <-> 2i+1: primes 3,5,7,11,13,17,19,23,29,31,37,41,43,47,53,59,61
    expect = 0
    for i in range(32):
        if oracle.trial_is_prime(2 * i + 1):
            expect |= 1 << i
    assert int(t[0]) == expect == 0x64B4CB6E
    # a limit that is not a multiple of 64 leaves the tail bits 0
    for limit in (1, 2, 3, 10, 64, 65, 100, 1001):
        tt = oracle.sieve_odd(limit)
        got = [v for v in range(1, limit, 2) if (int(tt[v >> 6]) >> ((v >> 1) & 31)) & 1]
        assert got == [v for v in range(3, limit, 2) if oracle.trial_is_prime(v)], limit
        assert _popcount_u32(tt) == len(got)


@pytest.mark.slow
def test_pi_2_32(oracle_table):
    """pi(2^32) = 203,280,221: the odd-only table holds all but the prime 2."""
    assert oracle_table.size == 1 << 26
    assert _popcount_u32(oracle_table) == 203280221 - 1
    assert int(oracle_table[0]) == 0x64B4CB6E


@pytest.mark.slow
def test_brute_force_below_2_24():
    """Every n < 2^24: trial division, the sieve, mr7 and dispatch agree."""
    a = np.arange(1 << 24, dtype=np.uint64)
    o1 = oracle.trial_array(a)
    assert int(o1.sum()) == 1077871  # pi(2^24)
    t = oracle.sieve_odd(1 << 24)
    bits = np.unpackbits(t.view(np.uint8), bitorder="little")
    o2 = np.zeros(1 << 24, dtype=np.uint8)
    o2[1::2] = bits[: 1 << 23]
    o2[2] = 1
    assert np.array_equal(o1, o2)
    o4 = oracle.mr7_array(a)
    o4[2] = 1
    assert np.array_equal(o1, o4)
    o5, _ = oracle.isprime_array(a, use_table=False)
    assert np.array_equal(o1, o5)


# --------------------------------------------------------- modular arithmetic


def test_mulmod_powmod_against_python_integers():
    rng = random.Random(0x21080479)
    moduli = [3, 5, (1 << 32) + 15, (1 << 61) - 1, (1 << 63) - 25, (1 << 63) + 29,
              U64 - 58, U64]
    moduli += [rng.getrandbits(64) | 1 for _ in range(200)]
    for n in moduli:
        edges = [0, 1, 2, n - 1, n - 2, n // 2, (n + 1) // 2]
        vals = [v % n for v in edges] + [rng.randrange(n) for _ in range(20)]
        for a in vals:
            for b in vals[:8]:
                assert oracle.mulmod(a, b, n) == a * b % n
        for _ in range(10):
            a, e = rng.randrange(n), rng.getrandbits(64)
            assert oracle.powmod(a, e, n) == pow(a, e, n)
    assert oracle.powmod(5, 0, 1) == 0


def test_strong_test_against_python_integers():
    rng = random.Random(7)
    for _ in range(3000):
        n = rng.getrandbits(rng.randrange(3, 65)) | 1
        if n < 3:
            continue
        a = rng.randrange(2, n) if n > 3 else 2
        assert oracle.strong_probable_prime(n, a) == int(_py_strong_test(n, a)), (n, a)


# ------------------------------------------------------------- fixed values

# 2^61-1, 2^64-59, 2^63-25, 2^32-5 (largest prime below 2^32), 2^32+15
# (smallest prime above it), 10^9+7.
PRIMES = [(1 << 61) - 1, U64 - 58, (1 << 63) - 25, (1 << 32) - 5, (1 << 32) + 15,
          1000000007]

SPSP = [2047, 1373653, 25326001, 3215031751, 2152302898747, 3474749660383,
        341550071728321, 3825123056546413051, (1 << 32) + 1]

CARMICHAEL = [561, 1105, 1729, 2465, 2821, 6601, 8911]


def test_fixed_primes_certified():
    for p in PRIMES:
        assert oracle.mr7(p) == 1, p
        assert oracle.is_prime(p) == 1, p
        assert oracle.pratt_certify(p) == 1, p
    assert (1 << 64) - 59 == 0xFFFFFFFFFFFFFFC5


def test_strong_pseudoprimes_are_composite():
    """Composites that pass the strong test for base 2 (and, for the larger
    ones, for every prime base up to 31): each is factored, each passes the
    base-2 round in the oracle, and the seven-base test rejects them."""
    for n in SPSP:
        f = oracle.find_factor(n)
        assert 1 < f < n and n % f == 0, n
        assert _py_strong_test(n, 2), n
        assert oracle.strong_probable_prime(n, 2) == 1, n
        assert oracle.mr7(n) == 0, n
        assert oracle.is_prime(n) == 0, n
    n = 3825123056546413051
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31):
        assert _py_strong_test(n, a) and oracle.strong_probable_prime(n, a) == 1
    for p in (11, 23, 29, 37, 41, 43, 47, 53, 59):
        m = (1 << p) - 1
        assert oracle.mr7(m) == 0 and oracle.strong_probable_prime(m, 2) == 1, p
    assert oracle.mr7(U64) == 0 and oracle.mr7((1 << 32) - 1) == 0


def _korselt(n: int, factors) -> bool:
    prod = 1
    for p in factors:
        prod *= p
    return prod == n and len(set(factors)) == len(factors) and all((n - 1) % (p - 1) == 0 for p in factors)


def test_carmichael_numbers_composite():
    for n in CARMICHAEL:
        fs, m, d = [], n, 2
        while m > 1:
            while m % d == 0:
                fs.append(d)
                m //= d
            d += 1
        assert _korselt(n, fs), n
        assert oracle.trial_is_prime(n) == 0 and oracle.mr7(n) == 0, n
        assert oracle.powmod(2, n - 1, n) == 1  # Fermat cannot see them


def test_chernick_list_and_verdicts():
    ks = [int(k) for k in workloads.chernick_k()]
    assert len(ks) == 1675 and ks[:8] == [1, 6, 35, 45, 51, 55, 56, 100]
    k_next = ks[-1] + 1
    while (6 * k_next + 1) * (12 * k_next + 1) * (18 * k_next + 1) < (1 << 64):
        assert not all(oracle.trial_is_prime(f) for f in
                       (6 * k_next + 1, 12 * k_next + 1, 18 * k_next + 1))
        k_next += 1
    vals = workloads.chernick_values()
    for k, n in zip(ks, vals.tolist()):
        fs = [6 * k + 1, 12 * k + 1, 18 * k + 1]
        assert _korselt(n, fs)
        assert all(oracle.trial_is_prime(f) for f in fs)
    assert int(oracle.mr7_array(vals).sum()) == 0
    big = vals[vals >= np.uint64(1 << 32)]
    base2 = sum(oracle.strong_probable_prime(int(n), 2) for n in big)
    assert base2 > 0  # some pass base 2, so later bases are exercised


# ------------------------------------------------------------- certificates

# The ten largest primes below 2^64, as 2^64 minus these offsets (the
# published list of primes just below powers of two).
TOP_PRIME_OFFSETS = [59, 83, 95, 179, 189, 257, 279, 323, 353, 363]


def test_pratt_is_two_sided():
    """Section 2.1 (Eq. 4) is checked above 2^32 by certificates that do not
    rest on the seven-base claim, so the Pratt certificate must never call a
    composite prime.  Its dangerous inputs are composites that pass Fermat's
    test to base 2 (the first witness it tries): strong pseudoprimes to base
    2 above 2^32, composite Mersenne numbers, and Carmichael numbers
    (Chernick's, which pass Fermat to every base coprime to them, some also
    the strong test to base 2).  Each must come out 0 or -1, never 1; and
    the published primes just below 2^64 must come out 1."""
    fermat2 = [n for n in SPSP if n >= 1 << 32]
    fermat2 += [(1 << p) - 1 for p in (37, 41, 43, 47, 53, 59)]
    vals = workloads.chernick_values()
    big = [int(n) for n in vals.tolist() if n >= 1 << 32]
    strong2 = [n for n in big if _py_strong_test(n, 2)]
    assert len(strong2) == 251
    fermat2 += strong2[::10] + big[::60]
    for n in fermat2:
        assert pow(2, n - 1, n) == 1, n  # base 2 cannot tell them from primes
        assert oracle.pratt_certify(n) != 1, n
    for off in TOP_PRIME_OFFSETS:
        assert oracle.pratt_certify((1 << 64) - off) == 1, off
    for n in ((1 << 64) - 61, (1 << 64) - 1, (1 << 64) - 57):  # composites between them
        assert oracle.pratt_certify(n) != 1, n


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_certificates_on_sampled_elements(name):
    """Every MR verdict above 2^32 on a sample is backed by a factor or a
    Pratt certificate, neither of which relies on the seven-base claim."""
    gen = workloads.c2_mr64 if name == "c2" else workloads.c3_mixed
    rng = np.random.default_rng(3)
    starts = rng.integers(0, 1 << 20, size=8)
    vals = np.concatenate([gen(64, start=int(s)) for s in starts])
    vals = vals[(vals >= np.uint64(1 << 32)) & ((vals & np.uint64(1)) == 1)]
    assert vals.size > 100
    for n in vals.tolist():
        if oracle.mr7(n):
            assert oracle.pratt_certify(n) == 1, n
        else:
            assert oracle.pratt_certify(n) != 1, n
            f = oracle.find_factor(n)
            if f == 0:  # a Fermat witness is enough to show compositeness
                assert pow(2, n - 1, n) != 1, n
            else:
                assert 1 < f < n and n % f == 0, n


def test_isprime_array_threads_and_tables(oracle_table):
    a = np.concatenate([np.arange(0, 5000, dtype=np.uint64),
                        np.array(PRIMES + SPSP, dtype=np.uint64),
                        workloads.c3_mixed(4096)])
    r1, used1 = oracle.isprime_array(a, nthreads=1, use_table=True)
    r8, used8 = oracle.isprime_array(a, nthreads=8, use_table=False)
    assert used1 == 1 and used8 == 8
    assert np.array_equal(r1, r8)
    for v, r in zip(a.tolist()[:5000], r1.tolist()[:5000]):
        assert r == oracle.trial_is_prime(v)


# -------------------------------------------------------------------- wheel


def _coprime_gaps(modulus: int) -> list:
    """Gaps between consecutive numbers coprime to `modulus` in [1, modulus + 1],
    from the definition (math.gcd), not from any printed list."""
    r = [v for v in range(1, modulus + 2) if math.gcd(v, modulus) == 1]
    return [b - a for a, b in zip(r, r[1:])]


def test_wheel_cycle_eq5_and_eq6():
    """The wheel's difference cycle against its definition; the derivation is
    itself checked on the two smaller cycles section 3 prints."""
    assert _coprime_gaps(6) == [4, 2]
    assert _coprime_gaps(30) == [6, 4, 2, 4, 2, 4, 6, 2]
    c = oracle.wheel_cycle()
    assert c == _coprime_gaps(210)
    assert len(c) == 48 and sum(c) == 210
    assert [int(v) for v in 1 + np.cumsum(c[:6])] == [11, 13, 17, 19, 23, 29]  # Eq. 6


def _largest_primes_per_residue(limit: int) -> list:
    """For each residue r coprime to 210, the largest prime p < limit with
    p = r (mod 210), found by O1."""
    out = []
    for r in range(1, 210):
        if math.gcd(r, 210) != 1:
            continue
        p = (limit - 1) - ((limit - 1 - r) % 210)
        while not oracle.trial_is_prime(p):
            p -= 210
        out.append(p)
    return out


def test_wheel_trial_division_brute_force_and_hard_cases():
    """O8 against the definition (O1) on every n < 2^20, then on squares and
    near-square products of primes from every residue class of the wheel
    near 2^20 (n just below 2^40: the last divisor tried is the factor)."""
    a = np.arange(1 << 20, dtype=np.uint64)
    w = oracle.wheel_array(a)
    assert np.array_equal(w, oracle.trial_array(a))
    assert int(w.sum()) == 82025  # pi(2^20)
    ps = _largest_primes_per_residue(1 << 20)
    assert len(ps) == 48
    cases = [p * p for p in ps] + [p * q for p, q in zip(ps, ps[1:])]
    cases += [p for p in ps] + [2, 3, 5, 7, 11, 121, 169, 221, 209 * 211]
    cases += [n for n in SPSP + CARMICHAEL + PRIMES if n < 1 << 42]
    for n in cases:
        assert n < 1 << 42
        assert oracle.wheel_is_prime(n) == oracle.trial_is_prime(n), n
    assert all(oracle.wheel_is_prime(p * p) == 0 for p in ps)
    assert all(oracle.wheel_is_prime(p) == 1 for p in ps)
