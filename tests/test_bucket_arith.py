"""Host checks of arithmetic that the kernels run on the device, written out
here in exact Python arithmetic: two pieces of the interval sieve's bucket
passes (csrc/range.hip) and the Montgomery constant 2^64 mod n of the
base-2 kernel (csrc/mont.h); the GPU tests (test_gpu_range.py,
test_gpu_parity.py) check the kernels' bytes.

1. lo mod d for 2^19 <= d < 2^34 in double precision: a reciprocal refined
   by two Newton steps, the quotient floor(lo * (1/d) - 1/2), and the
   remainder fma(-q, d, lo_hi) + lo_lo from the exact halves of lo, which
   is exact (the fused result is an integer below 2^35 in magnitude).  The
   first odd multiple of p at or above lo follows from m = lo mod 2p.
2. The hit bound of each group of primes: floor((len - 1) / 2p) + 1 per
   prime p in (2^21, root], with the primes above (len - 1) / 2 (bound 1
   each) counted from per-chunk prime counts and the group boundaries'
   partial chunks, and the root's word counted up to root.
3. 2^64 mod n for odd n >= 2^32: q = floor(2^64 (1/n) - 1/2) from the same
   refined reciprocal is floor(2^64 / n) or one less, and 2^64 - q n taken
   modulo 2^64 needs one conditional subtraction.
"""
import math
import random
from fractions import Fraction

import numpy as np


def _fma(a, b, c):
    """a * b + c rounded once to double (exact rational, then one rounding)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _mod_double(x, d, rel_err):
    """The device's mod_double with the reciprocal estimate off by rel_err."""
    xh = float(x & ~0xFFFFFFFF)
    xl = float(x & 0xFFFFFFFF)
    inv = (1.0 / d) * (1.0 + rel_err)
    inv = _fma(inv, _fma(-d, inv, 1.0), inv)
    inv = _fma(inv, _fma(-d, inv, 1.0), inv)
    q = math.floor(_fma(float(x), inv, -0.5))
    t = _fma(-q, d, xh)
    assert t == Fraction(xh) - q * int(d)  # the fused step is exact
    r = t + xl
    assert r == Fraction(t) + Fraction(xl)
    return r - d if r >= d else r


def _first_offset(lo, p, length, rel_err):
    """Offset of p's first odd multiple at or above lo, or length if none below it."""
    pd = float(p)
    m = _mod_double(lo, 2.0 * pd, rel_err)
    off = (pd if m <= pd else 3.0 * pd) - m
    return int(off) if off < float(length) else length


def test_first_odd_multiple_matches_integers():
    rng = random.Random(20210810)
    cases = 0
    for _ in range(6000):
        length = rng.choice([1 << 30, 1 << 28, rng.randint(1, 1 << 30)])
        lo = rng.choice([rng.getrandbits(64), (1 << 64) - length - rng.getrandbits(16),
                         rng.getrandbits(rng.randint(46, 64)), 1 << 63, (1 << 64) - length])
        lo = min(max(lo, 1 << 46), (1 << 64) - length)
        p = rng.choice([rng.randint((1 << 20) + 1, (1 << 32) - 1), (1 << 20) + 1 + rng.getrandbits(10),
                        (1 << 32) - 1 - rng.getrandbits(10), math.isqrt(lo) - rng.getrandbits(8)]) | 1
        if not (1 << 20) < p < (1 << 32) or p >= lo:
            continue
        # reciprocal estimates far worse than the hardware's
        err = rng.uniform(-2.0 ** -12, 2.0 ** -12)
        k = -(-lo // p)
        if k % 2 == 0:
            k += 1
        want = min(k * p - lo, length)
        assert _first_offset(lo, p, length, err) == want, (lo, p, length)
        cases += 1
    assert cases > 5000


def _table(n):
    """Odd-only sieve bits below n as uint32 words (bit i of word w <-> 64w + 2i + 1)."""
    odd = np.ones(n // 2, dtype=bool)
    odd[0] = False
    for i in range(1, math.isqrt(n) // 2 + 1):
        if odd[i]:
            p = 2 * i + 1
            odd[p * p // 2::p] = False
    bits = odd.reshape(-1, 32).astype(np.uint64) << np.arange(32, dtype=np.uint64)
    return bits.sum(axis=1).astype(np.uint32), 2 * np.nonzero(odd)[0] + 1


def test_group_bounds_from_chunk_counts():
    small = 1 << 21
    table, primes = _table(1 << 24)
    popc = np.unpackbits(table.view(np.uint8)).reshape(-1, 32).sum(axis=1).astype(np.int64)
    cum = np.concatenate([[0], np.cumsum(popc.reshape(-1, 64).sum(axis=1))])
    rng = random.Random(7)
    for _ in range(60):
        root = rng.randint(small + 64, (1 << 24) - 1)
        length = rng.choice([1 << 28, 1 << 30, rng.randint(1, 1 << 30), rng.randint(1, 1 << 22)])
        groups = rng.randint(1, 512)
        w_begin, w_end = (small + 1) >> 6, (root >> 6) + 1
        wsplit = [w_begin] + sorted(rng.randint(w_begin, w_end) for _ in range(groups - 1)) + [w_end]
        sel = primes[(primes > small) & (primes <= root)]
        words = sel >> 6
        per_prime = np.where(2 * sel > length - 1, 0, (length - 1) // (2 * sel)) + 1
        group = np.searchsorted(np.array(wsplit), words, side="right") - 1  # wsplit[q] <= word < wsplit[q+1]
        want = np.bincount(group, weights=per_prime, minlength=groups).astype(np.int64).tolist()
        # the words below w_mid prime by prime, the rest from the chunk counts
        lo_p = max((length - 1) // 2, small)
        w_mid = min(w_end, max(w_begin, (lo_p >> 6) + 1))
        below = words < w_mid
        got = np.bincount(group[below], weights=per_prime[below], minlength=groups).astype(np.int64).tolist()
        w_top = max(w_mid, w_end - 1)
        for g in range(groups + 1):
            w = min(max(wsplit[g], w_mid), w_top)
            count = int(cum[w >> 6]) + int(popc[(w >> 6) << 6:w].sum())
            if g > 0:
                got[g - 1] = (got[g - 1] + count) % (1 << 32)
            if g < groups:
                got[g] = (got[g] - count) % (1 << 32)
        if w_mid < w_end:
            nb = ((root & 63) + 1) >> 1
            mask = 0xFFFFFFFF if nb >= 32 else (1 << nb) - 1
            got[groups - 1] += bin(int(table[w_end - 1]) & mask).count("1")
        assert got == want, (root, length, groups)


def _r_mod_n_wide(n, rel_err):
    """The device's r_mod_n_wide with the reciprocal estimate off by rel_err."""
    d = float(n)
    inv = (1.0 / d) * (1.0 + rel_err)
    inv = _fma(inv, _fma(-d, inv, 1.0), inv)
    inv = _fma(inv, _fma(-d, inv, 1.0), inv)
    q = math.floor(_fma(2.0 ** 64, inv, -0.5))
    assert 0 <= q < 1 << 32
    r = -(q * n) % (1 << 64)
    r = r - n if r >= n else r
    return (1 << 64) - n if n >= 1 << 63 else r


def test_r_mod_n_matches_integers():
    rng = random.Random(64)
    for _ in range(20000):
        n = rng.choice([rng.getrandbits(64), rng.randint(1 << 32, 1 << 40), (1 << 32) + rng.getrandbits(8),
                        (1 << 63) - rng.getrandbits(8), (1 << 63) + rng.getrandbits(8),
                        rng.getrandbits(rng.randint(33, 64))]) | 1
        if n < 1 << 32:
            continue
        assert _r_mod_n_wide(n, rng.uniform(-2.0 ** -12, 2.0 ** -12)) == (1 << 64) % n, n
