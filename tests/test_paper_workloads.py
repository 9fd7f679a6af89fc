"""The paper's array workloads (sections 6.1.3 and 8.2), rebuilt from their
descriptions: the stored lists are checked here without the oracle that
wrote them (a plain sieve, Fermat tests with Python integers and a
vectorised interval sieve), and the generators for sizes, ranges and
determinism."""
import math

import numpy as np

import workloads as W

U64 = (1 << 64) - 1


def _plain_sieve(limit: int) -> np.ndarray:
    """Primes below limit, by the textbook sieve of Eratosthenes."""
    s = np.ones(limit, dtype=bool)
    s[:2] = False
    for p in range(2, math.isqrt(limit - 1) + 1):
        if s[p]:
            s[p * p::p] = False
    return np.nonzero(s)[0].astype(np.uint64)


def _fermat(n: int) -> bool:
    return all(pow(a, n - 1, n) == 1 for a in (2, 3, 5, 7, 11, 13))


def test_prime_pool_is_every_prime_below_2_17():
    pool = W._paper_list("primes_below_2_17")
    assert pool.size == 12251  # pi(2^17)
    assert np.array_equal(pool, _plain_sieve(1 << 17))


def test_largest_52_bit_prime():
    """2^52 - 47, and nothing between it and 2^52 passes a Fermat test."""
    p = int(W._paper_list("largest_prime_below_2_52")[0])
    assert p == (1 << 52) - 47 and _fermat(p)
    assert not any(_fermat(n) for n in range(p + 2, 1 << 52, 2))


def _survivors_near_top(span: int, bound: int) -> np.ndarray:
    """Odd n in [2^64 - span, 2^64) with no prime factor up to `bound`
    (vectorised: small primes by slicing, the rest one multiple each)."""
    lo = (1 << 64) - span
    keep = np.ones(span, dtype=bool)
    keep[lo & 1::2] = False  # even numbers
    primes = _plain_sieve(bound + 1)
    primes = primes[primes > 2]
    lo_u = np.uint64(lo)
    off = (primes - lo_u % primes) % primes  # first multiple of p at lo + off
    small = primes < np.uint64(span)
    for p, o in zip(primes[small].tolist(), off[small].tolist()):
        keep[o::p] = False
    big_off = off[~small]
    keep[big_off[big_off < np.uint64(span)].astype(np.int64)] = False
    return np.uint64(lo) + np.nonzero(keep)[0].astype(np.uint64)


def test_largest_64_bit_primes_and_composites_with_large_factors():
    """Between the smallest listed value and 2^64 - 1, the odd numbers with no
    prime factor up to 2*10^7 are exactly the 100 largest primes and the 100
    largest composites with every factor above 2*10^7; the primes start at the
    published top of the range, 2^64 - 59, 2^64 - 83, 2^64 - 95, ..."""
    primes = W._paper_list("largest_64bit_primes")
    comps = W._paper_list("largest_composites_factors_gt_2e7")
    assert primes.size == 100 and comps.size == 100
    assert [U64 + 1 - int(p) for p in primes[:10]] == [59, 83, 95, 179, 189, 257, 279, 323,
                                                      353, 363]
    surv = _survivors_near_top(12000, 20_000_000)
    fermat = np.array([_fermat(int(n)) for n in surv])
    lo_p, lo_c = int(primes.min()), int(comps.min())
    assert sorted(surv[fermat & (surv >= np.uint64(lo_p))].tolist(), reverse=True) == \
        primes.tolist()
    assert sorted(surv[~fermat & (surv >= np.uint64(lo_c))].tolist(), reverse=True) == \
        comps.tolist()


def test_paper_arrays_shapes_and_ranges():
    d = W.paper_arrays()
    pool = set(W._paper_list("primes_below_2_17").tolist())
    assert d["int16_primes_200"].shape == (200,)
    assert int(d["int16_primes_200"].max()) < (1 << 15)
    assert set(d["int16_primes_200"].tolist()) <= pool
    m = d["matrix_1000x1000_u32"]
    assert m.shape == (1000, 1000) and int(m.max()) < (1 << 32)
    npr = d["normal_primes_1m_mean_2_16"]
    assert npr.size == 10 ** 6 and set(np.unique(npr).tolist()) <= pool
    assert abs(float(npr.astype(np.float64).mean()) - 2 ** 16) < 50
    assert 0.9 * 2 ** 12 < float(npr.astype(np.float64).std()) < 1.1 * 2 ** 12
    odd = d["normal_odd_100k_mean_2_32"]
    assert odd.size == 10 ** 5 and bool(np.all(odd & np.uint64(1)))
    assert abs(float(odd.astype(np.float64).mean()) / 2 ** 32 - 1) < 0.01
    n53 = d["normal_1000_mean_2_53"].astype(np.float64)
    assert abs(n53.mean() / 2 ** 53 - 1) < 0.02
    assert bool(np.all(d["largest52_prime_x1000"] == np.uint64((1 << 52) - 47)))
    top = d["largest64_odd_5000"]
    assert int(top[0]) == U64 and int(top[-1]) == U64 - 9998
    assert np.array_equal(W.paper_arrays()["matrix_1000x1000_u32"], m)  # deterministic


def test_intervals():
    assert W.PAPER_INTERVALS["unix_2021"] == (1609477200, 31536001)
    lo, n = W.PAPER_INTERVALS["inc_1e4"]
    a = W.interval(lo, n)
    assert int(a[0]) == 1 and int(a[-1]) == 10 ** 4 and a.dtype == np.uint64
