"""GPU parity of the interval entry point isprime_range_u64: out[i] is the
primality of lo + i.  Checked against the oracle element by element on
intervals that cross the table bound (2^32), the bound where the segment
sieve stops being complete on its own (2^50), several segments with ragged
tails, the top of the 64-bit range, and a call larger than one piece
(sampled).  Tolerance: zero mismatching bytes."""
import os

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

U64 = (1 << 64) - 1
NTHREADS = min(16, os.cpu_count() or 1)
SEG = 1 << 19      # numbers per workgroup segment (2^20 in bucket mode and for long pieces whose primes pass 2^20)
SEG20 = 1 << 20
PIECE = 1 << 30    # numbers per piece of one call


@pytest.fixture(scope="module")
def isp():
    import paper_2108_04791_amd as isp
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    isp.init()
    return isp


def values(lo: int, length: int) -> np.ndarray:
    return np.uint64(lo) + np.arange(length, dtype=np.uint64)


def gpu_range(isp, lo: int, length: int) -> np.ndarray:
    out = isp.isprime_range(lo, length)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.uint8)


def check(isp, lo: int, length: int):
    a = values(lo, length)
    got = gpu_range(isp, lo, length)
    exp, _ = oracle.isprime_array(a, nthreads=NTHREADS, use_table=None)
    bad = np.nonzero(got != exp)[0]
    if bad.size:
        i = bad[:10]
        raise AssertionError("[%d, +%d): %d mismatches, first %s gpu %s oracle %s" % (
            lo, length, bad.size, a[i].tolist(), got[i].tolist(), exp[i].tolist()))
    return got


def test_small_interval_counts(isp):
    """pi(2^20) = 82025 and pi(10^6) = 78498 (standard values of the prime
    counting function)."""
    assert int(gpu_range(isp, 0, 1 << 20).sum()) == 82025
    assert int(gpu_range(isp, 0, 10 ** 6).sum()) == 78498


def test_below_2_20(isp):
    check(isp, 0, 1 << 20)


def test_across_table_bound(isp):
    check(isp, (1 << 32) - 300001, 600003)


def test_across_complete_bound(isp):
    """Six segments around 2^50: too few for a pass over the primes up to
    2^25 each, so the primes below 2^18 and Miller-Rabin decide them on both
    sides of the bound (the long intervals below cover the complete sieve
    next to Miller-Rabin in one call)."""
    check(isp, (1 << 50) - 3 * SEG - 17, 6 * SEG + 33)


def test_complete_at_several_magnitudes(isp):
    """Short intervals around 2^40, 2^44 and 2^48.  Around 2^40 every segment
    is complete, sieved by the primes up to 2^20.  Around 2^44 and 2^48 the
    primes up to the square root are too many for so few segments, so the
    primes below 2^18 and Miller-Rabin decide them instead."""
    check(isp, (1 << 40) - SEG - 5, 2 * SEG + 11)
    check(isp, (1 << 44) + 1, SEG + 7)
    check(isp, (1 << 48) - SEG // 2, SEG)


@pytest.mark.parametrize("lo,length", [
    (10 ** 12 + 7, 3 * SEG + 12345),
    ((1 << 33) + 1, SEG),
    ((1 << 33), SEG + 1),
    ((1 << 36) + 5, 2 * SEG - 1),
    ((1 << 61) - 1000, 200001),
    ((1 << 63) - 99999, 199999),
])
def test_segments_and_ragged_tails(isp, lo, length):
    check(isp, lo, length)


def test_top_of_range(isp):
    """The interval ends at 2^64 - 1 exactly."""
    length = 10 ** 6
    got = check(isp, U64 - length + 1, length)
    assert got[-1] == 0 and got[-59] == 1  # 2^64 - 59 is the largest 64-bit prime


@pytest.mark.parametrize("length", [1, 2, 3, 63, 64, 65, 1000])
def test_tiny(isp, length):
    for lo in (0, 1, 2, (1 << 32) - 2, (1 << 32) - 1, 1 << 32, (1 << 40) - 1, (1 << 61) - 1,
               U64 - length + 1):
        check(isp, lo, length)


def test_random_intervals(isp):
    rng = np.random.default_rng(20210810)
    for _ in range(12):
        lo = int(rng.integers(1 << 32, 1 << 63)) * 2 + int(rng.integers(0, 2))
        length = int(rng.integers(1, 200000))
        lo = min(lo, U64 - length + 1)
        check(isp, lo, length)


def test_equals_array_call(isp):
    """The interval call and the array call agree over several segments."""
    lo, length = (1 << 45) + 3, 5 * SEG + 999
    got = gpu_range(isp, lo, length)
    arr = torch.from_numpy(values(lo, length).view(np.int64)).cuda()
    ref = isp.isprime(arr).cpu().numpy().astype(np.uint8)
    assert np.array_equal(got, ref)


def test_empty_and_invalid(isp):
    assert gpu_range(isp, 123, 0).size == 0
    with pytest.raises(isp.IsprimeError):
        isp.isprime_range(U64 - 5, 7)
    with pytest.raises(isp.IsprimeError):
        isp.isprime_range(U64, 2)
    assert gpu_range(isp, U64, 1)[0] == 0


@pytest.mark.parametrize("lo,length", [((1 << 34) + 1, (1 << 27) + 5 * SEG + 3),
                                       ((1 << 44) + 3, 1 << 27),
                                       ((1 << 44) + 3, (1 << 28) + 3 * SEG20 + 12345),
                                       ((1 << 50) - (1 << 26) - 5, 1 << 27)])
def test_long_complete_pieces(isp, lo, length):
    """Intervals of at least 256 segments: below 2^50 every segment is
    complete, crossed off by all the primes up to its square root (2^17,
    2^22, 2^25); the third interval runs segments of 2^20 numbers (at least
    256 of them, primes past 2^20) with a ragged last one; the last interval
    crosses 2^50, where the segments switch to the primes below 2^22 and
    Miller-Rabin.  The whole interval equals the array call, and a sample
    (both ends and 20,000 random positions) equals the oracle."""
    got = isp.isprime_range(lo, length)
    arr = torch.arange(lo, lo + length, dtype=torch.int64, device="cuda")
    assert torch.equal(isp.isprime(arr), got)
    rng = np.random.default_rng(lo & 0xffff)
    idx = np.unique(np.concatenate([np.arange(0, 3000), np.arange(length - 3000, length),
                                    rng.integers(0, length, 20000)])).astype(np.int64)
    a = np.uint64(lo) + idx.astype(np.uint64)
    exp, _ = oracle.isprime_array(a, nthreads=NTHREADS, use_table=False)
    assert np.array_equal(got[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.uint8), exp)


@pytest.mark.parametrize("lo,length", [((1 << 56) + 12345, 1 << 26), ((1 << 62) - 3, 1 << 28),
                                       ((1 << 60) + 7, (1 << 27) + 3 * SEG20 + 999),
                                       ((1 << 64) - (1 << 29), 1 << 29)])
def test_bucket_mode_high_magnitude(isp, lo, length):
    """Intervals far above 2^50 that are long next to the number of primes up
    to their square root run as a complete bucketed sieve (every prime up to
    the square root, up to 2^32, crossed off; no Miller-Rabin): the whole
    interval equals the array call, and a sample equals the oracle.  The
    last case ends at 2^64 - 1."""
    got = isp.isprime_range(lo, length)
    base = lo if lo < (1 << 63) else lo - (1 << 64)
    arr = torch.arange(base, base + length, dtype=torch.int64, device="cuda")
    assert torch.equal(isp.isprime(arr), got)
    rng = np.random.default_rng(lo & 0xffff)
    idx = np.unique(np.concatenate([np.arange(0, 3000), np.arange(length - 3000, length),
                                    rng.integers(0, length, 20000)])).astype(np.int64)
    a = np.uint64(lo) + idx.astype(np.uint64)
    exp, _ = oracle.isprime_array(a, nthreads=NTHREADS, use_table=False)
    assert np.array_equal(got[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.uint8), exp)


@pytest.mark.parametrize("p,length", [(131071, 1 << 26), (4194301, 1 << 28),
                                      (2147483647, 1 << 28), (4294967291, 1 << 28)])
def test_interval_ending_at_a_prime_square(isp, p, length):
    """Intervals whose last number is p^2 for a prime p, so that p is exactly
    the square root of the last segment and its only sieving prime for p^2:
    131071 = 2^17 - 1 (segments of 2^19, complete), 4194301 (the largest
    prime below 2^22: segments of 2^20, complete), 2^31 - 1 and 4294967291
    (the largest prime below 2^32: bucket mode, p in the last table word the
    bucket passes count).  p^2 must come out composite, the whole interval
    must equal the array call, and a sample must equal the oracle."""
    lo = p * p - length + 1
    got = isp.isprime_range(lo, length)
    assert int(got[-1].item()) == 0
    base = lo if lo < (1 << 63) else lo - (1 << 64)
    arr = torch.arange(base, base + length, dtype=torch.int64, device="cuda")
    assert torch.equal(isp.isprime(arr), got)
    del arr
    rng = np.random.default_rng(p & 0xffff)
    idx = np.unique(np.concatenate([np.arange(0, 2000), np.arange(length - 5000, length),
                                    rng.integers(0, length, 20000)])).astype(np.int64)
    a = np.uint64(lo) + idx.astype(np.uint64)
    exp, _ = oracle.isprime_array(a, nthreads=NTHREADS, use_table=False)
    assert np.array_equal(got[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.uint8), exp)


def test_larger_than_one_piece_sampled(isp):
    """A call of more than 2^30 numbers runs in pieces; the outputs around the
    piece boundary and a random sample are checked one by one, and the whole
    equals the array call."""
    lo, length = (1 << 50) + 1, PIECE + 3 * SEG + 7
    out = isp.isprime_range(lo, length)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([
        np.arange(PIECE - 50000, PIECE + 50000, dtype=np.int64),
        np.arange(length - 20000, length, dtype=np.int64),
        rng.integers(0, length, 200000, dtype=np.int64)]))
    got = out[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.uint8)
    a = np.uint64(lo) + idx.astype(np.uint64)
    exp, _ = oracle.isprime_array(a, nthreads=NTHREADS, use_table=None)
    assert np.array_equal(got, exp)
    # whole-interval property: the array call on the same values agrees
    step = 1 << 28
    for s in range(0, length, step):
        n = min(step, length - s)
        arr = (torch.arange(n, dtype=torch.int64, device="cuda") + (lo + s))
        ref = isp.isprime(arr)
        assert torch.equal(ref, out[s:s + n].bool())
    del out
