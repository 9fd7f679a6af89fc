"""GPU parity of the wheel stage (wheel_log2 = b: every filter survivor below
2^b is decided by trial division on the 2/3/5/7 wheel of section 3 instead
of Miller-Rabin): identical bytes to the oracle's wheel route (O8) and to its
primality dispatch (O5), on squares and near-square products of primes from
every residue class of the wheel just below 2^40, on whole octaves from 2^32
to 2^40, with the filter on and off, through the plain and the batched
calls."""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def isp():
    import paper_2108_04791_amd as isp
    isp.init()
    return isp


def run(isp, a, **cfg):
    prev = isp.set_config(**cfg)
    try:
        out = isp.isprime(torch.from_numpy(a.view(np.int64)).cuda())
        torch.cuda.synchronize()
    finally:
        isp.set_config(**prev)
    return out.cpu().numpy().astype(np.uint8)


def largest_primes_per_residue(limit):
    """For each residue r coprime to 210, the largest prime p < limit with
    p = r (mod 210) (primality from the oracle)."""
    out = []
    for r in range(1, 210):
        if math.gcd(r, 210) != 1:
            continue
        p = (limit - 1) - ((limit - 1 - r) % 210)
        while not oracle.trial_is_prime(p):
            p -= 210
        out.append(p)
    return out


def hard_cases():
    """Composites whose smallest factor is the last divisor the wheel tries
    (p^2, p*q with q the next prime of the list) for primes from every
    residue class, the primes times themselves plus small offsets, and
    values at the octave edges."""
    vals = []
    for limit in (1 << 17, 1 << 18, 1 << 19, 1 << 20):
        ps = largest_primes_per_residue(limit)
        vals += [p * p for p in ps] + [p * q for p, q in zip(ps, ps[1:])]
        vals += [p * p + 2 for p in ps]
    vals += [(1 << 32) + 1, (1 << 32) + 15, (1 << 33) - 9, (1 << 36) - 5, (1 << 40) - 87,
             (1 << 40) - 1, 3 * ((1 << 38) + 1), 5 * 7 * 11 * 13 * 17 * 19 * 23 * 29 * 31 + 0]
    vals = [v for v in vals if (1 << 32) <= v < (1 << 40)]
    return np.array(vals, dtype=np.uint64)


@pytest.mark.parametrize("filt", [24, -1])
def test_wheel_hard_cases(isp, filt):
    a = hard_cases()
    assert a.size > 550
    got = run(isp, a, wheel_log2=40, filter_primes=filt)
    exp = oracle.wheel_array(a, nthreads=NTHREADS)
    assert np.array_equal(got, exp), a[np.nonzero(got != exp)[0][:10]]
    exp5, _ = oracle.isprime_array(a, nthreads=NTHREADS, use_table=False)
    assert np.array_equal(exp, exp5)


@pytest.mark.parametrize("bits", [33, 36, 40])
def test_wheel_octaves(isp, bits):
    a = W.odd_band(60000, bits)
    got = run(isp, a, wheel_log2=40)
    exp, _ = oracle.isprime_array(a, nthreads=NTHREADS, use_table=False)
    assert np.array_equal(got, exp)
    sub = a[:3000]
    assert np.array_equal(got[:3000], oracle.wheel_array(sub, nthreads=NTHREADS))
    assert 0 < int(got.sum()) < a.size


@pytest.mark.parametrize("b", [33, 36, 40])
def test_wheel_bound_splits_wheel_and_miller_rabin(isp, b):
    """Mixed magnitudes: below 2^b the wheel decides, above it Miller-Rabin;
    the bytes equal the default path's and the oracle's."""
    a = np.concatenate([W.c3_mixed(1 << 18, start=7), W.odd_band(20000, b),
                        W.odd_band(20000, b + 1), hard_cases()])
    got = run(isp, a, wheel_log2=b)
    exp, _ = oracle.isprime_array(a, nthreads=NTHREADS)
    assert np.array_equal(got, exp)
    assert np.array_equal(got, run(isp, a))


def test_wheel_small_call_and_empty(isp):
    """Calls of at most 65,536 elements skip the fused kernel when the wheel
    is on; an empty call is a no-op."""
    a = np.concatenate([hard_cases(), W.odd_band(5000, 38)])
    assert a.size <= 65536
    got = run(isp, a, wheel_log2=40)
    exp, _ = oracle.isprime_array(a, nthreads=NTHREADS, use_table=False)
    assert np.array_equal(got, exp)
    assert run(isp, np.zeros(0, dtype=np.uint64), wheel_log2=40).size == 0


def test_wheel_batched(isp):
    arrays = [W.odd_band(n, bits) for n, bits in ((1, 34), (3000, 40), (70000, 36), (17, 39))]
    arrays += [hard_cases(), W.c2_mr64(5000)]
    dev = [torch.from_numpy(x.view(np.int64)).cuda() for x in arrays]
    prev = isp.set_config(wheel_log2=40)
    try:
        outs = isp.isprime_batched(dev)
        torch.cuda.synchronize()
    finally:
        isp.set_config(**prev)
    for x, o in zip(arrays, outs):
        exp, _ = oracle.isprime_array(x, nthreads=NTHREADS, use_table=False)
        assert np.array_equal(o.cpu().numpy().astype(np.uint8), exp)

