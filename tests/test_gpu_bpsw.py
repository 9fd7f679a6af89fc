"""GPU parity of the Baillie-PSW alternative (rest_test=1: base-2 strong test,
then the strong Lucas test with Selfridge's parameters instead of the six
remaining Miller-Rabin bases): identical bytes to the oracle and to the
default path, including composites that pass the base-2 round."""
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


def base2_pseudoprimes_above_2_32():
    vals = [(1 << 32) + 1, 3825123056546413051, 341550071728321, 2152302898747,
            3474749660383]
    vals += [(1 << p) - 1 for p in (37, 41, 43, 47, 53, 59)]
    ch = [int(x) for x in W.chernick_values() if int(x) >= (1 << 32)]
    vals += [n for n in ch if oracle.strong_probable_prime(n, 2)]
    return np.array(vals, dtype=np.uint64)


@pytest.mark.parametrize("filt", [24, -1])
def test_bpsw_parity_hard_cases(isp, filt):
    spsp = base2_pseudoprimes_above_2_32()
    assert spsp.size > 200  # the Chernick numbers that pass base 2
    # squares of primes and products of close primes reach the Lucas round
    # when the filter is off
    sq = np.array([p * p for p in (4294967291, 4294967279, 65537, 1000003)] +
                  [4294967291 * 4294967279, 1000000007 * 998244353, 3 * ((1 << 62) + 1)],
                  dtype=np.uint64)
    a = np.concatenate([spsp, sq, W.chernick_values(), W.c2_mr64(20000, start=5)])
    got = run(isp, a, rest_test=1, filter_primes=filt)
    exp, _ = oracle.isprime_array(a, nthreads=NTHREADS, use_table=False)
    assert np.array_equal(got, exp), np.nonzero(got != exp)[0][:10]
    assert got[:spsp.size].sum() == 0


def test_bpsw_equals_default_on_workloads(isp):
    for a in (W.c2_mr64(), W.c3_mixed(1 << 22, start=1 << 20)):
        assert np.array_equal(run(isp, a, rest_test=1), run(isp, a))


def test_bpsw_full_c2_against_oracle(isp):
    a = W.c2_mr64()
    exp, _ = oracle.isprime_array(a, nthreads=NTHREADS)
    assert np.array_equal(run(isp, a, rest_test=1), exp)
