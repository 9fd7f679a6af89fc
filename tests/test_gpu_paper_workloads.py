"""GPU parity on the paper's array workloads (sections 6.1.3 and 8.2, rebuilt
from their descriptions): every output byte of the array call against the
oracle, shapes kept, and for the contiguous intervals the interval call
against the array call and the prime counts pi(10^k).  Tolerance: zero
mismatching bytes."""
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)
# pi(10^4) ... pi(10^8): standard values of the prime counting function
PI = {"inc_1e4": 1229, "inc_1e5": 9592, "inc_1e6": 78498, "inc_1e7": 664579,
      "inc_1e8": 5761455}


@pytest.fixture(scope="module")
def isp():
    import paper_2108_04791_amd as isp
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    isp.init()
    return isp


@pytest.mark.parametrize("name", sorted(W.paper_arrays().keys()))
def test_array_workload(isp, name):
    a = W.paper_arrays()[name]
    dev = torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()
    got = isp.isprime(dev)
    assert tuple(got.shape) == a.shape
    got = got.cpu().numpy().astype(np.uint8).ravel()
    exp, _ = oracle.isprime_array(a.ravel(), nthreads=NTHREADS, use_table=None)
    assert np.array_equal(got, exp)
    if name in ("int16_primes_200", "normal_primes_1m_mean_2_16", "largest64_primes_100",
                "largest52_prime_x1000"):
        assert got.all()
    if name == "composites_100_factors_gt_2e7":
        assert not got.any()


@pytest.mark.parametrize("name", sorted(W.PAPER_INTERVALS.keys()))
def test_interval_workload(isp, name):
    lo, length = W.PAPER_INTERVALS[name]
    arr = torch.arange(lo, lo + length, dtype=torch.int64, device="cuda")
    got = isp.isprime(arr)
    rng = isp.isprime_range(lo, length)
    assert torch.equal(got, rng)
    if name in PI:
        assert int(got.sum().item()) == PI[name]
    if length <= 10 ** 7 or name == "unix_2021":
        exp, _ = oracle.isprime_array(W.interval(lo, length), nthreads=NTHREADS, use_table=None)
        assert np.array_equal(rng.cpu().numpy().astype(np.uint8), exp)
