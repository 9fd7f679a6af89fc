"""The allocation-free entry point against the allocating one, through the
C ABI: isprime_u64_noalloc shares isprime_u64's kernels but takes its
workspace from a static device array, so two calls in a row -- the second
smaller, leaving the first call's survivors and counts behind in the array
-- must both give the bytes of isprime_u64 (and of the oracle) exactly."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2108_04791_amd as isp
    torch.cuda.set_device(0)
    isp.init(0)  # the table and the scratch address: the entry point allocates nothing
    return isp, torch


def _calls(isp, torch, a):
    """(allocating call's bytes, allocation-free call's bytes) on one stream."""
    L = isp.lib()
    dev = torch.from_numpy(a.view(np.int64)).cuda()
    ref = torch.full((a.size,), 7, dtype=torch.uint8, device="cuda")
    got = torch.full((a.size,), 7, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    assert L.isprime_u64(dev.data_ptr(), ref.data_ptr(), a.size, s.cuda_stream) == isp.ISP_OK
    st = L.isprime_u64_noalloc(dev.data_ptr(), got.data_ptr(), a.size, s.cuda_stream)
    assert st == isp.ISP_OK, isp._strerror(st)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_two_calls_then_smaller(env):
    isp, torch = env
    cap = isp.lib().isp_noalloc_max_len()
    assert cap == 1 << 20
    # first call: the maximum length, mixed magnitudes (every path), with the
    # paper's composites that pass base 2 and the largest primes mixed in
    big = W.c3_mixed(cap, start=11)
    big[:W.chernick_values().size] = W.chernick_values()
    big[-3:] = [(1 << 61) - 1, (1 << 64) - 59, 3215031751]
    # second call: smaller and ragged, 64-bit Miller-Rabin-heavy values
    small = W.c2_mr64(300001, start=5)
    for name, a in (("max", big), ("smaller", small)):
        ref, got = _calls(isp, torch, a)
        exp, _ = oracle.isprime_array(a, use_table=False)
        bad = np.nonzero(got != ref)[0]
        assert bad.size == 0, "%s: noalloc != isprime_u64 at %s" % (name, bad[:10].tolist())
        bad = np.nonzero(got != exp)[0]
        assert bad.size == 0, "%s: noalloc != oracle at %s" % (name, bad[:10].tolist())
        assert set(np.unique(got).tolist()) <= {0, 1}


def test_noalloc_small_and_limits(env):
    isp, torch = env
    L = isp.lib()
    # a call within the fused kernel's size, and the paper's worked example
    a = np.concatenate([np.arange(1, 6, dtype=np.uint64), W.c3_mixed(4000, start=3)])
    ref, got = _calls(isp, torch, a)
    assert np.array_equal(got, ref)
    assert got[:5].tolist() == [0, 1, 1, 0, 1]
    # beyond the maximum: refused before anything is enqueued
    cap = L.isp_noalloc_max_len()
    assert L.isprime_u64_noalloc(8, 8, cap + 1, None) == isp.ISP_ERANGE
    assert L.isprime_u64_noalloc(None, None, 0, None) == isp.ISP_OK
