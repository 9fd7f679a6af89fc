"""Host-side pieces of bench.py, checked without a GPU: the exit for more
than one GPU, the integer helpers behind the roofline's algorithmic work,
and the guard on the committed counter summary."""
import os
import subprocess
import sys

import numpy as np

import bench
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
U64 = (1 << 64) - 1


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bit_length_and_popcount_against_python():
    rng = np.random.default_rng(1)
    a = np.concatenate([np.array([0, 1, 2, 3, (1 << 32) - 1, 1 << 32, (1 << 63), U64],
                                 dtype=np.uint64),
                        rng.integers(0, U64, size=2000, dtype=np.uint64, endpoint=True)])
    assert bench.bit_length(a).tolist() == [int(x).bit_length() for x in a.tolist()]
    assert bench.popcount(a).tolist() == [bin(int(x)).count("1") for x in a.tolist()]


def test_mr_work_by_brute_force():
    """Squarings, doublings and products counted one element at a time."""
    rng = np.random.default_rng(2)
    a = np.concatenate([rng.integers(1 << 49, U64, size=300, dtype=np.uint64) | np.uint64(1),
                        np.array([(1 << 61) - 1, U64 - 58, 2047, 1 << 40, 3 * 5 * 7 * 313 * (1 << 30) + 0],
                                 dtype=np.uint64)])
    prime, _ = oracle.isprime_array(a, use_table=False)
    primes64 = bench.small_odd_primes(64)
    assert primes64[0] == 3 and primes64[-1] == 313
    for fp in (16, 0):
        work, surv, cand = bench.mr_work(a, prime, fp)
        sq = dbl = mm = ns = nc = 0
        for n in a.tolist():
            if n < (1 << 32) or n % 2 == 0:
                continue
            if fp and any(n % p == 0 for p in primes64):
                continue
            L = n.bit_length()
            ns += 1
            sq += L - 2
            dbl += bin(n - 1).count("1") - 1
        for n, pr in zip(a.tolist(), prime.tolist()):
            if pr and n >= (1 << 32):
                nc += 1
                d = n - 1
                while d % 2 == 0:
                    d //= 2
                mm += 6 * ((n.bit_length() - 2) + (bin(d).count("1") - 1))
        assert (surv, cand) == (ns, nc)
        assert work["mr_base2"]["montmul"] == sq and work["mr_base2"]["doublings"] == dbl
        assert work["mr_rest"]["montmul"] == mm


def test_counter_traffic_follows_the_source_hash():
    h = bench.kernel_source_hash()
    assert h == bench.kernel_source_hash() and len(h) == 16
    recorded = None
    for line in open(os.path.join(ROOT, "profiles", "pmc_c2_mr64.md")):
        if line.startswith("source_sha256_16:"):
            recorded = line.split(":", 1)[1].strip()
    t = bench.counter_traffic("mr_rest")
    if recorded == h:
        assert isinstance(t, int) and t > 0
    else:
        assert t is None
