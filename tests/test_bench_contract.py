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


def window_products(d: int) -> int:
    """Products of a^d by 3-bit fixed windows, one step at a time: the
    base's Montgomery form, the table a^2 .. a^7, then per further window
    three squarings and one multiplication."""
    nwin = -(-d.bit_length() // 3)
    count = 1 + 6
    for _ in range(nwin - 1):
        count += 3 + 1
    return count


def test_mr_work_by_brute_force():
    """Squarings, doublings and products counted one element at a time, and
    the instructions at each magnitude's product cost (lazy below 2^62)."""
    rng = np.random.default_rng(2)
    a = np.concatenate([rng.integers(1 << 49, U64, size=300, dtype=np.uint64) | np.uint64(1),
                        np.array([(1 << 61) - 1, U64 - 58, 2047, 1 << 40, 3 * 5 * 7 * 313 * (1 << 30) + 0],
                                 dtype=np.uint64)])
    prime, _ = oracle.isprime_array(a, use_table=False)
    primes64 = bench.small_odd_primes(64)
    assert primes64[0] == 3 and primes64[-1] == 313
    for fp in (16, 0):
        work, surv, cand = bench.mr_work(a, prime, fp)
        sq = dbl = mm = ns = nc = ops2 = ops_rest = 0
        for n in a.tolist():
            if n < (1 << 32) or n % 2 == 0:
                continue
            if fp and any(n % p == 0 for p in primes64):
                continue
            L = n.bit_length()
            ns += 1
            sq += L - 2
            dbl += bin(n - 1).count("1") - 1
            lazy = n < (1 << 62)
            ops2 += (L - 2) * (20 if lazy else 22) + (bin(n - 1).count("1") - 1) * (1 if lazy else 5)
        for n, pr in zip(a.tolist(), prime.tolist()):
            if pr and n >= (1 << 32):
                nc += 1
                d = n - 1
                while d % 2 == 0:
                    d //= 2
                mm += 6 * window_products(d)
                ops_rest += 6 * window_products(d) * (20 if n < (1 << 62) else 22)
        assert (surv, cand) == (ns, nc)
        assert work["mr_base2"]["montmul"] == sq and work["mr_base2"]["doublings"] == dbl
        assert work["mr_base2"]["ops"] == ops2
        assert work["mr_rest"]["montmul"] == mm and work["mr_rest"]["ops"] == ops_rest


def test_planted_pseudoprimes_by_the_oracle():
    """The bases a composite that passes base 2 runs (through its first
    failing one), against the oracle's strong-test round, on every Chernick
    number above 2^32 and on F5 = 2^32 + 1 and 3825123056546413051."""
    import workloads as W
    bases = oracle.mr_bases()
    assert tuple(bases[1:]) == bench.BASES_AFTER_2
    planted = np.concatenate([W.chernick_values(),
                              np.array([(1 << 32) + 1, 3825123056546413051], dtype=np.uint64)])
    a = np.concatenate([planted, np.array([2047, (1 << 61) - 1, 7], dtype=np.uint64)])
    got = bench.planted_pseudoprime_bases(a, planted)
    passers = 0
    for n, k in zip(a.tolist(), got.tolist()):
        if n < (1 << 32) or n % 2 == 0 or not oracle.strong_probable_prime(n, 2):
            assert k == 0, n
            continue
        ran = 0
        for b in bases[1:]:
            ran += 1
            if not oracle.strong_probable_prime(n, b):
                break
        else:
            ran = 0  # passes all seven (prime): not a planted pseudoprime
        assert k == ran, (n, k, ran)
        passers += k > 0
    # 251 of the Chernick numbers above 2^32 pass base 2, as do F5 and
    # 3825123056546413051 (a strong pseudoprime to every prime base below
    # 37), which passes 325 and 9375 and fails 28178
    assert passers == 253
    assert got[planted.size - 1] == 3


def test_mr_work_counts_planted_passers():
    import workloads as W
    cher = W.chernick_values()
    a = cher[cher >= np.uint64(1 << 32)]
    prime, _ = oracle.isprime_array(a, use_table=False)
    assert prime.sum() == 0
    work, _, _ = bench.mr_work(a, prime, 16, cher)
    nb = bench.planted_pseudoprime_bases(a, cher)
    mm = 0
    for n, k in zip(a.tolist(), nb.tolist()):
        d = n - 1
        while d % 2 == 0:
            d //= 2
        mm += k * window_products(d)
    assert work["mr_rest"]["montmul"] == mm > 0
    assert work["mr_rest"]["passers_counted"] == int((nb > 0).sum()) == 251


def test_classify_bytes_and_crossings():
    # table reads: odd values in [3, 2^32) coprime to 105 (11, 13, 2^32 - 5)
    a = np.array([0, 1, 2, 3, 4, 5, 9, 11, 13, 15, 21, 35, (1 << 32) - 5, (1 << 32) - 1,
                  1 << 32, (1 << 32) + 1], dtype=np.uint64)
    assert bench.classify_bytes(a) == 9 * a.size + 4 * 3
    # crossings: odd multiples of each prime 37 <= p < 2^16 from p^2 below 2^32
    ps = [p for p in range(37, 1 << 16, 2) if all(p % q for q in range(3, int(p ** 0.5) + 1, 2))]
    assert len(ps) == 6541 - 10
    assert bench.table_crossings() == sum(((1 << 32) - 1 - p * p) // (2 * p) + 1 for p in ps)


def test_counter_traffic_follows_the_source_hash():
    h = bench.kernel_source_hash()
    assert h == bench.kernel_source_hash() and len(h) == 16
    for summary in ("pmc_c3_mixed.md", "pmc_c2_mr64.md"):
        path = os.path.join(ROOT, "profiles", summary)
        if not os.path.exists(path):
            assert bench.counter_traffic("mr_rest", summary) is None
            continue
        recorded = None
        for line in open(path):
            if line.startswith("source_sha256_16:"):
                recorded = line.split(":", 1)[1].strip()
        t = bench.counter_traffic("mr_rest", summary)
        if recorded == h:
            assert isinstance(t, int) and t > 0
        else:
            assert t is None
