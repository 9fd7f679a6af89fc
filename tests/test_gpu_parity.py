"""GPU parity: the HIP path against the oracle, element by element, through
the C ABI.  Tolerance is zero mismatching bytes everywhere (primality is a
function; there is no rounding anywhere on either side)."""
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

U64 = (1 << 64) - 1
NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def isp():
    import paper_2108_04791_amd as isp
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    isp.init()
    return isp


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def gpu_isprime(isp, a: np.ndarray) -> np.ndarray:
    out = isp.isprime(to_dev(a))
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.uint8)


def expect(a: np.ndarray, use_table=None) -> np.ndarray:
    out, _ = oracle.isprime_array(a, nthreads=NTHREADS, use_table=use_table)
    return out


def assert_same(a, got, exp, what):
    bad = np.nonzero(got != exp)[0]
    if bad.size:
        i = bad[:10]
        raise AssertionError("%s: %d mismatches, first %s values %s gpu %s oracle %s" % (
            what, bad.size, i.tolist(), a[i].tolist(), got[i].tolist(), exp[i].tolist()))


EDGES = [0, 1, 2, 3, 4, 5, 7, 9, 11, 15, 21, 25, 35, 49, 121, 209, 211, 221, 2047, 65521,
         65535, 65537, (1 << 31) - 1, 4294967250, 4294967251, 4294967279,
         (1 << 32) - 5, (1 << 32) - 3, (1 << 32) - 1, 1 << 32, (1 << 32) + 1, (1 << 32) + 15,
         (1 << 32) + 17, 4294967291 * 4294967279, (1 << 61) - 1, (1 << 62) + 135,
         (1 << 63) - 25, (1 << 63) + 29, (1 << 63) + 1, U64 - 58, U64 - 2, U64 - 1, U64,
         3215031751, 3825123056546413051, 341550071728321, 2152302898747, 3474749660383,
         18446744073709551557, 18446744073709551533, 4611686018427388039,
         6700417 * 641, 1000000007 * 998244353]


def test_worked_example(isp):
    """Section 1: [1, 2, 3, 4, 5] -> 0 1 1 0 1, shape kept."""
    t = torch.tensor([[1, 2, 3, 4, 5]], dtype=torch.int64, device="cuda")
    out = isp.isprime(t)
    assert out.shape == t.shape and out.dtype == torch.bool
    assert out.cpu().int().tolist() == [[0, 1, 1, 0, 1]]


def test_table_equals_oracle(isp, oracle_table):
    tab = isp.table().cpu().numpy().view(np.uint32)
    assert tab.size == 1 << 26
    assert int(tab[0]) == 0x64B4CB6E
    neq = np.nonzero(tab != oracle_table)[0]
    assert neq.size == 0, "table words differ at %s" % neq[:10].tolist()


def test_wheel_table_equals_oracle(isp, oracle_table):
    """The table the array path reads, on the 2*3*5*7 wheel (section 3):
    bit 48 q + k stands for 210 q + r_k, r_k the k-th residue coprime to
    210; every word against the oracle's odd-only table (bit i <-> 2i + 1,
    so 210 q + r is bit 105 q + (r >> 1)), 0 at and above 2^32."""
    wt = isp.wheel_table().cpu().numpy().view(np.uint32)
    assert wt.size == 30678339
    res = np.array([r for r in range(210) if np.gcd(r, 210) == 1])
    assert res.size == 48 and res[1] == 11
    blocks = -(-(1 << 32) // 210)
    bits = np.unpackbits(oracle_table.view(np.uint8), bitorder="little")
    assert bits.size == 1 << 31
    bits = np.concatenate([bits, np.zeros(105 * blocks - bits.size, dtype=np.uint8)])
    exp = np.packbits(bits.reshape(blocks, 105)[:, res >> 1].reshape(-1),
                      bitorder="little").view(np.uint32)
    neq = np.nonzero(wt != exp)[0]
    assert neq.size == 0, "wheel table words differ at %s" % neq[:10].tolist()


def test_montmul_against_python(isp):
    rng = np.random.default_rng(11)
    mods = [(1 << 32) + 15, (1 << 63) - 25, (1 << 63) + 29, U64 - 58, U64, 3, 5, 65537,
            (1 << 61) - 1]
    mods += [int(x) | 1 for x in rng.integers(0, 1 << 63, size=200, dtype=np.uint64) * 2 + 1]
    A, B, N = [], [], []
    for n in mods:
        vals = [0, 1, 2 % n, n - 1, n - 2, n // 2] + [int(x) % n for x in
                                                     rng.integers(0, 1 << 63, size=8, dtype=np.uint64)]
        for a in vals:
            for b in vals[:6]:
                A.append(a)
                B.append(b)
                N.append(n)
    a, b, n = (np.array(x, dtype=np.uint64) for x in (A, B, N))
    got = isp.montmul(to_dev(a), to_dev(b), to_dev(n)).cpu().numpy().view(np.uint64)
    exp = np.array([x * y % m for x, y, m in zip(A, B, N)], dtype=np.uint64)
    assert_same(a, got, exp, "montmul")


def test_edge_values(isp):
    a = np.array(EDGES, dtype=np.uint64)
    got = gpu_isprime(isp, a)
    assert_same(a, got, expect(a, use_table=False), "edges")
    # known verdicts
    v = dict(zip(EDGES, got.tolist()))
    assert v[(1 << 61) - 1] == 1 and v[U64 - 58] == 1 and v[(1 << 32) + 15] == 1
    assert v[2047] == 0 and v[3215031751] == 0 and v[(1 << 32) + 1] == 0 and v[U64] == 0


def test_all_below_2_20(isp):
    a = np.arange(1 << 20, dtype=np.uint64)
    assert_same(a, gpu_isprime(isp, a), expect(a, use_table=False), "0..2^20")


def test_lookups_over_the_whole_table(isp, oracle_table):
    """2^22 values uniform in [0, 2^32) (the lookup workload's first ones),
    each an odd one read from the wheel table, against the oracle's table."""
    a = W.lookup32(1 << 22)
    assert_same(a, gpu_isprime(isp, a), expect(a, use_table=True), "lookups below 2^32")


def test_window_around_table_bound(isp):
    a = np.arange((1 << 32) - 50000, (1 << 32) + 50000, dtype=np.uint64)
    assert_same(a, gpu_isprime(isp, a), expect(a, use_table=False), "2^32 +- 50000")


def test_c1_full(isp):
    a = W.c1_uniform20()
    assert_same(a, gpu_isprime(isp, a), expect(a, use_table=False), "C1")


@pytest.mark.parametrize("size", [1, 2, 3, 63, 64, 65, 255, 256, 257, 1023, 1024, 1025, 4097,
                                  100003])
def test_ragged_sizes(isp, size):
    a = W.c3_mixed(size, start=size * 7)
    a[: min(size, 8)] = np.array(EDGES[-8:], dtype=np.uint64)[: min(size, 8)]
    assert_same(a, gpu_isprime(isp, a), expect(a, use_table=False), "ragged %d" % size)


def test_unaligned_views(isp):
    a = W.c2_mr64(5000)
    t = to_dev(a)
    for off in (1, 3):
        out = isp.isprime(t[off:])
        torch.cuda.synchronize()
        assert_same(a[off:], out.cpu().numpy().astype(np.uint8), expect(a[off:]), "offset %d" % off)


def test_empty_and_invalid(isp):
    t = torch.empty(0, dtype=torch.int64, device="cuda")
    assert isp.isprime(t).numel() == 0
    L = isp.lib()
    assert L.isprime_u64(None, None, 0, None) == isp.ISP_OK
    assert L.isprime_u64(None, None, 5, None) == isp.ISP_EINVAL
    assert L.isprime_u64(t.data_ptr() or 8, None, 5, None) == isp.ISP_EINVAL
    with pytest.raises(isp.IsprimeError):
        isp.set_config(classify_ept=3)


def test_c2_full(isp):
    a = W.c2_mr64()
    got = gpu_isprime(isp, a)
    assert_same(a, got, expect(a), "C2")
    assert 0.02 < got.mean() < 0.05


@pytest.mark.parametrize("bits", [33, 48, 59, 60, 61, 62, 63, 64])
def test_one_bit_length_per_array(isp, bits):
    """Arrays of a single bit length (the Miller-Rabin loops run one length per
    wavefront; below 2^62 the base-2 doubling is a plain shift), with base-2
    strong pseudoprimes of that length mixed in."""
    rng = np.random.default_rng(bits)
    lo = 1 << (bits - 1)
    a = (rng.integers(0, lo, 40000, dtype=np.uint64) + np.uint64(lo)) | np.uint64(1)
    ch = W.chernick_values()
    top = (1 << bits) - 1  # the largest value of this bit length
    ch = ch[(ch >= np.uint64(lo)) & (ch <= np.uint64(top))]
    a = np.concatenate([a, ch, np.array([lo + 1, top], dtype=np.uint64)])
    rng.shuffle(a)
    got = gpu_isprime(isp, a)
    assert_same(a, got, expect(a, use_table=False), "bit length %d" % bits)


def test_c3_full(isp, oracle_table):
    a = W.c3_mixed()
    got = gpu_isprime(isp, a)
    assert_same(a, got, expect(a, use_table=True), "C3")


def test_counts_match_host_accounting(isp):
    """Survivors = odd elements >= 2^32 with no factor among the filter
    primes (the first 64 odd primes when the filter is on); candidates =
    survivors passing the base-2 round (a call above the fused kernel's
    size, which keeps no counters)."""
    a = W.c2_mr64((1 << 16) + 1)
    cfg = isp.get_config()
    gpu_isprime(isp, a)
    surv, cand = isp.last_counts()
    # the classify kernel tests the first filter_primes odd primes and the
    # second stage the rest of the first 64
    F = cfg["filter_primes"]
    F = 0 if F <= 0 else max(F, 64)
    primes = [p for p in range(3, 2000, 2) if oracle.trial_is_prime(p)][:F]
    big = a[(a >= np.uint64(1 << 32)) & ((a & np.uint64(1)) == 1)]
    keep = np.ones(big.size, dtype=bool)
    for p in primes:
        keep &= (big % np.uint64(p)) != 0
    assert surv == int(keep.sum())
    assert cand == sum(oracle.strong_probable_prime(int(n), 2) for n in big[keep])


@pytest.mark.parametrize("cfg", [
    dict(classify_ept=1, classify_block=64),
    dict(classify_ept=2, classify_block=1024, classify_blocks_per_cu=1),
    dict(classify_ept=8, classify_block=128, classify_blocks_per_cu=16),
    dict(filter_primes=-1),
    dict(filter_primes=64), dict(filter_primes=8),
    dict(sort_survivors=-1),
    dict(mr_window=1), dict(mr_window=2), dict(mr_window=4),
    dict(mr_block=64, mr_blocks_per_cu=1),
    dict(mr_block=128, mr_blocks_per_cu=16),
    dict(mr_block=1024, mr_blocks_per_cu=1),
    dict(mr_block=512, mr_blocks_per_cu=4, mr_window=2),
])
def test_configs_do_not_change_bits(isp, cfg):
    # above the fused kernel's size, so every launch parameter is in play
    a = np.concatenate([np.array(EDGES, dtype=np.uint64), W.c3_mixed(70011, start=99),
                        W.chernick_values()])
    prev = isp.set_config(**cfg)
    try:
        got = gpu_isprime(isp, a)
    finally:
        isp.set_config(**prev)
    assert_same(a, got, expect(a, use_table=False), str(cfg))


def test_permutation_metamorphic(isp):
    a = W.c3_mixed(50000, start=12345)
    perm = np.random.default_rng(5).permutation(a.size)
    g1 = gpu_isprime(isp, a)
    g2 = gpu_isprime(isp, a[perm])
    assert np.array_equal(g1[perm], g2)


@pytest.mark.parametrize("size", [1, 64, 65535, 65536, 65537])
def test_fused_and_three_kernel_paths(isp, size):
    """Calls of up to 65,536 elements run as one fused kernel, larger ones as
    the three kernels: both equal the oracle on base-2 pseudoprimes, primes
    and composites of every length, at and around the size where the path
    changes, and the smallest call reads no counters."""
    base = np.concatenate([W.chernick_values(), np.array(EDGES, dtype=np.uint64),
                           W.c2_mr64(70000, start=3), W.c3_mixed(70000, start=4)])
    a = base[:size]
    assert_same(a, gpu_isprime(isp, a), expect(a, use_table=False), "size %d" % size)
    if size <= 65536:
        assert isp.last_counts() == (0, 0)


def test_two_streams(isp):
    a = W.c2_mr64(300000, start=777)
    b = W.c3_mixed(300000, start=888)
    ta, tb = to_dev(a), to_dev(b)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    oa = isp.isprime(ta, stream=s1)
    ob = isp.isprime(tb, stream=s2)
    torch.cuda.synchronize()
    assert_same(a, oa.cpu().numpy().astype(np.uint8), expect(a), "stream 1")
    assert_same(b, ob.cpu().numpy().astype(np.uint8), expect(b, use_table=False), "stream 2")


def test_larger_than_one_piece(isp):
    """A plain call of more than 2^28 elements runs in pieces of 2^28 (each
    piece's survivors share 32-bit counters): every output byte is checked.
    The bulk repeats 0 .. 2^20 - 1 (table lookups; the expected bytes are one
    oracle period, repeated on the device); a window of hard values (C2, C3,
    the edge values) straddles the piece boundary and is checked against the
    oracle directly."""
    piece, period = 1 << 28, 1 << 20
    n = piece + period + 13
    dev = torch.arange(n, dtype=torch.int64, device="cuda") % period
    hard = np.concatenate([W.c2_mr64(8192, start=11), W.c3_mixed(8192, start=5),
                           np.array(EDGES, dtype=np.uint64)])
    lo = piece - hard.size // 2
    dev[lo:lo + hard.size] = to_dev(hard)
    out = isp.isprime(dev).to(torch.uint8)
    torch.cuda.synchronize()
    base = torch.from_numpy(expect(np.arange(period, dtype=np.uint64), use_table=False)).cuda()
    exp = base.repeat(n // period + 1)[:n].clone()
    exp[lo:lo + hard.size] = torch.from_numpy(expect(hard)).cuda()
    bad = torch.nonzero(out != exp).flatten()
    assert bad.numel() == 0, (bad[:10].tolist(), dev[bad[:10]].tolist())
    assert int(out[lo:lo + hard.size].sum().item()) > 0



def test_many_passers_per_workgroup(isp):
    """More base-2 passers per workgroup than phase 1 groups (4 per thread,
    at most 4,096), whatever the tuned grid of at most 4096 workgroups: those
    workgroups keep the order found.  2^25 draws from primes of every
    magnitude class of the grouping (64-bit, 63-bit, shorter) and base-2
    strong pseudoprimes; each distinct value is checked by the oracle, and
    every byte against it."""
    vals = []
    for start in ((1 << 63) + 1, (1 << 62) + 1, (1 << 48) + 1, U64 - 4000):
        n, got = start | 1, 0
        while got < 64 and n < U64:
            if oracle.mr7(n):
                vals.append(n)
                got += 1
            n += 2
    spsp = [3825123056546413051, 341550071728321, 2152302898747, 3474749660383]
    uniq = np.array(sorted(set(vals + spsp)), dtype=np.uint64)
    exp_u = expect(uniq, use_table=False)
    assert int(exp_u.sum()) == len(set(vals))
    a = uniq[np.random.default_rng(2048).integers(0, uniq.size, size=1 << 25)]
    got = gpu_isprime(isp, a)
    assert_same(a, got, exp_u[np.searchsorted(uniq, a)], "many passers")
    _, passers = isp.last_counts()
    assert passers > 4096 * 4096  # above 4 per thread even on 4096 workgroups
