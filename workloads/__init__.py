"""Seeded synthetic inputs for elementwise uint64 primality.

This module is shared by the tests, the benchmark and the smoke check, and it
holds none of the method's arithmetic: it only draws numbers.  Every draw is
splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) used as a counter-based generator: draw k of the
stream with seed s is ``mix(s + (k + 1) * 0x9E3779B97F4A7C15)``, which is
exactly the k-th output of the sequential generator started at s.  Element i
of a workload owns the draws ``i * 8 + j`` for j < 8, so any element can be
regenerated alone and chunked generation gives the same bytes.

The one list this module reads, ``chernick_k.txt``, holds the k for which
(6k+1), (12k+1) and (18k+1) are all prime and their product is below 2^64.
It was written by ``make_chernick_k.py``, which calls only the oracle.

Workloads (sizes, value classes and mixes of the configurations the library
is measured on):

* ``c1_uniform20``   65,536 values uniform in [0, 2^20).
* ``c2_mr64``        2^24 values rejection-uniform in [2^49, 2^64); the low
                     bit is forced to 1 when a coin draw's top bit is set.
* ``c3_mixed``       2^26 values: 5% Chernick numbers, 1% one of
                     {2047, 3215031751, 2^61 - 1}, the rest octave-uniform
                     (bit length uniform, then uniform within the octave).
* ``c4_batched``     4096 arrays, lengths log-uniform in [1, 2^16], each
                     drawn from one magnitude class.
* ``c5_requests``    a Poisson request stream of arrays, lengths log-uniform
                     in [1, 2^20], classes as in ``c4_batched``.
* ``odd_band``       odd values uniform in one octave [2^(b-1), 2^b) (the
                     wheel-against-Miller-Rabin comparison, one octave at a
                     time).
* ``lookup32``       2^26 values uniform in [0, 2^32): the table lookup alone.

``paper_arrays()`` rebuilds the array workloads of the paper's
incrementing-sequence table (section 6.1.3) and array-performance table
(section 8.2) from their descriptions; ``PAPER_INTERVALS`` names the ones
that are contiguous intervals.  The lists they need that depend on
primality (primes below 2^17, the largest 52-bit prime, the 100 largest
64-bit primes, the 100 largest composites below 2^64 with every prime factor
above 2*10^7) are read from ``paper_lists.txt``, written by
``make_paper_lists.py`` with the oracle.  The normal distributions' standard
deviation is not printed in the paper; it is taken as mean / 16.
"""
from __future__ import annotations

import hashlib
import math
import os

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)
DRAWS_PER_ELEMENT = 8

SEED_C1 = 0x2108047900000001
SEED_C2 = 0x2108047900000002
SEED_C3 = 0x2108047900000003
SEED_C4 = 0x2108047900000004
SEED_C5 = 0x2108047900000005
SEED_PAPER = 0x2108047900000006
SEED_BAND = 0x2108047900000007
SEED_LOOKUP = 0x2108047900000008

# Magnitude classes of the batched and served workloads: [lo, hi) as
# (shift, lo): a draw r gives r >> shift, accepted when >= lo.
CLASSES = (
    (44, 0),            # [0, 2^20)
    (32, 1 << 20),      # [2^20, 2^32)
    (15, 1 << 32),      # [2^32, 2^49)
    (0, 1 << 49),       # [2^49, 2^64)
)

_HERE = os.path.dirname(os.path.abspath(__file__))
_CHUNK = 1 << 21


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * M1
    z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def draws(seed: int, k: np.ndarray) -> np.ndarray:
    """splitmix64 outputs number k (uint64 array) of the stream ``seed``."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(np.uint64(seed) + (k + np.uint64(1)) * GAMMA)


def element_draws(seed: int, idx: np.ndarray, j: int) -> np.ndarray:
    idx = np.asarray(idx, dtype=np.uint64)
    return draws(seed, idx * np.uint64(DRAWS_PER_ELEMENT) + np.uint64(j))


def _rejection(seed: int, idx: np.ndarray, shift: int, lo: int, first_j: int = 0,
               tries: int = 6) -> np.ndarray:
    """Uniform in [lo, 2^(64-shift)) by rejection on shifted draws j = first_j.."""
    out = np.zeros(idx.shape, dtype=np.uint64)
    done = np.zeros(idx.shape, dtype=bool)
    for j in range(first_j, first_j + tries):
        v = element_draws(seed, idx, j) >> np.uint64(shift)
        take = (~done) & (v >= np.uint64(lo))
        out[take] = v[take]
        done |= take
        if done.all():
            return out
    raise RuntimeError("rejection sampling did not terminate")  # probability < 2^-70


def c1_uniform20(n: int = 65536, seed: int = SEED_C1, start: int = 0) -> np.ndarray:
    idx = np.arange(start, start + n, dtype=np.uint64)
    return element_draws(seed, idx, 0) >> np.uint64(44)


def c2_mr64(n: int = 1 << 24, seed: int = SEED_C2, start: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    for c0 in range(0, n, _CHUNK):
        idx = np.arange(start + c0, start + min(n, c0 + _CHUNK), dtype=np.uint64)
        v = _rejection(seed, idx, 0, 1 << 49)
        coin = element_draws(seed, idx, 7) >> np.uint64(63)
        out[c0:c0 + idx.size] = v | coin
    return out


def odd_band(n: int, bits: int, seed: int = SEED_BAND, start: int = 0) -> np.ndarray:
    """n odd values uniform in [2^(bits-1), 2^bits), 2 <= bits <= 64."""
    if not 2 <= bits <= 64:
        raise ValueError("bits must be in [2, 64]")
    idx = np.arange(start, start + n, dtype=np.uint64)
    v = element_draws(seed ^ bits, idx, 0) >> np.uint64(65 - bits)
    return v | np.uint64(1 << (bits - 1)) | np.uint64(1)


def lookup32(n: int = 1 << 26, seed: int = SEED_LOOKUP, start: int = 0) -> np.ndarray:
    """n values uniform in [0, 2^32): the lookup path alone (every odd value
    is decided below the table bound; those coprime to 210 by one random
    read of the wheel table, spread over the whole of it)."""
    idx = np.arange(start, start + n, dtype=np.uint64)
    return element_draws(seed, idx, 0) >> np.uint64(32)


def chernick_k() -> np.ndarray:
    path = os.path.join(_HERE, "chernick_k.txt")
    vals = [int(x) for line in open(path) if not line.startswith("#") for x in line.split()]
    return np.array(vals, dtype=np.uint64)


def chernick_values() -> np.ndarray:
    k = [int(x) for x in chernick_k()]
    return np.array([(6 * x + 1) * (12 * x + 1) * (18 * x + 1) for x in k], dtype=np.uint64)


C3_FIXED = np.array([2047, 3215031751, (1 << 61) - 1], dtype=np.uint64)
# Thresholds on a 32-bit draw: 5% Chernick, then 1% fixed values.
C3_T_CHERNICK = 214748365          # round(0.05 * 2^32)
C3_T_FIXED = 214748365 + 42949673  # + round(0.01 * 2^32)


def c3_mixed(n: int = 1 << 26, seed: int = SEED_C3, start: int = 0) -> np.ndarray:
    cher = chernick_values()
    out = np.empty(n, dtype=np.uint64)
    one = np.uint64(1)
    for c0 in range(0, n, _CHUNK):
        idx = np.arange(start + c0, start + min(n, c0 + _CHUNK), dtype=np.uint64)
        sel = element_draws(seed, idx, 0) >> np.uint64(32)
        r1 = element_draws(seed, idx, 1)
        # octave-uniform: bit length b+1 with b uniform in [0, 64), value
        # 2^b + uniform in [0, 2^b)
        b = element_draws(seed, idx, 2) >> np.uint64(58)
        r3 = element_draws(seed, idx, 3)
        low = np.where(b == 0, np.uint64(0), r3 & ((one << b) - one))
        v = (one << b) | low
        is_ch = sel < np.uint64(C3_T_CHERNICK)
        is_fx = (~is_ch) & (sel < np.uint64(C3_T_FIXED))
        v[is_ch] = cher[(r1[is_ch] % np.uint64(cher.size)).astype(np.int64)]
        v[is_fx] = C3_FIXED[(r1[is_fx] % np.uint64(3)).astype(np.int64)]
        out[c0:c0 + idx.size] = v
    return out


def class_values(seed: int, idx: np.ndarray, cls: int) -> np.ndarray:
    shift, lo = CLASSES[cls]
    return _rejection(seed, idx, shift, lo)


def log_uniform_lengths(seed: int, count: int, max_len: int, first: int = 0) -> np.ndarray:
    """floor(2^(u * log2(max_len + 1))) for u = (r >> 11) * 2^-53: in [1, max_len]."""
    r = draws(seed, np.arange(first, first + count, dtype=np.uint64) * np.uint64(4))
    u = (r >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    L = np.floor(np.exp2(u * math.log2(max_len + 1))).astype(np.int64)
    return np.clip(L, 1, max_len)


def c4_batched(num_arrays: int = 4096, max_len: int = 1 << 16, seed: int = SEED_C4):
    """List of (uint64 array, class) pairs."""
    lens = log_uniform_lengths(seed, num_arrays, max_len)
    cls = (draws(seed, np.arange(num_arrays, dtype=np.uint64) * np.uint64(4) + np.uint64(1))
           % np.uint64(4)).astype(np.int64)
    vseed = int(draws(seed, np.array([1 << 40], dtype=np.uint64))[0])
    arrays, off = [], 0
    for L, c in zip(lens.tolist(), cls.tolist()):
        idx = np.arange(off, off + L, dtype=np.uint64)
        arrays.append((class_values(vseed, idx, c), c))
        off += L
    return arrays


def c5_requests(num: int = 2100, qps: float = 1000.0, max_len: int = 1 << 20,
                seed: int = SEED_C5):
    """Poisson request stream: list of (arrival_s, uint64 array, class)."""
    lens = log_uniform_lengths(seed, num, max_len)
    k = np.arange(num, dtype=np.uint64) * np.uint64(4)
    cls = (draws(seed, k + np.uint64(1)) % np.uint64(4)).astype(np.int64)
    u = (draws(seed, k + np.uint64(2)) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    gaps = -np.log1p(-u) / qps
    t = np.cumsum(gaps)
    vseed = int(draws(seed, np.array([1 << 40], dtype=np.uint64))[0])
    reqs, off = [], 0
    for i in range(num):
        L, c = int(lens[i]), int(cls[i])
        idx = np.arange(off, off + L, dtype=np.uint64)
        reqs.append((float(t[i]), class_values(vseed, idx, c), c))
        off += L
    return reqs


def _paper_list(name: str) -> np.ndarray:
    vals, cur = {}, None
    for line in open(os.path.join(_HERE, "paper_lists.txt")):
        if line.startswith("# "):
            parts = line.split()
            cur = parts[1] if len(parts) == 3 else None
            if cur:
                vals[cur] = []
        elif cur:
            vals[cur] += [int(x) for x in line.split()]
    return np.array(vals[name], dtype=np.uint64)


def _std_normal(seed: int, idx: np.ndarray, j: int) -> np.ndarray:
    """Standard normal deviates by the Box-Muller transform of draws j, j+1."""
    u1 = ((element_draws(seed, idx, j) >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (element_draws(seed, idx, j + 1) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def _normal_int(seed: int, n: int, mean: int, std: int) -> np.ndarray:
    """mean + round(std * z): exact integer offsets around a power of two."""
    z = _std_normal(seed, np.arange(n, dtype=np.uint64), 0)
    off = np.rint(z * std).astype(np.int64)  # |z| < 9, so mean + off stays in [0, 2^63)
    return (np.int64(mean) + off).astype(np.uint64)


# 1:N of the incrementing-sequence table and the Unix seconds of 2021
# (1609477200 through 1609477200 + 3600 * 24 * 365, inclusive): (lo, length).
PAPER_INTERVALS = {
    "inc_1e4": (1, 10 ** 4),
    "inc_1e5": (1, 10 ** 5),
    "inc_1e6": (1, 10 ** 6),
    "inc_1e7": (1, 10 ** 7),
    "inc_1e8": (1, 10 ** 8),
    "unix_2021": (1609477200, 3600 * 24 * 365 + 1),
}


def interval(lo: int, length: int) -> np.ndarray:
    return np.uint64(lo) + np.arange(length, dtype=np.uint64)


def paper_arrays(seed: int = SEED_PAPER, include_intervals: bool = False) -> dict:
    """name -> uint64 array (matrix workloads keep their 2-D shape)."""
    sub = [int(x) for x in draws(seed, np.arange(16, dtype=np.uint64) + np.uint64(1 << 40))]
    pool = _paper_list("primes_below_2_17")
    out = {}
    if include_intervals:
        for name, (lo, length) in PAPER_INTERVALS.items():
            out[name] = interval(lo, length)
    # 200 primes of int16 (below 2^15), uniform over that list
    p15 = pool[pool < np.uint64(1 << 15)]
    r = element_draws(sub[0], np.arange(200, dtype=np.uint64), 0)
    out["int16_primes_200"] = p15[(r % np.uint64(p15.size)).astype(np.int64)]
    # 1000 x 1000 random 32-bit integers
    r = element_draws(sub[1], np.arange(10 ** 6, dtype=np.uint64), 0) >> np.uint64(32)
    out["matrix_1000x1000_u32"] = r.reshape(1000, 1000)
    # 1M primes, normal around 2^16: each draw moves up to the next prime
    v = np.clip(_normal_int(sub[2], 10 ** 6, 1 << 16, 1 << 12), 2, (1 << 17) - 1)
    k = np.minimum(np.searchsorted(pool, v, side="left"), pool.size - 1)
    out["normal_primes_1m_mean_2_16"] = pool[k]
    # 100,000 odd numbers, normal around 2^32
    out["normal_odd_100k_mean_2_32"] = _normal_int(sub[3], 10 ** 5, 1 << 32, 1 << 28) | np.uint64(1)
    # 1000 numbers, normal around 2^53
    out["normal_1000_mean_2_53"] = _normal_int(sub[4], 1000, 1 << 53, 1 << 49)
    # the largest 52-bit prime, 1000 times
    out["largest52_prime_x1000"] = np.repeat(_paper_list("largest_prime_below_2_52"), 1000)
    # the 100 largest composites below 2^64 with all prime factors > 2*10^7
    out["composites_100_factors_gt_2e7"] = _paper_list("largest_composites_factors_gt_2e7")
    # the 100 largest 64-bit primes; the 5000 largest 64-bit odd integers
    out["largest64_primes_100"] = _paper_list("largest_64bit_primes")
    out["largest64_odd_5000"] = np.uint64((1 << 64) - 1) - np.uint64(2) * np.arange(5000, dtype=np.uint64)
    return out


def digest(a: np.ndarray) -> str:
    """Short SHA-256 of an array's bytes, recorded beside results."""
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]
