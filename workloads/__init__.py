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


def digest(a: np.ndarray) -> str:
    """Short SHA-256 of an array's bytes, recorded beside results."""
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]
