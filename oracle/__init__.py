"""Plain CPU oracle for elementwise uint64 primality (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product path (the HIP
library in ``paper_2108_04791_amd``) never imports, loads or calls it, and the
two share no code.

The arithmetic lives in ``oracle.c`` (plain C, built with gcc); this module
only loads it with ctypes and marshals arguments.  Function map:

=====================  ====================================================
``trial_is_prime``     O1, the definition (trial division), paper section 1
``sieve_odd``          O2, odd-only Eratosthenes, sections 1 and 4
``mulmod``/``powmod``  O3, 128-bit modular product, sections 2.3-2.4
``strong_probable``    one strong-test round, section 2.1 Eq. 1-3
``mr7``                O4, the seven bases of Eq. 4
``is_prime``           O5, table below 2^32, O4 above
``isprime_array``      O5 over an array, on POSIX threads
``find_factor``        O6, Pollard rho (Brent), composite certificate
``pratt_certify``      O6, Pratt certificate for primes
``numdiv``             O7, Table NumDiv of section 6
``wheel_is_prime``     O8, trial division on the 2/3/5/7 wheel, section 3
``wheel_cycle``        the wheel's difference cycle, Eq. 5
=====================  ====================================================
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TABLE_BOUND = 1 << 32

_lock = threading.Lock()
_table_lock = threading.Lock()
_lib = None
_table = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain C, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                        "-Wall", "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build()
        lib = ctypes.CDLL(_LIB)
        u64, i32 = ctypes.c_uint64, ctypes.c_int
        p = ctypes.c_void_p
        sig = {
            "oracle_trial_is_prime": (i32, [u64]),
            "oracle_sieve_words": (u64, [u64]),
            "oracle_sieve_odd": (None, [u64, p]),
            "oracle_mulmod": (u64, [u64, u64, u64]),
            "oracle_powmod": (u64, [u64, u64, u64]),
            "oracle_strong_probable_prime": (i32, [u64, u64]),
            "oracle_mr_base": (u64, [i32]),
            "oracle_mr7": (i32, [u64]),
            "oracle_is_prime": (i32, [u64, p]),
            "oracle_isprime_array": (i32, [p, p, u64, p, i32]),
            "oracle_trial_array": (i32, [p, p, u64, i32]),
            "oracle_mr7_array": (i32, [p, p, u64, i32]),
            "oracle_find_factor": (u64, [u64]),
            "oracle_pratt_certify": (i32, [u64]),
            "oracle_numdiv": (u64, [u64]),
            "oracle_wheel_cycle": (i32, [p]),
            "oracle_wheel_is_prime": (i32, [u64]),
            "oracle_wheel_array": (i32, [p, p, u64, i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def trial_is_prime(n: int) -> int:
    return _load().oracle_trial_is_prime(n)


def sieve_odd(limit: int) -> np.ndarray:
    """Odd-only table for numbers below ``limit``: bit i <-> 2i+1."""
    lib = _load()
    words = lib.oracle_sieve_words(limit)
    t = np.empty(words, dtype=np.uint32)
    lib.oracle_sieve_odd(limit, t.ctypes.data)
    return t


def table() -> np.ndarray:
    """The O2 table for limit 2^32 (256 MiB), built once per process."""
    global _table
    with _table_lock:
        if _table is None:
            _table = sieve_odd(TABLE_BOUND)
        return _table


def mulmod(a: int, b: int, n: int) -> int:
    return _load().oracle_mulmod(a, b, n)


def powmod(a: int, e: int, n: int) -> int:
    return _load().oracle_powmod(a, e, n)


def strong_probable_prime(n: int, a: int) -> int:
    return _load().oracle_strong_probable_prime(n, a)


def mr_bases() -> list:
    return [_load().oracle_mr_base(k) for k in range(7)]


def mr7(n: int) -> int:
    return _load().oracle_mr7(n)


def is_prime(n: int, use_table: bool = False) -> int:
    t = table() if use_table else None
    return _load().oracle_is_prime(n, None if t is None else t.ctypes.data)


def needs_table(n: np.ndarray) -> bool:
    """True when some odd element lies in [3, 2^32), i.e. O5 would look it up."""
    n = np.asarray(n, dtype=np.uint64)
    return bool(np.any((n < np.uint64(TABLE_BOUND)) & (n > np.uint64(2)) & ((n & np.uint64(1)) == 1)))


def isprime_array(n: np.ndarray, nthreads: int | None = None, use_table: bool | None = None):
    """O5 over a flat uint64 array; returns (uint8 array, threads used).

    ``use_table=None`` builds the 2^32 table only if some element needs it;
    without the table, elements below 2^32 go through trial division (O1).
    """
    n = np.ascontiguousarray(n, dtype=np.uint64)
    out = np.empty(n.shape, dtype=np.uint8)
    if use_table is None:
        use_table = needs_table(n)
    t = table() if use_table else None
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    used = _load().oracle_isprime_array(n.ctypes.data, out.ctypes.data, n.size,
                                        None if t is None else t.ctypes.data, nthreads)
    return out, used


def trial_array(n: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    """O1 alone over an array (threaded)."""
    n = np.ascontiguousarray(n, dtype=np.uint64)
    out = np.empty(n.shape, dtype=np.uint8)
    _load().oracle_trial_array(n.ctypes.data, out.ctypes.data, n.size, nthreads or os.cpu_count() or 1)
    return out


def mr7_array(n: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    """O4 alone over an array: mr7 for odd n >= 3, 0 otherwise (threaded)."""
    n = np.ascontiguousarray(n, dtype=np.uint64)
    out = np.empty(n.shape, dtype=np.uint8)
    _load().oracle_mr7_array(n.ctypes.data, out.ctypes.data, n.size, nthreads or os.cpu_count() or 1)
    return out


def find_factor(n: int) -> int:
    return _load().oracle_find_factor(n)


def pratt_certify(n: int) -> int:
    """1 certified prime, 0 certified composite, -1 undecided."""
    return _load().oracle_pratt_certify(n)


def numdiv(N: int) -> int:
    return _load().oracle_numdiv(N)


def wheel_cycle() -> list:
    """The 48 differences of the 2/3/5/7 wheel (Eq. 5)."""
    buf = (ctypes.c_uint8 * 48)()
    k = _load().oracle_wheel_cycle(buf)
    return list(buf)[:k]


def wheel_is_prime(n: int) -> int:
    return _load().oracle_wheel_is_prime(n)


def wheel_array(n: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    """O8 alone over an array (threaded)."""
    n = np.ascontiguousarray(n, dtype=np.uint64)
    out = np.empty(n.shape, dtype=np.uint8)
    _load().oracle_wheel_array(n.ctypes.data, out.ctypes.data, n.size, nthreads or os.cpu_count() or 1)
    return out
