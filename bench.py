"""Benchmark: uint64 primality tests/sec on one MI355X, bit-exact.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one isprime_u64 call over the whole workload (dispatch, table
lookup, trial filter + compaction, binning, Miller-Rabin base 2, Miller-Rabin
remaining bases, write-back), with the input already resident in HBM.  The
headline workload is the mixed-magnitude array: 2^26 uint64 values, 5%
Chernick numbers, 1% the values 2047, 3215031751 and 2^61 - 1, the rest
octave-uniform (splitmix64 seed 0x2108047900000003), which runs the lookup,
the filter, the compaction and both Miller-Rabin phases together.

Prints ONE JSON line: throughput, the roofline of the dominant kernel (its
duration measured here with HIP events on the stream it runs on), the
oracle timed on the host's cores on a bounded sample of the same input, the
parity of the whole workload against the oracle, the per-kernel times, then
the other workloads (64-bit Miller-Rabin array, small array, the lookup and
sieve paths, batched and served forms, the paper's array workloads,
intervals, the wheel comparison) and last a compact summary of the figures.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "uint64 primality tests/sec (bit-exact) + p50/p99 latency at fixed QPS vs plain"
HBM_PEAK_GBS = 8000.0
# Integer VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, in
# full-rate VALU lane-instructions per second (on gfx950 the 32-bit
# multiplies v_mad_u64_u32, v_mul_lo_u32 and v_mul_hi_u32 issue at full rate).
VALU_PEAK_GOPS = 256 * 4 * 16 * 2.4
# VALU instructions of the shortest gfx950 sequence known here for one 64-bit
# Montgomery product on 32-bit halves.  a*b: v_mul_lo_u32 and v_mul_hi_u32
# for a0*b0, three v_mad_u64_u32 (a1*b0, a0*b1 with its carry-out, a1*b1),
# one v_mov and one v_cndmask to form the carry pair: 7.  m = lo * n^-1: one
# v_mad_u64_u32, two v_mul_lo_u32, one v_add3_u32: 4.  floor(m*n / 2^64): one
# v_mul_hi_u32, three v_mad_u64_u32, one v_mov, one v_cndmask: 6.  The
# correction: subtract with borrow (2), two selects and one 64-bit add: 5.
# Total 22.  For n < 2^62 the lazy form (operands and result below 2n) drops
# the correction for (hi + n) - h: 20.  One modular doubling: shift, compare,
# two selects, add: 5; for n < 2^62, where x may stay below 2n, a shift: 1.
OPS_PER_MONTMUL = 22
OPS_PER_MONTMUL_LAZY = 20
OPS_PER_DOUBLING = 5
OPS_PER_DOUBLING_SHIFT = 1
LAZY_BELOW = 1 << 62
WINDOW_BITS = 3  # the remaining bases' fixed window
MR_BASES_AFTER_2 = 6
FILTER_STAGES_TO = 64  # the two filter stages together: the first 64 odd primes


# The sources of the array path's kernels (classify, both Miller-Rabin phases,
# the Lucas alternative) and their argument structs: a counter summary is
# valid while these are unchanged.
ARRAY_PATH_SOURCES = ("classify.hip", "compact.h", "mr.hip", "mont.h", "internal.h")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in ARRAY_PATH_SOURCES:
        with open(os.path.join(ROOT, "paper_2108_04791_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel: str, summary: str = "pmc_c3_mixed.md"):
    """HBM bytes per launch of `kernel` from a committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes scaled by the copy calibration), or
    None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and (line.startswith("source_sha256_16") or line.startswith("traffic_")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256_16") != kernel_source_hash():
        return None
    v = vals.get("traffic_bytes_per_launch." + kernel)
    return int(v) if v else None


def small_odd_primes(count: int) -> list:
    out, p = [], 3
    while len(out) < count:
        if all(p % q for q in out if q * q <= p):
            out.append(p)
        p += 2
    return out


def bit_length(a: np.ndarray) -> np.ndarray:
    """Exact bit length of each uint64 (0 for 0)."""
    x = a.copy()
    L = np.zeros(a.size, dtype=np.int64)
    for sh in (32, 16, 8, 4, 2, 1):
        m = x >= (np.uint64(1) << np.uint64(sh))
        L[m] += sh
        x[m] >>= np.uint64(sh)
    return L + (x > 0)


def popcount(x: np.ndarray) -> np.ndarray:
    return np.bitwise_count(np.asarray(x, dtype=np.uint64)).astype(np.int64)


BASES_AFTER_2 = (325, 9375, 28178, 450775, 9780504, 1795265022)


def _strong_round(n: int, a: int) -> bool:
    """One round of the strong probable-prime test (odd n > a)."""
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    x = pow(a, d, n)
    if x in (1, n - 1):
        return True
    for _ in range(s - 1):
        x = x * x % n
        if x == n - 1:
            return True
    return False


def planted_pseudoprime_bases(a: np.ndarray, planted: np.ndarray) -> np.ndarray:
    """Per element: how many of the six bases after 2 the textbook test runs
    on a composite that passes base 2 (up to and including the first base it
    fails), for the composites the workloads plant on purpose (`planted`:
    the Chernick numbers); 0 for every other element.  Strong pseudoprimes to
    base 2 among random 64-bit values are too rare to count (about 3e7 below
    2^64)."""
    out = np.zeros(a.size, dtype=np.int64)
    cand = np.unique(planted[(planted >= np.uint64(1 << 32)) & ((planted & np.uint64(1)) == 1)])
    runs = {}
    for v in cand.tolist():
        if not _strong_round(v, 2):
            continue
        k = 0
        for b in BASES_AFTER_2:
            k += 1
            if not _strong_round(v, b):
                break
        else:
            continue  # passes all seven: it would be counted as a prime
        runs[v] = k
    if not runs:
        return out
    keys = np.array(sorted(runs), dtype=np.uint64)
    cnt = np.array([runs[int(k)] for k in keys], dtype=np.int64)
    pos = np.minimum(np.searchsorted(keys, a), keys.size - 1)
    hit = keys[pos] == a
    out[hit] = cnt[pos[hit]]
    return out


def window_products(d: np.ndarray) -> np.ndarray:
    """Montgomery products of a^d with fixed windows of WINDOW_BITS bits for
    a base a below 2^32: the base's Montgomery form (1), the table a^2 ..
    a^(2^W - 1) (2^W - 2), then for each window after the first W squarings
    and one multiplication."""
    nwin = (bit_length(d) + WINDOW_BITS - 1) // WINDOW_BITS
    return 1 + (2 ** WINDOW_BITS - 2) + (WINDOW_BITS + 1) * (nwin - 1)


def mr_work(a: np.ndarray, prime: np.ndarray, filter_primes: int, planted=None):
    """Algorithmic work (VALU instructions) of the two Miller-Rabin launches,
    counted per element for the method the kernels implement, at the cost of
    the product form that element's magnitude allows (lazy below 2^62).

    The trial filter is the first `filter_primes` odd primes per element and,
    when that is on, the rest of the first 64 on its survivors (the second
    stage), so a survivor here has no factor among the first 64 odd primes.
    Base 2 (every filter survivor): L - 2 Montgomery squarings for bit length
    L and popcount(n - 1) - 1 modular doublings (left-to-right binary
    exponentiation).  Remaining bases: per base run, the products of a^d
    with 3-bit fixed windows (window_products), d = (n - 1) / 2^s; every
    prime >= 2^32 runs all six, a composite that passes base 2 runs them up
    to its first failing one (only the planted Chernick numbers are counted,
    `planted`).  Not credited: the -1 chain's squarings, the squarings and
    products of a wavefront's lanes beyond their own bit length, per-lane
    setup (n^-1, R mod n, R^2 mod n) and the bases run beyond a failing one.
    So the count is below what the kernels execute, and achieved / peak is
    at most their issue fraction.
    """
    big = (a >= np.uint64(1 << 32)) & ((a & np.uint64(1)) == 1)
    idx = np.nonzero(big)[0]
    vals = a[idx]
    nf = 0 if filter_primes <= 0 else max(filter_primes, FILTER_STAGES_TO)
    for p in small_odd_primes(nf):  # shrinking: each prime drops its multiples
        k = (vals % np.uint64(p)) != 0
        idx, vals = idx[k], vals[k]
    lazy = vals < np.uint64(LAZY_BELOW)
    L = bit_length(vals)
    sq = L - 2
    dbl = popcount(vals - np.uint64(1)) - 1
    sq2, dbl2 = int(sq.sum()), int(dbl.sum())
    base2_ops = int((sq * np.where(lazy, OPS_PER_MONTMUL_LAZY, OPS_PER_MONTMUL)).sum() +
                    (dbl * np.where(lazy, OPS_PER_DOUBLING_SHIFT, OPS_PER_DOUBLING)).sum())
    nb = np.where(prime.astype(bool) & big, MR_BASES_AFTER_2, 0).astype(np.int64)
    if planted is not None:
        nb = np.maximum(nb, planted_pseudoprime_bases(a, planted))
    sel = np.nonzero(nb)[0]
    v = a[sel]
    d = v - np.uint64(1)
    while True:
        ev = (d & np.uint64(1)) == 0
        if not ev.any():
            break
        d[ev] >>= np.uint64(1)
    prods = nb[sel] * window_products(d)
    mm_rest = int(prods.sum())
    rest_ops = int((prods * np.where(v < np.uint64(LAZY_BELOW), OPS_PER_MONTMUL_LAZY,
                                     OPS_PER_MONTMUL)).sum())
    work = {"mr_base2": {"montmul": sq2, "doublings": dbl2, "ops": base2_ops},
            "mr_rest": {"montmul": mm_rest, "doublings": 0, "ops": rest_ops,
                        "passers_counted": int(sel.size)}}
    return work, int(idx.size), int((prime.astype(bool) & big).sum())


# The paper's MATLAB seconds for its array workloads (Intel Core i7-9750H,
# MATLAB R2020b): Table IncrementingSequence (section 6.1.3) for 1:N and
# Table ArrayPerformance (section 8.2) for the rest.  Context from another
# machine and another program, not a target.
PAPER_MATLAB_S = {
    "inc_1e4": 0.000829, "inc_1e5": 0.005502, "inc_1e6": 0.05697, "inc_1e7": 0.6294,
    "inc_1e8": 6.728, "unix_2021": 12.26, "int16_primes_200": 5.0952e-05,
    "matrix_1000x1000_u32": 3.927, "normal_primes_1m_mean_2_16": 0.1623,
    "normal_odd_100k_mean_2_32": 2.689, "normal_1000_mean_2_53": 5.07,
    "largest52_prime_x1000": 58.270, "composites_100_factors_gt_2e7": 0.4852,
    "largest64_primes_100": 0.1442, "largest64_odd_5000": 76.201,
}


def _time_ms(torch, stream, fn, reps: int) -> float:
    """Median of `reps` single calls, each bracketed by HIP events."""
    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def bench_paper_suite(isp, W, torch, reps: int = 7) -> dict:
    """The paper's array workloads, rebuilt from their descriptions: the array
    call on each (inputs resident), and for the contiguous intervals also the
    interval call.  Values stay on the device; nothing is copied back inside
    a timed call."""
    stream = torch.cuda.current_stream()
    res = {}
    arrays = W.paper_arrays()
    for name, (lo, length) in W.PAPER_INTERVALS.items():
        dev = torch.arange(lo, lo + length, dtype=torch.int64, device="cuda")
        out = torch.empty(length, dtype=torch.uint8, device="cuda")
        rout = torch.empty(length, dtype=torch.bool, device="cuda")
        ms = _time_ms(torch, stream, lambda: isp.isprime_into(dev, out, stream), reps)
        rms = _time_ms(torch, stream, lambda: isp.isprime_range(lo, length, rout, stream), reps)
        same = bool(torch.equal(out.bool(), rout))
        res[name] = {"elements": length, "ms": ms, "tests_per_s": length / (ms * 1e-3),
                     "interval_ms": rms, "interval_tests_per_s": length / (rms * 1e-3),
                     "interval_equals_array": same, "primes": int(out.sum().item())}
        del dev, out, rout
    for name, a in arrays.items():
        dev = torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()
        out = torch.empty(a.shape, dtype=torch.uint8, device="cuda")
        ms = _time_ms(torch, stream, lambda: isp.isprime_into(dev, out, stream), reps)
        res[name] = {"elements": int(a.size), "ms": ms, "tests_per_s": a.size / (ms * 1e-3),
                     "primes": int(out.sum().item()), "input_sha256_16": W.digest(a)}
    for name, r in res.items():
        r["paper_matlab_s"] = PAPER_MATLAB_S[name]
        best = min(r["ms"], r.get("interval_ms", r["ms"])) * 1e-3
        r["x_vs_paper_matlab"] = PAPER_MATLAB_S[name] / best
    return res


INTERVAL_CASES = (("2^34+[0,2^28)", 1 << 34, 1 << 28), ("2^44+[0,2^28)", 1 << 44, 1 << 28),
                  ("2^50+[0,2^28)", 1 << 50, 1 << 28), ("2^63+[0,2^28)", 1 << 63, 1 << 28),
                  ("2^64-2^28+[0,2^28)", (1 << 64) - (1 << 28), 1 << 28),
                  ("2^63+[0,2^24)", 1 << 63, 1 << 24))


def bench_intervals(isp, torch, reps: int = 5, array_call: bool = True, only=None) -> dict:
    """The interval call above 2^32, where each workgroup sieves a segment of
    2^20 or 2^19 numbers in LDS, in each of its modes: segments decided by the primes
    up to their square root (2^34, 2^44), the bucket sieve of the primes
    above 2^21 (2^50, 2^63, 2^64 - 2^28), and, for an interval short next
    to the number of primes up to its square root, the primes below 2^22
    followed by Miller-Rabin on the survivors (2^24 numbers at 2^63); each
    against the array call on the same values."""
    stream = torch.cuda.current_stream()
    res = {}
    for name, lo, length in INTERVAL_CASES:
        if only is not None and name != only:
            continue
        rout = torch.empty(length, dtype=torch.bool, device="cuda")
        rms = _time_ms(torch, stream, lambda: isp.isprime_range(lo, length, rout, stream), reps)
        if not array_call:
            res[name] = {"elements": length, "interval_ms": rms,
                         "interval_tests_per_s": length / (rms * 1e-3),
                         "primes": int(rout.sum().item())}
            del rout
            continue
        # the same values as an array (int64 view of the uint64 values)
        base = lo if lo < (1 << 63) else lo - (1 << 64)
        dev = torch.arange(base, base + length, dtype=torch.int64, device="cuda")
        out = torch.empty(length, dtype=torch.uint8, device="cuda")
        ms = _time_ms(torch, stream, lambda: isp.isprime_into(dev, out, stream), reps)
        res[name] = {"elements": length, "interval_ms": rms,
                     "interval_tests_per_s": length / (rms * 1e-3), "array_ms": ms,
                     "array_tests_per_s": length / (ms * 1e-3),
                     "same_bytes": bool(torch.equal(out.bool(), rout)),
                     "primes": int(rout.sum().item())}
        del dev, out, rout
    return res


WHEEL_OCTAVES = (33, 34, 36, 38, 40)


def bench_wheel(isp, W, torch, reps: int = 3, n: int = 1 << 20) -> dict:
    """The paper's medium-integer method (trial division on the 2/3/5/7 wheel
    up to the square root) against Miller-Rabin on the same filter
    survivors: 2^20 odd values uniform in each octave [2^(b-1), 2^b), one
    plain call with the wheel stage on (wheel_log2 = 40) and one without."""
    stream = torch.cuda.current_stream()
    res = {}
    for bits in WHEEL_OCTAVES:
        a = W.odd_band(n, bits)
        dev = torch.from_numpy(a.view(np.int64)).cuda()
        out_mr = torch.empty(n, dtype=torch.uint8, device="cuda")
        out_wh = torch.empty(n, dtype=torch.uint8, device="cuda")
        mr_ms = _time_ms(torch, stream, lambda: isp.isprime_into(dev, out_mr, stream), reps)
        prev = isp.set_config(wheel_log2=40)
        try:
            wh_ms = _time_ms(torch, stream, lambda: isp.isprime_into(dev, out_wh, stream), reps)
        finally:
            isp.set_config(**prev)
        res["2^%d" % bits] = {"elements": n, "miller_rabin_ms": mr_ms, "wheel_ms": wh_ms,
                              "wheel_over_mr": wh_ms / mr_ms,
                              "same_bytes": bool(torch.equal(out_mr, out_wh)),
                              "primes": int(out_mr.sum().item())}
        del dev, out_mr, out_wh
    return res


def bench_batched(isp, W, torch, reps: int = 5) -> dict:
    """4096 arrays of log-uniform length in [1, 2^16], magnitude class per
    array: one isprime_u64_batched call (graph replay; its host arrays of
    pointers prepared once, as a C caller holds them) vs one isprime_u64
    call per array on the same stream."""
    arrays = W.c4_batched()
    total = sum(a.size for a, _ in arrays)
    dev = [torch.from_numpy(a.view(np.int64)).cuda() for a, _ in arrays]
    outs = [torch.empty(a.size, dtype=torch.uint8, device="cuda") for a, _ in arrays]
    stream = torch.cuda.current_stream()

    prepared = isp.Batch(dev, outs)  # the host pointer arrays, built once

    def batched():
        prepared.run(stream)

    def plain():
        for d, o in zip(dev, outs):
            isp.isprime_into(d, o, stream)

    res = {}
    for name, fn in (("batched", batched), ("plain_per_array", plain)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = {"ms": ms, "tests_per_s": total / (ms * 1e-3)}
    res["arrays"] = len(arrays)
    res["elements"] = total
    res["speedup"] = res["plain_per_array"]["ms"] / res["batched"]["ms"]
    return res


SERVED_PASSES = 3


def _lat_stats(lat_ms: np.ndarray, elems: int, span_s: float) -> dict:
    return {"p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
            "mean_ms": float(lat_ms.mean()), "tests_per_s": elems / span_s}


def _passes(run, arrive, warm, elems, passes=SERVED_PASSES) -> dict:
    """`passes` runs over the same arrival times: the pass with the median
    p99, every pass's p99, and the p50/p99 of all passes' latencies pooled."""
    lats, res = [], []
    for _ in range(passes):
        lat, span = run(arrive)
        m = lat[warm:] * 1e3
        lats.append(m)
        res.append(_lat_stats(m, elems, span))
    order = sorted(range(passes), key=lambda i: res[i]["p99_ms"])
    out = dict(res[order[len(order) // 2]])
    out["p99_ms_passes"] = [res[i]["p99_ms"] for i in range(passes)]
    pooled = np.concatenate(lats)
    out["pooled_p50_ms"] = float(np.percentile(pooled, 50))
    out["pooled_p99_ms"] = float(np.percentile(pooled, 99))
    out["worst_pass_p99_ms"] = max(r["p99_ms"] for r in res)
    out["qps"] = float(len(arrive) / (arrive[-1] - arrive[0])) if len(arrive) > 1 else 0.0
    return out


def bench_served(isp, W, torch, num: int = 2100, warm: int = 100, max_inflight: int = 8,
                 max_batch_elems: int = 1 << 18, loads=(0.25, 0.5, 0.7, 0.9)) -> dict:
    """Poisson request stream (lengths log-uniform in [1, 2^20], magnitude
    class per request) served by the continuous-batching server (its default
    8 slots of 2^18 elements) at several fractions of its measured capacity (the
    headline at 0.7), and the same stream served FIFO by serial plain calls
    (copy in, isprime_u64, copy out, synchronise) at 0.7 of their own
    capacity (a load they sustain) and at the server's 0.7 rate (which they
    do not).  The server also runs at the serial calls' sustainable rate, so
    the two are compared at one QPS both sustain.  Latency = arrival to
    result in the caller's host array.  Every served request's bytes are
    compared with a plain isprime_u64 call on the same values afterwards."""
    import threading
    reqs = W.c5_requests(num, qps=1.0)  # arrival times for rate 1; rescaled below
    arrays = [r for _, r, _ in reqs]
    unit_t = np.array([t for t, _, _ in reqs])
    elems = sum(a.size for a in arrays[warm:])
    stream = torch.cuda.current_stream()

    # plain results of every request (device call), the reference for the
    # served bytes
    plain_out = []
    for a in arrays:
        d = torch.from_numpy(a.view(np.int64)).cuda()
        o = torch.empty(a.size, dtype=torch.uint8, device="cuda")
        isp.isprime_into(d, o, stream)
        plain_out.append(o)
    torch.cuda.synchronize()
    plain_out = [o.cpu().numpy() for o in plain_out]

    # Python's cyclic collector is paused and its thread switch interval
    # shortened while requests are timed: a collection pass over the many
    # request arrays, or a 5 ms wait for the interpreter lock, would delay
    # the submitting and waiting threads, not the server
    switch = sys.getswitchinterval()
    mismatched = set()
    srv = isp.Server(max_inflight=max_inflight, max_batch_elems=max_batch_elems)
    footprint = srv.footprint()
    outs = [np.full(a.size, 2, np.uint8) for a in arrays]

    def check():
        for i, (o, p) in enumerate(zip(outs, plain_out)):
            if not np.array_equal(o, p):
                mismatched.add(i)
            o.fill(2)

    try:
        # capacity: everything submitted at once (after one untimed pass, so
        # that the output pages and the server's buffers are already mapped)
        for rep in range(2):
            t0 = time.perf_counter()
            tk = [srv.submit(a, o) for a, o in zip(arrays, outs)]
            for t in tk:
                srv.wait(t)
            cap_s = time.perf_counter() - t0
            check()
        capacity = num / cap_s

        def run_served(arrive):
            done_t = np.zeros(num)
            tickets = [None] * num
            ready = threading.Semaphore(0)
            base = time.perf_counter() + 0.01

            def waiter():
                for i in range(num):
                    ready.acquire()
                    srv.wait(tickets[i])
                    done_t[i] = time.perf_counter() - base

            th = threading.Thread(target=waiter)
            th.start()
            for i in range(num):
                d = base + arrive[i] - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets[i] = srv.submit(arrays[i], outs[i])
                ready.release()
            th.join()
            check()
            return done_t - arrive, done_t[-1] - arrive[warm]

        def run_plain(arrive):
            lat = np.zeros(num)
            base = time.perf_counter() + 0.01
            t_free = 0.0
            for i, a in enumerate(arrays):
                now = time.perf_counter() - base
                if now < arrive[i]:
                    time.sleep(arrive[i] - now)
                d = torch.from_numpy(a.view(np.int64)).cuda()
                o = torch.empty(a.size, dtype=torch.uint8, device="cuda")
                isp.isprime_into(d, o, stream)
                o.cpu()
                t_free = time.perf_counter() - base
                lat[i] = t_free - arrive[i]
            return lat, t_free - arrive[warm]

        by_load = {}
        gc.disable()
        sys.setswitchinterval(1e-4)
        try:
            run_served(unit_t / (0.7 * capacity))  # untimed: threads and pages warm
            # a pass lasts about 2000 / (load x capacity) s (~60 ms at 0.7), so
            # one stall of the host of a few ms decides a pass's p99 alone:
            # each load runs SERVED_PASSES passes over the same stream
            for load in loads:
                by_load[str(load)] = _passes(run_served, unit_t / (load * capacity), warm, elems)
            # serial plain calls: their capacity (back to back), then at 0.7 of
            # it and at the server's 0.7 rate; the server at the former too
            lat, _ = run_plain(np.zeros(num))  # every request waiting at time 0
            plain_capacity = num / lat[-1]
            plain_own = _passes(run_plain, unit_t / (0.7 * plain_capacity), warm, elems)
            plain_at_server = _passes(run_plain, unit_t / (0.7 * capacity), warm, elems, passes=1)
            served_at_plain = _passes(run_served, unit_t / (0.7 * plain_capacity), warm, elems)
        finally:
            sys.setswitchinterval(switch)
            gc.enable()
    finally:
        srv.close()

    head = by_load.get("0.7")
    return {"requests": num - warm, "warmup_requests": warm, "elements": int(elems),
            "server": {"max_inflight": max_inflight, "max_batch_elems": max_batch_elems,
                       "footprint_device_bytes": footprint[0],
                       "footprint_pinned_bytes": footprint[1]},
            "capacity_req_per_s": capacity, "qps": 0.7 * capacity,
            "served": head, "served_by_load": by_load,
            "serial_plain_capacity_req_per_s": plain_capacity,
            "serial_plain_at_own_0.7": plain_own,
            "served_at_serial_plain_0.7": served_at_plain,
            "serial_plain_at_server_0.7": plain_at_server,
            "bytes_checked_requests": num * (3 + SERVED_PASSES * (len(loads) + 1)),
            "served_bytes_equal_plain": not mismatched,
            "mismatched_requests": sorted(mismatched)[:20]}


def table_crossings() -> int:
    """Odd multiples the sieve kernel crosses off below 2^32: for each odd
    prime 37 <= p < 2^16 (3..31 come from a periodic pre-sieve mask), every
    odd multiple from p^2 up."""
    lim = 1 << 16
    s = np.ones(lim, dtype=bool)
    s[:2] = False
    for q in range(2, 256):
        if s[q]:
            s[q * q::q] = False
    p = np.nonzero(s)[0].astype(np.int64)
    p = p[p >= 37]
    return int((((1 << 32) - 1 - p * p) // (2 * p) + 1).sum())


WHEEL_TABLE_BYTES = 30678339 * 4  # 48 bits per 210 numbers below 2^32


def bench_sieve(isp, reps: int = 5) -> dict:
    """The table build: base primes + segment sieve kernels, then the wheel
    table derived from the sieve table, each timed by HIP events."""
    runs = [isp.table_rebuild_ms() for _ in range(reps)]
    times = sorted(r[0] for r in runs)
    wtimes = sorted(r[1] for r in runs)
    ms, wms = times[len(times) // 2], wtimes[len(wtimes) // 2]
    table_bytes = 1 << 28
    cr = table_crossings()
    return {"kernel_ms": ms, "kernel_ms_all": times, "table_bytes": table_bytes,
            "write_GBps": table_bytes / (ms * 1e-3) / 1e9,
            "write_frac_of_hbm": table_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "crossings": cr, "crossings_per_s": cr / (ms * 1e-3),
            "wheel_table_ms": wms, "wheel_table_bytes": WHEEL_TABLE_BYTES,
            "wheel_table_GBps": (table_bytes + WHEEL_TABLE_BYTES) / (wms * 1e-3) / 1e9}


def classify_bytes(a: np.ndarray) -> int:
    """Algorithmic HBM bytes of classify_kernel: 8 B read and 1 B written
    per element, plus one 4-byte table word per element that needs a table
    read: odd, in [3, 2^32) and coprime to 3, 5 and 7 (the others are
    decided by their residue mod 210)."""
    look = (a > np.uint64(2)) & (a < np.uint64(1 << 32)) & ((a & np.uint64(1)) == 1)
    for p in (3, 5, 7):
        look &= (a % np.uint64(p)) != 0
    return 9 * a.size + 4 * int(look.sum())


def measure_plain(isp, torch, a: np.ndarray, steps: int, warmup: int, stages: bool = True) -> dict:
    """K timed steps of one plain call over a resident array (HIP events on
    the call's stream), then K profiled steps (events around each kernel)."""
    dev = torch.from_numpy(a.view(np.int64)).cuda()
    out = torch.empty(a.size, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        isp.isprime_into(dev, out, stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        isp.isprime_into(dev, out, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    res = {"len": int(a.size), "ms_per_step": ms, "tests_per_s": a.size / (ms * 1e-3),
           "got": out.cpu().numpy()}
    res["survivors"], res["base2_passers"] = isp.last_counts(stream)
    if stages:
        isp.profile(True)
        for _ in range(steps):
            isp.isprime_into(dev, out, stream)
        prof = isp.profile_read()
        isp.profile(False)
        calls = max(1, prof["calls"])
        res["stage_ms"] = {k: prof[k] / calls for k in isp.STAGES}
    del dev, out
    return res


def roofline_of(a: np.ndarray, got: np.ndarray, stage_ms: dict, filter_primes: int,
                planted, summary: str):
    """The roofline of the slowest kernel of one call, and the VALU fraction
    of both Miller-Rabin kernels."""
    work, n_surv, n_prime = mr_work(a, got, filter_primes, planted)
    dom = max(("classify", "filter2", "mr_base2", "mr_rest"), key=lambda k: stage_ms[k])
    other = {}
    for k in ("mr_base2", "mr_rest"):
        ach = work[k]["ops"] / (stage_ms[k] * 1e-3) / 1e9
        other[k] = {"achieved": ach, "frac": ach / VALU_PEAK_GOPS}
    if dom in ("classify", "filter2"):
        b = classify_bytes(a)
        ach = b / (stage_ms["classify"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": counter_traffic("classify", summary),
                "kernel": "classify", "bytes_per_launch": b, "ms_per_launch": stage_ms["classify"]}
    else:
        ach = work[dom]["ops"] / (stage_ms[dom] * 1e-3) / 1e9
        roof = {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_GOPS,
                "unit": "Gop/s", "frac": ach / VALU_PEAK_GOPS,
                "traffic": counter_traffic(dom, summary),
                "kernel": dom, "op": "VALU lane-instruction",
                "ms_per_launch": stage_ms[dom],
                "montmul_per_launch": work[dom]["montmul"],
                "doublings_per_launch": work[dom]["doublings"],
                "ops_per_montmul": {"n_below_2^62": OPS_PER_MONTMUL_LAZY,
                                    "n_from_2^62": OPS_PER_MONTMUL},
                "ops_per_doubling": {"n_below_2^62": OPS_PER_DOUBLING_SHIFT,
                                     "n_from_2^62": OPS_PER_DOUBLING},
                "window_bits": WINDOW_BITS}
    return roof, other, work, n_surv, n_prime


def host_cpus() -> dict:
    """The host's CPU model, its logical CPU count, this process's affinity
    set and its cgroup CPU quota (when one is set)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    quota = None
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()
        if q != "max":
            quota = int(q) / int(per)
    except (OSError, ValueError):
        pass
    aff = len(os.sched_getaffinity(0))
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": aff,
            "cgroup_cpu_quota": quota}


# The share of host CPUs a one-GPU job gets on the measuring machine; the
# oracle's thread count never exceeds it (more threads than the share only
# time-slice against each other).
JOB_CPU_SHARE = 16


def cpu_baseline(W, a: np.ndarray, got: np.ndarray, one_len: int = 1 << 21,
                 all_len: int = 1 << 24, runs: int = 3):
    """The oracle (plain C: table below 2^32, Miller-Rabin with 128-bit
    products above) on the host: its 2^32 table build timed alone, then a
    bounded prefix of the same input on 1 thread and on the job's CPUs,
    median of `runs` each; then the whole workload once on the job's CPUs
    for parity (not timed)."""
    import oracle
    info = host_cpus()
    threads = info["affinity_cpus"]
    if info["cgroup_cpu_quota"]:
        threads = min(threads, max(1, int(info["cgroup_cpu_quota"])))
    threads = min(threads, JOB_CPU_SHARE)
    t0 = time.perf_counter()
    oracle.table()
    table_s = time.perf_counter() - t0

    def median_rate(sample, nthreads):
        times, used = [], 0
        for _ in range(runs):
            t1 = time.perf_counter()
            _, used = oracle.isprime_array(sample, nthreads=nthreads, use_table=True)
            times.append(time.perf_counter() - t1)
        times.sort()
        return sample.size / times[len(times) // 2], used, times

    one_rate, _, one_t = median_rate(a[:one_len], 1)
    all_rate, used, all_t = median_rate(a[:all_len], threads)
    exp, _ = oracle.isprime_array(a, nthreads=threads, use_table=True)
    bit_exact = bool(np.array_equal(exp, got))
    cpu = {"value": all_rate, "unit": "tests/s", "cores": used, "kind": "oracle",
           "sample": "the first %d elements of the workload on %d threads (median of %d runs: "
                     "%s s); 1 thread: the first %d elements, median of %d (%s s); the oracle's "
                     "2^32 table build (%.2f s) timed apart" % (
                         all_len, used, runs, "/".join("%.2f" % t for t in all_t), one_len,
                         runs, "/".join("%.2f" % t for t in one_t), table_s),
           "one_thread_tests_per_s": one_rate, "all_threads_tests_per_s": all_rate,
           "threads": used, "table_build_s": table_s, "runs": runs}
    cpu.update(info)
    return cpu, bit_exact


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip everything after the headline and 64-bit workloads")
    ap.add_argument("--workload", default=None, choices=("c3_mixed", "c2_mr64", "lookup32"),
                    help="only time this workload's plain calls (--warmup, then --steps timed "
                         "and --steps with per-kernel events; for profiling)")
    ap.add_argument("--intervals-only", action="store_true",
                    help="only time the interval call on its cases (for profiling its kernels)")
    ap.add_argument("--interval-case", choices=[c[0] for c in INTERVAL_CASES], default=None,
                    help="with --intervals-only: only this case")
    ap.add_argument("--wheel-only", action="store_true",
                    help="only time the wheel stage against Miller-Rabin per octave")
    ap.add_argument("--sieve-only", action="store_true",
                    help="only rebuild the table --steps times (for profiling the sieve kernel)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (the reference "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path needs no exchange between devices, "
              "so --gpus must be 1 (got %d)" % args.gpus, file=sys.stderr)
        return 2

    import torch
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.int64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": src.numel() * 8, "copies": 5}))
        return 0
    import paper_2108_04791_amd as isp
    import workloads as W

    torch.cuda.set_device(0)
    isp.init(0)
    torch.cuda.synchronize()
    if args.sieve_only:
        print(json.dumps({"sieve": bench_sieve(isp, reps=args.steps)}))
        return 0
    if args.intervals_only:
        print(json.dumps({"intervals": bench_intervals(isp, torch, reps=args.steps,
                                                       array_call=False, only=args.interval_case)}))
        return 0
    if args.wheel_only:
        print(json.dumps({"wheel_vs_miller_rabin": bench_wheel(isp, W, torch, reps=args.steps)}))
        return 0

    from paper_2108_04791_amd import tune
    defaults = isp.get_config()

    def with_tuning(key, length, fn):
        isp.set_config(**defaults)
        tuned = tune.apply(key, length) is not None
        res = fn()
        res["tuning"] = isp.get_config()
        res["tuning_source"] = "autotuner database" if tuned else "library defaults"
        isp.set_config(**defaults)
        return res

    gens = {"c3_mixed": W.c3_mixed, "c2_mr64": W.c2_mr64, "lookup32": W.lookup32}
    if args.workload:
        a = gens[args.workload]()
        r = with_tuning(args.workload, a.size,
                        lambda: measure_plain(isp, torch, a, args.steps, args.warmup))
        r.pop("got")
        print(json.dumps({"workload": args.workload, **r}))
        return 0

    # ---- the headline: the mixed-magnitude array
    a = W.c3_mixed()
    n = a.size
    head = with_tuning("c3_mixed", n, lambda: measure_plain(isp, torch, a, args.steps, args.warmup))
    got = head.pop("got")
    cfg = head["tuning"]
    stage_ms = head["stage_ms"]
    roofline, alu_other, work, n_surv, n_prime = roofline_of(
        a, got, stage_ms, max(0, cfg["filter_primes"]), W.chernick_values(), "pmc_c3_mixed.md")
    lookup_bytes = classify_bytes(a)
    classify_gbps = lookup_bytes / (stage_ms["classify"] * 1e-3) / 1e9

    # the Baillie-PSW alternative on the same input (base 2, then a strong
    # Lucas test instead of the six remaining bases): same bytes, timed alike
    def bpsw():
        isp.set_config(rest_test=1)
        r = measure_plain(isp, torch, a, args.steps, 1)
        return {"stage_ms": r["stage_ms"], "ms_per_step": r["ms_per_step"],
                "tests_per_s": r["tests_per_s"], "same_bytes": bool(np.array_equal(r["got"], got))}
    alt = {"bpsw": with_tuning("c3_mixed", n, bpsw)}

    # ---- the 64-bit Miller-Rabin array (the Montgomery kernels at full width)
    a2 = W.c2_mr64()
    c2 = with_tuning("c2_mr64", a2.size, lambda: measure_plain(isp, torch, a2, args.steps, args.warmup))
    got2 = c2.pop("got")
    c2_roof, c2_alu, _, _, _ = roofline_of(a2, got2, c2["stage_ms"],
                                           max(0, c2["tuning"]["filter_primes"]), None,
                                           "pmc_c2_mr64.md")
    c2.update({"workload": "c2_mr64: 2^24 uint64 rejection-uniform in [2^49, 2^64), half forced "
                           "odd, splitmix64 seed 0x2108047900000002",
               "input_sha256_16": W.digest(a2), "roofline": c2_roof, "alu_frac_by_kernel": c2_alu,
               "primes": int(got2.sum())})

    forms = {}
    if not args.no_forms:
        c1 = W.c1_uniform20()
        r1 = with_tuning("c1_uniform20", c1.size, lambda: measure_plain(isp, torch, c1, 50, 5))
        r1.pop("got")
        forms["c1_uniform20"] = r1
        lk = W.lookup32()
        rl = with_tuning("lookup32", lk.size, lambda: measure_plain(isp, torch, lk, args.steps, 2))
        rl.pop("got")
        b = classify_bytes(lk)
        rl.update({"workload": "2^26 uint64 uniform in [0, 2^32) (every odd value a table lookup), "
                               "splitmix64 seed 0x2108047900000008",
                   "classify_bytes": b,
                   "classify_GBps": b / (rl["stage_ms"]["classify"] * 1e-3) / 1e9})
        rl["classify_frac_of_hbm"] = rl["classify_GBps"] / HBM_PEAK_GBS
        del lk
        forms["lookup32"] = rl
        forms["sieve"] = bench_sieve(isp)
        forms["batched"] = with_tuning("c4_batched", 25341952, lambda: bench_batched(isp, W, torch))
        forms["served"] = bench_served(isp, W, torch)
        isp.set_config(**defaults)
        forms["paper_workloads"] = bench_paper_suite(isp, W, torch)
        forms["intervals"] = bench_intervals(isp, torch)
        forms["wheel_vs_miller_rabin"] = bench_wheel(isp, W, torch)

    cpu, bit_exact = None, None
    if not args.no_cpu_baseline:
        cpu, bit_exact = cpu_baseline(W, a, got)

    line = {
        "metric": METRIC,
        "value": n / (head["ms_per_step"] * 1e-3),
        "unit": "tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "c3_mixed: 2^26 uint64, 5% Chernick numbers, 1% {2047, 3215031751, "
                               "2^61-1}, the rest octave-uniform, splitmix64 seed 0x2108047900000003",
                   "len": n, "input_sha256_16": W.digest(a),
                   "tuning_source": head["tuning_source"], "tuning": cfg},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "bit_exact_vs_oracle": bit_exact,
        "stage_ms": stage_ms,
        "alu_frac_by_kernel": alu_other,
        "classify_GBps": classify_gbps,
        "survivors": n_surv,
        "base2_passers": head["base2_passers"],
        "primes": int(got.sum()),
        "alternatives": alt,
        "c2_mr64": c2,
    }
    line.update(forms)
    # last: the figures in brief (scalars only)
    summ = {"c3_tests_per_s": line["value"], "c3_ms": head["ms_per_step"],
            "c3_bit_exact": bit_exact, "roofline_kernel": roofline["kernel"],
            "roofline_frac": roofline["frac"]}
    summ.update({"c3_%s_ms" % k: v for k, v in stage_ms.items()})
    summ.update({"c2_tests_per_s": c2["tests_per_s"], "c2_ms": c2["ms_per_step"],
                 "c2_mr_rest_frac": c2_alu["mr_rest"]["frac"],
                 "c2_mr_base2_frac": c2_alu["mr_base2"]["frac"],
                 "c3_mr_rest_frac": alu_other["mr_rest"]["frac"],
                 "c3_mr_base2_frac": alu_other["mr_base2"]["frac"],
                 "c3_classify_GBps": classify_gbps,
                 "bpsw_c3_ms": alt["bpsw"]["ms_per_step"]})
    if forms:
        sv = forms["served"]
        summ.update({"c1_ms": forms["c1_uniform20"]["ms_per_step"],
                     "lookup32_classify_GBps": forms["lookup32"]["classify_GBps"],
                     "lookup32_ms": forms["lookup32"]["ms_per_step"],
                     "sieve_kernel_ms": forms["sieve"]["kernel_ms"],
                     "sieve_write_GBps": forms["sieve"]["write_GBps"],
                     "sieve_crossings_per_s": forms["sieve"]["crossings_per_s"],
                     "batched_ms": forms["batched"]["batched"]["ms"],
                     "batched_speedup": forms["batched"]["speedup"],
                     "served_p50_ms": sv["served"]["p50_ms"], "served_p99_ms": sv["served"]["p99_ms"],
                     "served_pooled_p99_ms": sv["served"]["pooled_p99_ms"],
                     "served_bytes_equal_plain": sv["served_bytes_equal_plain"],
                     "plain_own07_p50_ms": sv["serial_plain_at_own_0.7"]["p50_ms"],
                     "plain_own07_p99_ms": sv["serial_plain_at_own_0.7"]["p99_ms"],
                     "served_at_plain07_p50_ms": sv["served_at_serial_plain_0.7"]["p50_ms"],
                     "served_at_plain07_p99_ms": sv["served_at_serial_plain_0.7"]["p99_ms"]})
    if cpu:
        summ.update({"cpu_1t_tests_per_s": cpu["one_thread_tests_per_s"],
                     "cpu_all_tests_per_s": cpu["all_threads_tests_per_s"],
                     "cpu_threads": cpu["threads"], "cpu_nproc": cpu["nproc"]})
    line["summary"] = summ
    print(json.dumps(line), flush=True)
    ok = bit_exact in (None, True) and (not forms or forms["served"]["served_bytes_equal_plain"])
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
