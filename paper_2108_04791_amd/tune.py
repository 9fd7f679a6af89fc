"""Autotuner for the library's launch parameters.

The parameters (isp_config) never change an output bit, only speed: the
classify block size, elements per thread and grid; the trial-filter size;
the magnitude binning (survivors ordered by bit length, or not); the
Miller-Rabin block size, grid and window width.  The tuner times
configurations on a sample of a workload class by coordinate descent (one
parameter at a time, two sweeps), rejects any configuration whose output
bytes differ from the default configuration's, and records the fastest in a
JSON database keyed by workload class and length bucket:

    python -m paper_2108_04791_amd.tune --workload c2_mr64 --db tuning.json

``apply(db, key, length)`` loads the entry nearest in length for a class.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import torch

from . import Batch, get_config, isprime_into, set_config

SPACE = {
    "classify_ept": [2, 4, 8],
    "classify_block": [256, 512, 1024],
    "classify_blocks_per_cu": [1, 2, 4, 8, 16],
    "filter_primes": [8, 16, 24, 32, 48, 64],
    "sort_survivors": [1, -1],
    "mr_block": [256, 512, 1024],
    "mr_blocks_per_cu": [1, 2, 4, 8],
    "mr_window": [2, 3, 4],
}

DEFAULT_DB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")


def length_bucket(n: int) -> int:
    """log2 bucket of a call length (0 for empty)."""
    return 0 if n <= 0 else int(math.log2(n))


def _timer(fn, reps: int, trials: int = 3) -> float:
    """Per-call time of `reps` calls back to back between two events on the
    stream (as the benchmark times them: the part holds a lower clock under
    sustained issue-bound work than for isolated calls, which ranked some
    configurations differently), median of `trials` such runs."""
    stream = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(trials):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / reps)
    times.sort()
    return times[len(times) // 2]


def tune(arrays, reps: int = 7, sweeps: int = 2, log=print) -> dict:
    """Tune on a list of device tensors (one: plain calls; several: batched).

    Returns {"config": best, "ms": best_ms, "default_ms": (the starting
    configuration's time), "tried": n}.
    """
    batched = len(arrays) > 1
    outs = [torch.empty(a.shape, dtype=torch.uint8, device=a.device) for a in arrays]
    prepared = Batch(arrays, outs) if batched else None  # pointer arrays built once

    def run():
        if batched:
            prepared.run()
        else:
            isprime_into(arrays[0], outs[0])

    start = get_config()
    try:
        run()
        torch.cuda.synchronize()
        reference = [o.clone() for o in outs]
        # bring the part to its sustained clock before the first timing (the
        # first calls after an idle spell run up to 15% slower)
        for _ in range(3 * reps):
            run()
        torch.cuda.synchronize()
        best = dict(start)
        best_ms = _timer(run, reps)
        default_ms = best_ms
        tried = 1
        for _ in range(sweeps):
            for key, values in SPACE.items():
                for v in values:
                    if v == best[key]:
                        continue
                    cand = dict(best)
                    cand[key] = v
                    try:
                        set_config(**cand)
                    except Exception:
                        continue
                    ms = _timer(run, reps)
                    tried += 1
                    same = all(torch.equal(o, r) for o, r in zip(outs, reference))
                    if not same:
                        raise RuntimeError("configuration %s changed output bytes" % cand)
                    if ms < best_ms * 0.99:
                        best, best_ms = cand, ms
                        log("  %s=%s -> %.4f ms" % (key, v, ms))
                set_config(**best)
        return {"config": best, "ms": best_ms, "default_ms": default_ms, "tried": tried}
    finally:
        set_config(**start)


def load(db_path: str = DEFAULT_DB) -> dict:
    if not os.path.exists(db_path):
        return {"version": 1, "entries": {}}
    with open(db_path) as f:
        return json.load(f)


def save(db: dict, db_path: str = DEFAULT_DB) -> None:
    tmp = db_path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, db_path)


def lookup(db: dict, key: str, length: int):
    """Entry of class `key` whose length bucket is nearest `length`."""
    best, dist = None, None
    for name, e in db.get("entries", {}).items():
        k, b = name.rsplit("|", 1)
        if k != key:
            continue
        d = abs(int(b) - length_bucket(length))
        if dist is None or d < dist:
            best, dist = e, d
    return best


def apply(key: str, length: int, db_path: str = DEFAULT_DB) -> dict | None:
    """Set the configuration tuned for (class, length); returns it or None."""
    e = lookup(load(db_path), key, length)
    if e is None:
        return None
    set_config(**e["config"])
    return e["config"]


def _workload(name: str):
    import numpy as np

    import workloads as W
    if name == "c4_batched":
        return [torch.from_numpy(a.view(np.int64)).cuda() for a, _ in W.c4_batched()]
    gen = {"c1_uniform20": W.c1_uniform20, "c2_mr64": W.c2_mr64, "c3_mixed": W.c3_mixed,
           "lookup32": W.lookup32}[name]
    return [torch.from_numpy(gen().view(np.int64)).cuda()]


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", action="append", required=True,
                    help="c1_uniform20, c2_mr64, c3_mixed, lookup32 or c4_batched (repeatable)")
    ap.add_argument("--db", default=DEFAULT_DB)
    ap.add_argument("--reps", type=int, default=7)
    args = ap.parse_args()
    db = load(args.db)
    db["device"] = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    base = get_config()
    for name in args.workload:
        arrays = _workload(name)
        n = sum(a.numel() for a in arrays)
        t0 = time.perf_counter()
        print("tuning %s (%d elements)" % (name, n), flush=True)
        # the descent starts from the entry already recorded for this class
        # and length, if any (coordinate descent finds a local optimum)
        set_config(**base)
        known = lookup(db, name, n)
        if known is not None:
            set_config(**known["config"])
        res = tune(arrays, reps=args.reps, log=lambda s: print(s, flush=True))
        res["seconds"] = time.perf_counter() - t0
        db.setdefault("entries", {})["%s|%d" % (name, length_bucket(n))] = res
        print("  best %.4f ms (default %.4f ms): %s" % (res["ms"], res["default_ms"], res["config"]),
              flush=True)
        save(db, args.db)


if __name__ == "__main__":
    main()
