"""Timing harness of the CPU baselines -- TEST INFRASTRUCTURE (the benchmark's CPU legs).

The oracle is built a second time for timing only, ``-O3 -march=native`` for the host that runs
it (the checker build, ``liboracle.so`` at ``-O2``, is left as it is), and timed with the
protocol of the paper's Section 4: warm-up runs first, then 5 to 50 timed runs per matrix
(fewer for larger matrices), and the mean after dropping the fastest and slowest tenth.  One
matrix is timed at a time on one pinned core (the caller starts this module under
``taskset -c <core>``); the all-cores figure pins one pool thread per allowed core.

Kinds timed (all plain C from ``oracle.c``):
  dp_full    : the recurrence of Section 2.1 eq. (1), full table (the oracle's map mode)
  dp_rolling : the same with two rolling rows, largest side only (the O(n)-space DP the
               paper's Section 4 compares against)
  freq       : the frequency-based method of Section 3 (largest side only)

    python -m oracle.cpu_timing --kinds dp_full,dp_rolling,freq --sample grid15 [--threads N]
prints one JSON object.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import subprocess
import sys
import threading
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle_native.so")
CFLAGS = ["-O3", "-march=native", "-std=c99"]
WARMUP = 3
TRIM = 0.10

_p = ctypes.c_void_p
_i64 = ctypes.c_int64


def build_native() -> str:
    """Compile oracle.c for this host (always recompiles: -march=native must match it)."""
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc"] + CFLAGS + ["-shared", "-fPIC", _SRC, "-o", tmp])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    L = ctypes.CDLL(_LIB)
    L.oracle_square_map_u8.argtypes = [_p, _i64, _i64, _i64, _p, _i64, _p]
    L.oracle_max_square_u8.argtypes = [_p, _i64, _i64, _i64, _p]
    L.oracle_freq_alg1_u8.argtypes = [_p, _i64, _i64, _i64, _p, _p]
    for f in (L.oracle_square_map_u8, L.oracle_max_square_u8, L.oracle_freq_alg1_u8):
        f.restype = ctypes.c_int
    return L


def _runner(L, kind, a):
    """A no-argument callable running `kind` once on the uint8 matrix a (buffers made here)."""
    m, n = a.shape
    pa = a.ctypes.data_as(_p)
    res = np.zeros(3, np.int64)
    pr = res.ctypes.data_as(_p)
    if kind == "dp_full":
        dp = np.empty((m, n), np.int32)
        pd = dp.ctypes.data_as(_p)
        return lambda: L.oracle_square_map_u8(pa, m, n, n, pd, n, pr), res
    if kind == "dp_rolling":
        return lambda: L.oracle_max_square_u8(pa, m, n, n, pr), res
    if kind == "freq":
        return lambda: L.oracle_freq_alg1_u8(pa, m, n, n, pr, None), res
    raise ValueError(kind)


def iterations(cells: int) -> int:
    """50 timed runs for a 1000^2 matrix down to 5 for the largest, as in the paper's protocol."""
    return int(max(5, min(50, round(5e7 / max(cells, 1)))))


def trimmed_mean(ts) -> float:
    ts = sorted(ts)
    k = int(len(ts) * TRIM)
    kept = ts[k:len(ts) - k] if len(ts) - 2 * k > 0 else ts
    return sum(kept) / len(kept)


def time_one(L, kind, a):
    """(trimmed mean seconds, runs) of `kind` on a: WARMUP untimed runs, then the timed ones."""
    fn, res = _runner(L, kind, a)
    for _ in range(WARMUP):
        if fn() != 0:
            raise RuntimeError("oracle %s failed" % kind)
    ts = []
    for _ in range(iterations(a.size)):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return trimmed_mean(ts), len(ts), tuple(int(x) for x in res)


def sample_grid(name: str):
    """The grid matrices of a named sample: grid15 = p in {0.1, 0.5, 0.9} at every side,
    grid45 = all of them."""
    sys.path.insert(0, os.path.dirname(_HERE))
    import workloads as W
    keep = {"grid15": (1, 5, 9), "grid45": tuple(range(1, 10))}[name]
    return [((n, d), W.gen_bernoulli(n, n, p, seed)) for n, d, p, seed in W.paper_grid()
            if d in keep]


def host():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model


def single_core(kinds, mats):
    L = _load()
    out = {}
    for kind in kinds:
        total_t, total_cells, runs, per = 0.0, 0, 0, []
        for (n, d), a in mats:
            t, r, res = time_one(L, kind, a)
            total_t += t
            total_cells += a.size
            runs += r
            per.append({"n": n, "p": d / 10, "s": t, "runs": r, "side": res[0]})
        out[kind] = {"gcells_s": total_cells / total_t / 1e9, "cells": total_cells,
                     "seconds_per_pass": total_t, "timed_runs": runs, "per_matrix": per}
    return out


def all_cores(kinds, mats, threads):
    """One pass list per kind: every matrix timed as above, the matrices dealt over `threads`
    pool threads, each pinned to its own allowed core; the figure is cells over wall time of
    the whole timed set."""
    from concurrent.futures import ThreadPoolExecutor
    L = _load()
    cores = sorted(os.sched_getaffinity(0))[:threads]
    slot = threading.local()
    counter = iter(range(1 << 30))
    lock = threading.Lock()

    def pin():
        if not getattr(slot, "pinned", False):
            with lock:
                k = next(counter)
            os.sched_setaffinity(threading.get_native_id(), {cores[k % len(cores)]})
            slot.pinned = True

    out = {"threads": len(cores)}
    order = sorted(mats, key=lambda x: -x[1].size)
    for kind in kinds:
        def job(item):
            pin()
            fn, _ = _runner(L, kind, item[1])
            for _ in range(WARMUP):
                fn()
            r = iterations(item[1].size)
            for _ in range(r):
                fn()
            return item[1].size * r
        t0 = time.perf_counter()
        with ThreadPoolExecutor(len(cores)) as ex:
            cells = sum(ex.map(job, order))
        t = time.perf_counter() - t0
        out[kind] = {"gcells_s": cells / t / 1e9, "cells": cells, "seconds": t}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kinds", default="dp_full,dp_rolling,freq")
    ap.add_argument("--sample", default="grid15")
    ap.add_argument("--threads", type=int, default=0, help="0: one pinned core")
    args = ap.parse_args()
    build_native()
    kinds = [k for k in args.kinds.split(",") if k]
    mats = sample_grid(args.sample)
    allowed = sorted(os.sched_getaffinity(0))
    rec = {"cpu": host(), "compiler": "gcc " + " ".join(CFLAGS), "warmup": WARMUP,
           "trim_each_side": TRIM, "sample": args.sample, "matrices": len(mats),
           "allowed_cores": allowed if len(allowed) <= 8 else "%d cores" % len(allowed)}
    if args.threads:
        rec.update(all_cores(kinds, mats, args.threads))
    else:
        rec["cores"] = len(allowed)
        rec.update(single_core(kinds, mats))
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
