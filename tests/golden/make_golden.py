"""Write tests/golden/oracle_configs.json: the oracle's (S, row, col) for every full-size
workload, plus a sha256 of the packed input so a consumer can confirm it regenerated the
same bits.  Calls only the oracle and the input generators.

    python tests/golden/make_golden.py [--only c1,c2,c3a,c3b,c3c]
"""
import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "oracle_configs.json")


def sha(bits):
    return hashlib.sha256(bits.tobytes()).hexdigest()


def record(name, bits, m, n, extra=None):
    t = time.time()
    s, r, c = oracle.max_square_packed(bits, n)
    rec = {"m": m, "n": n, "side": s, "row": r, "col": c, "sha256_packed": sha(bits)}
    rec.update(extra or {})
    print(name, rec, "%.1fs" % (time.time() - t), flush=True)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="c1,c2,c3a,c3b,c3c")
    args = ap.parse_args()
    want = set(args.only.split(","))
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data["_note"] = ("Written by tests/golden/make_golden.py from the oracle only. "
                     "side/row/col: largest all-ones square and its row-major-first bottom-right corner.")
    if "c1" in want:
        data["c1"] = record("c1", W.pack_rows(W.c1()), 1000, 1000, {"p": 0.7, "seed": 0})
    if "c2" in want:
        grid = {}
        for n, d, p, seed in W.paper_grid():
            grid["%d_%d" % (n, d)] = record("c2 %d %.1f" % (n, p), W.gen_bernoulli_packed(n, n, p, seed),
                                           n, n, {"p": p, "seed": seed})
        data["c2"] = grid
    if "c3a" in want:
        data["c3a"] = record("c3a", W.gen_bernoulli_packed(32768, 32768, 0.9, 1), 32768, 32768,
                             {"p": 0.9, "seed": 1})
    if "c3b" in want:
        bits, r0, c0 = W.gen_planted_packed(4096, 262144, 0.5, 1500, 2)
        data["c3b"] = record("c3b", bits, 4096, 262144, {"p": 0.5, "seed": 2, "planted": [r0, c0, 1500]})
        del bits
    if "c3c" in want:
        a = W.gen_blob(16384, 16384, 8.0, 60.0, 3)
        dens = float(a.mean())
        bits = W.pack_rows(a)
        del a
        data["c3c"] = record("c3c", bits, 16384, 16384, {"sigma": 8.0, "percentile": 60.0, "seed": 3,
                                                          "density": dens})
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
