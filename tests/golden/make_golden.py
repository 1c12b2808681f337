"""Write tests/golden/oracle_configs.json: the oracle's (S, row, col) for every full-size
workload, plus a sha256 of the packed input so a consumer can confirm it regenerated the
same bits.  Calls only the oracle and the input generators.

    python tests/golden/make_golden.py [--only c1,c2,c3a,c3b,c3c,c4]
    python tests/golden/make_golden.py --rect [--only c1,c2,c3a,c3c]

--rect adds, to the existing records, the oracle's largest all-ones rectangle as
"rect": [area, row, col, height, width] (rows of at most 32768 columns only).
--cube writes "volumes": the oracle's largest all-ones cube (side, z, y, x) of every benchmark
volume, with a sha256 of the packed volume.

The batched workload's 10000 results go to c4_results.txt instead (one line per matrix).
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
OUT_C4 = os.path.join(HERE, "c4_results.txt")


def sha(bits):
    return hashlib.sha256(bits.tobytes()).hexdigest()


def record(name, bits, m, n, extra=None):
    t = time.time()
    s, r, c = oracle.max_square_packed(bits, n)
    rec = {"m": m, "n": n, "side": s, "row": r, "col": c, "sha256_packed": sha(bits)}
    rec.update(extra or {})
    print(name, rec, "%.1fs" % (time.time() - t), flush=True)
    return rec


def write_c4(count=10000):
    """Oracle (side, row, col) for every matrix of the batched workload, and a sha256 over
    all packed inputs in order."""
    from concurrent.futures import ThreadPoolExecutor
    t = time.time()
    mats, m, n, p = W.batch_packed(count)
    h = hashlib.sha256()
    for a in mats:
        h.update(a.tobytes())
    with ThreadPoolExecutor(8) as ex:   # the oracle's C call releases the GIL
        res = list(ex.map(lambda k: oracle.max_square_packed(mats[k], int(n[k])), range(count)))
    with open(OUT_C4, "w") as f:
        f.write("# Written by tests/golden/make_golden.py from the oracle only.\n")
        f.write("# batched workload: %d matrices, sha256 of the packed inputs in order %s\n"
                % (count, h.hexdigest()))
        f.write("# index m n side row col\n")
        for k, (s_, r_, c_) in enumerate(res):
            f.write("%d %d %d %d %d %d\n" % (k, m[k], n[k], s_, r_, c_))
    print("c4", count, "matrices, %.1fs" % (time.time() - t), flush=True)


def add_rects(data, want):
    """The oracle's largest rectangle for each wanted record (input regenerated and checked
    against the stored sha256 first)."""
    from concurrent.futures import ThreadPoolExecutor

    def one(rec, bits):
        if sha(bits) != rec["sha256_packed"]:
            raise SystemExit("regenerated input differs from the recorded one")
        t = time.time()
        rec["rect"] = list(oracle.max_rect_packed(bits, rec["n"]))
        print(rec["m"], rec["n"], rec.get("p"), rec["rect"], "%.1fs" % (time.time() - t),
              flush=True)

    if "c1" in want:
        one(data["c1"], W.pack_rows(W.c1()))
    if "c2" in want:
        jobs = [(data["c2"]["%d_%d" % (n, d)], (n, p, seed)) for n, d, p, seed in W.paper_grid()]
        with ThreadPoolExecutor(6) as ex:   # the oracle's C call releases the GIL
            list(ex.map(lambda j: one(j[0], W.gen_bernoulli_packed(j[1][0], j[1][0], j[1][1],
                                                                   j[1][2])), jobs))
    for name in ("c3a", "c3c"):
        if name in want:
            bits, m, n, _ = W.large_packed(name)
            one(data[name], bits)
            del bits


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="c1,c2,c3a,c3b,c3c")
    ap.add_argument("--rect", action="store_true")
    ap.add_argument("--cube", action="store_true")
    args = ap.parse_args()
    want = set(args.only.split(","))
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    if args.cube:
        vols = {}
        for name in sorted(W.VOLUMES):
            t = time.time()
            bits, D, M, N = W.volume_packed(name)
            s_, z, y, x = oracle.max_cube_packed(bits, N)
            vols[name] = {"D": D, "M": M, "N": N, "side": s_, "z": z, "y": y, "x": x,
                          "sha256_packed": sha(bits)}
            print(name, vols[name], "%.1fs" % (time.time() - t), flush=True)
        data["volumes"] = vols
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        return
    if args.rect:
        add_rects(data, want)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        return
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
    for name in ("c3a", "c3b", "c3c"):
        if name in want:
            bits, m, n, extra = W.large_packed(name)
            extra = dict(extra)
            for k, v in W.LARGE[name].items():
                if k not in ("m", "n", "side"):
                    extra[k] = v
            if name == "c3c":
                extra["density"] = float(W.unpack_rows(bits, n).mean())
            data[name] = record(name, bits, m, n, extra)
            del bits
    if "c4" in want:
        write_c4()
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
