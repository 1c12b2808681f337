"""Full-size parity on the large single matrices: side and corner against the stored oracle
values, and every cell of the int32 map against the rolling-row oracle, chunk by chunk."""
import hashlib
import json
import os
import time

import numpy as np
import pytest

import oracle
import workloads as W
import paper_2503_18974_amd as M
from gpu_util import announce

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_configs.json")))


def make_input(name):
    g = GOLDEN[name]
    if name == "c3a":
        bits = W.gen_bernoulli_packed(g["m"], g["n"], g["p"], g["seed"])
    elif name == "c3b":
        bits, r0, c0 = W.gen_planted_packed(g["m"], g["n"], g["p"], g["planted"][2], g["seed"])
        assert [r0, c0] == g["planted"][:2]
    else:
        bits = W.pack_rows(W.gen_blob(g["m"], g["n"], g["sigma"], g["percentile"], g["seed"]))
    assert hashlib.sha256(bits.tobytes()).hexdigest() == g["sha256_packed"], "input differs"
    return bits, g


@pytest.mark.parametrize("name", ["c3a", "c3b", "c3c"])
def test_large_config(dev, name):
    import torch
    announce("large", name, "generating")
    t0 = time.time()
    bits, g = make_input(name)
    announce("large", name, "input ready %.1fs" % (time.time() - t0))
    m, n = g["m"], g["n"]
    d = torch.from_numpy(bits.view(np.int64)).to(dev)
    torch.cuda.synchronize()
    t1 = time.time()
    sq = M.max_square(d, n)
    announce("large", name, "max_square %s in %.3fs" % (sq, time.time() - t1))
    assert (sq.side, sq.row, sq.col) == (g["side"], g["row"], g["col"])
    t2 = time.time()
    dp, sq2 = M.square_map(d, n)
    torch.cuda.synchronize()
    announce("large", name, "square_map in %.3fs" % (time.time() - t2))
    assert (sq2.side, sq2.row, sq2.col) == (g["side"], g["row"], g["col"])
    # every cell against the oracle's rolling rows
    st = oracle.Stream(bits, n)
    rows = max(1, (64 << 20) // (4 * n))
    t3 = time.time()
    for r0 in range(0, m, rows):
        ref = st.next(rows)
        got = dp[r0:r0 + ref.shape[0]].cpu().numpy()
        if not np.array_equal(got, ref):
            bad = np.argwhere(got != ref)[0]
            raise AssertionError("map differs at (%d, %d): %d vs %d" % (
                r0 + bad[0], bad[1], got[tuple(bad)], ref[tuple(bad)]))
    assert st.result() == (g["side"], g["row"], g["col"])
    announce("large", name, "map verified in %.1fs" % (time.time() - t3))
