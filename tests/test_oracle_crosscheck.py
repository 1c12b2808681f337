"""The oracle against values computed independently of it for every benchmark input: the single
1000 x 1000 matrix, the 45-matrix grid of the paper's sizes and densities (Section 4's test
matrices), and the three large matrices.  The stored values (tests/golden/
independent_crosscheck.json) come from a vectorized evaluation of the identity
dp = min(H, W, dp[i-1][j-1] + 1) written separately from oracle/, so a mistake in the oracle's
recurrence, its tie-break or its unpacker shows up here as well as in the brute-force pins.
These also pin the input generators: a different draw gives different squares."""
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import workloads as W

XC = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                  "independent_crosscheck.json")))


def test_c1_matches_independent_value():
    assert list(oracle.max_square(W.c1())) == XC["c1"]


def test_grid_matches_independent_values():
    grid = W.paper_grid()
    assert len(grid) == len(XC["c2"]) == 45

    def one(cell):
        n, d, p, seed = cell
        bits = W.gen_bernoulli_packed(n, n, p, seed)
        return "%d_%d" % (n, d), list(oracle.max_square_packed(bits, n))

    with ThreadPoolExecutor(8) as ex:   # the oracle's C calls release the GIL
        got = dict(ex.map(one, grid))
    bad = {k: (got[k], v) for k, v in XC["c2"].items() if got[k] != v}
    assert not bad, bad


@pytest.mark.slow
@pytest.mark.parametrize("name", ["c3a", "c3b", "c3c"])
def test_large_matches_independent_values(name):
    bits, m, n, extra = W.large_packed(name)
    if name == "c3b":
        assert extra["planted"][:2] == XC["c3b_planted_top_left"]
    if name == "c3c":
        density = float(np.unpackbits(bits.view(np.uint8)).sum()) / (m * n)
        assert abs(density - XC["c3c_density"]) < 1e-7
    assert list(oracle.max_square_packed(bits, n)) == XC[name]
