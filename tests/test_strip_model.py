"""CPU model of the strip sweep's arithmetic (the pass for squares too wide for the windowed
kernels), checked against the oracle's map of eq. (1).  It restates, lane by lane, what one wave
does per row and per 64-column word of its strip, and what one strip hands the next per row
(the row run and the dp at its last column, the run capped at RUN_CAP).  It pins the design,
not the GPU code: the cap argument (min(m, n) < cap keeps every minimum exact, tried here with
a cap of 25 on 20-row matrices) and the hand-over order (the previous row's dp left of a word,
taken before that word's lanes are updated).  The GPU parity of the kernels themselves is in
test_gpu_strips.py."""
import numpy as np
import pytest

import oracle

STRIP_WORDS = 2
ONES = (1 << 64) - 1


def _clz64(v):
    return 64 if v == 0 else 64 - v.bit_length()


def _pack(a):
    m, n = a.shape
    nw = (n + 63) // 64
    out = [[0] * nw for _ in range(m)]
    for i in range(m):
        for c in np.flatnonzero(a[i]):
            out[i][c // 64] |= 1 << (int(c) % 64)
    return out, nw


def sweep(a, run_cap=(1 << 20) - 1, handover=True):
    """dp map and (side, first corner as i * n + j) by strips of STRIP_WORDS words, the strips
    taken left to right (the order the kernels' tickets follow)."""
    m, n = a.shape
    words, nw = _pack(a)
    ns = (nw + STRIP_WORDS - 1) // STRIP_WORDS
    dp = np.zeros((m, n), dtype=np.int64)
    run_in = [0] * m   # row run at the last column of the strip to the left, per row
    dp_in = [0] * m    # dp there
    best = (0, -1)
    for s in range(ns):
        H = [[0] * 64 for _ in range(STRIP_WORDS)]
        D = [[0] * 64 for _ in range(STRIP_WORDS)]
        dl = 0
        run_out, dp_out = [0] * m, [0] * m
        for i in range(m):
            wc = run_in[i]
            dleft = dl
            dl = dp_in[i]
            for u in range(STRIP_WORDS):
                k = s * STRIP_WORDS + u
                x = words[i][k] if k < nw else 0
                dprev = [dleft] + D[u][:63]   # lane 0 takes the previous row's dp left of it
                dleft = D[u][63]
                for lane in range(64):
                    bit = (x >> lane) & 1
                    lo = _clz64(~(x << (63 - lane)) & ONES)
                    w = ((lane + 1 + wc) if lo == lane + 1 else lo) if bit else 0
                    h = H[u][lane] + 1 if bit else 0
                    d = min(h, w, dprev[lane] + 1) if bit else 0
                    H[u][lane], D[u][lane] = h, d
                    c = k * 64 + lane
                    if c < n:
                        dp[i, c] = d
                        if d > best[0]:
                            best = (d, i * n + c)
                wc = min(wc + 64, run_cap) if x == ONES else _clz64(~x & ONES)
            run_out[i], dp_out[i] = wc, D[STRIP_WORDS - 1][63]
        if handover:
            run_in, dp_in = run_out, dp_out
    return dp, best


@pytest.mark.parametrize("m,n,p,seed", [(5, 300, 0.9, 1), (70, 130, 1.0, 2), (130, 260, 0.97, 3),
                                        (1, 129, 1.0, 4), (40, 1, 1.0, 5), (65, 257, 1.0, 6)])
def test_strip_model_matches_oracle(m, n, p, seed):
    rng = np.random.default_rng(seed)
    a = (rng.random((m, n)) < p).astype(np.uint8)
    if p == 1.0 and m > 60:
        a[m // 2, n // 3] = 0
    dp, best = sweep(a)
    ref_dp, (side, row, col) = oracle.square_map(a)
    np.testing.assert_array_equal(dp, ref_dp)
    assert best[0] == side
    if side:
        assert divmod(best[1], n) == (row, col)


def test_strip_model_run_cap_exact_below_min_side():
    """A run cap at or above min(m, n) changes no value (here m = 20 < cap = 25 < n)."""
    a = np.ones((20, 400), np.uint8)
    a[3, 7] = 0
    dp, _ = sweep(a, run_cap=25)
    np.testing.assert_array_equal(dp, oracle.square_map(a)[0])


def test_strip_model_dropped_handover_is_caught():
    """The model is not vacuous: without the hand-over between strips it goes wrong on a square
    that spans two strips."""
    a = np.zeros((200, 300), np.uint8)
    a[10:160, 60:210] = 1   # crosses the strip edge at column 128
    dp, best = sweep(a, handover=False)
    assert not np.array_equal(dp, oracle.square_map(a)[0])
