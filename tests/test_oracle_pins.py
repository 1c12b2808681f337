"""Pins of the CPU oracle against things other than itself (brute force, closed forms,
invariants, the paper's Algorithm 1, probability bounds).  CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute, stats
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("m,n", [(m, n) for m in range(1, 6) for n in range(1, 6) if m * n <= 20])
def test_exhaustive_small_shapes(m, n):
    """Every m x n 0/1 matrix (m*n <= 20): S and corner equal brute-force enumeration."""
    side_o, corner_o = oracle.all_masks(m, n)
    side_b, corner_b = brute.all_masks(m, n)
    np.testing.assert_array_equal(side_o, side_b)
    np.testing.assert_array_equal(corner_o, corner_b)


@pytest.mark.slow
@pytest.mark.parametrize("m,n", [(4, 5), (5, 4), (5, 5)])
def test_exhaustive_5x5(m, n):
    """All 2^25 5x5 matrices (and 2^20 4x5 / 5x4)."""
    side_o, corner_o = oracle.all_masks(m, n)
    side_b, corner_b = brute.all_masks(m, n)
    assert np.array_equal(side_o, side_b)
    assert np.array_equal(corner_o, corner_b)


def _random_cases(count, max_side, seed):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        m = int(rng.integers(1, max_side + 1))
        n = int(rng.integers(1, max_side + 1))
        p = float(rng.choice([0.3, 0.6, 0.8, 0.9, 0.97]))
        yield (rng.random((m, n)) < p).astype(np.uint8)


def test_random_small_map_vs_brute():
    """Per-cell side map (the definition in Section 1) on random matrices up to 16 x 16."""
    for a in _random_cases(300, 16, 1):
        dp, res = oracle.square_map(a)
        np.testing.assert_array_equal(dp, brute.side_map(a))
        assert res == brute.max_square(a)
        assert oracle.max_square(a) == res


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("m,n", [(1, 1), (1, 7), (7, 1), (3, 9), (9, 3), (64, 65), (100, 100)])
def test_all_ones(m, n):
    k = min(m, n)
    a = np.ones((m, n), np.uint8)
    assert oracle.max_square(a) == (k, k - 1, k - 1)
    dp, _ = oracle.square_map(a)
    i, j = np.indices((m, n))
    np.testing.assert_array_equal(dp, np.minimum(i, j) + 1)


@pytest.mark.parametrize("m,n", [(1, 1), (5, 8), (100, 100)])
def test_all_zeros(m, n):
    a = np.zeros((m, n), np.uint8)
    assert oracle.max_square(a) == (0, -1, -1)
    dp, _ = oracle.square_map(a)
    assert not dp.any()


def test_empty_shapes():
    for m, n in [(0, 0), (0, 5), (5, 0)]:
        assert oracle.max_square(np.zeros((m, n), np.uint8)) == (0, -1, -1)


def test_paper_edge_cases_fixture():
    """The paper's edge cases (Section 4, Edge Case Testing): 100 x 100 all-zero / all-one."""
    with open(os.path.join(GOLDEN, "paper_edge_cases.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        a = np.full((c["m"], c["n"]), c["fill"], np.uint8)
        s, r, col = oracle.max_square(a)
        assert (s, r, col) == tuple(c["expect"])
        assert s * s == c["area"]


@pytest.mark.parametrize("m,n", [(1, 1), (1, 6), (6, 1), (2, 2), (7, 9), (50, 31)])
@pytest.mark.parametrize("phase", [0, 1])
def test_checkerboard(m, n, phase):
    i, j = np.indices((m, n))
    a = (((i + j + phase) % 2) == 0).astype(np.uint8)
    res = oracle.max_square(a)
    if not a.any():
        assert res == (0, -1, -1)
    elif phase == 0:
        assert res == (1, 0, 0)
    else:
        assert res == ((1, 0, 1) if n >= 2 else (1, 1, 0))


def test_planted_with_border():
    """A planted s x s block framed by zeros in sparse noise whose window is below s."""
    rng = np.random.default_rng(5)
    for s in (6, 8, 17, 40):
        m, n = 200, 300
        a = (rng.random((m, n)) < 0.2).astype(np.uint8)
        lo, hi = stats.window(m, n, 0.2, 1e-9)
        assert hi < s
        r0, c0 = int(rng.integers(1, m - s - 1)), int(rng.integers(1, n - s - 1))
        a[r0 - 1:r0 + s + 1, c0 - 1:c0 + s + 1] = 0
        a[r0:r0 + s, c0:c0 + s] = 1
        assert oracle.max_square(a) == (s, r0 + s - 1, c0 + s - 1)


# ---------------------------------------------------------------- invariants

def test_transpose_invariance():
    for a in _random_cases(100, 40, 2):
        dp, _ = oracle.square_map(a)
        dpt, _ = oracle.square_map(np.ascontiguousarray(a.T))
        np.testing.assert_array_equal(dpt, dp.T)
        # the transpose's row-major-first corner is A's column-major-first dp == S cell
        s = dp.max()
        if s:
            cells = np.argwhere(dp.T == s)
            i, j = cells[0]
            assert oracle.max_square(a.T) == (int(s), int(i), int(j))


def test_monotone_under_setting_bits():
    rng = np.random.default_rng(3)
    for a in _random_cases(60, 48, 4):
        dp, _ = oracle.square_map(a)
        b = a.copy()
        b[rng.random(a.shape) < 0.1] = 1
        dpb, _ = oracle.square_map(b)
        assert (dpb >= dp).all()


def _erosion_brute(a, k):
    """E_k: the k x k square ending at (i, j) is all ones (sliding windows, no recurrence)."""
    m, n = a.shape
    e = np.zeros((m, n), bool)
    if k <= min(m, n):
        v = np.lib.stride_tricks.sliding_window_view(a != 0, (k, k))
        e[k - 1:, k - 1:] = v.all(axis=(2, 3))
    return e


def test_map_vs_erosion_counts():
    """popcount(E_k) = #{dp >= k} and E_k == (dp >= k) for every k <= S + 1."""
    for a in _random_cases(40, 64, 6):
        dp, (s, r, c) = oracle.square_map(a)
        assert dp.max() == s
        if s:
            flat = int(np.argmax(dp == s))
            assert (r, c) == divmod(flat, a.shape[1])
        for k in range(1, s + 2):
            e = _erosion_brute(a, k)
            np.testing.assert_array_equal(e, dp >= k)


def test_identity_heights_runs():
    """dp = min(H, W, dp[i-1][j-1] + 1) on ones, with H / W the vertical / horizontal run
    lengths computed here by direct counting."""
    for a in _random_cases(30, 40, 7):
        dp, _ = oracle.square_map(a)
        m, n = a.shape
        for i in range(m):
            for j in range(n):
                if not a[i, j]:
                    assert dp[i, j] == 0
                    continue
                h = 0
                while i - h >= 0 and a[i - h, j]:
                    h += 1
                w = 0
                while j - w >= 0 and a[i, j - w]:
                    w += 1
                d = dp[i - 1, j - 1] + 1 if i and j else 1
                assert dp[i, j] == min(h, w, d)


# ---------------------------------------------------------------- packed reader

def test_packed_bit_order():
    """Column j is bit j & 63 of word j >> 6, least significant first."""
    bits = np.zeros((1, 3), np.uint64)
    bits[0, 1] = np.uint64(2)           # column 65
    assert oracle.max_square_packed(bits, 130) == (1, 0, 65)
    bits[0, 1] = np.uint64(1 << 63)     # column 127
    assert oracle.max_square_packed(bits, 130) == (1, 0, 127)
    bits[0, 1] = np.uint64(0)
    bits[0, 2] = np.uint64(1 << 1)      # column 129
    assert oracle.max_square_packed(bits, 130) == (1, 0, 129)
    bits[0, 2] = np.uint64(1 << 2)      # column 130 is padding
    assert oracle.max_square_packed(bits, 130) == (0, -1, -1)


def test_packed_matches_u8_and_padding_ignored():
    for a in _random_cases(50, 150, 8):
        m, n = a.shape
        ref = oracle.max_square(a)
        bits = oracle.pack(a, ld_words=(n + 63) // 64 + 2)
        assert oracle.max_square_packed(bits, n) == ref
        # padding bits and padding words set to ones change nothing
        junk = bits.copy()
        if n % 64:
            junk[:, n // 64] |= np.uint64(~((1 << (n % 64)) - 1) & 0xFFFFFFFFFFFFFFFF)
        junk[:, (n + 63) // 64:] = np.uint64(0xFFFFFFFFFFFFFFFF)
        assert oracle.max_square_packed(junk, n) == ref
        dp_u8, _ = oracle.square_map(a)
        dp_p, _ = oracle.square_map_packed(junk, n)
        np.testing.assert_array_equal(dp_u8, dp_p)


def test_two_independent_packers_agree():
    """The oracle's C packer and the generator module's numpy encoder agree, and unpacking
    inverts both."""
    for a in _random_cases(50, 200, 9):
        n = a.shape[1]
        p1 = oracle.pack(a)
        p2 = W.pack_rows(a)
        np.testing.assert_array_equal(p1, p2)
        np.testing.assert_array_equal(oracle.unpack(p1, n), a)
        np.testing.assert_array_equal(W.unpack_rows(p1, n), a)


def test_stream_equals_full_map():
    for a in _random_cases(20, 300, 10):
        bits = oracle.pack(a)
        dp, res = oracle.square_map(a)
        st = oracle.Stream(bits, a.shape[1])
        rows = []
        while True:
            r = st.next(7)
            if r.shape[0] == 0:
                break
            rows.append(r)
        got = np.concatenate(rows) if rows else np.zeros((0, a.shape[1]), np.int32)
        np.testing.assert_array_equal(got, dp)
        assert st.result() == res


# ---------------------------------------------------------------- Algorithm 1 witness

def test_algorithm1_witness_random():
    """The paper's Algorithm 1 (Section 3) gives the same side, its last increment sits at the
    oracle's corner, and its per-row value is the running maximum of the dp rows."""
    for a in list(_random_cases(200, 40, 11)) + [W.gen_bernoulli(300, 500, p, 77) for p in (0.5, 0.9)]:
        (f, fr, fc), trace = oracle.freq_alg1(a)
        dp, res = oracle.square_map(a)
        assert (f, fr, fc) == res
        np.testing.assert_array_equal(trace, np.maximum.accumulate(dp.max(axis=1)))


def test_algorithm1_witness_exhaustive_4x4():
    side, corner = oracle.all_masks(4, 4)
    for mask in range(1 << 16):
        a = ((mask >> np.arange(16)) & 1).astype(np.uint8).reshape(4, 4)
        (f, fr, fc), _ = oracle.freq_alg1(a)
        assert f == side[mask]
        assert (fr * 4 + fc if f else -1) == corner[mask]


# ---------------------------------------------------------------- probability window

@pytest.mark.parametrize("n,p,seed", [(1000, 0.1, 1), (1000, 0.5, 2), (1000, 0.7, 0),
                                      (1000, 0.9, 3), (2000, 0.8, 4)])
def test_bernoulli_window(n, p, seed):
    a = W.gen_bernoulli(n, n, p, seed)
    lo, hi = stats.window(n, n, p, 1e-6)
    s, _, _ = oracle.max_square(a)
    assert lo <= s <= hi
    # Sun-Nobel's non-contiguous scale only bounds from above here
    assert s <= stats.sun_nobel_shape(n, p)


def test_oracle_rejects_bad_dims():
    L = oracle.lib()
    res = np.zeros(3, np.int64)
    assert L.oracle_max_square_u8(None, -1, 3, 3, res.ctypes.data) != 0
    assert L.oracle_max_square_packed(None, 3, 3, 1, res.ctypes.data) != 0
    assert L.oracle_max_square_packed(res.ctypes.data, 3, 130, 2, res.ctypes.data) != 0
