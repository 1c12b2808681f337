"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle, on seeded inputs
spanning several tiles with ragged tails, edge cases and every launch-shape candidate."""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_2503_18974_amd as M
from gpu_util import announce, set_padding_bits, to_dev_bits

pytestmark = pytest.mark.gpu


def run_both(a_u8, dev, ctx=None, ld_extra=0, pad_ones=False, dp_extra=0):
    import torch
    m, n = a_u8.shape
    bits = oracle.pack(a_u8)
    if pad_ones:
        bits = set_padding_bits(bits, n)
    d = to_dev_bits(bits, dev, ld_words=W.words_per_row(n) + ld_extra,
                    pad_fill=0xFFFFFFFFFFFFFFFF if pad_ones else 0)
    sq = M.max_square(d, n, ctx=ctx)
    dp = torch.full((m, n + dp_extra), -7, dtype=torch.int32, device=dev)
    dpv = dp[:, :n] if dp_extra else dp
    _, sq2 = M.square_map(d, n, ctx=ctx, dp=dpv)
    ref_dp, ref = oracle.square_map(a_u8)
    got = dp.cpu().numpy()
    return sq, sq2, got, ref, ref_dp


def assert_same(a_u8, dev, **kw):
    sq, sq2, got, ref, ref_dp = run_both(a_u8, dev, **kw)
    n = a_u8.shape[1]
    assert (sq.side, sq.row, sq.col) == ref, (sq, ref)
    assert (sq2.side, sq2.row, sq2.col) == ref, (sq2, ref)
    np.testing.assert_array_equal(got[:, :n], ref_dp)
    if got.shape[1] > n:
        assert (got[:, n:] == -7).all(), "map wrote beyond n"


SHAPES = [(1, 1), (1, 200), (200, 1), (2, 3), (63, 64), (64, 65), (65, 127), (127, 128),
          (129, 129), (300, 1000), (1000, 63), (257, 4097), (1500, 1100)]


@pytest.mark.parametrize("m,n", SHAPES)
@pytest.mark.parametrize("p", [0.5, 0.9])
def test_random_shapes(dev, m, n, p):
    announce("random", m, n, p)
    a = W.gen_bernoulli(m, n, p, 1000 * m + n)
    assert_same(a, dev)


@pytest.mark.parametrize("p", [0.0, 0.05, 0.3, 0.7, 0.95, 0.99, 1.0])
def test_densities(dev, p):
    announce("density", p)
    a = W.gen_bernoulli(700, 900, p, 7)
    assert_same(a, dev)


def test_padding_ones_and_strides(dev):
    announce("padding")
    for (m, n) in [(50, 70), (33, 130), (200, 191)]:
        a = W.gen_bernoulli(m, n, 0.8, m + n)
        assert_same(a, dev, ld_extra=3, pad_ones=True, dp_extra=5)


@pytest.mark.parametrize("m,n", [(1, 1), (64, 64), (300, 17), (17, 300), (2100, 2100)])
def test_all_ones(dev, m, n):
    announce("all-ones", m, n)
    a = np.ones((m, n), np.uint8)
    assert_same(a, dev)


def test_all_zeros_and_empty(dev):
    import torch
    announce("zeros/empty")
    assert_same(np.zeros((130, 70), np.uint8), dev)
    for m, n in [(0, 0), (0, 5), (5, 0)]:
        d = torch.zeros((max(m, 1), max(W.words_per_row(n), 1)), dtype=torch.int64, device=dev)[:m]
        sq = M.max_square(d, n)
        assert (sq.side, sq.row, sq.col) == (0, -1, -1)


@pytest.mark.parametrize("phase", [0, 1])
def test_checkerboard(dev, phase):
    announce("checkerboard", phase)
    i, j = np.indices((333, 517))
    assert_same((((i + j + phase) % 2) == 0).astype(np.uint8), dev)


@pytest.mark.parametrize("side", [1, 15, 16, 17, 31, 32, 33, 64, 65, 200, 700])
def test_planted_blocks(dev, side):
    """Squares around the erosion tile's certified bound and the window sizes."""
    announce("planted", side)
    rng = np.random.default_rng(side)
    m, n = 1200, 1500
    a = (rng.random((m, n)) < 0.6).astype(np.uint8)
    r0, c0 = int(rng.integers(0, m - side)), int(rng.integers(0, n - side))
    a[r0:r0 + side, c0:c0 + side] = 1
    assert_same(a, dev)


def test_blob(dev):
    announce("blob")
    a = W.gen_blob(1024, 1536, 8.0, 60.0, 3)
    assert_same(a, dev)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("shape,sigma,pct,seed", [((1500, 4100), 9.0, 50.0, 21),
                                                  ((2200, 2900), 12.0, 45.0, 22)])
def test_blob_grouped_resolve(dev, variant, shape, sigma, pct, seed):
    """Blob images where most tiles saturate: the resolve pass takes neighbouring tiles of a tile
    row together (ragged tile columns, groups with unsaturated members), for every probe tile."""
    announce("blob groups", variant, shape, seed)
    a = W.gen_blob(shape[0], shape[1], sigma, pct, seed)
    r0, c0 = shape[0] // 3, 2800  # a square across tile columns 2 and 3 (two groups)
    a[r0:r0 + 120, c0:c0 + 120] = 1
    ctx = M.Context()
    try:
        M.ms_set_config(ctx.handle, dict(probe_variant=variant, map_cols=4, map_band_rows=64))
        assert_same(a, dev, ctx=ctx)
    finally:
        ctx.close()


def test_every_candidate_identical(dev):
    """Every launch shape gives the same bits (a race or a missed barrier would differ)."""
    import torch
    rng = np.random.default_rng(11)
    a = (rng.random((900, 1300)) < 0.85).astype(np.uint8)
    a[100:160, 200:260] = 1
    ref_dp, ref = oracle.square_map(a)
    d = to_dev_bits(oracle.pack(a), dev)
    ctx = M.Context()
    try:
        for i in range(M.ms_num_candidates()):
            cfg = M.ms_candidate(i)
            announce("candidate", cfg)
            M.ms_set_config(ctx.handle, cfg)
            sq = M.max_square(d, 1300, ctx=ctx)
            dp, sq2 = M.square_map(d, 1300, ctx=ctx)
            assert (sq.side, sq.row, sq.col) == ref
            assert (sq2.side, sq2.row, sq2.col) == ref
            assert torch.equal(dp.cpu(), torch.from_numpy(ref_dp))
    finally:
        ctx.close()


def test_pack_parity(dev):
    import torch
    rng = np.random.default_rng(5)
    for (m, n) in [(1, 1), (3, 15), (7, 16), (5, 17), (9, 64), (11, 100), (40, 1000), (64, 4099)]:
        announce("pack", m, n)
        a = rng.integers(0, 4, size=(m, n)).astype(np.uint8)   # non-zero bytes other than 1
        ref = oracle.pack(a)
        ta = torch.from_numpy(a).to(dev)
        got = M.pack_u8(ta).cpu().numpy().view(np.uint64)
        np.testing.assert_array_equal(got[:, : ref.shape[1]], ref)
        # unaligned row stride: a view into a wider buffer, offset by 3 bytes
        wide = torch.zeros((m, n + 13), dtype=torch.uint8, device=dev)
        wide[:, 3:3 + n] = ta
        got2 = M.pack_u8(wide[:, 3:3 + n]).cpu().numpy().view(np.uint64)
        np.testing.assert_array_equal(got2[:, : ref.shape[1]], ref)


def test_c1(dev):
    """1000 x 1000 Bernoulli(0.7) from seed 0: side, corner and the full int32 map."""
    announce("c1")
    a = W.c1()
    assert_same(a, dev)


def test_repeated_calls_reuse_scratch(dev):
    """The scratch clears itself: alternating inputs give each input's own answer."""
    announce("repeat")
    a1 = W.gen_bernoulli(500, 700, 0.9, 1)
    a2 = np.zeros((800, 300), np.uint8)
    a3 = W.gen_bernoulli(64, 64, 0.99, 2)
    ds = [(to_dev_bits(oracle.pack(a), dev), a.shape[1], oracle.max_square(a)) for a in (a1, a2, a3)]
    for _ in range(3):
        for d, n, ref in ds:
            sq = M.max_square(d, n)
            assert (sq.side, sq.row, sq.col) == ref


@pytest.mark.parametrize("where", ["top_left", "bottom_right", "tile_seams", "far_right"])
@pytest.mark.parametrize("side", [40, 130, 1000])
def test_saturated_tiles_at_edges(dev, where, side):
    """Squares beyond the tiles' certified side, placed against the matrix borders (column
    heights reaching row 0, windows clipped at column 0 and at n) and across tile seams."""
    announce("saturated", where, side)
    rng = np.random.default_rng([side, len(where)])
    m, n = (1200, 7000) if where == "far_right" else (1300, 2100)
    a = (rng.random((m, n)) < 0.7).astype(np.uint8)
    if where == "top_left":
        r0, c0 = 0, 0
    elif where == "bottom_right":
        r0, c0 = m - side, n - side
    elif where == "tile_seams":
        r0, c0 = max(0, 113 * 3 - side // 2), max(0, 960 - side // 2)
    else:
        r0, c0 = 100, n - side - 3
    a[r0:r0 + side, c0:c0 + side] = 1
    assert_same(a, dev)


@pytest.mark.parametrize("layout", ["same_row", "earlier_row_later_col", "touching"])
def test_equal_squares_first_corner(dev, layout):
    """Several squares of the maximal side: the reported corner is the first bottom-right
    corner in row-major order."""
    announce("ties", layout)
    rng = np.random.default_rng(len(layout))
    m, n = 900, 2500
    a = (rng.random((m, n)) < 0.5).astype(np.uint8)
    s = 60
    if layout == "same_row":
        spots = [(300, 1800), (300, 200), (300, 1000)]
    elif layout == "earlier_row_later_col":
        spots = [(500, 100), (200, 2300), (350, 1200)]
    else:
        spots = [(100, 100), (100, 100 + s), (100 + s, 100)]
    for r0, c0 in spots:
        a[r0:r0 + s, c0:c0 + s] = 1
    assert_same(a, dev)


# Probe tiles per variant: (owned rows TR, certified side KC).  The owned rows of a tile at
# offset >= KC from its first row (the "deep" rows) are exact inside the probe's register tile
# for sides up to 2 KC; the resolve pass then finishes only the first KC rows of the tile.
PROBE_TILES = {0: (49, 16), 1: (113, 16), 2: (97, 32), 3: (65, 64)}


def _deep_rows_cases(TR, KC):
    """(name, [(bottom row offset in tile row 1, side)]): squares whose bottom-right corners sit
    in the first KC rows or the deep rows of one tile, around every boundary that matters."""
    last = TR - 1
    return [
        ("tie_top_last_vs_deep_first", [(KC - 1, KC + 3), (KC, KC + 3)]),
        ("deep_larger", [(2, KC + 1), (last, 2 * KC - 1)]),
        ("deep_full", [(3, KC + 2), (last, 2 * KC + 2)]),
        ("top_only", [(KC - 1, KC + 4)]),
        ("deep_exactly_2kc", [(0, 2 * KC - 1), (last, 2 * KC)]),
        ("tie_2kc_minus_1", [(1, 2 * KC - 1), (KC + 1, 2 * KC - 1)]),
        ("deep_reaches_tile_above", [(KC, 2 * KC - 1)]),
        ("deep_2kc_from_register_row_0", [(KC, 2 * KC)]),
        ("deep_past_register_tile", [(KC, 2 * KC + 1)]),
        ("deep_below_kc_top_kc", [(KC - 2, KC), (KC + 5, KC - 1)]),
        # first-row squares reaching deep into the tile above, whose last row then holds a
        # square of side s - KC: below KC, between KC and 2 KC, and beyond 2 KC
        ("first_rows_above_unsaturated", [(KC - 1, 2 * KC - 1)]),
        ("first_rows_above_deep", [(KC - 1, 2 * KC + 5)]),
        ("first_rows_above_full", [(KC - 1, 3 * KC + 2)]),
    ]


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_deep_rows_of_saturated_tiles(dev, variant):
    """Saturated tiles whose deep rows the probe finishes: ties between the first rows and the
    deep rows, sides at 2 KC - 1, 2 KC and beyond, squares reaching into the tile above, a
    tile whose deep rows stay below KC, and first-row squares reaching deep into the tile
    above."""
    TR, KC = PROBE_TILES[variant]
    ctx = M.Context()
    try:
        M.ms_set_config(ctx.handle, dict(probe_variant=variant, map_cols=4, map_band_rows=64))
        for k, (name, squares) in enumerate(_deep_rows_cases(TR, KC)):
            announce("deep rows", variant, name)
            rng = np.random.default_rng([variant, k])
            m, n = 3 * TR + 7, 2100
            a = (rng.random((m, n)) < 0.5).astype(np.uint8)
            ta = TR  # tile row 1; tile column 1 owns columns 960..1919
            for q, (off, side) in enumerate(squares):
                r1 = ta + off
                c1 = 1100 + q * 400  # the square's right column
                side = min(side, r1 + 1)  # the 64-certified tile's rows: keep it in the matrix
                a[r1 - side + 1:r1 + 1, c1 - side + 1:c1 + 1] = 1
            assert_same(a, dev, ctx=ctx)
    finally:
        ctx.close()


def test_resolve_falls_back_to_serial(dev):
    """A square so wide that the column-height window exceeds one word per lane: the serial
    pass finishes the matrix."""
    announce("serial fallback 3300")
    assert_same(np.ones((3300, 3300), np.uint8), dev)


@pytest.mark.parametrize("side", [300, 449, 700, 1500, 2100])
def test_map_from_max_wide(dev, side):
    """The map from an earlier search's device result, in both of its forms: handed the
    search's own result buffer (the context still holds that search's per-tile bounds, so the
    halos follow them) and a copy of it (no per-tile bounds: one S halo everywhere).  The
    2048-column block kernel for 448 < S <= 1984, the one-wave sweep beyond, the narrow kernel
    below."""
    import torch
    announce("map_from_max", side)
    rng = np.random.default_rng([side, 11])
    m, n = side + 260, side + 410
    a = (rng.random((m, n)) < 0.7).astype(np.uint8)
    r0, c0 = int(rng.integers(0, m - side)), int(rng.integers(0, n - side))
    a[r0:r0 + side, c0:c0 + side] = 1
    d = to_dev_bits(oracle.pack(a), dev)
    ref_dp, ref = oracle.square_map(a)
    res = M.max_square(d, n, sync=False)
    dp = torch.full((m, n), -7, dtype=torch.int32, device=dev)
    M.square_map_from_max(d, n, res, dp=dp)           # by region
    assert tuple(res.cpu().tolist()) == ref
    np.testing.assert_array_equal(dp.cpu().numpy(), ref_dp)
    dp2 = torch.full((m, n), -7, dtype=torch.int32, device=dev)
    M.square_map_from_max(d, n, res.clone(), dp=dp2)  # one halo
    np.testing.assert_array_equal(dp2.cpu().numpy(), ref_dp)


@pytest.mark.parametrize("spots", [1, 3])
def test_map_regions_mixed(dev, spots):
    """Several wide squares in small-square noise: the map splits tiles by their search bound
    (wide halos only around the big squares), so seams between the classes must agree."""
    announce("map_regions", spots)
    rng = np.random.default_rng([spots, 12])
    m, n = 1800, 5200
    a = (rng.random((m, n)) < 0.8).astype(np.uint8)
    sides = [900, 520, 470][:spots]
    for k, s in enumerate(sides):
        r0 = int(rng.integers(0, m - s))
        c0 = 1700 * k + int(rng.integers(0, 1700 - s))
        a[r0:r0 + s, c0:c0 + s] = 1
    assert_same(a, dev)


def test_wide_map_unaligned_rows(dev):
    """A square beyond the narrow reach with a map row stride that is not a multiple of four:
    the block-wide kernel's scalar stores, in both halo classes."""
    announce("wide map unaligned")
    rng = np.random.default_rng(77)
    a = (rng.random((1000, 1500)) < 0.75).astype(np.uint8)
    a[200:800, 300:900] = 1
    assert_same(a, dev, dp_extra=3)
