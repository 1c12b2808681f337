"""The strip sweep: squares too wide for the windowed passes (the map beyond S = 1984, the search
when a saturated tile's window exceeds one word per lane), computed by many waves that walk
column strips and hand each other the row run and dp at a strip's last column.  Bit-exact
against the oracle's map and result (eq. (1) over the whole matrix): all-ones and planted
squares, ragged last strips, row strides and padding ones, a tie across strips, repeated calls
on one context, and graph replays."""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_2503_18974_amd as M
from gpu_util import announce, set_padding_bits, to_dev_bits

pytestmark = pytest.mark.gpu


def planted(m, n, side, p, seed):
    rng = np.random.default_rng([m, n, side, seed])
    a = (rng.random((m, n)) < p).astype(np.uint8)
    r0, c0 = int(rng.integers(0, m - side + 1)), int(rng.integers(0, n - side + 1))
    a[r0:r0 + side, c0:c0 + side] = 1
    return a


def check(a, dev, ctx=None, ld_extra=0, pad_ones=False):
    import torch
    m, n = a.shape
    bits = oracle.pack(a)
    if pad_ones:
        bits = set_padding_bits(bits, n)
    d = to_dev_bits(bits, dev, ld_words=W.words_per_row(n) + ld_extra,
                    pad_fill=0xFFFFFFFFFFFFFFFF if pad_ones else 0)
    ref_dp, ref = oracle.square_map(a)
    sq = M.max_square(d, n, ctx=ctx)
    assert (sq.side, sq.row, sq.col) == ref, (sq, ref)
    dp = torch.full((m, n), -7, dtype=torch.int32, device=dev)
    _, sq2 = M.square_map(d, n, ctx=ctx, dp=dp)
    assert (sq2.side, sq2.row, sq2.col) == ref, (sq2, ref)
    np.testing.assert_array_equal(dp.cpu().numpy(), ref_dp)
    # the map from a copy of the result: no per-tile bounds, the sweep alone
    dp.fill_(-7)
    res = torch.tensor([ref[0], ref[1], ref[2]], dtype=torch.int64, device=dev)
    M.square_map_from_max(d, n, res, ctx=ctx, dp=dp)
    np.testing.assert_array_equal(dp.cpu().numpy(), ref_dp)
    return ref


@pytest.mark.parametrize("m,n,side,p", [
    (3300, 3300, 3300, 1.0),   # all ones: the search and the map sweep
    (2200, 2300, 2100, 0.7),   # map sweep only (the search's windows still fit)
    (3100, 9000, 3050, 0.9),   # 141 words: a one-word last strip with a partial word
    (5000, 3200, 3150, 0.8),   # taller than wide
    (3200, 3257, 3200, 0.5),   # a square over the full height, one column of the last word
])
def test_strip_shapes(dev, m, n, side, p):
    announce("strips", m, n, side, p)
    check(planted(m, n, side, p, 1), dev)


def test_strip_stride_and_padding_ones(dev):
    announce("strips stride/padding")
    check(planted(3300, 3333, 3250, 0.9, 2), dev, ld_extra=3, pad_ones=True)


def test_strip_tie_across_strips(dev):
    """Two squares of the same side: the one whose bottom-right corner (the reported cell)
    comes first in row-major order lies in a strip to the right of the other's."""
    announce("strips tie")
    m, n = 3200, 7000
    a = np.zeros((m, n), np.uint8)
    a[50:3150, 3500:6600] = 1   # corner (3149, 6599)
    a[60:3160, 0:3100] = 1      # corner (3159, 3099): later in row-major order
    ref = check(a, dev)
    assert ref == (3100, 3149, 6599)


def test_strip_large(dev):
    """An all-ones 8192^2 matrix and a 4096 x 32768 matrix holding a 4000-wide square in
    Bernoulli(0.9) noise."""
    announce("strips 8192^2 ones")
    check(np.ones((8192, 8192), np.uint8), dev)
    announce("strips 4096 x 32768")
    check(planted(4096, 32768, 4000, 0.9, 3), dev)


def test_strip_repeated_calls_one_context(dev):
    """Each launch tags its boundary words with its own epoch: calls of different shapes in a
    row on one context never read an earlier call's words."""
    announce("strips repeated")
    ctx = M.Context()
    try:
        for (m, n, side, p, seed) in [(3300, 3300, 3300, 1.0, 4), (2500, 2600, 2200, 0.6, 5),
                                      (3300, 3300, 3300, 1.0, 4), (1500, 1100, 900, 0.8, 6),
                                      (3400, 3100, 3090, 0.9, 7)]:
            check(planted(m, n, side, p, seed), dev, ctx=ctx)
    finally:
        ctx.close()


def test_strip_graph_replay(dev):
    """The search and the map recorded in one graph, replayed three times with the outputs
    cleared between replays: the epoch lives on the device, so every replay has its own."""
    import torch
    announce("strips graph")
    a = planted(3300, 3300, 3280, 0.9, 8)
    m, n = a.shape
    ref_dp, ref = oracle.square_map(a)
    d = to_dev_bits(oracle.pack(a), dev)
    dp = torch.full((m, n), -7, dtype=torch.int32, device=dev)
    out = torch.zeros(3, dtype=torch.int64, device=dev)
    ctx = M.Context()
    try:
        L = M.lib()
        st = torch.cuda.Stream(device=dev)

        def call():
            rc = L.ms_square_map(ctx.handle, d.data_ptr(), m, n, W.words_per_row(n),
                                 dp.data_ptr(), n, out.data_ptr(), st.cuda_stream)
            assert rc == 0, rc

        with torch.cuda.stream(st):
            call()  # eager once: allocates the context's scratch outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st):
            call()
        for rep in range(3):
            dp.fill_(-7)
            out.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert tuple(out.cpu().tolist()) == ref, rep
            np.testing.assert_array_equal(dp.cpu().numpy(), ref_dp)
        del g
    finally:
        ctx.close()
