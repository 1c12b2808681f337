"""Bit-exact parity of the largest all-ones rectangle (HIP, through the C ABI) with the CPU
oracle: random shapes with ragged tails at every row width the kernel distinguishes, densities,
closed forms, planted rectangles, ties, padding and strides, and repeated calls."""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_2503_18974_amd as M
from gpu_util import announce, set_padding_bits, to_dev_bits

pytestmark = pytest.mark.gpu


def check(a, dev, ld_extra=0, pad_ones=False, ctx=None):
    m, n = a.shape
    bits = oracle.pack(a)
    if pad_ones:
        bits = set_padding_bits(bits, n)
    d = to_dev_bits(bits, dev, ld_words=W.words_per_row(n) + ld_extra,
                    pad_fill=0xFFFFFFFFFFFFFFFF if pad_ones else 0)
    got = M.max_rectangle(d, n, ctx=ctx)
    want = oracle.max_rect(a)
    assert (got.area, got.row, got.col, got.height, got.width) == want, (got, want)
    return got


WIDTHS = [1, 2, 63, 64, 65, 127, 300, 4096, 4097, 8192, 8200, 16384, 16447, 32768]


@pytest.mark.parametrize("n", WIDTHS)
@pytest.mark.parametrize("p", [0.5, 0.9])
def test_widths(dev, n, p):
    m = 90 if n <= 300 else 24
    announce("rect width", m, n, p)
    check(W.gen_bernoulli(m, n, p, 77 * n + int(p * 10)), dev)


@pytest.mark.parametrize("m,n", [(1, 1), (1, 500), (500, 1), (3, 7), (257, 129), (700, 900)])
def test_random_shapes(dev, m, n):
    announce("rect random", m, n)
    check(W.gen_bernoulli(m, n, 0.8, 31 * m + n), dev)


@pytest.mark.parametrize("p", [0.0, 0.05, 0.3, 0.7, 0.95, 0.99, 1.0])
def test_densities(dev, p):
    announce("rect density", p)
    check(W.gen_bernoulli(300, 700, p, 5), dev)


@pytest.mark.parametrize("m,n", [(1, 1), (1, 300), (200, 1), (64, 64), (150, 4097)])
def test_all_ones(dev, m, n):
    announce("rect ones", m, n)
    got = check(np.ones((m, n), np.uint8), dev)
    assert got.area == m * n


def test_empty_and_zero(dev):
    import torch
    announce("rect empty")
    for m, n in [(0, 5), (5, 0), (0, 0)]:
        d = torch.zeros((m, max(W.words_per_row(n), 1)), dtype=torch.int64, device=dev)
        r = M.max_rectangle(d, n)
        assert (r.area, r.row, r.col, r.height, r.width) == (0, -1, -1, 0, 0)
    check(np.zeros((40, 100), np.uint8), dev)


@pytest.mark.parametrize("phase", [0, 1])
def test_checkerboard(dev, phase):
    announce("rect checkerboard", phase)
    i, j = np.indices((333, 517))
    check((((i + j + phase) % 2) == 0).astype(np.uint8), dev)


@pytest.mark.parametrize("h,w", [(9, 31), (40, 3), (1, 200), (250, 1), (64, 64), (3, 2000)])
def test_planted(dev, h, w):
    announce("rect planted", h, w)
    rng = np.random.default_rng([h, w, 3])
    m, n = 600, 2600
    a = (rng.random((m, n)) < 0.6).astype(np.uint8)
    r0, c0 = int(rng.integers(1, m - h - 1)), int(rng.integers(1, n - w - 1))
    a[r0:r0 + h, c0:c0 + w] = 1
    check(a, dev)


@pytest.mark.parametrize("layout", ["same_corner", "same_row", "earlier_row"])
def test_ties(dev, layout):
    """Equal largest areas: the first bottom-right corner in row-major order, then the
    smallest height."""
    announce("rect ties", layout)
    a = np.zeros((200, 3000), np.uint8)
    if layout == "same_corner":
        a[50:53, 100:103] = 1
        a[50, 100] = 0          # a 2 x 3 and a 3 x 2 end at (52, 102)
    elif layout == "same_row":
        a[60:64, 2000:2010] = 1
        a[60:64, 500:510] = 1   # equal rectangles, the left one first
    else:
        a[100:105, 50:58] = 1   # 5 x 8
        a[30:38, 2500:2505] = 1  # 8 x 5 ending in an earlier row
    check(a, dev)


def test_padding_ones_and_strides(dev):
    announce("rect padding")
    a = W.gen_bernoulli(200, 4150, 0.9, 12)
    check(a, dev, pad_ones=True)
    check(a, dev, ld_extra=3)


def test_blob(dev):
    announce("rect blob")
    check(W.gen_blob(1024, 1536, 8.0, 60.0, 3), dev)


def test_c1_and_paper_sized(dev):
    announce("rect c1")
    check(W.c1(), dev)
    announce("rect 5000 p=0.9")
    check(W.gen_bernoulli(5000, 5000, 0.9, 50009), dev)


def test_repeated_calls_share_scratch(dev):
    """Calls on one context reuse its scratch; a smaller matrix after a larger one and the
    same matrix twice give the oracle's results."""
    announce("rect repeated")
    ctx = M.Context()
    try:
        for a in (W.gen_bernoulli(900, 3000, 0.85, 1), W.gen_bernoulli(40, 70, 0.6, 2),
                  W.gen_bernoulli(40, 70, 0.6, 2), np.ones((5, 9), np.uint8)):
            check(a, dev, ctx=ctx)
    finally:
        ctx.close()


def test_too_wide_reports_unsupported(dev):
    import torch
    announce("rect too wide")
    d = torch.zeros((3, 513), dtype=torch.int64, device=dev)
    with pytest.raises(M.MaxsqError) as e:
        M.max_rectangle(d, 32769)
    assert e.value.status == 5
