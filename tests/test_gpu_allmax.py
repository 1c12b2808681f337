"""All maximal squares: the row-major list of cells whose side equals the largest side S, against
the oracle's side map, on random shapes, ties, degenerate inputs, truncation and wide squares."""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_2503_18974_amd as M
from gpu_util import announce, to_dev_bits

pytestmark = pytest.mark.gpu


def expected(a):
    dp, (s, r, c) = oracle.square_map(a)
    if s == 0:
        return np.zeros(0, np.int64), 0
    pos = np.flatnonzero(dp.ravel() == s).astype(np.int64)
    assert pos[0] == r * a.shape[1] + c
    return pos, s


def check(a, dev, capacity=None):
    d = to_dev_bits(oracle.pack(a), dev)
    pos, count = M.all_max_squares(d, a.shape[1], capacity=capacity)
    ref, _ = expected(a)
    assert count == len(ref), (count, len(ref))
    got = pos.cpu().numpy()
    k = len(ref) if capacity is None else min(capacity, len(ref))
    np.testing.assert_array_equal(got[:k], ref[:k])
    return count


SHAPES = [(1, 1), (1, 300), (300, 1), (63, 64), (130, 129), (300, 1100), (1100, 300),
          (257, 4097), (1000, 1000)]


@pytest.mark.parametrize("m,n", SHAPES)
@pytest.mark.parametrize("p", [0.3, 0.7, 0.95])
def test_random(dev, m, n, p):
    announce("allmax random", m, n, p)
    check(W.gen_bernoulli(m, n, p, 31 * m + n), dev)


def test_ties_and_touching(dev):
    announce("allmax ties")
    rng = np.random.default_rng(4)
    a = (rng.random((900, 2500)) < 0.5).astype(np.uint8)
    for r0, c0 in ((100, 100), (100, 160), (160, 100), (500, 2300), (300, 1100)):
        a[r0:r0 + 60, c0:c0 + 60] = 1
    assert check(a, dev) >= 5


@pytest.mark.parametrize("m,n", [(1, 1), (7, 300), (300, 7), (700, 700), (2100, 2050)])
def test_all_ones(dev, m, n):
    """All-ones m x n: the squares of side min(m, n) slide along the longer side."""
    announce("allmax ones", m, n)
    assert check(np.ones((m, n), np.uint8), dev) == abs(m - n) + 1


def test_zeros_and_empty(dev):
    import torch
    announce("allmax zeros")
    assert check(np.zeros((50, 70), np.uint8), dev) == 0
    empty = torch.zeros((0, 2), dtype=torch.int64, device=dev)
    pos, count = M.all_max_squares(empty, 100)
    assert count == 0 and pos.numel() == 0


@pytest.mark.parametrize("capacity", [0, 1, 7])
def test_capacity_truncates(dev, capacity):
    announce("allmax capacity", capacity)
    a = np.ones((5, 400), np.uint8)              # 396 maximal squares
    assert check(a, dev, capacity=capacity) == 396


def test_blob(dev):
    announce("allmax blob")
    check(W.gen_blob(1024, 1536, 6.0, 55.0, 8), dev)


def test_too_wide_reports_unsupported(dev):
    announce("allmax unsupported")
    d = to_dev_bits(oracle.pack(np.ones((3100, 3100), np.uint8)), dev)
    with pytest.raises(M.MaxsqError):
        M.all_max_squares(d, 3100)


def test_corners_spread_over_many_scan_chunks(dev):
    """Equal squares planted down the whole matrix: the row-major prefix of the per-row counts
    crosses many scan chunks (and the chunks' own prefix), so every carry is exercised."""
    announce("allmax many chunks")
    m, n = 9000, 4100
    a = (np.random.default_rng(8).random((m, n)) < 0.3).astype(np.uint8)
    for r0 in range(7, m - 30, 41):
        for c0 in range(3 + (r0 % 5) * 61, n - 30, 397):
            a[r0 - 1:r0 + 21, c0 - 1:c0 + 21] = 0
            a[r0:r0 + 20, c0:c0 + 20] = 1
    assert check(a, dev) > 2000
    check(a, dev, capacity=1500)
