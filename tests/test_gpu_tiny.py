"""Every matrix of every tiny shape through the library, against the oracle's exhaustive
enumeration (oracle.all_masks: each m x n 0/1 matrix, its side and first row-major corner).
Tile edges, halos and padding masks are off by one at these sizes if anywhere:

  * batched: every matrix of every shape m, n <= 5 with m n <= 20 (2,239,754 matrices) in one
    ms_max_square_batched call, and every 5 x 5 matrix (2^25) in four calls of 2^23;
  * single calls: ms_square_map on every matrix of every shape up to 4 x 4 (74,954 maps,
    each map compared cell by cell with the oracle's table), and ms_max_square on every 4 x 4.

Matrix number `mask` of shape (m, n) has A[i][j] = bit i n + j of mask (the enumeration's
order).  Odd masks carry ones in their padding bits (columns n..63), which must be ignored."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2503_18974_amd as M
from gpu_util import announce

pytestmark = pytest.mark.gpu

PAD_ONES = np.uint64(0xFFFFFFFFFFFFFFFF)


def packed_rows(m, n, masks):
    """uint64 (len(masks), m): row i of matrix `mask` is bits i n .. i n + n - 1 of the mask;
    odd masks get their padding bits set."""
    masks = masks.astype(np.uint64)
    rows = np.empty((masks.size, m), np.uint64)
    low = np.uint64((1 << n) - 1)
    pad = np.where(masks & np.uint64(1), PAD_ONES ^ low, np.uint64(0)).astype(np.uint64)
    for i in range(m):
        rows[:, i] = ((masks >> np.uint64(i * n)) & low) | pad
    return rows


def expected(m, n):
    side, corner = oracle.all_masks(m, n)
    row = np.where(corner >= 0, corner // n, -1)
    col = np.where(corner >= 0, corner % n, -1)
    return np.stack([side, row, col], axis=1)


def run_batched(dev, shapes_masks):
    """One ms_max_square_batched call over the given (m, n, masks) groups; returns the int64
    (count, 3) results."""
    import torch
    blocks, descs = [], []
    word = 0
    for m, n, masks in shapes_masks:
        rows = packed_rows(m, n, masks)
        blocks.append(rows.reshape(-1))
        k = masks.size
        d = np.zeros((k, 4), np.int64)
        d[:, 0] = word + np.arange(k, dtype=np.int64) * m   # word offset, made a pointer below
        d[:, 1], d[:, 2], d[:, 3] = m, n, 1
        descs.append(d)
        word += k * m
    flat = np.concatenate(blocks)
    desc = np.concatenate(descs)
    count = desc.shape[0]
    bits = torch.from_numpy(flat.view(np.int64)).to(dev)
    desc[:, 0] = bits.data_ptr() + desc[:, 0] * 8
    assert ctypes.sizeof(M._Matrix) == 32
    h_mats = np.ascontiguousarray(desc)
    d_mats = torch.from_numpy(h_mats.view(np.uint8).reshape(-1)).to(dev)
    out = torch.full((count, 3), -7, dtype=torch.int64, device=dev)
    L = M.lib()
    ws_n = ctypes.c_size_t()
    assert L.ms_batched_workspace_size(None, h_mats.ctypes.data, count, ctypes.byref(ws_n)) == 0
    ws = torch.empty(ws_n.value, dtype=torch.uint8, device=dev)
    rc = L.ms_max_square_batched(None, h_mats.ctypes.data, d_mats.data_ptr(), count,
                                 out.data_ptr(), ws.data_ptr(), ws_n.value,
                                 torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    got = out.cpu().numpy()
    del bits, d_mats, ws, out
    return got


def test_batched_every_matrix_up_to_20_cells(dev):
    groups, refs = [], []
    for m in range(1, 6):
        for n in range(1, 6):
            if m * n > 20:
                continue
            groups.append((m, n, np.arange(1 << (m * n), dtype=np.int64)))
            refs.append(expected(m, n))
    ref = np.concatenate(refs)
    announce("tiny batched", len(groups), "shapes", ref.shape[0], "matrices")
    got = run_batched(dev, groups)
    bad = np.flatnonzero(np.any(got != ref, axis=1))
    if bad.size:
        k = int(bad[0])
        for m, n, masks in groups:
            if k < masks.size:
                raise AssertionError("shape %dx%d mask %d: %s vs oracle %s" % (
                    m, n, k, got[bad[0]], ref[bad[0]]))
            k -= masks.size


@pytest.mark.parametrize("quarter", range(4))
def test_batched_every_5x5_matrix(dev, quarter):
    ref = expected(5, 5)
    q = 1 << 23
    masks = np.arange(quarter * q, (quarter + 1) * q, dtype=np.int64)
    announce("tiny batched 5x5 quarter", quarter)
    got = run_batched(dev, [(5, 5, masks)])
    bad = np.flatnonzero(np.any(got != ref[masks], axis=1))
    assert bad.size == 0, "5x5 mask %d: %s vs oracle %s" % (
        masks[bad[0]], got[bad[0]], ref[masks[bad[0]]])


def test_single_map_every_matrix_up_to_4x4(dev):
    """ms_square_map (search + map in one call) on each matrix of each shape up to 4 x 4, every
    call on its own slice of one device buffer, then all compared at once."""
    import torch
    L = M.lib()
    sp = torch.cuda.current_stream().cuda_stream
    for m in range(1, 5):
        for n in range(1, 5):
            masks = np.arange(1 << (m * n), dtype=np.int64)
            k = masks.size
            announce("tiny single maps", m, n, k)
            rows = packed_rows(m, n, masks)
            bits = torch.from_numpy(rows.reshape(-1).view(np.int64)).to(dev)
            dp = torch.full((k, m, n), -5, dtype=torch.int32, device=dev)
            res = torch.full((k, 3), -7, dtype=torch.int64, device=dev)
            pb, pd, pr = bits.data_ptr(), dp.data_ptr(), res.data_ptr()
            for t in range(k):
                rc = L.ms_square_map(None, pb + t * m * 8, m, n, 1, pd + t * m * n * 4, n,
                                     pr + t * 24, sp)
                assert rc == 0
            got_dp = dp.cpu().numpy()
            got = res.cpu().numpy()
            ref = expected(m, n)
            bad = np.flatnonzero(np.any(got != ref, axis=1))
            assert bad.size == 0, "%dx%d mask %d: %s vs %s" % (m, n, bad[0], got[bad[0]],
                                                               ref[bad[0]])
            # the oracle's table for every mask (bit i n + j of the mask is A[i][j])
            cells = ((masks[:, None] >> np.arange(m * n)) & 1).astype(np.uint8)
            for t in range(k):
                ref_dp, _ = oracle.square_map(cells[t].reshape(m, n))
                if not np.array_equal(got_dp[t], ref_dp):
                    raise AssertionError("%dx%d mask %d map %s vs oracle %s" % (
                        m, n, t, got_dp[t].tolist(), ref_dp.tolist()))


def test_single_search_every_4x4(dev):
    import torch
    L = M.lib()
    sp = torch.cuda.current_stream().cuda_stream
    masks = np.arange(1 << 16, dtype=np.int64)
    rows = packed_rows(4, 4, masks)
    bits = torch.from_numpy(rows.reshape(-1).view(np.int64)).to(dev)
    res = torch.full((masks.size, 3), -7, dtype=torch.int64, device=dev)
    pb, pr = bits.data_ptr(), res.data_ptr()
    announce("tiny single search 4x4")
    for t in range(masks.size):
        assert L.ms_max_square(None, pb + t * 32, 4, 4, 1, pr + t * 24, sp) == 0
    got = res.cpu().numpy()
    ref = expected(4, 4)
    bad = np.flatnonzero(np.any(got != ref, axis=1))
    assert bad.size == 0, "4x4 mask %d: %s vs %s" % (bad[0], got[bad[0]], ref[bad[0]])
