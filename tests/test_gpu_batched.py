"""Batched entry point: every result equals the single-matrix call and the oracle, under mixed
shapes, empty matrices, duplicates and shuffled order."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
import paper_2503_18974_amd as M
from gpu_util import announce, to_dev_bits

pytestmark = pytest.mark.gpu


def make_mix(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        m = int(np.exp(rng.uniform(np.log(16), np.log(1500))))
        n = int(np.exp(rng.uniform(np.log(16), np.log(1500))))
        a = (rng.random((m, n)) < rng.uniform(0.1, 0.95)).astype(np.uint8)
        if k % 7 == 3:   # planted squares beyond the erosion tile's certified side
            s = min(m, n, int(rng.integers(17, 200)))
            r0, c0 = int(rng.integers(0, m - s + 1)), int(rng.integers(0, n - s + 1))
            a[r0:r0 + s, c0:c0 + s] = 1
        out.append(a)
    return out


def check_batch(mats, dev):
    items = [(to_dev_bits(oracle.pack(a), dev), a.shape[1]) for a in mats]
    got = M.max_square_batched(items)
    for a, g, (d, n) in zip(mats, got, items):
        ref = oracle.max_square(a)
        assert (g.side, g.row, g.col) == ref, (a.shape, g, ref)
        single = M.max_square(d, n)
        assert (single.side, single.row, single.col) == ref


def test_batched_small_mix(dev):
    announce("batched mix 40")
    check_batch(make_mix(1, 40), dev)


def test_batched_edges(dev):
    announce("batched edges")
    mats = [np.zeros((0, 5), np.uint8), np.ones((1, 1), np.uint8), np.zeros((33, 70), np.uint8),
            np.ones((300, 200), np.uint8), W.gen_bernoulli(64, 4096, 0.9, 3),
            np.zeros((5, 0), np.uint8), W.gen_bernoulli(1, 5000, 0.5, 4)]
    check_batch(mats, dev)


def test_batched_many_blocks_with_empty_runs(dev):
    """More matrices than one init block of 256: empty matrices at both ends of every block and
    a whole block of empty matrices (its tile start equals the next block's), so the two-level
    lookup of a tile's matrix meets equal starts within and across blocks."""
    announce("batched 700, empty runs")
    rng = np.random.default_rng(17)
    mats = []
    for k in range(700):
        empty = k % 256 in (0, 1, 254, 255) or 256 <= k < 512 or k == 699
        if empty:
            mats.append(np.zeros((int(rng.integers(0, 3)), 0), np.uint8) if k % 2 else
                        np.zeros((0, int(rng.integers(0, 40))), np.uint8))
        else:
            m, n = int(rng.integers(1, 90)), int(rng.integers(1, 200))
            mats.append((rng.random((m, n)) < rng.uniform(0.3, 0.95)).astype(np.uint8))
    items = [(to_dev_bits(oracle.pack(a), dev), a.shape[1]) for a in mats]
    got = M.max_square_batched(items)
    for a, g in zip(mats, got):
        assert (g.side, g.row, g.col) == oracle.max_square(a), (a.shape, g)


def test_batched_empty_batch(dev):
    announce("batched count 0")
    assert M.max_square_batched([]) == []


def test_batched_large_square_serial_path(dev):
    """A square far beyond the erosion tile's certified side (the resolve pass bounds it by the
    runs of saturated tiles and takes it in one window of 33 words)."""
    announce("batched serial")
    mats = [np.ones((2100, 2050), np.uint8), W.gen_bernoulli(500, 500, 0.7, 5)]
    check_batch(mats, dev)


def test_batched_serial_flags_spread(dev):
    """Serial-pass matrices in different 64-matrix groups of a larger batch (the final kernel
    finds them by a ballot per group), run twice on one workspace (the count is cleared)."""
    announce("batched serial spread")
    mats = make_mix(6, 150)
    # 66 words per row: the resolve window of the right-most tiles outgrows one word per lane
    for k, i in enumerate((5, 70, 149)):
        big = np.ones((4200, 4200), np.uint8)
        big[4199 - 300 * k, 4199 - 7 * k] = 0
        mats[i] = big
    items = [(to_dev_bits(oracle.pack(a), dev), a.shape[1]) for a in mats]
    b = M.Batch(items)
    refs = [oracle.max_square(a) for a in mats]
    for _ in range(2):
        b.run()
        assert [(g.side, g.row, g.col) for g in b.results()] == refs


def test_batched_order_and_duplicates(dev):
    announce("batched order")
    mats = make_mix(2, 12)
    mats = mats + mats[:4]
    perm = np.random.default_rng(3).permutation(len(mats))
    check_batch([mats[i] for i in perm], dev)


def test_batched_repeat_reuses_workspace(dev):
    announce("batched repeat")
    mats = make_mix(4, 20)
    items = [(to_dev_bits(oracle.pack(a), dev), a.shape[1]) for a in mats]
    b = M.Batch(items)
    refs = [oracle.max_square(a) for a in mats]
    for _ in range(3):
        b.run()
        got = b.results()
        assert [(g.side, g.row, g.col) for g in got] == refs


# MAXSQ_GRAPH unset: the library's default (a repeated batch is captured on its second call
# and replayed after); "1": captured on the first call; "0": eager launches only.
GRAPH_MODES = [None, "1", "0"]


def _graph_mode(monkeypatch, mode):
    if mode is None:
        monkeypatch.delenv("MAXSQ_GRAPH", raising=False)
    else:
        monkeypatch.setenv("MAXSQ_GRAPH", mode)


@pytest.mark.parametrize("mode", GRAPH_MODES)
def test_batched_graph_replays(dev, monkeypatch, mode):
    """The launch sequence recorded once into a HIP graph: every replay (with eager work and
    synchronisation between replays) gives the oracle's results."""
    import torch
    announce("batched graph", mode)
    _graph_mode(monkeypatch, mode)
    mats = make_mix(5, 16)
    items = [(to_dev_bits(oracle.pack(a), dev), a.shape[1]) for a in mats]
    b = M.Batch(items)
    refs = [oracle.max_square(a) for a in mats]
    for k in range(4):
        b.out.fill_(-5)
        b.run()
        torch.cuda.synchronize()
        got = b.results()
        assert [(g.side, g.row, g.col) for g in got] == refs, "replay %d" % k
        d, n = items[k]
        single = M.max_square(d, n)       # eager work between replays
        assert (single.side, single.row, single.col) == refs[k]


@pytest.mark.parametrize("mode", [M.GRAPHS_OFF, M.GRAPHS_ON_REPEAT, M.GRAPHS_ALWAYS])
def test_batched_context_graph_modes(dev, monkeypatch, mode):
    """The per-context submission mode (no MAXSQ_GRAPH override): four calls of one batch on
    one context, each equal to the oracle."""
    import torch
    announce("batched context graph mode", mode)
    monkeypatch.delenv("MAXSQ_GRAPH", raising=False)
    mats = make_mix(9, 12)
    items = [(to_dev_bits(oracle.pack(a), dev), a.shape[1]) for a in mats]
    refs = [oracle.max_square(a) for a in mats]
    ctx = M.Context()
    try:
        M.ms_set_batched_graphs(ctx.handle, mode)
        b = M.Batch(items, ctx=ctx)
        for k in range(4):
            b.out.fill_(-6)
            b.run()
            torch.cuda.synchronize()
            assert [(g.side, g.row, g.col) for g in b.results()] == refs, "call %d" % k
        del b
    finally:
        ctx.close()


@pytest.mark.parametrize("mode", GRAPH_MODES)
def test_batched_graph_same_buffers_new_shapes(dev, monkeypatch, mode):
    """Graph mode with the descriptor buffer, count, output and workspace reused for a batch
    of different shapes: no call may replay another shape set's launch sequence."""
    import ctypes
    import torch
    announce("batched graph new shapes", mode)
    _graph_mode(monkeypatch, mode)
    sets = [make_mix(6, 10), make_mix(7, 10)]
    items = [[(to_dev_bits(oracle.pack(a), dev), a.shape[1]) for a in s] for s in sets]
    count = 10
    h = [(M._Matrix * count)() for _ in sets]
    for k in range(2):
        for i, (bits, n) in enumerate(items[k]):
            h[k][i] = M._Matrix(bits.data_ptr(), bits.size(0), n, M._ld_words(bits, n))
    ws_bytes = max(M.ms_batched_workspace_size(None, h[k], count) for k in range(2))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    d_mats = torch.empty(ctypes.sizeof(M._Matrix) * count, dtype=torch.uint8, device=dev)
    out = torch.empty((count, 3), dtype=torch.int64, device=dev)
    sp = torch.cuda.current_stream().cuda_stream
    for rep in range(3):
        for k in (0, 0, 1) if rep < 2 else (1, 0):
            raw = bytes(h[k])
            d_mats.copy_(torch.frombuffer(bytearray(raw), dtype=torch.uint8))
            out.fill_(-7)
            rc = M.ms_max_square_batched(None, h[k], d_mats.data_ptr(), count, out.data_ptr(),
                                         ws.data_ptr(), ws_bytes, sp)
            assert rc == 0
            got = [tuple(r) for r in out.cpu().tolist()]
            assert got == [oracle.max_square(a) for a in sets[k]], (rep, k)


def test_mismatched_device_descriptors_fail_every_result(dev):
    """The host and device copies of the descriptors list the same two matrices in a different
    order: the tile total agrees, the shapes per index do not.  The device must refuse the batch
    (every result -1) rather than search with the host's workspace layout."""
    import ctypes
    import torch
    announce("batched mismatched descriptors")
    a = W.gen_bernoulli(100, 200, 0.6, 21)
    b = W.gen_bernoulli(200, 100, 0.6, 22)
    da, db = to_dev_bits(oracle.pack(a), dev), to_dev_bits(oracle.pack(b), dev)
    ma = M._Matrix(da.data_ptr(), 100, 200, da.stride(0))
    mb = M._Matrix(db.data_ptr(), 200, 100, db.stride(0))
    h_mats = (M._Matrix * 2)(ma, mb)
    swapped = (M._Matrix * 2)(mb, ma)
    d_mats = torch.frombuffer(bytearray(bytes(swapped)), dtype=torch.uint8).to(dev)
    nbytes = M.ms_batched_workspace_size(None, h_mats, 2)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    out = torch.zeros((2, 3), dtype=torch.int64, device=dev)
    st = M.ms_max_square_batched(None, h_mats, d_mats.data_ptr(), 2, out.data_ptr(),
                                 ws.data_ptr(), nbytes, torch.cuda.current_stream().cuda_stream)
    assert st == 0
    assert out.cpu().tolist() == [[-1, -1, -1], [-1, -1, -1]]
    # the same call with matching copies is answered normally
    d_ok = torch.frombuffer(bytearray(bytes(h_mats)), dtype=torch.uint8).to(dev)
    st = M.ms_max_square_batched(None, h_mats, d_ok.data_ptr(), 2, out.data_ptr(),
                                 ws.data_ptr(), nbytes, torch.cuda.current_stream().cuda_stream)
    assert st == 0
    assert [tuple(r) for r in out.cpu().tolist()] == [oracle.max_square(a), oracle.max_square(b)]


# the narrow tile of the batched path: 241 owned rows, certified side 16
NARROW_TILE = (241, 16)


def _deep_row_mats(TR, KC, seed, n, cols):
    """One matrix per deep-row case (tile row 1 of a TR-row tile, squares with their right
    columns at `cols`), 0.5-dense noise around them."""
    from test_gpu_parity import _deep_rows_cases
    out = []
    for k, (name, squares) in enumerate(_deep_rows_cases(TR, KC)):
        rng = np.random.default_rng([seed, k])
        m = 3 * TR + 7
        a = (rng.random((m, n)) < 0.5).astype(np.uint8)
        for q, (off, side) in enumerate(squares):
            r1 = TR + off
            c1 = cols[q]
            side = min(side, r1 + 1, c1 + 1)
            a[r1 - side + 1:r1 + 1, c1 - side + 1:c1 + 1] = 1
        out.append((name, a))
    return out


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_batched_deep_rows(dev, variant, tmp_path):
    """The deep-row cases of the single-matrix search, every one in one batch: wide matrices on
    the variant's own tile (never narrow), and 150-column matrices on the narrow tile (the
    default tile-width rule picks it there), each result against the oracle."""
    import torch
    from test_gpu_parity import PROBE_TILES
    TR, KC = PROBE_TILES[variant]
    cases = _deep_row_mats(TR, KC, [variant, 21], 2100, (1100, 1500))
    cases += _deep_row_mats(*NARROW_TILE, [variant, 22], 150, (60, 120))
    for q in (0, 4):
        announce("batched deep rows", variant, q)
        table = os.path.join(tmp_path, "deep_%d_%d.txt" % (variant, q))
        with open(table, "w") as f:
            f.write("batched %d %d\n" % (variant, q))
        ctx = M.Context()
        try:
            M.ms_autotune_load(ctx.handle, table)
            items = [(to_dev_bits(oracle.pack(a), dev), a.shape[1]) for _, a in cases]
            b = M.Batch(items, ctx=ctx)
            got = b.run().cpu().tolist()
            torch.cuda.synchronize()
            for (name, a), g in zip(cases, got):
                assert tuple(g) == oracle.max_square(a), (variant, q, name, a.shape, g)
            del b
        finally:
            ctx.close()
