"""The paper-shaped grid (45 square Bernoulli matrices, n = 1000..5000, p = 0.1..0.9: the sizes
and densities of Section 4's test matrices) through exactly the per-matrix call sequence the
benchmark times -- uint8 resident on the device, ms_pack_u8, ms_max_square,
ms_square_map_from_max -- with every cell of every dp map compared to the oracle's full table,
and side and corner to the stored oracle values.  Run once on one stream, eagerly, and once as
the benchmark's headline runs it: the matrices dealt over four streams with a context each,
the launches recorded into one HIP graph and replayed."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W
import paper_2503_18974_amd as M
from gpu_util import announce

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "oracle_configs.json")))["c2"]


@pytest.fixture(scope="module")
def grid(dev):
    import torch
    announce("grid", "generating 45 matrices")
    cells = W.paper_grid()
    A, B, DP = [], [], []
    for n, d, p, seed in cells:
        a = W.gen_bernoulli(n, n, p, seed)
        A.append(torch.from_numpy(a).to(dev))
        B.append(torch.full((n, W.words_per_row(n)), -1, dtype=torch.int64, device=dev))
        DP.append(torch.full((n, n), -3, dtype=torch.int32, device=dev))
    RES = torch.full((len(cells), 3), -9, dtype=torch.int64, device=dev)
    return cells, A, B, DP, RES


def calls_of(grid):
    cells, A, B, DP, RES = grid
    return [(n, A[i].data_ptr(), B[i].data_ptr(), B[i].stride(0), DP[i].data_ptr(),
             RES[i].data_ptr()) for i, (n, d, p, seed) in enumerate(cells)]


def run_calls(L, h, sp, calls):
    for (n, pa, pb, ldw, pdp, pres) in calls:
        assert L.ms_pack_u8(h, pa, n, n, n, pb, ldw, sp) == 0
        assert L.ms_max_square(h, pb, n, n, ldw, pres, sp) == 0
        assert L.ms_square_map_from_max(h, pb, n, n, ldw, pres, pdp, n, sp) == 0


def check_all(grid, tag):
    import torch
    cells, A, B, DP, RES = grid
    torch.cuda.synchronize()
    res = RES.cpu().numpy()
    for i, (n, d, p, seed) in enumerate(cells):
        announce("grid", tag, n, p)
        g = GOLDEN["%d_%d" % (n, d)]
        assert tuple(res[i]) == (g["side"], g["row"], g["col"]), (n, d, res[i], g)
        a = A[i].cpu().numpy()
        assert np.array_equal(B[i].cpu().numpy().view(np.uint64), oracle.pack(a)), (n, d)
        ref_dp, ref = oracle.square_map(a)
        assert ref == (g["side"], g["row"], g["col"])
        got = DP[i].cpu().numpy()
        if not np.array_equal(got, ref_dp):
            bad = np.argwhere(got != ref_dp)[0]
            raise AssertionError("%s: %dx%d p=%.1f map differs at %s: %d vs %d" % (
                tag, n, n, p, tuple(bad), got[tuple(bad)], ref_dp[tuple(bad)]))


def reset(grid):
    cells, A, B, DP, RES = grid
    for b in B:
        b.fill_(-1)
    for dp in DP:
        dp.fill_(-3)
    RES.fill_(-9)


def test_grid_single_stream_eager(dev, grid):
    import torch
    announce("grid", "single stream")
    reset(grid)
    ctx = M.Context()
    try:
        run_calls(M.lib(), ctx.handle, torch.cuda.current_stream().cuda_stream, calls_of(grid))
        check_all(grid, "single stream")
    finally:
        ctx.close()


def test_grid_four_streams_graph_replay(dev, grid):
    """Largest matrices first to the least-loaded of four streams, recorded once as one graph
    (side streams fork from and join the capturing stream), replayed twice with the outputs
    cleared in between."""
    import torch
    announce("grid", "four streams, graph")
    L = M.lib()
    calls = calls_of(grid)
    nst = 4
    streams = [torch.cuda.Stream(device=dev) for _ in range(nst)]
    ctxs = [M.Context() for _ in range(nst)]
    try:
        load = [0] * nst
        lanes = [[] for _ in range(nst)]
        for i in sorted(range(len(calls)), key=lambda k: -calls[k][0]):
            s = min(range(nst), key=lambda k: load[k])
            load[s] += calls[i][0] ** 2
            lanes[s].append(calls[i])

        def mstep():
            for s in range(nst):
                run_calls(L, ctxs[s].handle, streams[s].cuda_stream, lanes[s])

        # eager once (allocates every context's scratch outside the capture)
        mstep()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            cs = torch.cuda.current_stream()
            for st in streams:
                st.wait_stream(cs)
            mstep()
            for st in streams:
                cs.wait_stream(st)
        for rep in range(2):
            reset(grid)
            torch.cuda.synchronize()
            g.replay()
            check_all(grid, "graph replay %d" % rep)
        del g
    finally:
        for c in ctxs:
            c.close()


def test_grid_graph_per_stream(dev, grid):
    """The headline submission: the same four lanes, each recorded as a graph of its own on its
    stream and replayed there; three replays, the outputs cleared and an eager step run
    between them."""
    import torch
    announce("grid", "a graph per stream")
    L = M.lib()
    calls = calls_of(grid)
    nst = 4
    streams = [torch.cuda.Stream(device=dev) for _ in range(nst)]
    ctxs = [M.Context() for _ in range(nst)]
    try:
        load = [0] * nst
        lanes = [[] for _ in range(nst)]
        for i in sorted(range(len(calls)), key=lambda k: -calls[k][0]):
            s = min(range(nst), key=lambda k: load[k])
            load[s] += calls[i][0] ** 2
            lanes[s].append(calls[i])
        for s in range(nst):  # eager once: every context's scratch allocated outside a capture
            run_calls(L, ctxs[s].handle, streams[s].cuda_stream, lanes[s])
        torch.cuda.synchronize()
        graphs = []
        for s in range(nst):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=streams[s]):
                run_calls(L, ctxs[s].handle, streams[s].cuda_stream, lanes[s])
            graphs.append(g)
        for rep in range(3):
            reset(grid)
            torch.cuda.synchronize()
            for s in range(nst):
                with torch.cuda.stream(streams[s]):
                    graphs[s].replay()
            check_all(grid, "graph per stream, replay %d" % rep)
            reset(grid)
            torch.cuda.synchronize()
            for s in range(nst):
                run_calls(L, ctxs[s].handle, streams[s].cuda_stream, lanes[s])
            check_all(grid, "eager between replays %d" % rep)
        del graphs
    finally:
        for c in ctxs:
            c.close()


def test_grid_streams_scratch_grows_mid_run(dev, grid):
    """Fresh contexts on four streams, each stream's smallest matrices first: every context
    grows its scratch partway through the run while the other streams are busy.  The grown
    scratch's header must be zeroed in order on the call's own stream; zeroed on the null
    stream, it was once cleared after the probe had pushed its keys (right side, later corner)."""
    import torch
    announce("grid", "four streams, scratch growing mid-run")
    L = M.lib()
    calls = calls_of(grid)
    nst = 4
    streams = [torch.cuda.Stream(device=dev) for _ in range(nst)]
    ctxs = [M.Context() for _ in range(nst)]
    try:
        load = [0] * nst
        lanes = [[] for _ in range(nst)]
        for i in sorted(range(len(calls)), key=lambda k: -calls[k][0]):
            s = min(range(nst), key=lambda k: load[k])
            load[s] += calls[i][0] ** 2
            lanes[s].append(calls[i])
        lanes = [lst[::-1] for lst in lanes]  # smallest first: the scratch grows as sizes rise
        reset(grid)
        torch.cuda.synchronize()
        for s in range(nst):
            run_calls(L, ctxs[s].handle, streams[s].cuda_stream, lanes[s])
        check_all(grid, "scratch growing mid-run")
    finally:
        for c in ctxs:
            c.close()
