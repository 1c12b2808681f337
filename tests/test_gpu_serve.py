"""Serving on the GPU: every request served in the mix (continuous batching over several
streams, under a small HBM budget) gives the same side, corner and dp map as the same request
run alone through the single-matrix calls, and as the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_2503_18974_amd as M
from paper_2503_18974_amd.serve import GpuExecutor, Server, make_requests
from gpu_util import announce

pytestmark = pytest.mark.gpu


def pool_of(count, hi):
    pool = [W.serving_request(k, hi=hi)[:3] for k in range(count)]
    # two planted squares wider than the erosion tile's certified side
    for k, s in ((0, 90), (1, 300)):
        bits, m, n = W.gen_bernoulli_packed(400, 500, 0.5, [55, k]), 400, 500
        W.set_block_packed(bits, 37, 101, s, s)
        pool.append((bits, m, n))
    return pool


def test_served_in_mix_equals_alone(dev):
    import torch
    announce("serve mix")
    pool = pool_of(30, hi=1024)
    budget = 24 << 20
    ex = GpuExecutor(budget, slots=4, max_batch=64, max_n=1024)
    pinned = [(ex.host_bits(b), m, n) for b, m, n in pool]
    reqs = make_requests(pinned, 160, rate=20000.0, map_fraction=0.3, seed=[30000, 7])
    maps = {}

    def keep(r, view):
        if view is not None:
            maps[r.rid] = view.cpu().numpy()

    st = Server(ex, budget, slots=4, max_batch=64, on_complete=keep).run(reqs)
    ex.close()
    s = st.summary()
    announce("serve mix", s)
    assert st.completed == len(reqs) and st.rejected == 0
    assert st.batches < len(reqs) and max(st.batch_sizes) > 1     # requests were batched
    assert st.peak_bytes <= budget
    alone = []
    for bits, m, n in pool:
        d = torch.from_numpy(np.ascontiguousarray(bits).view(np.int64)).to(dev)
        sq = M.max_square(d, n)
        dp, sq2 = M.square_map(d, n)
        ref = oracle.max_square_packed(bits, n)
        assert (sq.side, sq.row, sq.col) == ref == (sq2.side, sq2.row, sq2.col)
        alone.append((ref, dp.cpu().numpy()))
    for r in reqs:
        k = r.rid % len(pool)
        assert r.result == alone[k][0], (r.rid, r.m, r.n, r.result, alone[k][0])
        if r.want_map:
            assert np.array_equal(maps[r.rid], alone[k][1]), (r.rid, r.m, r.n)
    for k in {r.rid % len(pool) for r in reqs if r.want_map}:
        bits, m, n = pool[k]
        assert np.array_equal(alone[k][1], oracle.square_map_packed(bits, n)[0])
