"""The autotuner on the GPU: tuning picks a listed candidate, tuned calls stay bit-exact with
the oracle, and tables survive a save/load round trip (batched choice included)."""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_2503_18974_amd as M
from gpu_util import announce, to_dev_bits

pytestmark = pytest.mark.gpu


def test_autotune_single_matrix_and_table(dev, tmp_path):
    import torch
    announce("autotune single")
    m, n = 1500, 1700
    a = W.gen_bernoulli(m, n, 0.85, 11)
    d = to_dev_bits(oracle.pack(a), dev)
    ctx = M.Context()
    dp = torch.empty((m, n), dtype=torch.int32, device=dev)
    M.ms_autotune(ctx.handle, d.data_ptr(), m, n, d.stride(0), dp.data_ptr(), n,
                  torch.cuda.current_stream().cuda_stream)
    cfg = M.ms_get_config(ctx.handle, m, n)
    assert cfg in [M.ms_candidate(i) for i in range(M.ms_num_candidates())]
    ref_dp, ref = oracle.square_map(a)
    sq = M.max_square(d, n, ctx=ctx)
    dp2, sq2 = M.square_map(d, n, ctx=ctx)
    assert (sq.side, sq.row, sq.col) == ref == (sq2.side, sq2.row, sq2.col)
    np.testing.assert_array_equal(dp2.cpu().numpy(), ref_dp)
    path = str(tmp_path / "table.txt")
    M.ms_autotune_save(ctx.handle, path)
    ctx2 = M.Context()
    M.ms_autotune_load(ctx2.handle, path)
    assert M.ms_get_config(ctx2.handle, m, n) == cfg
    bad = tmp_path / "bad.txt"
    for text in ("1 9 4 64\n",        # probe variant out of range
                 "batched 1 3\n",     # tile-width weight not among the tuned ones
                 "batched 5 4\n"):    # batched probe variant out of range
        bad.write_text(text)
        with pytest.raises(M.MaxsqError):
            M.ms_autotune_load(ctx2.handle, str(bad))
    assert M.ms_get_config(ctx2.handle, m, n) == cfg   # a rejected table changes nothing
    ctx.close()
    ctx2.close()


def test_autotune_batched(dev, tmp_path):
    announce("autotune batched")
    rng = np.random.default_rng(5)
    mats = []
    for k in range(30):
        mm, nn = int(rng.integers(16, 900)), int(rng.integers(16, 900))
        x = (rng.random((mm, nn)) < rng.uniform(0.3, 0.95)).astype(np.uint8)
        if k % 5 == 0:
            s = min(mm, nn, 40 + k)
            x[:s, :s] = 1
        mats.append(x)
    items = [(to_dev_bits(oracle.pack(x), dev), x.shape[1]) for x in mats]
    refs = [oracle.max_square(x) for x in mats]
    ctx = M.Context()
    b = M.Batch(items, ctx=ctx)
    b.autotune()
    assert [(s.side, s.row, s.col) for s in b.results()] == refs
    b.out.fill_(-3)
    b.run()
    assert [(s.side, s.row, s.col) for s in b.results()] == refs
    path = str(tmp_path / "table.txt")
    M.ms_autotune_save(ctx.handle, path)
    batched = [line.split() for line in open(path) if line.startswith("batched ")]
    assert len(batched) == 1 and len(batched[0]) == 3          # variant and tile-width weight
    assert int(batched[0][1]) in (0, 1, 2, 3) and int(batched[0][2]) in (4, 0, 2, 8)
    ctx2 = M.Context()
    M.ms_autotune_load(ctx2.handle, path)
    b2 = M.Batch(items, ctx=ctx2)
    b2.run()
    assert [(s.side, s.row, s.col) for s in b2.results()] == refs
    ctx.close()
    ctx2.close()
