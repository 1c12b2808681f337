"""Bit-exact parity of the largest all-ones cube (HIP passes and their search, through the C
ABI) with the CPU oracle: random volumes across shapes and densities, closed forms, planted
cubes, cubes wider than a word (shifts of whole words), padding and strides, blobs."""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_2503_18974_amd as M
from gpu_util import announce

pytestmark = pytest.mark.gpu


def check(v, dev, ld_extra=0, pad_ones=False, ctx=None):
    import torch
    D, Mr, N = v.shape
    bits = W.pack_volume(v, W.words_per_row(N) + ld_extra)
    if pad_ones and N % 64:
        bits[:, :, N // 64] |= np.uint64((~((1 << (N % 64)) - 1)) & 0xFFFFFFFFFFFFFFFF)
    if ld_extra:
        bits[:, :, W.words_per_row(N):] = np.uint64(0xFFFFFFFFFFFFFFFF)
    d = torch.from_numpy(bits.view(np.int64)).to(dev)
    got = M.max_cube(d, N, ctx=ctx)
    want = oracle.max_cube(v)
    assert (got.side, got.z, got.y, got.x) == want, (got, want)
    return got


SHAPES = [(1, 1, 1), (1, 40, 50), (30, 1, 70), (12, 17, 1), (9, 33, 63), (9, 33, 64),
          (9, 33, 65), (20, 24, 200), (6, 8, 4100), (64, 64, 64)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("p", [0.6, 0.95])
def test_random_shapes(dev, shape, p):
    announce("cube random", shape, p)
    check(W.gen_bernoulli_volume(*shape, p, sum(shape) + int(p * 100)), dev)


@pytest.mark.parametrize("p", [0.0, 0.1, 0.5, 0.9, 0.99, 1.0])
def test_densities(dev, p):
    announce("cube density", p)
    check(W.gen_bernoulli_volume(40, 50, 90, p, 3), dev)


@pytest.mark.parametrize("shape", [(3, 4, 5), (70, 70, 140), (130, 131, 200)])
def test_all_ones(dev, shape):
    """All-ones: the side is the shortest extent; 130 needs shifts of whole words."""
    announce("cube ones", shape)
    got = check(np.ones(shape, np.uint8), dev)
    assert got.side == min(shape)


def test_empty_and_zero(dev):
    import torch
    announce("cube empty")
    for shape in [(0, 4, 5), (4, 0, 5), (4, 5, 0)]:
        d = torch.zeros((shape[0], shape[1], 1), dtype=torch.int64, device=dev)
        c = M.max_cube(d, shape[2])
        assert (c.side, c.z, c.y, c.x) == (0, -1, -1, -1)
    check(np.zeros((10, 20, 30), np.uint8), dev)


@pytest.mark.parametrize("side", [2, 5, 17, 66])
def test_planted(dev, side):
    announce("cube planted", side)
    rng = np.random.default_rng([side, 9])
    D, Mr, N = side + 20, side + 30, side + 150
    v = (rng.random((D, Mr, N)) < 0.5).astype(np.uint8)
    z0, y0, x0 = (int(rng.integers(1, d - side - 1)) for d in (D, Mr, N))
    v[z0:z0 + side, y0:y0 + side, x0:x0 + side] = 1
    check(v, dev)


def test_equal_cubes_first_corner(dev):
    announce("cube ties")
    v = np.zeros((30, 40, 300), np.uint8)
    for z0, y0, x0 in ((10, 5, 200), (10, 5, 20), (4, 30, 250), (20, 1, 1)):
        v[z0:z0 + 6, y0:y0 + 6, x0:x0 + 6] = 1
    check(v, dev)


def test_single_plane_stack_matches_square(dev):
    """A plane stacked k times: the cube side is min(S, k) (the plane's largest square S)."""
    announce("cube stacked plane")
    a = W.gen_bernoulli(200, 300, 0.9, 4)
    s = oracle.max_square(a)[0]
    for k in (1, s, s + 3):
        got = check(np.repeat(a[None], k, axis=0), dev)
        assert got.side == min(s, k)


def test_padding_and_strides(dev):
    announce("cube padding")
    v = W.gen_bernoulli_volume(20, 30, 130, 0.9, 5)
    check(v, dev, pad_ones=True)
    check(v, dev, ld_extra=2)


def test_blob(dev):
    announce("cube blob")
    check(W.gen_blob_volume(48, 64, 96, 3.0, 60.0, 6), dev)


def test_repeated_calls(dev):
    announce("cube repeated")
    ctx = M.Context()
    try:
        for v in (W.gen_bernoulli_volume(30, 40, 200, 0.9, 1), W.gen_bernoulli_volume(5, 6, 7, 0.8, 2),
                  np.ones((4, 4, 4), np.uint8), W.gen_bernoulli_volume(30, 40, 200, 0.9, 1)):
            check(v, dev, ctx=ctx)
    finally:
        ctx.close()


def test_benchmark_volumes(dev):
    """The benchmark's volumes (up to 512^3) against the oracle's stored results."""
    import hashlib
    import json
    import os
    import torch
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                         "oracle_configs.json")))["volumes"]
    for name in sorted(W.VOLUMES):
        announce("cube volume", name)
        bits, D, Mr, N = W.volume_packed(name)
        g = golden[name]
        assert hashlib.sha256(bits.tobytes()).hexdigest() == g["sha256_packed"]
        c = M.max_cube(torch.from_numpy(bits.view(np.int64)).to(dev), N)
        assert (c.side, c.z, c.y, c.x) == (g["side"], g["z"], g["y"], g["x"])
