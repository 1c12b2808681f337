"""The allocation-free search (ms_max_square_noalloc) through the C ABI: the same results as
ms_max_square and the oracle on consecutive calls that share the library's fixed scratch (the
second call smaller than the first), its size limits, and its required context."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_2503_18974_amd as M
from gpu_util import announce, set_padding_bits, to_dev_bits

pytestmark = pytest.mark.gpu

WORKSPACE_TOO_SMALL = 2
INVALID = 1


def planted(m, n, p, side, seed):
    a = W.gen_bernoulli(m, n, p, seed)
    rng = np.random.default_rng(seed + 1)
    r0, c0 = int(rng.integers(0, m - side + 1)), int(rng.integers(0, n - side + 1))
    a[r0:r0 + side, c0:c0 + side] = 1
    return a


def noalloc(ctx, bits, n, stream):
    out = torch.full((3,), -7, dtype=torch.int64, device=bits.device)
    m = bits.size(0)
    ldw = bits.stride(0) if (m and n) else max(M.words_per_row(n), 1)
    st = M.ms_max_square_noalloc(ctx.handle, bits.data_ptr() if bits.numel() else None, m, n,
                                 ldw, out.data_ptr(), stream.cuda_stream)
    assert st == 0, M.lib().ms_status_string(st)
    return out


def plain(ctx, bits, n, stream):
    out = torch.full((3,), -7, dtype=torch.int64, device=bits.device)
    m = bits.size(0)
    ldw = bits.stride(0) if (m and n) else max(M.words_per_row(n), 1)
    st = M.ms_max_square(ctx.handle, bits.data_ptr() if bits.numel() else None, m, n, ldw,
                         out.data_ptr(), stream.cuda_stream)
    assert st == 0, M.lib().ms_status_string(st)
    return out


def run_sequence(dev, mats):
    """Each matrix through the allocation-free call and through ms_max_square, in order, on
    one stream; every result against the other and the oracle."""
    stream = torch.cuda.current_stream()
    with M.Context() as c_free, M.Context() as c_plain:
        got = []
        for a in mats:
            announce("noalloc", a.shape)
            n = a.shape[1]
            bits = to_dev_bits(set_padding_bits(oracle.pack(a), n), dev)  # padding ignored
            r1 = noalloc(c_free, bits, n, stream)
            r2 = plain(c_plain, bits, n, stream)
            got.append((a, r1, r2))
        torch.cuda.synchronize()
        for a, r1, r2 in got:
            ref = oracle.max_square(a)
            assert tuple(r1.cpu().tolist()) == ref, (a.shape, r1, ref)
            assert tuple(r2.cpu().tolist()) == ref, (a.shape, r2, ref)


def test_two_calls_second_smaller(dev):
    """A large matrix with saturated probe tiles (resolve pass), then a smaller one."""
    run_sequence(dev, [planted(2000, 3000, 0.8, 150, 11), W.gen_bernoulli(300, 700, 0.7, 12)])


def test_sequence_of_kinds(dev):
    """Search-only, saturated, serial-pass, empty and tiny matrices back to back: each call
    starts from the state the previous one left in the shared array."""
    mats = [W.gen_bernoulli(1000, 1000, 0.7, 0),
            np.ones((3300, 3400), np.uint8),        # square wider than the resolve window
            np.zeros((0, 5), np.uint8),
            planted(700, 900, 0.5, 40, 13),
            np.ones((1, 1), np.uint8),
            np.zeros((37, 65), np.uint8),
            W.gen_bernoulli(129, 4097, 0.9, 14)]
    run_sequence(dev, mats)


def test_limits_and_context(dev):
    """Beyond the fixed scratch: MS_ERR_WORKSPACE_TOO_SMALL before any launch; no context:
    invalid argument."""
    announce("noalloc limits")
    L = M.lib()
    buf = ctypes.create_string_buffer(24)
    p = ctypes.addressof(buf)  # never dereferenced: these calls return before any HIP call
    with M.Context() as c:
        # a row of 262145 columns needs 4097 words of serial state
        assert L.ms_max_square_noalloc(c.handle, p, 1, 262145, 4097, p, None) == \
            WORKSPACE_TOO_SMALL
        # more than 2^21 probe tiles (49-row tiles of one word each)
        m = (1 << 21) * 49 + 1
        assert L.ms_max_square_noalloc(c.handle, p, m, 64, 1, p, None) == WORKSPACE_TOO_SMALL
        assert L.ms_max_square_noalloc(c.handle, p, 5, 5, 1, None, None) == INVALID
    assert L.ms_max_square_noalloc(None, p, 5, 5, 1, p, None) == INVALID
