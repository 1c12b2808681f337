"""Helpers shared by the GPU tests: move seeded numpy inputs to the device and compare the
HIP path with the oracle."""
import numpy as np


def to_dev_bits(bits_u64: np.ndarray, device, ld_words=None, pad_fill=0):
    """numpy uint64 (m, w) -> int64 CUDA tensor (m, ld_words) with padding words = pad_fill."""
    import torch
    m, w = bits_u64.shape
    ld = w if ld_words is None else ld_words
    host = np.full((m, max(ld, 1)), np.uint64(pad_fill), dtype=np.uint64)
    host[:, :w] = bits_u64
    return torch.from_numpy(host.view(np.int64)).to(device)


def set_padding_bits(bits_u64: np.ndarray, n: int) -> np.ndarray:
    """Copy with every padding bit (columns >= n in the last word) set to one."""
    out = bits_u64.copy()
    if n % 64 and out.shape[0]:
        out[:, n // 64] |= np.uint64((~((1 << (n % 64)) - 1)) & 0xFFFFFFFFFFFFFFFF)
    return out


def announce(*what):
    print("[gpu-case]", *what, flush=True)
