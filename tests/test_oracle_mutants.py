"""Plant mistakes in copies of the oracle (CPU only) and check that the pins catch each one:
a dropped term, a wrong index, a reversed bit order, a wrong tie-break, a transposed operand.
The real oracle is never modified."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import brute

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "dropped_diag": ("cur[j] = 1 + min3(up, left, diag);", "cur[j] = 1 + min3(up, left, left);"),
    "wrong_diag_index": ("? prev[j - 1] : 0;", "? prev[j] : 0;"),
    "last_not_first_corner": ("if (row[j] > res[0]) {", "if (row[j] >= res[0] && row[j]) {"),
    "reversed_bit_order": ("return (int)((word >> (j % 64)) & 1u);",
                           "return (int)((word >> (63 - j % 64)) & 1u);"),
    "transposed_operand": ("return a[i * ld + j] != 0;", "return a[j * ld + i] != 0;"),
    "masks_dropped_up": ("int32_t up = i > 0 ? dp[k - n] : 0;", "int32_t up = 99;"),
}


def _build(tmp_path, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, name
    src = tmp_path / (name + ".c")
    src.write_text(text.replace(old, new))
    so = tmp_path / (name + ".so")
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", str(src), "-o", str(so)])
    return str(so)


def _pins_pass() -> bool:
    """A quick subset of the pin battery; False as soon as one pin fails."""
    rng = np.random.default_rng(123)
    # exhaustive 3x3 and 3x4 against brute force
    for m, n in [(3, 3), (3, 4)]:
        so, co = oracle.all_masks(m, n)
        sb, cb = brute.all_masks(m, n)
        if not (np.array_equal(so, sb) and np.array_equal(co, cb)):
            return False
    # per-cell map against brute force on random square and non-square inputs
    for _ in range(40):
        m = n = int(rng.integers(2, 12))
        a = (rng.random((m, n)) < 0.8).astype(np.uint8)
        dp, res = oracle.square_map(a)
        if not np.array_equal(dp, brute.side_map(a)) or res != brute.max_square(a):
            return False
    # bit-order pin of the packed reader
    bits = np.zeros((1, 3), np.uint64)
    bits[0, 1] = np.uint64(2)
    if oracle.max_square_packed(bits, 130) != (1, 0, 65):
        return False
    return True


@pytest.fixture
def swap_lib():
    saved = oracle._lib

    def use(path):
        L = ctypes.CDLL(path)
        oracle._lib = None
        real = oracle._LIB
        try:
            oracle._LIB = path
            oracle.lib()
        finally:
            oracle._LIB = real
        return L

    yield use
    oracle._lib = saved


def test_real_oracle_passes_battery():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, swap_lib):
    old, new = MUTANTS[name]
    swap_lib(_build(tmp_path, name, old, new))
    assert not _pins_pass(), "planted mistake %s not caught" % name
