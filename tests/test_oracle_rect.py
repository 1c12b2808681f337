"""Pins of the oracle's largest all-ones rectangle (CPU only): brute force over every
rectangle, the textbook histogram-and-stack method, closed forms, invariants and the
tie-break."""
import numpy as np
import pytest

import oracle
from oracle import brute


def _mask_matrix(mask, m, n):
    return np.array([[(mask >> (i * n + j)) & 1 for j in range(n)] for i in range(m)], np.uint8)


@pytest.mark.parametrize("m,n", [(1, 1), (1, 5), (5, 1), (2, 2), (2, 5), (3, 3), (3, 4),
                                 (4, 3), (2, 7), (4, 4)])
def test_exhaustive_against_brute(m, n):
    want = brute.rect_all_masks(m, n)
    for mask in range(1 << (m * n)):
        a = _mask_matrix(mask, m, n)
        got = oracle.max_rect(a)
        assert got == tuple(int(x) for x in want[mask]), (mask, got, want[mask])


def test_random_small_against_brute():
    rng = np.random.default_rng(5)
    for _ in range(150):
        m, n = int(rng.integers(1, 9)), int(rng.integers(1, 10))
        a = (rng.random((m, n)) < rng.choice([0.3, 0.6, 0.85])).astype(np.uint8)
        assert oracle.max_rect(a) == brute.max_rect(a), a


@pytest.mark.parametrize("p", [0.2, 0.5, 0.8, 0.95])
def test_area_matches_histogram_stack(p):
    """The paper's related-work method (per-row histograms, stack pass) gives the same area."""
    rng = np.random.default_rng(int(p * 100))
    for _ in range(6):
        m, n = int(rng.integers(20, 70)), int(rng.integers(20, 90))
        a = (rng.random((m, n)) < p).astype(np.uint8)
        assert oracle.max_rect(a)[0] == brute.rect_area_histogram_stack(a)


@pytest.mark.parametrize("m,n", [(1, 1), (1, 9), (7, 1), (5, 8), (13, 4)])
def test_all_ones(m, n):
    assert oracle.max_rect(np.ones((m, n), np.uint8)) == (m * n, m - 1, n - 1, m, n)


def test_all_zeros_and_empty():
    assert oracle.max_rect(np.zeros((6, 9), np.uint8)) == (0, -1, -1, 0, 0)
    assert oracle.max_rect(np.zeros((0, 4), np.uint8)) == (0, -1, -1, 0, 0)
    assert oracle.max_rect(np.zeros((4, 0), np.uint8)) == (0, -1, -1, 0, 0)


@pytest.mark.parametrize("phase", [0, 1])
def test_checkerboard(phase):
    i, j = np.indices((7, 9))
    a = ((i + j + phase) % 2 == 0).astype(np.uint8)
    assert oracle.max_rect(a) == (1, 0, phase, 1, 1)


def test_single_row_and_column():
    a = np.zeros((6, 10), np.uint8)
    a[3, :] = 1
    assert oracle.max_rect(a) == (10, 3, 9, 1, 10)
    b = np.zeros((6, 10), np.uint8)
    b[:, 4] = 1
    assert oracle.max_rect(b) == (6, 5, 4, 6, 1)


@pytest.mark.parametrize("h,w", [(7, 13), (20, 3), (1, 40), (33, 1)])
def test_planted_rectangle_with_border(h, w):
    """A rectangle with a zero border in sparse noise, larger than any noise rectangle."""
    rng = np.random.default_rng([h, w])
    m, n = 120, 150
    a = (rng.random((m, n)) < 0.05).astype(np.uint8)
    r0, c0 = int(rng.integers(1, m - h - 1)), int(rng.integers(1, n - w - 1))
    a[r0 - 1:r0 + h + 1, c0 - 1:c0 + w + 1] = 0
    a[r0:r0 + h, c0:c0 + w] = 1
    assert brute.rect_area_histogram_stack(a) == h * w
    assert oracle.max_rect(a) == (h * w, r0 + h - 1, c0 + w - 1, h, w)


def test_tie_same_corner_takes_smaller_height():
    """3x3 ones minus its top-left cell: a 2x3 and a 3x2 rectangle share the corner (2, 2)."""
    a = np.ones((3, 3), np.uint8)
    a[0, 0] = 0
    assert oracle.max_rect(a) == (6, 2, 2, 2, 3)


def test_tie_takes_first_corner():
    a = np.zeros((8, 12), np.uint8)
    a[5:7, 1:4] = 1     # 2 x 3, corner (6, 3)
    a[1:4, 8:10] = 1    # 3 x 2, corner (3, 9): earlier row
    assert oracle.max_rect(a) == (6, 3, 9, 3, 2)


def test_packed_reader_and_padding():
    rng = np.random.default_rng(9)
    a = (rng.random((40, 130)) < 0.7).astype(np.uint8)
    bits = oracle.pack(a)
    bits[:, -1] |= np.uint64(0xFFFFFFFFFFFFFFFF) << np.uint64(130 - 128)
    assert oracle.max_rect_packed(bits, 130) == oracle.max_rect(a)


def test_invariants():
    rng = np.random.default_rng(11)
    for _ in range(25):
        m, n = int(rng.integers(5, 40)), int(rng.integers(5, 40))
        a = (rng.random((m, n)) < rng.choice([0.5, 0.8, 0.9])).astype(np.uint8)
        area = oracle.max_rect(a)[0]
        # transposition keeps the area; a square is a rectangle; so is any row run
        assert oracle.max_rect(a.T.copy())[0] == area
        assert area >= oracle.max_square(a)[0] ** 2
        runs = max((len(s) for row in a for s in "".join(map(str, row)).split("0")), default=0)
        assert area >= runs
        # setting bits never shrinks the largest rectangle
        b = a.copy()
        b[rng.random((m, n)) < 0.1] = 1
        assert oracle.max_rect(b)[0] >= area
        # the reported rectangle is all ones and has the reported area
        ar, r, c, h, w = oracle.max_rect(a)
        assert h * w == ar and a[r - h + 1:r + 1, c - w + 1:c + 1].all()


# ---- planted mistakes in copies of the rectangle oracle must fail the pins ----
import ctypes  # noqa: E402
import os  # noqa: E402
import subprocess  # noqa: E402

RECT_MUTANTS = {
    "height_off_by_one": ("if (h <= H[j] && h * W[h] > res[0]) {",
                          "if (h < H[j] && h * W[h] > res[0]) {"),
    "last_not_first_tie": ("if (h <= H[j] && h * W[h] > res[0]) {",
                           "if (h <= H[j] && h * W[h] >= res[0] && W[h]) {"),
    "width_strict": ("W[h] = H[j] >= h ? W[h] + 1 : 0;", "W[h] = H[j] > h ? W[h] + 1 : 0;"),
    "height_not_reset": ("H[j] = cell(r, i, j) ? H[j] + 1 : 0;",
                         "H[j] = cell(r, i, j) ? H[j] + 1 : H[j];"),
}


def _rect_pins_pass() -> bool:
    for m, n in [(3, 3), (2, 4)]:
        want = brute.rect_all_masks(m, n)
        for mask in range(1 << (m * n)):
            if oracle.max_rect(_mask_matrix(mask, m, n)) != tuple(int(x) for x in want[mask]):
                return False
    a = np.ones((3, 3), np.uint8)
    a[0, 0] = 0
    if oracle.max_rect(a) != (6, 2, 2, 2, 3):
        return False
    rng = np.random.default_rng(3)
    for _ in range(20):
        a = (rng.random((12, 15)) < 0.8).astype(np.uint8)
        if oracle.max_rect(a) != brute.max_rect(a):
            return False
    return True


@pytest.mark.parametrize("name", sorted(RECT_MUTANTS))
def test_rect_mutant_is_caught(name, tmp_path):
    old, new = RECT_MUTANTS[name]
    src = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")
    text = open(src).read()
    assert text.count(old) == 1, name
    (tmp_path / "m.c").write_text(text.replace(old, new))
    so = str(tmp_path / "m.so")
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", str(tmp_path / "m.c"),
                           "-o", so])
    saved, real = oracle._lib, oracle._LIB
    try:
        oracle._lib = None
        oracle._LIB = so
        oracle.lib()
        assert not _rect_pins_pass(), "planted mistake %s not caught" % name
    finally:
        oracle._lib, oracle._LIB = saved, real
    assert _rect_pins_pass()
