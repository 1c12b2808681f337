"""Brute-force enumeration of all-ones squares -- TEST INFRASTRUCTURE (pins the oracle).

Straight from the problem statement (Section 1: the largest contiguous square submatrix made
entirely of ones), with no recurrence: every candidate square is checked cell by cell, or,
for exhaustive tiny shapes, as a bit mask over all 2^(m*n) matrices at once.
"""
from __future__ import annotations

import numpy as np


def square_all_ones(a: np.ndarray, i: int, j: int, s: int) -> bool:
    """Is the s x s square with bottom-right corner (i, j) inside A and all ones?"""
    if s <= 0 or i - s + 1 < 0 or j - s + 1 < 0:
        return False
    return bool(np.all(a[i - s + 1:i + 1, j - s + 1:j + 1] != 0))


def cell_side(a: np.ndarray, i: int, j: int) -> int:
    """Largest s such that the s x s square ending at (i, j) is all ones (0 if none)."""
    s = 0
    while square_all_ones(a, i, j, s + 1):
        s += 1
    return s


def side_map(a: np.ndarray) -> np.ndarray:
    m, n = a.shape
    out = np.zeros((m, n), np.int32)
    for i in range(m):
        for j in range(n):
            out[i, j] = cell_side(a, i, j)
    return out


def max_square(a: np.ndarray) -> tuple[int, int, int]:
    """(S, row, col): largest side, and the first bottom-right corner in row-major order."""
    a = np.asarray(a)
    m, n = a.shape
    best = 0
    for s in range(1, min(m, n) + 1):
        if any(square_all_ones(a, i, j, s) for i in range(s - 1, m) for j in range(s - 1, n)):
            best = s
        else:
            break
    if best == 0:
        return 0, -1, -1
    for i in range(m):
        for j in range(n):
            if square_all_ones(a, i, j, best):
                return best, i, j
    raise AssertionError("unreachable")


def all_masks(m: int, n: int):
    """Exhaustive over every m x n 0/1 matrix (A[i][j] = bit i*n + j of the mask).
    Returns (side, corner) arrays indexed by mask; corner = i*n + j or -1."""
    cnt = 1 << (m * n)
    masks = np.arange(cnt, dtype=np.uint32)
    side = np.zeros(cnt, np.int64)
    corner = np.full(cnt, -1, np.int64)
    for s in range(1, min(m, n) + 1):
        first = np.full(cnt, -1, np.int64)
        # visit bottom-right corners in reverse row-major order so the first one wins
        for i in reversed(range(s - 1, m)):
            for j in reversed(range(s - 1, n)):
                sq = 0
                for r in range(i - s + 1, i + 1):
                    for c in range(j - s + 1, j + 1):
                        sq |= 1 << (r * n + c)
                sq = np.uint32(sq)
                hit = (masks & sq) == sq
                first[hit] = i * n + j
        has = first >= 0
        side[has] = s
        corner[has] = first[has]
    return side, corner
