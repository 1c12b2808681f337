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


# ---- largest all-ones rectangle (the future-work extension of Section 6) ----

def max_rect(a: np.ndarray) -> tuple[int, int, int, int, int]:
    """Every rectangle checked cell by cell through a 2-D prefix sum.  Returns (area, row, col,
    height, width): the largest area; among rectangles reaching it, the bottom-right corner
    first in row-major order, then the smallest height; (0, -1, -1, 0, 0) when none."""
    a = (np.asarray(a) != 0).astype(np.int64)
    m, n = a.shape
    P = np.zeros((m + 1, n + 1), np.int64)
    P[1:, 1:] = a.cumsum(0).cumsum(1)
    best = (0, -1, -1, 0, 0)
    for i in range(m):
        for j in range(n):
            for h in range(1, i + 2):
                for w in range(j + 1, 0, -1):
                    ones = P[i + 1, j + 1] - P[i + 1 - h, j + 1] - P[i + 1, j + 1 - w] \
                        + P[i + 1 - h, j + 1 - w]
                    if ones == h * w:
                        if h * w > best[0]:
                            best = (h * w, i, j, h, w)
                        break
    return best


def rect_all_masks(m: int, n: int) -> np.ndarray:
    """Exhaustive over every m x n 0/1 matrix (A[i][j] = bit i*n + j of the mask): an array
    (2^(m*n), 5) of (area, row, col, height, width) as max_rect defines them."""
    cnt = 1 << (m * n)
    masks = np.arange(cnt, dtype=np.uint32)
    A = np.zeros((cnt, m, n), np.int64)
    for i in range(m):
        for j in range(n):
            A[:, i, j] = (masks >> (i * n + j)) & 1
    P = np.zeros((cnt, m + 1, n + 1), np.int64)
    P[:, 1:, 1:] = A.cumsum(1).cumsum(2)
    out = np.zeros((cnt, 5), np.int64)
    out[:, 1:3] = -1
    for i in range(m):
        for j in range(n):
            for h in range(1, i + 2):
                for w in range(j + 1, 0, -1):
                    ones = P[:, i + 1, j + 1] - P[:, i + 1 - h, j + 1] \
                        - P[:, i + 1, j + 1 - w] + P[:, i + 1 - h, j + 1 - w]
                    hit = (ones == h * w) & (h * w > out[:, 0])
                    out[hit] = (h * w, i, j, h, w)
    return out


def rect_area_histogram_stack(a: np.ndarray) -> int:
    """Largest all-ones rectangle area by the histogram method the paper's related work
    describes (Section 2.3): per row, the heights of the runs of ones ending there, and the
    textbook stack pass for the largest rectangle under a histogram."""
    a = np.asarray(a) != 0
    m, n = a.shape
    heights = [0] * n
    best = 0
    for i in range(m):
        for j in range(n):
            heights[j] = heights[j] + 1 if a[i, j] else 0
        stack = []  # column indices with increasing heights
        for j in range(n + 1):
            cur = heights[j] if j < n else 0
            while stack and heights[stack[-1]] >= cur:
                top = stack.pop()
                left = stack[-1] + 1 if stack else 0
                best = max(best, heights[top] * (j - left))
            stack.append(j)
    return best


# ---- largest all-ones cube of a volume (the higher-dimensional generalization of Section 6) ----

def max_cube(v: np.ndarray) -> tuple[int, int, int, int]:
    """Every cube checked through a 3-D prefix sum: (side, z, y, x) of its far corner (largest
    z, y, x), the first in (z, y, x) order among the largest; (0, -1, -1, -1) when none."""
    v = (np.asarray(v) != 0).astype(np.int64)
    D, M, N = v.shape
    P = np.zeros((D + 1, M + 1, N + 1), np.int64)
    P[1:, 1:, 1:] = v.cumsum(0).cumsum(1).cumsum(2)

    def ones(z, y, x, s):
        z0, y0, x0 = z + 1 - s, y + 1 - s, x + 1 - s
        return (P[z + 1, y + 1, x + 1] - P[z0, y + 1, x + 1] - P[z + 1, y0, x + 1]
                - P[z + 1, y + 1, x0] + P[z0, y0, x + 1] + P[z0, y + 1, x0]
                + P[z + 1, y0, x0] - P[z0, y0, x0])

    best = (0, -1, -1, -1)
    for s in range(1, min(D, M, N) + 1):
        hit = None
        for z in range(s - 1, D):
            for y in range(s - 1, M):
                for x in range(s - 1, N):
                    if ones(z, y, x, s) == s ** 3:
                        hit = (s, z, y, x)
                        break
                if hit:
                    break
            if hit:
                break
        if hit is None:
            break
        best = hit
    return best
