"""Probability window for the largest all-ones square of an i.i.d. Bernoulli(p) matrix --
TEST INFRASTRUCTURE (a statistical pin on the oracle).

Section 2.2 of the paper cites Sun and Nobel's concentration s(n) = 2 log_b n - 2 log_b log_b n
+ C, b = 1/p.  That scaling is for square submatrices over arbitrary (non-contiguous) row and
column sets, and its constant C is not given, so it cannot pin a contiguous square.  For a
contiguous square the two elementary bounds below are rigorous and tight enough:

* union bound over the (m-k+1)(n-k+1) positions:  P(S >= k) <= (m-k+1)(n-k+1) p^(k^2);
* floor(m/k) * floor(n/k) disjoint k x k tiles are independent: P(S < k) <= (1 - p^(k^2))^tiles.

``window(m, n, p, alpha)`` returns [lo, hi] with P(S < lo) <= alpha and P(S > hi) <= alpha.
``sun_nobel_shape`` is kept only to show the non-contiguous scale is far above (an upper shape).
"""
from __future__ import annotations

import math


def _log_p_ge(m: int, n: int, p: float, k: int) -> float:
    if k > min(m, n):
        return -math.inf
    if p >= 1.0:
        return 0.0
    if p <= 0.0:
        return -math.inf
    return math.log((m - k + 1) * (n - k + 1)) + k * k * math.log(p)


def _log_p_lt(m: int, n: int, p: float, k: int) -> float:
    tiles = (m // k) * (n // k)
    if tiles == 0:
        return 0.0
    q = p ** (k * k)
    if q >= 1.0:
        return -math.inf
    return tiles * math.log1p(-q)


def window(m: int, n: int, p: float, alpha: float = 1e-6) -> tuple[int, int]:
    la = math.log(alpha)
    hi = min(m, n)
    for k in range(1, min(m, n) + 1):
        if _log_p_ge(m, n, p, k) <= la:
            hi = k - 1
            break
    lo = 0
    for k in range(1, min(m, n) + 1):
        if _log_p_lt(m, n, p, k) <= la:
            lo = k
        else:
            break
    return lo, hi


def sun_nobel_shape(n: int, p: float) -> float:
    """2 log_b n - 2 log_b log_b n with b = 1/p (constant C omitted)."""
    b = 1.0 / p
    lb = math.log(n) / math.log(b)
    return 2.0 * lb - 2.0 * math.log(lb) / math.log(b)
