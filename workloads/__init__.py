"""Seeded synthetic binary-matrix generators shared by the oracle tests and the HIP path.

This module holds input generation and the packed input *encoding* only; none of the
method's arithmetic (no heights, no erosion, no dp).  Every input the tests and the
benchmark use comes from here, so both sides read the same bits.

Workloads follow the paper's experimental setup (Section 4, "Test Matrix Generation"):
uniform-random binary matrices, square, sides up to 5000, densities 0.1-0.9.  The paper
draws with mt19937 and does not say how a draw maps to a bit; here a cell is
``rng.random() < p`` with numpy's PCG64 ``default_rng(seed)``, drawn row chunk by row chunk
(a chunked draw equals a full draw because the stream is consumed in C order).

Packed encoding: row i is ``ld_words >= ceil(n/64)`` little-endian uint64 words; column j is
bit ``j & 63`` of word ``j >> 6`` (LSB first).  Padding bits beyond n are zero here, and the
consumers of packed input ignore them anyway.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "words_per_row", "pack_rows", "unpack_rows", "gen_bernoulli", "gen_bernoulli_packed",
    "gen_planted_packed", "gen_blob", "paper_grid", "paper_grid_seed", "c1", "batch_shapes",
    "gen_batch_matrix", "batch_packed", "large_packed", "LARGE", "serving_request", "CHUNK_ROWS",
    "gen_bernoulli_volume", "gen_blob_volume", "pack_volume", "VOLUMES", "volume_packed",
]

CHUNK_ROWS = 256


def words_per_row(n: int) -> int:
    return (int(n) + 63) // 64


def pack_rows(a: np.ndarray, ld_words: int | None = None) -> np.ndarray:
    """uint8/bool (m, n) -> uint64 (m, ld_words) in the packed encoding above."""
    a = np.asarray(a)
    m, n = a.shape
    w = words_per_row(n)
    ld = w if ld_words is None else int(ld_words)
    if ld < w:
        raise ValueError("ld_words < ceil(n/64)")
    out = np.zeros((m, ld * 8), dtype=np.uint8)
    if m and n:
        b = np.packbits(a != 0, axis=1, bitorder="little")
        out[:, : b.shape[1]] = b
    return out.view("<u8").reshape(m, ld)


def unpack_rows(bits: np.ndarray, n: int) -> np.ndarray:
    """Inverse of pack_rows (padding ignored)."""
    bits = np.ascontiguousarray(bits, dtype="<u8")
    m = bits.shape[0]
    if m == 0 or n == 0:
        return np.zeros((m, n), dtype=np.uint8)
    b = np.unpackbits(bits.view(np.uint8).reshape(m, -1), axis=1, bitorder="little")
    return np.ascontiguousarray(b[:, :n])


def gen_bernoulli(m: int, n: int, p: float, seed, chunk_rows: int = CHUNK_ROWS) -> np.ndarray:
    """uint8 (m, n), cell = rng.random() < p, drawn in row chunks."""
    rng = np.random.default_rng(seed)
    out = np.empty((m, n), dtype=np.uint8)
    for r in range(0, m, chunk_rows):
        rr = min(chunk_rows, m - r)
        out[r:r + rr] = rng.random((rr, n)) < p
    return out


def gen_bernoulli_packed(m: int, n: int, p: float, seed, chunk_rows: int = CHUNK_ROWS,
                         rng: np.random.Generator | None = None) -> np.ndarray:
    """Same bits as gen_bernoulli, produced directly in packed form (bounded host memory)."""
    rng = np.random.default_rng(seed) if rng is None else rng
    out = np.empty((m, words_per_row(n)), dtype=np.uint64)
    for r in range(0, m, chunk_rows):
        rr = min(chunk_rows, m - r)
        out[r:r + rr] = pack_rows(rng.random((rr, n)) < p)
    return out


def gen_planted_packed(m: int, n: int, p: float, side: int, seed, chunk_rows: int = CHUNK_ROWS):
    """Bernoulli(p) noise, then an all-ones side x side block at a position drawn from the same
    generator after the noise.  Returns (packed, r0, c0) with (r0, c0) the block's top-left."""
    rng = np.random.default_rng(seed)
    bits = gen_bernoulli_packed(m, n, p, None, chunk_rows, rng=rng)
    r0 = int(rng.integers(0, m - side + 1))
    c0 = int(rng.integers(0, n - side + 1))
    set_block_packed(bits, r0, c0, side, side)
    return bits, r0, c0


def set_block_packed(bits: np.ndarray, r0: int, c0: int, h: int, w: int) -> None:
    """Set an h x w block of ones with top-left (r0, c0) in a packed matrix, in place."""
    c1 = c0 + w
    for wd in range(c0 >> 6, (c1 + 63) >> 6):
        lo = max(c0, wd * 64) - wd * 64
        hi = min(c1, wd * 64 + 64) - wd * 64
        mask = ((1 << (hi - lo)) - 1) << lo
        bits[r0:r0 + h, wd] |= np.uint64(mask)


def gen_blob(m: int, n: int, sigma: float, percentile: float, seed) -> np.ndarray:
    """'Blob image': standard-normal noise smoothed by a Gaussian of width sigma pixels
    (reflect boundary, truncate at 4 sigma), thresholded above its given percentile."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((m, n), dtype=np.float32)
    g = gaussian_filter(g, sigma, mode="reflect", truncate=4.0)
    thr = np.percentile(g, percentile)
    return (g > thr).astype(np.uint8)


def paper_grid_seed(n: int, d: int) -> int:
    """Seed for the paper-shaped grid cell (n, p = d/10): 10*n + d (integer-safe form of
    n*10 + p*10)."""
    return 10 * int(n) + int(d)


def paper_grid(sizes=(1000, 2000, 3000, 4000, 5000), deciles=range(1, 10)):
    """[(n, d, p, seed)] for the paper-shaped grid: square n x n, p = d/10."""
    return [(n, d, d / 10.0, paper_grid_seed(n, d)) for n in sizes for d in deciles]


def c1() -> np.ndarray:
    """Single 1000 x 1000 Bernoulli(0.7) matrix from seed 0."""
    return gen_bernoulli(1000, 1000, 0.7, 0)


def batch_shapes(count: int = 10000, lo: int = 16, hi: int = 4096, seed: int = 10000):
    """Shapes and densities for the batched workload: m, n independently log-uniform in
    [lo, hi], p uniform in [0.1, 0.9]; returns int64 m, n and float64 p arrays."""
    rng = np.random.default_rng(seed)
    u = rng.random((count, 3))
    a, b = math.log(lo), math.log(hi + 1)
    m = np.floor(np.exp(a + u[:, 0] * (b - a))).astype(np.int64)
    n = np.floor(np.exp(a + u[:, 1] * (b - a))).astype(np.int64)
    m = np.clip(m, lo, hi)
    n = np.clip(n, lo, hi)
    p = 0.1 + 0.8 * u[:, 2]
    return m, n, p


def gen_batch_matrix(i: int, m: int, n: int, p: float, seed: int = 10000) -> np.ndarray:
    """Matrix i of the batched workload, packed."""
    return gen_bernoulli_packed(int(m), int(n), float(p), [seed, int(i)])


def batch_packed(count: int = 10000, threads: int = 16, seed: int = 10000):
    """The whole batched workload, packed: (list of packed matrices, m, n, p).  Matrices are
    independent streams, so a thread pool draws them in parallel with the same bits."""
    from concurrent.futures import ThreadPoolExecutor
    m, n, p = batch_shapes(count, seed=seed)
    with ThreadPoolExecutor(max(1, int(threads))) as ex:
        mats = list(ex.map(lambda i: gen_batch_matrix(i, m[i], n[i], p[i], seed), range(count)))
    return mats, m, n, p


# The large single matrices: (a) 32768^2 Bernoulli(0.9), seed 1; (b) 4096 x 262144
# Bernoulli(0.5), seed 2, with an all-ones 1500^2 block planted at a position drawn after the
# noise; (c) 16384^2 blob image, sigma 8 px, threshold at the 60th percentile, seed 3.
LARGE = {
    "c3a": {"m": 32768, "n": 32768, "p": 0.9, "seed": 1},
    "c3b": {"m": 4096, "n": 262144, "p": 0.5, "seed": 2, "side": 1500},
    "c3c": {"m": 16384, "n": 16384, "sigma": 8.0, "percentile": 60.0, "seed": 3},
}


def large_packed(name: str):
    """(packed bits, m, n, extra) for one of the LARGE matrices; extra holds the planted
    block's [row, col, side] for c3b."""
    c = LARGE[name]
    if name == "c3a":
        return gen_bernoulli_packed(c["m"], c["n"], c["p"], c["seed"]), c["m"], c["n"], {}
    if name == "c3b":
        bits, r0, c0 = gen_planted_packed(c["m"], c["n"], c["p"], c["side"], c["seed"])
        return bits, c["m"], c["n"], {"planted": [r0, c0, c["side"]]}
    a = gen_blob(c["m"], c["n"], c["sigma"], c["percentile"], c["seed"])
    return pack_rows(a), c["m"], c["n"], {}


def serving_request(k: int, lo: int = 32, hi: int = 8192, seed: int = 30001):
    """Request k of the serving pool: (packed bits, m, n, kind, params).
    Sides log-uniform in [lo, hi]; 70 % Bernoulli(p ~ U[0.1, 0.9]), 30 % blobs with
    sigma ~ U[2, 16] px and threshold percentile ~ U[40, 80]."""
    rng = np.random.default_rng([seed, int(k)])
    a, b = math.log(lo), math.log(hi + 1)
    m = int(min(hi, math.floor(math.exp(a + rng.random() * (b - a)))))
    n = int(min(hi, math.floor(math.exp(a + rng.random() * (b - a)))))
    if rng.random() < 0.7:
        p = 0.1 + 0.8 * rng.random()
        bits = gen_bernoulli_packed(m, n, p, None, rng=rng)
        return bits, m, n, "bernoulli", {"p": p}
    sigma = 2.0 + 14.0 * rng.random()
    pct = 40.0 + 40.0 * rng.random()
    sub = int(rng.integers(0, 2**31 - 1))
    a8 = gen_blob(m, n, sigma, pct, sub)
    return pack_rows(a8), m, n, "blob", {"sigma": sigma, "percentile": pct}


# ---- binary volumes (the higher-dimensional generalization the paper names as future work) ----

def gen_bernoulli_volume(D: int, M: int, N: int, p: float, seed) -> np.ndarray:
    """uint8 (D, M, N), voxels i.i.d. Bernoulli(p): ``default_rng(seed).random() < p`` drawn
    plane by plane (equal to one full draw)."""
    rng = np.random.default_rng(seed)
    out = np.empty((D, M, N), np.uint8)
    for z in range(D):
        out[z] = rng.random((M, N)) < p
    return out


def gen_blob_volume(D: int, M: int, N: int, sigma: float, percentile: float, seed) -> np.ndarray:
    """3-D 'blob' volume: standard-normal noise smoothed by a Gaussian of width sigma voxels
    (reflect boundary, truncate at 4 sigma), thresholded above its given percentile."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((D, M, N), dtype=np.float32)
    g = gaussian_filter(g, sigma, mode="reflect", truncate=4.0)
    return (g > np.percentile(g, percentile)).astype(np.uint8)


def pack_volume(v: np.ndarray, ld_words: int | None = None) -> np.ndarray:
    """uint8/bool (D, M, N) -> uint64 (D, M, ld_words): every plane packed like a matrix."""
    D, M, N = v.shape
    ld = words_per_row(N) if ld_words is None else ld_words
    out = np.zeros((D, M, max(ld, 1)), np.uint64)
    for z in range(D):
        if M and N:
            out[z] = pack_rows(v[z], ld)
    return out


# Volumes for the cube benchmark: Bernoulli volumes at the densities where cubes of a few voxels
# appear, and a blob volume whose cubes are tens of voxels wide.
VOLUMES = {
    "v256_p90": dict(D=256, M=256, N=256, kind="bernoulli", p=0.9, seed=41),
    "v512_p95": dict(D=512, M=512, N=512, kind="bernoulli", p=0.95, seed=42),
    "v256_blob": dict(D=256, M=256, N=256, kind="blob", sigma=4.0, pct=60.0, seed=43),
}


def volume_packed(name: str):
    """(packed (D, M, W) uint64, D, M, N) of a named benchmark volume."""
    c = VOLUMES[name]
    if c["kind"] == "bernoulli":
        v = gen_bernoulli_volume(c["D"], c["M"], c["N"], c["p"], c["seed"])
    else:
        v = gen_blob_volume(c["D"], c["M"], c["N"], c["sigma"], c["pct"], c["seed"])
    return pack_volume(v), c["D"], c["M"], c["N"]
