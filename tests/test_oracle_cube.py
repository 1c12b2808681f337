"""Pins of the oracle's largest all-ones cube (CPU only): brute force over every cube, the
reduction to the plane case, the characterisation by ANDs of consecutive planes, closed forms
and invariants."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import brute


@pytest.mark.parametrize("shape", [(2, 2, 2), (2, 2, 3), (3, 2, 2), (2, 3, 2), (1, 3, 4)])
def test_exhaustive_against_brute(shape):
    D, M, N = shape
    cells = D * M * N
    for mask in range(1 << cells):
        v = np.array([(mask >> k) & 1 for k in range(cells)], np.uint8).reshape(shape)
        assert oracle.max_cube(v) == brute.max_cube(v), (mask, shape)


def test_random_against_brute():
    rng = np.random.default_rng(21)
    for _ in range(60):
        shape = tuple(int(x) for x in rng.integers(1, 8, 3))
        v = (rng.random(shape) < rng.choice([0.5, 0.8, 0.95])).astype(np.uint8)
        assert oracle.max_cube(v) == brute.max_cube(v), shape


def test_single_plane_is_the_square():
    """One plane: cubes are 1 x 1 x 1, and stacking a plane k times gives its largest square
    capped at k."""
    rng = np.random.default_rng(3)
    a = (rng.random((40, 50)) < 0.8).astype(np.uint8)
    s, r, c = oracle.max_square(a)
    assert oracle.max_cube(a[None]) == (1, 0, *divmod(int(np.flatnonzero(a)[0]), 50))
    dp, _ = oracle.square_map(a)
    for k in (1, 2, 3, s, s + 2):
        v = np.repeat(a[None], k, axis=0)
        side = min(s, k)
        # the first far corner: plane side - 1, the plane's first cell with a square >= side
        first = int(np.flatnonzero(dp.ravel() >= side)[0])
        assert oracle.max_cube(v) == (side, side - 1, first // 50, first % 50)
        if k > s:
            assert first == r * 50 + c


def _plane_and_characterisation(v):
    """S = max{k : some k consecutive planes AND to a plane holding a k x k square}."""
    D = v.shape[0]
    best = 0
    for k in range(1, D + 1):
        ok = False
        for z in range(k - 1, D):
            plane = np.logical_and.reduce(v[z - k + 1:z + 1], axis=0).astype(np.uint8)
            if oracle.max_square(plane)[0] >= k:
                ok = True
                break
        if not ok:
            break
        best = k
    return best


def test_plane_and_characterisation():
    rng = np.random.default_rng(5)
    for _ in range(25):
        shape = (int(rng.integers(3, 12)), int(rng.integers(5, 30)), int(rng.integers(5, 90)))
        v = (rng.random(shape) < rng.choice([0.7, 0.9, 0.97])).astype(np.uint8)
        assert oracle.max_cube(v)[0] == _plane_and_characterisation(v), shape


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 4, 5), (6, 2, 9), (5, 5, 5), (7, 70, 3)])
def test_all_ones(shape):
    s = min(shape)
    assert oracle.max_cube(np.ones(shape, np.uint8)) == (s, s - 1, s - 1, s - 1)


def test_zeros_and_empty():
    assert oracle.max_cube(np.zeros((3, 4, 5), np.uint8)) == (0, -1, -1, -1)
    for shape in [(0, 3, 3), (3, 0, 3), (3, 3, 0)]:
        assert oracle.max_cube(np.zeros(shape, np.uint8)) == (0, -1, -1, -1)


def test_checkerboard():
    z, y, x = np.indices((5, 6, 7))
    v = ((z + y + x) % 2 == 1).astype(np.uint8)
    assert oracle.max_cube(v) == (1, 0, 0, 1)


@pytest.mark.parametrize("side", [2, 4, 7])
def test_planted_cube_with_border(side):
    rng = np.random.default_rng(side)
    D, M, N = 20, 30, 140
    v = (rng.random((D, M, N)) < 0.1).astype(np.uint8)
    z0, y0, x0 = (int(rng.integers(1, d - side - 1)) for d in (D, M, N))
    v[z0 - 1:z0 + side + 1, y0 - 1:y0 + side + 1, x0 - 1:x0 + side + 1] = 0
    v[z0:z0 + side, y0:y0 + side, x0:x0 + side] = 1
    assert oracle.max_cube(v) == (side, z0 + side - 1, y0 + side - 1, x0 + side - 1)


def test_invariants():
    rng = np.random.default_rng(9)
    for _ in range(15):
        shape = tuple(int(x) for x in rng.integers(3, 14, 3))
        v = (rng.random(shape) < 0.85).astype(np.uint8)
        s = oracle.max_cube(v)[0]
        # the side does not depend on which axis is which
        for perm in itertools.permutations(range(3)):
            assert oracle.max_cube(np.ascontiguousarray(v.transpose(perm)))[0] == s
        # setting voxels never shrinks it; every plane's square bounds it
        w = v.copy()
        w[rng.random(shape) < 0.1] = 1
        assert oracle.max_cube(w)[0] >= s
        assert s <= max(oracle.max_square(v[z])[0] for z in range(shape[0]))
        # the reported cube is all ones
        s, z, y, x = oracle.max_cube(v)
        assert v[z - s + 1:z + 1, y - s + 1:y + 1, x - s + 1:x + 1].all()


# ---- planted mistakes in copies of the cube oracle must fail the pins ----
import os  # noqa: E402
import subprocess  # noqa: E402

CUBE_MUTANTS = {
    "dropped_diagonal": ("if (a == 0 && b == 0 && d == 0) continue;",
                         "if ((a == 0 && b == 0 && d == 0) || (a && b && d)) continue;"),
    "planes_swapped": ("c = (a ? prev : cur)[(y - b) * N + (x - d)];",
                       "c = (a ? cur : prev)[(y - b) * N + (x - d)];"),
    "last_not_first": ("if (v > res[0]) {", "if (v >= res[0] && v) {"),
}


def _cube_pins_pass() -> bool:
    for shape in [(2, 2, 2), (2, 2, 3)]:
        D, M, N = shape
        for mask in range(1 << (D * M * N)):
            v = np.array([(mask >> k) & 1 for k in range(D * M * N)], np.uint8).reshape(shape)
            if oracle.max_cube(v) != brute.max_cube(v):
                return False
    rng = np.random.default_rng(2)
    for _ in range(10):
        v = (rng.random((6, 7, 8)) < 0.9).astype(np.uint8)
        if oracle.max_cube(v) != brute.max_cube(v):
            return False
    return True


@pytest.mark.parametrize("name", sorted(CUBE_MUTANTS))
def test_cube_mutant_is_caught(name, tmp_path):
    old, new = CUBE_MUTANTS[name]
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
        assert not _cube_pins_pass(), "planted mistake %s not caught" % name
    finally:
        oracle._lib, oracle._LIB = saved, real
    assert _cube_pins_pass()
