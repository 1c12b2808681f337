"""CPU oracle for maximal all-ones square detection -- TEST INFRASTRUCTURE.

Only tests, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may import
this package.  The product (the HIP library and its binding) never calls it, and it never
calls the product: the two share no code.

The arithmetic lives in plain C (``oracle.c``: the dp recurrence of Section 2.1 eq. (1) in
full-table and rolling-row form, its own bit unpacker/packer, the paper's Algorithm 1 as a
second witness, the largest all-ones rectangle by its plain definition, and the largest
all-ones cube of a volume by the seven-neighbour recurrence); this module only marshals numpy
arrays through ctypes and builds the shared object with gcc when it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain C, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        for name, args in {
            "oracle_max_square_u8": [_p, _i64, _i64, _i64, _p],
            "oracle_max_square_packed": [_p, _i64, _i64, _i64, _p],
            "oracle_square_map_u8": [_p, _i64, _i64, _i64, _p, _i64, _p],
            "oracle_square_map_packed": [_p, _i64, _i64, _i64, _p, _i64, _p],
            "oracle_pack_u8": [_p, _i64, _i64, _i64, _p, _i64],
            "oracle_unpack": [_p, _i64, _i64, _i64, _p, _i64],
            "oracle_freq_alg1_u8": [_p, _i64, _i64, _i64, _p, _p],
            "oracle_all_masks": [ctypes.c_int, ctypes.c_int, _p, _p],
            "oracle_max_rect_u8": [_p, _i64, _i64, _i64, _p],
            "oracle_max_rect_packed": [_p, _i64, _i64, _i64, _p],
            "oracle_max_cube_packed": [_p, _i64, _i64, _i64, _i64, _p],
            "oracle_stream_next": [_p, _i64, _p, _i64],
            "oracle_stream_result": [_p, _p],
            "oracle_stream_close": [_p],
        }.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int if name not in ("oracle_stream_next",) else _i64
        L.oracle_stream_open_packed.argtypes = [_p, _i64, _i64, _i64]
        L.oracle_stream_open_packed.restype = _p
        L.oracle_stream_result.restype = None
        L.oracle_stream_close.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def _check(rc: int):
    if rc != 0:
        raise ValueError("oracle error %d" % rc)


def _u8(a) -> np.ndarray:
    a = np.asarray(a)
    if a.dtype != np.uint8:
        a = (a != 0).astype(np.uint8)
    return np.ascontiguousarray(a)


def max_square(a) -> tuple[int, int, int]:
    """(S, row, col) of the first row-major maximal square's bottom-right corner."""
    a = _u8(a)
    m, n = a.shape
    res = np.zeros(3, np.int64)
    _check(lib().oracle_max_square_u8(_ptr(a), m, n, n, _ptr(res)))
    return int(res[0]), int(res[1]), int(res[2])


def max_square_packed(bits: np.ndarray, n: int) -> tuple[int, int, int]:
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    m, ldw = bits.shape
    res = np.zeros(3, np.int64)
    _check(lib().oracle_max_square_packed(_ptr(bits), m, n, ldw, _ptr(res)))
    return int(res[0]), int(res[1]), int(res[2])


def square_map(a):
    """(dp int32 (m, n), (S, row, col))."""
    a = _u8(a)
    m, n = a.shape
    dp = np.zeros((m, n), np.int32)
    res = np.zeros(3, np.int64)
    _check(lib().oracle_square_map_u8(_ptr(a), m, n, n, _ptr(dp), n, _ptr(res)))
    return dp, (int(res[0]), int(res[1]), int(res[2]))


def square_map_packed(bits: np.ndarray, n: int):
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    m, ldw = bits.shape
    dp = np.zeros((m, n), np.int32)
    res = np.zeros(3, np.int64)
    _check(lib().oracle_square_map_packed(_ptr(bits), m, n, ldw, _ptr(dp), n, _ptr(res)))
    return dp, (int(res[0]), int(res[1]), int(res[2]))


class Stream:
    """Rolling-row evaluation over packed input: next(rows) returns the next dp rows."""

    def __init__(self, bits: np.ndarray, n: int):
        self.bits = np.ascontiguousarray(bits, dtype=np.uint64)
        self.m, ldw = self.bits.shape
        self.n = int(n)
        self.h = lib().oracle_stream_open_packed(_ptr(self.bits), self.m, self.n, ldw)
        if not self.h:
            raise ValueError("oracle stream open failed")

    def next(self, rows: int) -> np.ndarray:
        out = np.empty((rows, max(self.n, 1)), np.int32)
        got = lib().oracle_stream_next(self.h, rows, _ptr(out), out.shape[1])
        return out[:got, : self.n]

    def result(self) -> tuple[int, int, int]:
        res = np.zeros(3, np.int64)
        lib().oracle_stream_result(self.h, _ptr(res))
        return int(res[0]), int(res[1]), int(res[2])

    def close(self):
        if self.h:
            lib().oracle_stream_close(self.h)
            self.h = None

    def __del__(self):
        self.close()


def pack(a, ld_words: int | None = None) -> np.ndarray:
    """The oracle's own packer (column j -> bit j & 63 of word j >> 6)."""
    a = _u8(a)
    m, n = a.shape
    ldw = (n + 63) // 64 if ld_words is None else int(ld_words)
    bits = np.zeros((m, max(ldw, 1) if m else 0), np.uint64)
    if m and n:
        _check(lib().oracle_pack_u8(_ptr(a), m, n, n, _ptr(bits), bits.shape[1]))
    return bits


def unpack(bits: np.ndarray, n: int) -> np.ndarray:
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    m, ldw = bits.shape
    a = np.zeros((m, n), np.uint8)
    if m and n:
        _check(lib().oracle_unpack(_ptr(bits), m, n, ldw, _ptr(a), n))
    return a


def freq_alg1(a):
    """The paper's Algorithm 1: ((found, row, col) at the last increment, per-row found)."""
    a = _u8(a)
    m, n = a.shape
    res = np.zeros(3, np.int64)
    trace = np.zeros(max(m, 1), np.int64)
    _check(lib().oracle_freq_alg1_u8(_ptr(a), m, n, n, _ptr(res), _ptr(trace)))
    return (int(res[0]), int(res[1]), int(res[2])), trace[:m]


def all_masks(m: int, n: int):
    """S and corner (i*n + j, or -1) of every m x n 0/1 matrix, indexed by bit mask."""
    cnt = 1 << (m * n)
    side = np.zeros(cnt, np.int64)
    corner = np.zeros(cnt, np.int64)
    _check(lib().oracle_all_masks(m, n, _ptr(side), _ptr(corner)))
    return side, corner


def max_rect(a) -> tuple[int, int, int, int, int]:
    """Largest all-ones rectangle of a uint8/bool (m, n) array: (area, row, col, height, width)
    with (row, col) its bottom-right corner, first in row-major order among the largest, then
    the smallest height; (0, -1, -1, 0, 0) when there is none."""
    a = _u8(a)
    m, n = a.shape
    res = np.zeros(5, np.int64)
    _check(lib().oracle_max_rect_u8(_ptr(a), m, n, max(n, 1), _ptr(res)))
    return tuple(int(x) for x in res)


def max_rect_packed(bits: np.ndarray, n: int) -> tuple[int, int, int, int, int]:
    """As max_rect, from packed uint64 rows (column j = bit j & 63 of word j >> 6)."""
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    m = bits.shape[0]
    res = np.zeros(5, np.int64)
    _check(lib().oracle_max_rect_packed(_ptr(bits), m, n, max(bits.shape[1], 1), _ptr(res)))
    return tuple(int(x) for x in res)


def pack_volume(v) -> np.ndarray:
    """uint8/bool (D, M, N) -> packed (D, M, ceil(N/64)) uint64, by the oracle's own packer."""
    v = (np.asarray(v) != 0).astype(np.uint8)
    D, M, N = v.shape
    w = max((N + 63) // 64, 1)
    out = np.zeros((D, M, w), np.uint64)
    for z in range(D):
        if M and N:
            out[z] = pack(np.ascontiguousarray(v[z]))
    return out


def max_cube(v) -> tuple[int, int, int, int]:
    """Largest all-ones cube of a (D, M, N) volume: (side, z, y, x) of its far corner, the first
    in (z, y, x) order among the largest; (0, -1, -1, -1) when there is none."""
    v = np.asarray(v)
    D, M, N = v.shape
    return max_cube_packed(pack_volume(v), N)


def max_cube_packed(bits: np.ndarray, n: int) -> tuple[int, int, int, int]:
    """As max_cube, from packed planes (D, M, ld_words) uint64."""
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    D, M, ldw = bits.shape
    res = np.zeros(4, np.int64)
    _check(lib().oracle_max_cube_packed(_ptr(bits), D, M, n, max(ldw, 1), _ptr(res)))
    return tuple(int(x) for x in res)
