"""Python binding of libmaxsq (maximal all-ones square detection on MI355X).

Argument marshalling only: every step of the computation runs in the HIP kernels of
``libmaxsq.so``; PyTorch provides device memory and streams.  The functions ``ms_*`` mirror
the C ABI in ``include/maxsq.h`` one to one (raw device pointers and sizes); the helpers below
them take torch tensors.

Problem and conventions (Bhandari, Section 1 and Section 2.1 eq. (1)): the side S of the
largest all-ones square, the first bottom-right corner (row, col) in row-major order among the
cells whose dp value is S, and the dp map itself.  The paper's Algorithm 1 returns the area;
``area(S) = S * S``.

Packed layout: row i is ``ld_words >= ceil(n/64)`` uint64 words; column j is bit ``j & 63`` of
word ``j >> 6`` (LSB first).  Torch has no uint64 arithmetic on ROCm, so packed tensors are
``torch.int64`` carrying the same bits.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

__all__ = [
    "MaxsqError", "Square", "lib", "library_path", "ms_create", "ms_destroy", "ms_pack_u8",
    "ms_max_square", "ms_max_square_noalloc", "ms_square_map", "ms_square_map_from_max", "ms_batched_workspace_size", "ms_max_square_batched",
    "ms_set_config", "ms_get_config", "ms_candidate", "ms_num_candidates", "ms_autotune",
    "ms_autotune_save", "ms_autotune_load", "ms_set_batched_graphs", "GRAPHS_OFF",
    "GRAPHS_ON_REPEAT", "GRAPHS_ALWAYS", "Context", "pack_u8", "max_square", "square_map",
    "max_square_batched", "square_map_from_max", "area", "words_per_row",
    "Rect", "ms_max_rectangle", "max_rectangle", "Cube", "ms_max_cube",
    "ms_max_cube_workspace_size", "max_cube",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmaxsq.so")

MS_OK = 0
STATUS = {0: "ok", 1: "invalid argument", 2: "workspace too small", 3: "out of memory",
          4: "HIP runtime error", 5: "unsupported"}


class MaxsqError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__("%s: %s (status %d)" % (where, STATUS.get(status, "?"), status))
        self.status = status


class _Square(ctypes.Structure):
    _fields_ = [("side", ctypes.c_int64), ("row", ctypes.c_int64), ("col", ctypes.c_int64)]


class _Matrix(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("ld_words", ctypes.c_int64)]


class _Config(ctypes.Structure):
    _fields_ = [("probe_variant", ctypes.c_int32), ("map_cols", ctypes.c_int32),
                ("map_band_rows", ctypes.c_int32)]


@dataclass(frozen=True)
class Square:
    side: int
    row: int
    col: int

    @property
    def area(self) -> int:
        return self.side * self.side


@dataclass(frozen=True)
class Rect:
    """Largest all-ones rectangle: area, bottom-right corner (row, col), height and width."""
    area: int
    row: int
    col: int
    height: int
    width: int


@dataclass(frozen=True)
class Cube:
    """Largest all-ones cube of a volume: side and far corner (z, y, x)."""
    side: int
    z: int
    y: int
    x: int


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libmaxsq.so (built in-tree by ``paper_2503_18974_amd.build``); never falls back."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError("libmaxsq.so is not built; run `python -m paper_2503_18974_amd.build`"
                              " (or __graft_entry__.build())")
        L = ctypes.CDLL(_LIB_PATH)
        sig = {
            "ms_create": [ctypes.POINTER(_P), ctypes.c_int],
            "ms_destroy": [_P],
            "ms_pack_u8": [_P, _P, _I64, _I64, _I64, _P, _I64, _P],
            "ms_max_square": [_P, _P, _I64, _I64, _I64, _P, _P],
            "ms_max_square_noalloc": [_P, _P, _I64, _I64, _I64, _P, _P],
            "ms_square_map": [_P, _P, _I64, _I64, _I64, _P, _I64, _P, _P],
            "ms_square_map_from_max": [_P, _P, _I64, _I64, _I64, _P, _P, _I64, _P],
            "ms_batched_workspace_size": [_P, _P, _I64, ctypes.POINTER(ctypes.c_size_t)],
            "ms_max_square_batched": [_P, _P, _P, _I64, _P, _P, ctypes.c_size_t, _P],
            "ms_candidate": [ctypes.c_int, ctypes.POINTER(_Config)],
            "ms_set_config": [_P, ctypes.POINTER(_Config)],
            "ms_get_config": [_P, _I64, _I64, ctypes.POINTER(_Config)],
            "ms_autotune": [_P, _P, _I64, _I64, _I64, _P, _I64, _P],
            "ms_autotune_batched": [_P, _P, _P, _I64, _P, _P, ctypes.c_size_t, _P],
            "ms_all_max_squares_workspace_size": [_P, _I64, _I64, ctypes.POINTER(ctypes.c_size_t)],
            "ms_all_max_squares": [_P, _P, _I64, _I64, _I64, _P, _P, _I64, _P, _P,
                                   ctypes.c_size_t, _P],
            "ms_max_rectangle": [_P, _P, _I64, _I64, _I64, _P, _P],
            "ms_max_cube_workspace_size": [_P, _I64, _I64, _I64, ctypes.POINTER(ctypes.c_size_t)],
            "ms_max_cube": [_P, _P, _I64, _I64, _I64, _I64, _P, _P, ctypes.c_size_t, _P],
            "ms_autotune_save": [_P, ctypes.c_char_p],
            "ms_autotune_load": [_P, ctypes.c_char_p],
            "ms_set_batched_graphs": [_P, ctypes.c_int],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.ms_num_candidates.argtypes = []
        L.ms_num_candidates.restype = ctypes.c_int
        L.ms_status_string.argtypes = [ctypes.c_int]
        L.ms_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != MS_OK:
        raise MaxsqError(status, where)


# ------------------------------------------------------------------ raw C ABI mirrors

def ms_create(hip_device: int = -1) -> int:
    h = _P()
    _check(lib().ms_create(ctypes.byref(h), hip_device), "ms_create")
    return h.value


def ms_destroy(ctx: int) -> None:
    _check(lib().ms_destroy(ctx), "ms_destroy")


def ms_pack_u8(ctx, d_a, m, n, ld_bytes, d_bits, ld_words, stream) -> int:
    return lib().ms_pack_u8(ctx, d_a, m, n, ld_bytes, d_bits, ld_words, stream)


def ms_max_square(ctx, d_bits, m, n, ld_words, d_out, stream) -> int:
    return lib().ms_max_square(ctx, d_bits, m, n, ld_words, d_out, stream)


def ms_max_square_noalloc(ctx, d_bits, m, n, ld_words, d_out, stream) -> int:
    return lib().ms_max_square_noalloc(ctx, d_bits, m, n, ld_words, d_out, stream)


def ms_square_map(ctx, d_bits, m, n, ld_words, d_dp, ld_dp, d_out, stream) -> int:
    return lib().ms_square_map(ctx, d_bits, m, n, ld_words, d_dp, ld_dp, d_out, stream)


def ms_square_map_from_max(ctx, d_bits, m, n, ld_words, d_max, d_dp, ld_dp, stream) -> int:
    return lib().ms_square_map_from_max(ctx, d_bits, m, n, ld_words, d_max, d_dp, ld_dp, stream)


def ms_batched_workspace_size(ctx, h_mats, count) -> int:
    out = ctypes.c_size_t()
    _check(lib().ms_batched_workspace_size(ctx, h_mats, count, ctypes.byref(out)),
           "ms_batched_workspace_size")
    return out.value


def ms_max_square_batched(ctx, h_mats, d_mats, count, d_out, d_ws, ws_bytes, stream) -> int:
    return lib().ms_max_square_batched(ctx, h_mats, d_mats, count, d_out, d_ws, ws_bytes, stream)


def ms_num_candidates() -> int:
    return lib().ms_num_candidates()


def ms_candidate(i: int) -> dict:
    c = _Config()
    _check(lib().ms_candidate(i, ctypes.byref(c)), "ms_candidate")
    return {"probe_variant": c.probe_variant, "map_cols": c.map_cols,
            "map_band_rows": c.map_band_rows}


GRAPHS_OFF, GRAPHS_ON_REPEAT, GRAPHS_ALWAYS = 0, 1, 2


def ms_set_batched_graphs(ctx, mode: int) -> None:
    """How batched calls on ctx submit their launches (see include/maxsq.h)."""
    _check(lib().ms_set_batched_graphs(ctx, int(mode)), "ms_set_batched_graphs")


def ms_set_config(ctx, cfg: dict | None) -> None:
    if cfg is None:
        _check(lib().ms_set_config(ctx, None), "ms_set_config")
        return
    c = _Config(cfg["probe_variant"], cfg["map_cols"], cfg["map_band_rows"])
    _check(lib().ms_set_config(ctx, ctypes.byref(c)), "ms_set_config")


def ms_get_config(ctx, m: int, n: int) -> dict:
    c = _Config()
    _check(lib().ms_get_config(ctx, m, n, ctypes.byref(c)), "ms_get_config")
    return {"probe_variant": c.probe_variant, "map_cols": c.map_cols,
            "map_band_rows": c.map_band_rows}


def ms_autotune(ctx, d_bits, m, n, ld_words, d_dp, ld_dp, stream) -> None:
    _check(lib().ms_autotune(ctx, d_bits, m, n, ld_words, d_dp, ld_dp, stream), "ms_autotune")


def ms_autotune_batched(ctx, h_mats, d_mats, count, d_out, d_ws, ws_bytes, stream) -> None:
    _check(lib().ms_autotune_batched(ctx, h_mats, d_mats, count, d_out, d_ws, ws_bytes, stream),
           "ms_autotune_batched")


def ms_autotune_save(ctx, path: str) -> None:
    _check(lib().ms_autotune_save(ctx, path.encode()), "ms_autotune_save")


def ms_autotune_load(ctx, path: str) -> None:
    _check(lib().ms_autotune_load(ctx, path.encode()), "ms_autotune_load")


# ------------------------------------------------------------------ torch helpers

def _torch():
    import torch
    return torch


def words_per_row(n: int) -> int:
    return (int(n) + 63) // 64


def area(side: int) -> int:
    return int(side) * int(side)


def _stream(stream=None) -> int:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


class Context:
    """Owns an ms_ctx bound to one device (its scratch and tuning table)."""

    def __init__(self, device: int = -1):
        self.handle = ms_create(device)

    def close(self):
        if self.handle:
            ms_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _ctx(ctx) -> int | None:
    if ctx is None:
        return None
    return ctx.handle if isinstance(ctx, Context) else int(ctx)


def _check_bits(bits, n):
    torch = _torch()
    if bits.dtype != torch.int64 or bits.dim() != 2 or not bits.is_cuda:
        raise ValueError("packed bits must be a 2-D int64 CUDA tensor")
    if bits.size(0) == 0 or n == 0:
        return
    if bits.stride(1) != 1:
        raise ValueError("packed rows must be contiguous")
    if bits.size(1) < words_per_row(n):
        raise ValueError("packed rows are shorter than ceil(n/64) words")


def _ld_words(bits, n) -> int:
    return bits.stride(0) if (bits.size(0) and n) else max(words_per_row(n), 0)


def pack_u8(a, ld_words: int | None = None, ctx=None, stream=None):
    """uint8 (m, n) CUDA tensor -> packed int64 (m, ld_words) CUDA tensor."""
    torch = _torch()
    if a.dtype not in (torch.uint8, torch.bool) or a.dim() != 2 or not a.is_cuda:
        raise ValueError("expected a 2-D uint8 CUDA tensor")
    if a.stride(1) != 1:
        a = a.contiguous()
    m, n = a.shape
    ldw = words_per_row(n) if ld_words is None else int(ld_words)
    bits = torch.empty((m, max(ldw, 1)), dtype=torch.int64, device=a.device)
    _check(ms_pack_u8(_ctx(ctx), a.data_ptr(), m, n, a.stride(0), bits.data_ptr(), bits.stride(0),
                      _stream(stream)), "ms_pack_u8")
    return bits


def max_square(bits, n: int, ctx=None, stream=None, out=None, sync: bool = True):
    """Largest square of a packed (m, >= ceil(n/64)) int64 CUDA tensor.  Returns Square when
    sync, else the int64 (3,) device tensor the result is written to."""
    torch = _torch()
    _check_bits(bits, n)
    m = bits.size(0)
    res = torch.empty(3, dtype=torch.int64, device=bits.device) if out is None else out
    _check(ms_max_square(_ctx(ctx), bits.data_ptr(), m, n, _ld_words(bits, n), res.data_ptr(),
                         _stream(stream)), "ms_max_square")
    if not sync:
        return res
    v = res.cpu().tolist()
    return Square(int(v[0]), int(v[1]), int(v[2]))


def square_map(bits, n: int, ctx=None, stream=None, out=None, dp=None, sync: bool = True):
    """dp map (int32 (m, n) CUDA tensor) and, when sync, the Square."""
    torch = _torch()
    _check_bits(bits, n)
    m = bits.size(0)
    if dp is None:
        dp = torch.empty((m, n), dtype=torch.int32, device=bits.device)
    res = torch.empty(3, dtype=torch.int64, device=bits.device) if out is None else out
    _check(ms_square_map(_ctx(ctx), bits.data_ptr(), m, n, _ld_words(bits, n), dp.data_ptr(),
                         dp.stride(0) if dp.numel() else max(n, 1), res.data_ptr(),
                         _stream(stream)), "ms_square_map")
    if not sync:
        return dp, res
    v = res.cpu().tolist()
    return dp, Square(int(v[0]), int(v[1]), int(v[2]))


def square_map_from_max(bits, n: int, result, ctx=None, stream=None, dp=None):
    """dp map given the int64 (3,) device tensor that max_square(..., sync=False) returned for
    the same bits (skips the second search)."""
    torch = _torch()
    _check_bits(bits, n)
    m = bits.size(0)
    if dp is None:
        dp = torch.empty((m, n), dtype=torch.int32, device=bits.device)
    _check(ms_square_map_from_max(_ctx(ctx), bits.data_ptr(), m, n, _ld_words(bits, n),
                                  result.data_ptr(), dp.data_ptr(),
                                  dp.stride(0) if dp.numel() else max(n, 1), _stream(stream)),
           "ms_square_map_from_max")
    return dp


def ms_max_rectangle(ctx, d_bits, m, n, ld_words, d_out, stream) -> int:
    return lib().ms_max_rectangle(ctx, d_bits, m, n, ld_words, d_out, stream)


def max_rectangle(bits, n: int, ctx=None, stream=None, out=None, sync: bool = True):
    """Largest all-ones rectangle of a packed (m, >= ceil(n/64)) int64 CUDA tensor.  Returns a
    Rect when sync, else the int64 (5,) device tensor (area, row, col, height, width)."""
    torch = _torch()
    _check_bits(bits, n)
    m = bits.size(0)
    res = torch.empty(5, dtype=torch.int64, device=bits.device) if out is None else out
    _check(ms_max_rectangle(_ctx(ctx), bits.data_ptr(), m, n, _ld_words(bits, n), res.data_ptr(),
                            _stream(stream)), "ms_max_rectangle")
    if not sync:
        return res
    return Rect(*(int(x) for x in res.cpu().tolist()))


def ms_max_cube_workspace_size(ctx, D, M, N) -> int:
    n = ctypes.c_size_t()
    _check(lib().ms_max_cube_workspace_size(ctx, D, M, N, ctypes.byref(n)),
           "ms_max_cube_workspace_size")
    return n.value


def ms_max_cube(ctx, d_bits, D, M, N, ld_words, d_out, d_ws, ws_bytes, stream) -> int:
    return lib().ms_max_cube(ctx, d_bits, D, M, N, ld_words, d_out, d_ws, ws_bytes, stream)


def max_cube(bits, n: int, ctx=None, stream=None, workspace=None) -> Cube:
    """Largest all-ones cube of a packed volume: an int64 CUDA tensor (D, M, >= ceil(n/64))
    whose last dimension is contiguous and whose planes are contiguous rows.  Blocks until the
    result is known (the search steers itself from the host)."""
    torch = _torch()
    if bits.dtype != torch.int64 or bits.dim() != 3 or not bits.is_cuda:
        raise ValueError("packed volume must be a 3-D int64 CUDA tensor")
    D, M, ldw = bits.shape
    if D and M and n:
        if bits.stride(2) != 1 or bits.stride(1) != ldw or bits.stride(0) != M * ldw:
            raise ValueError("packed volume must be contiguous")
        if ldw < words_per_row(n):
            raise ValueError("packed rows are shorter than ceil(n/64) words")
    need = ms_max_cube_workspace_size(_ctx(ctx), D, M, n)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=bits.device)
    out = torch.empty(4, dtype=torch.int64, device=bits.device)
    _check(ms_max_cube(_ctx(ctx), bits.data_ptr(), D, M, n, max(ldw, 1), out.data_ptr(),
                       workspace.data_ptr(), workspace.numel(), _stream(stream)), "ms_max_cube")
    return Cube(*(int(x) for x in out.cpu().tolist()))


def all_max_squares(bits, n: int, result=None, capacity: int | None = None, ctx=None,
                    stream=None):
    """Row-major positions i * n + j (int64 CUDA tensor) of the bottom-right corners of every
    largest all-ones square of a packed matrix, and their count.  `result`: the int64 (3,)
    device result of max_square(..., sync=False) for the same bits (computed if None).  With
    the default capacity the call is repeated once with room for every corner if needed."""
    torch = _torch()
    _check_bits(bits, n)
    m = bits.size(0)
    if result is None:
        result = max_square(bits, n, ctx=ctx, stream=stream, sync=False)
    ws_n = ctypes.c_size_t()
    _check(lib().ms_all_max_squares_workspace_size(_ctx(ctx), m, n, ctypes.byref(ws_n)),
           "ms_all_max_squares_workspace_size")
    ws = torch.empty(max(ws_n.value, 1), dtype=torch.uint8, device=bits.device)
    count = torch.empty(1, dtype=torch.int64, device=bits.device)
    cap = 4096 if capacity is None else int(capacity)
    while True:
        pos = torch.empty(max(cap, 1), dtype=torch.int64, device=bits.device)
        _check(lib().ms_all_max_squares(_ctx(ctx), bits.data_ptr(), m, n, _ld_words(bits, n),
                                        result.data_ptr(), pos.data_ptr(), cap,
                                        count.data_ptr(), ws.data_ptr(), ws_n.value,
                                        _stream(stream)), "ms_all_max_squares")
        c = int(count.item())
        if c < 0:
            raise MaxsqError(5, "ms_all_max_squares (square wider than the enumeration supports)")
        if capacity is not None or c <= cap:
            return pos[: min(c, cap)], c
        cap = c


class Batch:
    """Device descriptors, result buffer and workspace for ms_max_square_batched."""

    def __init__(self, items, ctx=None):
        """items: list of (packed int64 CUDA tensor, n)."""
        torch = _torch()
        self.items = list(items)
        count = len(self.items)
        self.count = count
        self.h_mats = (_Matrix * max(count, 1))()
        dev = None
        for i, (bits, n) in enumerate(self.items):
            _check_bits(bits, n)
            dev = bits.device
            self.h_mats[i] = _Matrix(bits.data_ptr(), bits.size(0), int(n), _ld_words(bits, n))
        dev = dev or torch.device("cuda")
        raw = bytes(self.h_mats)[: ctypes.sizeof(_Matrix) * count]
        self.d_mats = torch.frombuffer(bytearray(raw) or bytearray(1), dtype=torch.uint8).to(dev)
        self.out = torch.empty((max(count, 1), 3), dtype=torch.int64, device=dev)
        self.ctx = _ctx(ctx)
        self.ws_bytes = ms_batched_workspace_size(self.ctx, self.h_mats, count)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=dev)

    def run(self, stream=None):
        _check(ms_max_square_batched(self.ctx, self.h_mats, self.d_mats.data_ptr(), self.count,
                                     self.out.data_ptr(), self.ws.data_ptr(), self.ws_bytes,
                                     _stream(stream)), "ms_max_square_batched")
        return self.out[: self.count]

    def autotune(self, stream=None):
        """Time every probe variant on this batch; later runs on the same context use the
        fastest (the results of this call are left in `out`)."""
        ms_autotune_batched(self.ctx, self.h_mats, self.d_mats.data_ptr(), self.count,
                            self.out.data_ptr(), self.ws.data_ptr(), self.ws_bytes,
                            _stream(stream))
        return self.out[: self.count]

    def results(self):
        rows = self.out[: self.count].cpu().tolist()
        if any(r[0] < 0 for r in rows):
            raise MaxsqError(4, "ms_max_square_batched (device reported an inconsistent batch)")
        return [Square(*map(int, r)) for r in rows]


def max_square_batched(items, ctx=None, stream=None):
    """Largest square of every (packed tensor, n) in items, in one batched launch sequence."""
    b = Batch(items, ctx)
    b.run(stream)
    return b.results()
