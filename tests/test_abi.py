"""The C ABI library loads, exports every symbol its header declares, and rejects invalid
arguments before touching the device.  CPU only (no kernel is launched)."""
import ctypes
import os
import re

import pytest

import paper_2503_18974_amd as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "maxsq.h")

INVALID = 1


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ms_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = M.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name


def test_status_strings():
    L = M.lib()
    for s in range(6):
        assert L.ms_status_string(s)
    assert L.ms_status_string(99) == b"unknown status"


OUT = ctypes.create_string_buffer(24)
P = ctypes.addressof(OUT)  # a non-null pointer; never dereferenced by these calls


@pytest.mark.parametrize("args", [
    (None, None, -1, 5, 1, P, None),          # negative m
    (None, None, 5, -1, 1, P, None),          # negative n
    (None, None, 5, 5, 1, P, None),           # null bits with cells
    (None, P, 5, 130, 2, P, None),            # ld_words < ceil(n/64)
    (None, P, 5, 5, 1, None, None),           # null result
    (None, P, 1 << 22, 1 << 22, 1 << 16, P, None),  # m*n beyond the 2^44 key range
    (None, P, 5, 5, -1, P, None),             # negative ld
])
def test_max_square_invalid(args):
    assert M.lib().ms_max_square(*args) == INVALID


@pytest.mark.parametrize("args", [
    (None, P, 5, 5, 1, None, 5, P, None),     # null map with cells
    (None, P, 5, 5, 1, P, 4, P, None),        # ld_dp < n
    (None, P, 5, 5, 1, P, -3, P, None),       # negative ld_dp
    (None, None, 5, 5, 1, P, 5, P, None),     # null bits
    (None, P, 1 << 40, 2, 1, P, 1 << 40, P, None),  # m * ld_dp overflows
])
def test_square_map_invalid(args):
    assert M.lib().ms_square_map(*args) == INVALID


@pytest.mark.parametrize("args", [
    (None, None, 5, 5, 5, P, 1, None),        # null input
    (None, P, 5, 5, 4, P, 1, None),           # ld_bytes < n
    (None, P, 5, 130, 130, P, 2, None),       # ld_words < ceil(n/64)
    (None, P, 5, 5, 5, None, 1, None),        # null output
    (None, P, -2, 5, 5, P, 1, None),          # negative m
])
def test_pack_invalid(args):
    assert M.lib().ms_pack_u8(*args) == INVALID


def test_batched_invalid():
    L = M.lib()
    size = ctypes.c_size_t()
    assert L.ms_batched_workspace_size(None, None, -1, ctypes.byref(size)) == INVALID
    assert L.ms_batched_workspace_size(None, None, 3, ctypes.byref(size)) == INVALID
    mats = (M._Matrix * 2)(M._Matrix(P, 4, 4, 1), M._Matrix(None, 4, 4, 1))
    assert L.ms_batched_workspace_size(None, mats, 2, ctypes.byref(size)) == INVALID
    mats[1] = M._Matrix(P, 4, 200, 3)   # ld_words < ceil(200/64)
    assert L.ms_batched_workspace_size(None, mats, 2, ctypes.byref(size)) == INVALID
    assert L.ms_max_square_batched(None, None, P, 1, P, P, 1 << 20, None) == INVALID
    assert L.ms_max_square_batched(None, mats, P, -1, P, P, 1 << 20, None) == INVALID
    assert L.ms_max_square_batched(None, mats, None, 2, P, P, 1 << 20, None) == INVALID
    # count == 0 is a no-op that succeeds without touching the device
    assert L.ms_max_square_batched(None, None, None, 0, None, None, 0, None) == 0


def test_workspace_size_is_host_only():
    mats = (M._Matrix * 3)(M._Matrix(P, 100, 100, 2), M._Matrix(P, 0, 7, 1),
                           M._Matrix(P, 4096, 4096, 64))
    a = M.ms_batched_workspace_size(None, mats, 3)
    b = M.ms_batched_workspace_size(None, mats, 1)
    assert a > b > 0


def test_candidates_and_config_validation():
    n = M.ms_num_candidates()
    assert n >= 6
    seen = set()
    for i in range(n):
        c = M.ms_candidate(i)
        seen.add(tuple(sorted(c.items())))
    assert len(seen) == n
    L = M.lib()
    bad = M._Config(7, 4, 64)
    assert L.ms_set_config(None, ctypes.byref(bad)) == INVALID
    bad = M._Config(0, 5, 64)
    assert L.ms_set_config(None, ctypes.byref(bad)) == INVALID
    assert L.ms_candidate(n, ctypes.byref(M._Config())) == INVALID
    # batched submission modes: only the three declared ones (checked before any context)
    for mode in (-1, 3, 99):
        assert L.ms_set_batched_graphs(None, mode) == INVALID


def test_default_config_by_size():
    """Untuned defaults (no context: host only): the 49-row probe tile below 2^24 cells, the
    113-row 16-certified tile up to 2^26, the 32-certified tile from there on."""
    def variant(m, n):
        return M.ms_get_config(None, m, n)["probe_variant"]
    assert variant(1000, 1000) == 0
    assert variant(4096, 4095) == 0
    assert variant(4096, 4096) == 1
    assert variant(5000, 5000) == 1
    assert variant(8191, 8192) == 1
    assert variant(8192, 8192) == 2
    assert variant(4096, 262144) == 2
    assert M.ms_get_config(None, 5000, 5000)["map_cols"] == 4
    assert M.ms_get_config(None, 1000, 1000)["map_cols"] == 4
    assert M.ms_get_config(None, 1000, 1000) in [M.ms_candidate(i)
                                                 for i in range(M.ms_num_candidates())]


def test_create_rejects_bad_args():
    L = M.lib()
    assert L.ms_create(None, 0) == INVALID
    h = ctypes.c_void_p()
    assert L.ms_create(ctypes.byref(h), -5) == INVALID
    assert L.ms_destroy(None) == INVALID


@pytest.mark.parametrize("args", [
    (None, P, 5, 5, 1, P, P, -1, P, P, 1 << 20, None),     # negative capacity
    (None, P, 5, 5, 1, P, None, 4, P, P, 1 << 20, None),   # null positions with capacity
    (None, P, 5, 5, 1, P, P, 4, None, P, 1 << 20, None),   # null count
    (None, P, 5, 5, 1, None, P, 4, P, P, 1 << 20, None),   # null device result
    (None, P, 5, 5, 1, P, P, 4, P, None, 1 << 20, None),   # null workspace
    (None, None, 5, 5, 1, P, P, 4, P, P, 1 << 20, None),   # null bits
    (None, P, 5, 130, 2, P, P, 4, P, P, 1 << 20, None),    # ld_words < ceil(n/64)
])
def test_all_max_squares_invalid(args):
    assert M.lib().ms_all_max_squares(*args) == INVALID


def test_all_max_squares_workspace():
    L = M.lib()
    size = ctypes.c_size_t()
    assert L.ms_all_max_squares_workspace_size(None, -1, 5, ctypes.byref(size)) == INVALID
    assert L.ms_all_max_squares_workspace_size(None, 1000, 2000, ctypes.byref(size)) == 0
    big = size.value
    assert L.ms_all_max_squares_workspace_size(None, 10, 2000, ctypes.byref(size)) == 0
    assert 0 < size.value < big
    # a workspace below the required size is refused before any device work
    assert L.ms_all_max_squares(None, P, 1000, 2000, 32, P, P, 4, P, P, 16, None) == 2


@pytest.mark.parametrize("args", [
    (None, None, -1, 5, 1, P, None),          # negative m
    (None, None, 5, 5, 1, P, None),           # null bits with cells
    (None, P, 5, 130, 2, P, None),            # ld_words < ceil(n/64)
    (None, P, 5, 5, 1, None, None),           # null result
    (None, P, 1 << 22, 1 << 22, 1 << 16, P, None),  # m*n beyond the 2^44 key range
])
def test_max_rectangle_invalid(args):
    assert M.lib().ms_max_rectangle(*args) == INVALID


def test_max_rectangle_too_wide_is_unsupported():
    """Rows wider than 512 words are refused before any device work."""
    assert M.lib().ms_max_rectangle(None, P, 4, 32769, 513, P, None) == 5


@pytest.mark.parametrize("args", [
    (None, None, -1, 5, 5, 1, P, P, 1 << 20, None),        # negative D
    (None, None, 2, 5, 5, 1, P, P, 1 << 20, None),         # null bits with voxels
    (None, P, 2, 5, 130, 2, P, P, 1 << 20, None),          # ld_words < ceil(N/64)
    (None, P, 2, 5, 5, 1, None, P, 1 << 20, None),         # null result
    (None, P, 2, 5, 5, 1, P, None, 1 << 20, None),         # null workspace
    (None, P, 1 << 15, 1 << 15, 1 << 15, 512, P, P, 1, None),  # D*M*N beyond 2^44
])
def test_max_cube_invalid(args):
    assert M.lib().ms_max_cube(*args) == INVALID


def test_max_cube_workspace_checked():
    import ctypes as C
    n = C.c_size_t()
    assert M.lib().ms_max_cube_workspace_size(None, 3, 4, 130, C.byref(n)) == 0
    assert n.value >= 3 * 3 * 4 * 3 * 8
    assert M.lib().ms_max_cube(None, P, 3, 4, 130, 3, P, P, n.value - 1, None) == 2


def test_side_beyond_key_field_is_unsupported():
    """The result key holds sides below 2^20, so a matrix whose shorter dimension reaches 2^20
    (e.g. an all-ones 2^20 x 2^20 matrix, 128 GiB packed) is refused before any device work
    instead of coming back with a truncated side; one row or column less is accepted by the
    host checks."""
    L = M.lib()
    unsupported = 5
    big = 1 << 20
    assert L.ms_max_square(None, P, big, big, big // 64, P, None) == unsupported
    assert L.ms_square_map(None, P, big, big, big // 64, P, big, P, None) == unsupported
    assert L.ms_square_map_from_max(None, P, big, big, big // 64, P, P, big, None) == unsupported
    assert L.ms_all_max_squares(None, P, big, big, big // 64, P, P, 4, P, P, 1 << 40,
                                None) == unsupported
    size = ctypes.c_size_t()
    mats = (M._Matrix * 2)(M._Matrix(P, 4, 4, 1), M._Matrix(P, big, big, big // 64))
    assert L.ms_batched_workspace_size(None, mats, 2, ctypes.byref(size)) == unsupported
    assert L.ms_max_square_batched(None, mats, P, 2, P, P, 1 << 40, None) == unsupported
    mats[1] = M._Matrix(P, big - 1, big, big // 64)
    assert L.ms_batched_workspace_size(None, mats, 2, ctypes.byref(size)) == 0
