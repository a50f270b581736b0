"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point declared in include/rici.h, and refuses to run without a
gfx950 device instead of falling back to anything."""

import ctypes
import os
import re

import pytest

import paper_2007_02306_amd as rici
from paper_2007_02306_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "rici.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rici_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ["rici_create", "rici_destroy", "rici_generate", "rici_distance_rank", "rici_distance_matrix",
                 "rici_sync", "rici_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTS) == _declared()


def test_no_gpu_means_an_error_not_a_fallback():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = _lib.load()
    h = ctypes.c_void_p()
    rc = lib.rici_create(ctypes.byref(h), 0)
    assert rc == -5 and not h.value
    assert b"no HIP device" in lib.rici_last_error()
    with pytest.raises(RuntimeError):
        rici.Context(0)


def test_null_handle_is_rejected():
    lib = _lib.load()
    assert lib.rici_generate(None, None, 0, None, 0, None, None, 1, ctypes.c_float(0.3), None, None) == -1
    assert lib.rici_distance_rank(None, None, 1, None, 1, None, None, None, None) == -1
    assert lib.rici_sync(None, None) == -1
    assert b"NULL handle" in lib.rici_last_error()


def test_noalloc_constants_match_the_header():
    """The binding's limit and the serving budget's workspace charge follow the
    header's triangle limit: 16 B spheres + 48 B vertex records per triangle and
    16 B per 64-triangle cluster, each region rounded up to 256 B."""
    text = open(HEADER).read()
    m = re.search(r"#define RICI_NOALLOC_MAX_TRIANGLES \(1u << (\d+)\)", text)
    assert m
    n = 1 << int(m.group(1))
    up = lambda x: (x + 255) // 256 * 256
    assert rici.NOALLOC_MAX_TRIANGLES == n
    assert rici.NOALLOC_WORKSPACE_BYTES == up(16 * n) + up((n + 63) // 64 * 16) + up(48 * n)
