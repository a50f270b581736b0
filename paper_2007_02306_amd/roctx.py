"""ROCTx ranges for the host control loops (serving), so that a
`rocprofv3 --marker-trace` run shows admission, describe and scan steps on the
timeline next to the kernels.  Markers are annotations only: when neither ROCTx
library can be loaded, push/pop do nothing and nothing else changes."""

from __future__ import annotations

import ctypes
import contextlib

_CANDIDATES = ("librocprofiler-sdk-roctx.so.1", "/opt/rocm/lib/librocprofiler-sdk-roctx.so.1",
               "libroctx64.so.4", "/opt/rocm/lib/libroctx64.so.4")
_lib = None
_tried = False


def _load():
    global _lib, _tried
    if _tried:
        return _lib
    _tried = True
    for name in _CANDIDATES:
        try:
            lib = ctypes.CDLL(name)
            lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
            lib.roctxRangePushA.restype = ctypes.c_int
            lib.roctxRangePop.argtypes = []
            lib.roctxRangePop.restype = ctypes.c_int
            _lib = lib
            break
        except (OSError, AttributeError):
            continue
    return _lib


def available() -> bool:
    return _load() is not None


def push(name: str) -> None:
    lib = _load()
    if lib is not None:
        lib.roctxRangePushA(name.encode())


def pop() -> None:
    lib = _load()
    if lib is not None:
        lib.roctxRangePop()


@contextlib.contextmanager
def range(name: str):  # noqa: A001 - mirrors the ROCTx name
    push(name)
    try:
        yield
    finally:
        pop()
