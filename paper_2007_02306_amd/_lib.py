"""ctypes loader for librici.so (the C ABI of include/rici.h).

Argument marshalling only: every step of the pipeline runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librici.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "rici.h")

EXPORTS = [
    "rici_create", "rici_destroy", "rici_last_error", "rici_sync", "rici_device_errors",
    "rici_generate", "rici_generate_noalloc", "rici_distance_rank", "rici_distance_matrix",
    "rici_timing_enable", "rici_timing_reset", "rici_timing_get",
    "rici_batch_create", "rici_batch_run", "rici_batch_destroy", "rici_batch_scratch_bytes",
    "rici_batch_kernel_ms",
    "rici_db_create", "rici_db_tiles", "rici_db_scratch_bytes", "rici_db_destroy",
    "rici_query_create", "rici_query_footprint", "rici_query_destroy", "rici_db_scan",
    "rici_set_tuning", "rici_get_tuning",
    "rici_spin_generate", "rici_spin_rank", "rici_spin_correlation_matrix",
    "rici_clutter_areas",
]


class MeshJob(ctypes.Structure):
    """rici_mesh_job of include/rici.h."""
    _fields_ = [
        ("positions", ctypes.c_void_p), ("num_vertices", ctypes.c_uint32),
        ("triangles", ctypes.c_void_p), ("num_triangles", ctypes.c_uint32),
        ("op_positions", ctypes.c_void_p),
        ("op_normals", ctypes.c_void_p), ("num_points", ctypes.c_uint32),
        ("out_images", ctypes.c_void_p),
        ("true_index", ctypes.c_void_p),
        ("out_rank", ctypes.c_void_p),
        ("out_true_distance", ctypes.c_void_p),
    ]

RICI_OK = 0
STATUS = {0: "RICI_OK", -1: "RICI_ERR_INVALID", -2: "RICI_ERR_OOM", -3: "RICI_ERR_HIP",
          -4: "RICI_ERR_DEVICE", -5: "RICI_ERR_UNSUPPORTED"}

_lock = threading.Lock()
_lib = None


class RiciError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS.get(code, code)}: {message}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load librici.so and declare its prototypes (raises if it is missing)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with paper_2007_02306_amd/build.py "
                              "(there is no CPU fallback)")
        lib = ctypes.CDLL(path)
        P, U32, I32, F32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int, ctypes.c_float
        lib.rici_create.argtypes = [ctypes.POINTER(P), I32]
        lib.rici_create.restype = I32
        lib.rici_destroy.argtypes = [P]
        lib.rici_destroy.restype = None
        lib.rici_last_error.argtypes = []
        lib.rici_last_error.restype = ctypes.c_char_p
        lib.rici_sync.argtypes = [P, P]
        lib.rici_sync.restype = I32
        lib.rici_device_errors.argtypes = [P]
        lib.rici_device_errors.restype = U32
        lib.rici_generate.argtypes = [P, P, U32, P, U32, P, P, U32, F32, P, P]
        lib.rici_generate.restype = I32
        lib.rici_generate_noalloc.argtypes = [P, P, U32, P, U32, P, P, U32, F32, P, P]
        lib.rici_generate_noalloc.restype = I32
        lib.rici_spin_generate.argtypes = [P, P, U32, P, P, U32, F32, P, P]
        lib.rici_spin_generate.restype = I32
        lib.rici_spin_rank.argtypes = [P, P, U32, P, U32, P, P, P, P]
        lib.rici_spin_rank.restype = I32
        lib.rici_spin_correlation_matrix.argtypes = [P, P, U32, P, U32, P, P]
        lib.rici_spin_correlation_matrix.restype = I32
        lib.rici_clutter_areas.argtypes = [P, P, U32, P, U32, U32, U32, P, P, U32, F32, P, P, P]
        lib.rici_clutter_areas.restype = I32
        lib.rici_distance_rank.argtypes = [P, P, U32, P, U32, P, P, P, P]
        lib.rici_distance_rank.restype = I32
        lib.rici_distance_matrix.argtypes = [P, P, U32, P, U32, P, P]
        lib.rici_distance_matrix.restype = I32
        lib.rici_timing_enable.argtypes = [P, I32]
        lib.rici_timing_enable.restype = I32
        lib.rici_timing_reset.argtypes = [P]
        lib.rici_timing_reset.restype = I32
        lib.rici_timing_get.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_uint64)]
        lib.rici_timing_get.restype = I32
        lib.rici_batch_create.argtypes = [P, ctypes.POINTER(MeshJob), U32, F32, ctypes.POINTER(P)]
        lib.rici_batch_create.restype = I32
        lib.rici_batch_run.argtypes = [P, P]
        lib.rici_batch_run.restype = I32
        lib.rici_batch_destroy.argtypes = [P]
        lib.rici_batch_destroy.restype = None
        lib.rici_batch_scratch_bytes.argtypes = [P]
        lib.rici_batch_scratch_bytes.restype = ctypes.c_uint64
        lib.rici_batch_kernel_ms.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(F32)]
        lib.rici_batch_kernel_ms.restype = I32
        U64 = ctypes.c_uint64
        lib.rici_db_create.argtypes = [P, P, U32, P, ctypes.POINTER(P)]
        lib.rici_db_create.restype = I32
        lib.rici_db_tiles.argtypes = [P]
        lib.rici_db_tiles.restype = U32
        lib.rici_db_scratch_bytes.argtypes = [P]
        lib.rici_db_scratch_bytes.restype = U64
        lib.rici_db_destroy.argtypes = [P]
        lib.rici_db_destroy.restype = None
        lib.rici_query_create.argtypes = [P, P, P, U32, P, P, P, P, U64, P, ctypes.POINTER(P)]
        lib.rici_query_create.restype = I32
        lib.rici_query_footprint.argtypes = [P, U32]
        lib.rici_query_footprint.restype = U64
        lib.rici_query_destroy.argtypes = [P]
        lib.rici_query_destroy.restype = None
        lib.rici_db_scan.argtypes = [P, P, ctypes.POINTER(P), U32, U32, U32, P]
        lib.rici_db_scan.restype = I32
        lib.rici_set_tuning.argtypes = [P, ctypes.c_char_p, I32]
        lib.rici_set_tuning.restype = I32
        lib.rici_get_tuning.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(I32)]
        lib.rici_get_tuning.restype = I32
        _lib = lib
    return _lib


def check(code: int) -> None:
    if code != RICI_OK:
        msg = load().rici_last_error()
        raise RiciError(code, msg.decode() if msg else "")
