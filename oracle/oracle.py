"""ctypes wrapper around rici_oracle.c -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module.  Array checks and marshalling only; every result is computed by the
C oracle (FP64 geometry, int64 distances).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

NBINS = 64
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rici_oracle.c")
_LIB = os.path.join(_HERE, "librici_oracle.so")
_lock = threading.Lock()
_lib = None


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-D_GNU_SOURCE",
               "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=False)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            U32, I32, I64, F32 = ctypes.c_uint32, ctypes.c_int, ctypes.c_int64, ctypes.c_float
            lib.oracle_rici_rowrange.argtypes = [P, U32, P, U32, P, P, U32, F32, P, P, P, I32]
            lib.oracle_rici_rowrange.restype = I32
            lib.oracle_rici_brute.argtypes = [P, U32, P, U32, P, P, U32, F32, P, P, I32]
            lib.oracle_rici_brute.restype = I32
            F64 = ctypes.c_double
            lib.oracle_rici_rowrange_f64.argtypes = [P, U32, P, U32, P, P, U32, F64, P, P, P, I32]
            lib.oracle_rici_rowrange_f64.restype = I32
            lib.oracle_rici_brute_f64.argtypes = [P, U32, P, U32, P, P, U32, F64, P, P, I32]
            lib.oracle_rici_brute_f64.restype = I32
            lib.oracle_project.argtypes = [P, P, P, I64, I32, P, P, P]
            lib.oracle_project.restype = None
            lib.oracle_crd.argtypes = [P, P]
            lib.oracle_crd.restype = I64
            lib.oracle_rank.argtypes = [P, U32, P, U32, P, P, P, I32]
            lib.oracle_rank.restype = I32
            lib.oracle_distance_matrix.argtypes = [P, U32, P, U32, P, I32]
            lib.oracle_distance_matrix.restype = I32
            lib.oracle_threads.argtypes = [I32]
            lib.oracle_threads.restype = I32
            lib.oracle_spin_images.argtypes = [P, I64, P, P, U32, F32, P, P, P, I32]
            lib.oracle_spin_images.restype = I32
            lib.oracle_pearson.argtypes = [P, P]
            lib.oracle_pearson.restype = F64
            lib.oracle_pearson_rank.argtypes = [P, U32, P, U32, P, F64, P, P, P, P, I32]
            lib.oracle_pearson_rank.restype = I32
            lib.oracle_pearson_matrix.argtypes = [P, U32, P, U32, P, I32]
            lib.oracle_pearson_matrix.restype = I32
            lib.oracle_clutter_areas.argtypes = [P, U32, P, U32, U32, U32, P, P, U32, F32, P, P, I32]
            lib.oracle_clutter_areas.restype = I32
            lib.oracle_triangle_area_in_volume.argtypes = [P, P, P, F64]
            lib.oracle_triangle_area_in_volume.restype = F64
            _lib = lib
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _mesh_args(positions, triangles, op_positions, op_normals, dtype=np.float32):
    pos = _c(positions, dtype).reshape(-1, 3)
    tri = _c(triangles, np.uint32).reshape(-1, 3)
    opp = _c(op_positions, dtype).reshape(-1, 3)
    opn = _c(op_normals, dtype).reshape(-1, 3)
    if opp.shape != opn.shape:
        raise ValueError("op_positions and op_normals differ in shape")
    return pos, tri, opp, opn


def _check(rc: int, what: str):
    if rc == -1:
        raise ValueError(f"{what} out of range")
    if rc != 0:
        raise MemoryError("the oracle ran out of host memory")


def threads(nthreads: int = 0) -> int:
    return int(load().oracle_threads(int(nthreads)))


def rici_rowrange(positions, triangles, op_positions, op_normals, support_radius: float,
                  nthreads: int = 0, f64: bool = False):
    """Row-range oracle: returns (images u32 [N,64,64], flags bool [N,64,64],
    work u64 [N,5] = (triangles visited, slices, pixel updates, triangles and
    slices that come closer to the axis than R)).  Inputs are
    fp32 (the library's input type) unless `f64`, which passes positions,
    oriented points and the support radius in FP64."""
    dt = np.float64 if f64 else np.float32
    pos, tri, opp, opn = _mesh_args(positions, triangles, op_positions, op_normals, dt)
    n = opp.shape[0]
    images = np.zeros((n, NBINS, NBINS), dtype=np.uint32)
    flags = np.zeros((n, NBINS, NBINS), dtype=np.uint8)
    work = np.zeros((n, 5), dtype=np.uint64)
    fn = load().oracle_rici_rowrange_f64 if f64 else load().oracle_rici_rowrange
    rc = fn(_ptr(pos), pos.shape[0], _ptr(tri), tri.shape[0], _ptr(opp), _ptr(opn), n, float(support_radius),
            _ptr(images), _ptr(flags), _ptr(work), int(nthreads))
    _check(rc, "triangle index")
    return images, flags.astype(bool), work


def rici_brute(positions, triangles, op_positions, op_normals, support_radius: float,
               nthreads: int = 0, f64: bool = False):
    """Brute-force oracle (plain definition): returns (images, flags)."""
    dt = np.float64 if f64 else np.float32
    pos, tri, opp, opn = _mesh_args(positions, triangles, op_positions, op_normals, dt)
    n = opp.shape[0]
    images = np.zeros((n, NBINS, NBINS), dtype=np.uint32)
    flags = np.zeros((n, NBINS, NBINS), dtype=np.uint8)
    fn = load().oracle_rici_brute_f64 if f64 else load().oracle_rici_brute
    rc = fn(_ptr(pos), pos.shape[0], _ptr(tri), tri.shape[0], _ptr(opp), _ptr(opn), n, float(support_radius),
            _ptr(images), _ptr(flags), int(nthreads))
    _check(rc, "triangle index")
    return images, flags.astype(bool)


def project(spin_vertex, spin_normal, points, printed_eq1: bool = False):
    """Eq. 1-5 projection: returns (alpha, beta, (T_x, T_y)) in FP64."""
    sv = _c(spin_vertex, np.float32).reshape(3)
    sn = _c(spin_normal, np.float32).reshape(3)
    pts = _c(points, np.float64).reshape(-1, 3)
    n = pts.shape[0]
    alpha = np.zeros(n)
    beta = np.zeros(n)
    txy = np.zeros((n, 2))
    load().oracle_project(_ptr(sv), _ptr(sn), _ptr(pts), n, int(bool(printed_eq1)), _ptr(alpha), _ptr(beta),
                          _ptr(txy))
    return alpha, beta, txy


def crd(needle, haystack) -> int:
    nd = _c(needle, np.uint32).reshape(NBINS, NBINS)
    hs = _c(haystack, np.uint32).reshape(NBINS, NBINS)
    return int(load().oracle_crd(_ptr(nd), _ptr(hs)))


def distance_matrix(needles, haystack, nthreads: int = 0) -> np.ndarray:
    nd = _c(needles, np.uint32).reshape(-1, NBINS, NBINS)
    hs = _c(haystack, np.uint32).reshape(-1, NBINS, NBINS)
    out = np.zeros((nd.shape[0], hs.shape[0]), dtype=np.int64)
    rc = load().oracle_distance_matrix(_ptr(nd), nd.shape[0], _ptr(hs), hs.shape[0], _ptr(out), int(nthreads))
    _check(rc, "index")
    return out


def rank(needles, haystack, true_index, nthreads: int = 0):
    """Returns (rank u32 [Nn], true distance i64 [Nn])."""
    nd = _c(needles, np.uint32).reshape(-1, NBINS, NBINS)
    hs = _c(haystack, np.uint32).reshape(-1, NBINS, NBINS)
    ti = _c(true_index, np.uint32).reshape(-1)
    if ti.shape[0] != nd.shape[0]:
        raise ValueError("true_index must have one entry per needle")
    rk = np.zeros(nd.shape[0], dtype=np.uint32)
    ds = np.zeros(nd.shape[0], dtype=np.int64)
    rc = load().oracle_rank(_ptr(nd), nd.shape[0], _ptr(hs), hs.shape[0], _ptr(ti), _ptr(rk), _ptr(ds),
                            int(nthreads))
    _check(rc, "true_index")
    return rk, ds


# ------------------------------------------------------------------ spin images

def spin_images(samples, op_positions, op_normals, support_radius: float, nthreads: int = 0):
    """Spin Images (Sec. 2.1 with the Sec. 3.1.1 projection; readings S1-S2):
    returns (images f64 [N,64,64], counts u32 [N,64,64] of non-zero weights
    per pixel, flags bool [N,64,64] of pixels a sample near the support
    boundary reaches)."""
    smp = _c(samples, np.float32).reshape(-1, 3)
    opp = _c(op_positions, np.float32).reshape(-1, 3)
    opn = _c(op_normals, np.float32).reshape(-1, 3)
    n = opp.shape[0]
    images = np.zeros((n, NBINS, NBINS), dtype=np.float64)
    counts = np.zeros((n, NBINS, NBINS), dtype=np.uint32)
    flags = np.zeros((n, NBINS, NBINS), dtype=np.uint8)
    rc = load().oracle_spin_images(_ptr(smp), smp.shape[0], _ptr(opp), _ptr(opn), n, float(support_radius),
                                   _ptr(images), _ptr(counts), _ptr(flags), int(nthreads))
    _check(rc, "sample")
    return images, counts, flags.astype(bool)


def pearson(a, b) -> float:
    """Pearson correlation of two images (reading S3: 0 for a constant image)."""
    x = _c(a, np.float32).reshape(NBINS * NBINS)
    y = _c(b, np.float32).reshape(NBINS * NBINS)
    return float(load().oracle_pearson(_ptr(x), _ptr(y)))


def pearson_matrix(needles, haystack, nthreads: int = 0) -> np.ndarray:
    nd = _c(needles, np.float32).reshape(-1, NBINS, NBINS)
    hs = _c(haystack, np.float32).reshape(-1, NBINS, NBINS)
    out = np.zeros((nd.shape[0], hs.shape[0]), dtype=np.float64)
    load().oracle_pearson_matrix(_ptr(nd), nd.shape[0], _ptr(hs), hs.shape[0], _ptr(out), int(nthreads))
    return out


def pearson_rank(needles, haystack, true_index, band: float = 0.0, nthreads: int = 0):
    """Rank of the true match under correlation (reading S4).  Returns (rank,
    lo, hi, rho_true): lo / hi count h != true with rho above rho_true + band /
    rho_true - band, the range of ranks allowed to an implementation whose
    correlations are within band / 2 of these."""
    nd = _c(needles, np.float32).reshape(-1, NBINS, NBINS)
    hs = _c(haystack, np.float32).reshape(-1, NBINS, NBINS)
    ti = _c(true_index, np.uint32).reshape(-1)
    if ti.shape[0] != nd.shape[0]:
        raise ValueError("true_index must have one entry per needle")
    n = nd.shape[0]
    rk, lo, hi = (np.zeros(n, dtype=np.uint32) for _ in range(3))
    rt = np.zeros(n, dtype=np.float64)
    rc = load().oracle_pearson_rank(_ptr(nd), n, _ptr(hs), hs.shape[0], _ptr(ti), float(band), _ptr(rk), _ptr(lo),
                                    _ptr(hi), _ptr(rt), int(nthreads))
    _check(rc, "true_index")
    return rk, lo, hi, rt


# ---------------------------------------------------------------- clutter

def clutter_areas(positions, triangles, object_first: int, object_count: int, op_positions, op_normals,
                  support_radius: float, nthreads: int = 0):
    """Surface areas inside each oriented point's support volume (reading C1):
    (A_all, A_object) float64 [N]; the object is triangles object_first ..
    object_first + object_count - 1.  Eq. 8: clutter = (A_all - A_object) /
    A_all."""
    pos, tri, opp, opn = _mesh_args(positions, triangles, op_positions, op_normals, np.float32)
    n = opp.shape[0]
    a_all = np.zeros(n, dtype=np.float64)
    a_obj = np.zeros(n, dtype=np.float64)
    rc = load().oracle_clutter_areas(_ptr(pos), pos.shape[0], _ptr(tri), tri.shape[0], int(object_first),
                                     int(object_count), _ptr(opp), _ptr(opn), n, float(support_radius),
                                     _ptr(a_all), _ptr(a_obj), int(nthreads))
    _check(rc, "triangle index")
    return a_all, a_obj


def triangle_area_in_volume(p0, p1, p2, support_radius: float) -> float:
    """Area of one triangle, given in the frame of the axis (z) and the Spin
    Vertex (origin), inside the support volume."""
    a, b, c = (_c(np.asarray(x, np.float64), np.float64).reshape(3) for x in (p0, p1, p2))
    return float(load().oracle_triangle_area_in_volume(_ptr(a), _ptr(b), _ptr(c), float(support_radius)))
