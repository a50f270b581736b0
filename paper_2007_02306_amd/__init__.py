"""MI355X (gfx950) RICI pipeline: descriptor generation and clutter-resistant
rank search (van Blokland & Theoharis 2020, Sec. 3.1-3.2, Sec. 4.1).

Thin binding over librici.so (include/rici.h).  Tensors are ROCm torch tensors;
PyTorch only supplies device memory and the current stream, every step runs in
the library's HIP kernels.

    ctx = Context()
    images = ctx.generate(positions, triangles, op_positions, op_normals, 0.3)
    rank, dist = ctx.distance_rank(needle_images, haystack_images, true_index)
"""

from __future__ import annotations

import ctypes

from ._lib import EXPORTS, LIB_PATH, MeshJob, RiciError, check, load  # noqa: F401

NBINS = 64
NOALLOC_MAX_TRIANGLES = 1 << 20          # RICI_NOALLOC_MAX_TRIANGLES
NOALLOC_WORKSPACE_BYTES = 67_371_008     # the static generation workspace per GPU

__all__ = ["Context", "Batch", "RiciError", "NBINS", "load", "EXPORTS", "LIB_PATH"]


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, name, dtype, shape_tail=None, device=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU (got {t.device})")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name} is on cuda:{t.device.index}, the context on cuda:{device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [N, {', '.join(map(str, shape_tail))}] (got {tuple(t.shape)})")
    return t


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


class Context:
    """One librici handle bound to one GPU.  Not safe for concurrent calls:
    use one Context per stream that issues work concurrently."""

    def __init__(self, device: int | None = None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no ROCm GPU visible: the RICI pipeline runs only on gfx950")
        self.device = torch.cuda.current_device() if device is None else int(device)
        self._lib = load()
        h = ctypes.c_void_p()
        check(self._lib.rici_create(ctypes.byref(h), self.device))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.rici_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---------------------------------------------------------------- calls
    def generate(self, positions, triangles, op_positions, op_normals, support_radius: float,
                 out=None, stream=None):
        """RICIs of the oriented points: uint32 [N, 64, 64] (int32 tensor viewed as uint32)."""
        torch = _torch()
        dev = self.device
        pos = _dev(positions, "positions", torch.float32, (3,), dev)
        tri = _dev(triangles, "triangles", torch.int32, (3,), dev)
        opp = _dev(op_positions, "op_positions", torch.float32, (3,), dev)
        opn = _dev(op_normals, "op_normals", torch.float32, (3,), dev)
        if opp.shape != opn.shape:
            raise ValueError("op_positions and op_normals differ in shape")
        n = opp.shape[0]
        if out is None:
            out = torch.empty((n, NBINS, NBINS), dtype=torch.int32, device=opp.device)
        else:
            _dev(out, "out", torch.int32, (NBINS, NBINS), dev)
            if out.shape[0] != n:
                raise ValueError("out must have one image per oriented point")
        check(self._lib.rici_generate(self._h, _ptr(pos), pos.shape[0], _ptr(tri), tri.shape[0], _ptr(opp),
                                      _ptr(opn), n, float(support_radius), _ptr(out), _stream_ptr(stream)))
        return out

    def generate_noalloc(self, positions, triangles, op_positions, op_normals, support_radius: float, out,
                         stream=None):
        """rici_generate_noalloc: like generate() into a caller tensor `out`, with
        the library's static per-GPU workspace (at most NOALLOC_MAX_TRIANGLES
        triangles; calls that overlap on one GPU race)."""
        torch = _torch()
        dev = self.device
        pos = _dev(positions, "positions", torch.float32, (3,), dev)
        tri = _dev(triangles, "triangles", torch.int32, (3,), dev)
        opp = _dev(op_positions, "op_positions", torch.float32, (3,), dev)
        opn = _dev(op_normals, "op_normals", torch.float32, (3,), dev)
        _dev(out, "out", torch.int32, (NBINS, NBINS), dev)
        if opp.shape != opn.shape or out.shape[0] != opp.shape[0]:
            raise ValueError("op_positions, op_normals and out must agree in length")
        check(self._lib.rici_generate_noalloc(self._h, _ptr(pos), pos.shape[0], _ptr(tri), tri.shape[0], _ptr(opp),
                                              _ptr(opn), opp.shape[0], float(support_radius), _ptr(out),
                                              _stream_ptr(stream)))
        return out

    def clutter_areas(self, positions, triangles, object_first: int, object_count: int, op_positions, op_normals,
                      support_radius: float, stream=None):
        """(A_all, A_object) float64 [N]: surface areas inside each oriented
        point's support volume; Eq. 8 clutter = (A_all - A_object) / A_all."""
        torch = _torch()
        dev = self.device
        pos = _dev(positions, "positions", torch.float32, (3,), dev)
        tri = _dev(triangles, "triangles", torch.int32, (3,), dev)
        opp = _dev(op_positions, "op_positions", torch.float32, (3,), dev)
        opn = _dev(op_normals, "op_normals", torch.float32, (3,), dev)
        if opp.shape != opn.shape:
            raise ValueError("op_positions and op_normals differ in shape")
        n = opp.shape[0]
        a_all = torch.empty(n, dtype=torch.float64, device=opp.device)
        a_obj = torch.empty(n, dtype=torch.float64, device=opp.device)
        check(self._lib.rici_clutter_areas(self._h, _ptr(pos), pos.shape[0], _ptr(tri), tri.shape[0],
                                           int(object_first), int(object_count), _ptr(opp), _ptr(opn), n,
                                           float(support_radius), _ptr(a_all), _ptr(a_obj), _stream_ptr(stream)))
        return a_all, a_obj

    # ------------------------------------------------------ spin images
    def spin_generate(self, samples, op_positions, op_normals, support_radius: float, out=None, stream=None):
        """Spin Images of the oriented points over the point samples: float32 [N, 64, 64]."""
        torch = _torch()
        dev = self.device
        smp = _dev(samples, "samples", torch.float32, (3,), dev)
        opp = _dev(op_positions, "op_positions", torch.float32, (3,), dev)
        opn = _dev(op_normals, "op_normals", torch.float32, (3,), dev)
        if opp.shape != opn.shape:
            raise ValueError("op_positions and op_normals differ in shape")
        n = opp.shape[0]
        if out is None:
            out = torch.empty((n, NBINS, NBINS), dtype=torch.float32, device=opp.device)
        else:
            _dev(out, "out", torch.float32, (NBINS, NBINS), dev)
            if out.shape[0] != n:
                raise ValueError("out must have one image per oriented point")
        check(self._lib.rici_spin_generate(self._h, _ptr(smp), smp.shape[0], _ptr(opp), _ptr(opn), n,
                                           float(support_radius), _ptr(out), _stream_ptr(stream)))
        return out

    def spin_rank(self, needles, haystack, true_index, out_rank=None, out_true_correlation=None, stream=None):
        """Rank of the true match under Pearson correlation: (rank int32 [Nn]
        holding uint32, true correlation float64 [Nn])."""
        torch = _torch()
        dev = self.device
        nd = _dev(needles, "needles", torch.float32, (NBINS, NBINS), dev)
        hs = _dev(haystack, "haystack", torch.float32, (NBINS, NBINS), dev)
        ti = _dev(true_index, "true_index", torch.int32, None, dev)
        n = nd.shape[0]
        if ti.numel() != n:
            raise ValueError("true_index must have one entry per needle")
        if out_rank is None:
            out_rank = torch.empty(n, dtype=torch.int32, device=nd.device)
        if out_true_correlation is None:
            out_true_correlation = torch.empty(n, dtype=torch.float64, device=nd.device)
        check(self._lib.rici_spin_rank(self._h, _ptr(nd), n, _ptr(hs), hs.shape[0], _ptr(ti), _ptr(out_rank),
                                       _ptr(out_true_correlation), _stream_ptr(stream)))
        return out_rank, out_true_correlation

    def spin_correlation_matrix(self, needles, haystack, out=None, stream=None):
        """Pearson correlations float32 [Nn, Nh] from the fp32 contraction."""
        torch = _torch()
        dev = self.device
        nd = _dev(needles, "needles", torch.float32, (NBINS, NBINS), dev)
        hs = _dev(haystack, "haystack", torch.float32, (NBINS, NBINS), dev)
        if out is None:
            out = torch.empty((nd.shape[0], hs.shape[0]), dtype=torch.float32, device=nd.device)
        check(self._lib.rici_spin_correlation_matrix(self._h, _ptr(nd), nd.shape[0], _ptr(hs), hs.shape[0],
                                                     _ptr(out), _stream_ptr(stream)))
        return out

    def distance_rank(self, needles, haystack, true_index, out_rank=None, out_true_distance=None, stream=None):
        """(rank int32 [Nn], true-match CRD int64 [Nn]) of each needle's true match."""
        torch = _torch()
        dev = self.device
        nd = _dev(needles, "needles", torch.int32, (NBINS, NBINS), dev)
        hs = _dev(haystack, "haystack", torch.int32, (NBINS, NBINS), dev)
        ti = _dev(true_index, "true_index", torch.int32, None, dev)
        nn = nd.shape[0]
        if ti.dim() != 1 or ti.shape[0] != nn:
            raise ValueError("true_index must be [num_needles]")
        if out_rank is None:
            out_rank = torch.empty(nn, dtype=torch.int32, device=nd.device)
        if out_true_distance is None:
            out_true_distance = torch.empty(nn, dtype=torch.int64, device=nd.device)
        _dev(out_rank, "out_rank", torch.int32, None, dev)
        _dev(out_true_distance, "out_true_distance", torch.int64, None, dev)
        check(self._lib.rici_distance_rank(self._h, _ptr(nd), nn, _ptr(hs), hs.shape[0], _ptr(ti), _ptr(out_rank),
                                           _ptr(out_true_distance), _stream_ptr(stream)))
        return out_rank, out_true_distance

    def distance_matrix(self, needles, haystack, out=None, stream=None):
        """CRD(needle_i, haystack_j) as int64 [Nn, Nh]."""
        torch = _torch()
        dev = self.device
        nd = _dev(needles, "needles", torch.int32, (NBINS, NBINS), dev)
        hs = _dev(haystack, "haystack", torch.int32, (NBINS, NBINS), dev)
        if out is None:
            out = torch.empty((nd.shape[0], hs.shape[0]), dtype=torch.int64, device=nd.device)
        _dev(out, "out", torch.int64, (hs.shape[0],), dev)
        check(self._lib.rici_distance_matrix(self._h, _ptr(nd), nd.shape[0], _ptr(hs), hs.shape[0], _ptr(out),
                                             _stream_ptr(stream)))
        return out

    def sync(self, stream=None):
        """Wait for the stream and raise on errors the kernels reported."""
        check(self._lib.rici_sync(self._h, _stream_ptr(stream)))

    def device_errors(self) -> int:
        return int(self._lib.rici_device_errors(self._h))

    def batch(self, jobs, support_radius: float):
        """Plan a batched describe-and-rank (see Batch)."""
        return Batch(self, jobs, support_radius)

    # --------------------------------------------------------------- tuning
    def set_tuning(self, key: str, value: int):
        check(self._lib.rici_set_tuning(self._h, key.encode(), int(value)))

    def get_tuning(self, key: str) -> int:
        v = ctypes.c_int()
        check(self._lib.rici_get_tuning(self._h, key.encode(), ctypes.byref(v)))
        return v.value

    # --------------------------------------------------------------- timing
    def timing(self, on: bool = True):
        check(self._lib.rici_timing_enable(self._h, int(bool(on))))

    def timing_reset(self):
        check(self._lib.rici_timing_reset(self._h))

    def timing_get(self, kernel: str):
        ms = ctypes.c_double()
        n = ctypes.c_uint64()
        check(self._lib.rici_timing_get(self._h, kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


class Batch:
    """A recorded describe-and-rank plan over many meshes (rici_batch_*).

    jobs: list of dicts with device tensors
        positions [V,3] f32, triangles [T,3] i32, op_positions [N,3] f32,
        op_normals [N,3] f32, and optionally true_index [N] i32 (ranks each RICI
        of the mesh against the mesh's own RICIs).
    The plan allocates the outputs: images[k] ([N,64,64] i32), rank[k] and
    true_distance[k] (None for describe-only jobs).  run() replays the plan.
    """

    def __init__(self, ctx: Context, jobs, support_radius: float):
        torch = _torch()
        dev = ctx.device
        self._ctx = ctx
        self._keep = []
        self.images, self.rank, self.true_distance = [], [], []
        arr = (MeshJob * max(len(jobs), 1))()
        for k, j in enumerate(jobs):
            pos = _dev(j["positions"], "positions", torch.float32, (3,), dev)
            tri = _dev(j["triangles"], "triangles", torch.int32, (3,), dev)
            opp = _dev(j["op_positions"], "op_positions", torch.float32, (3,), dev)
            opn = _dev(j["op_normals"], "op_normals", torch.float32, (3,), dev)
            n = opp.shape[0]
            img = torch.empty((n, NBINS, NBINS), dtype=torch.int32, device=opp.device)
            ti = j.get("true_index")
            rk = ds = None
            if ti is not None:
                ti = _dev(ti, "true_index", torch.int32, None, dev)
                rk = torch.empty(n, dtype=torch.int32, device=opp.device)
                ds = torch.empty(n, dtype=torch.int64, device=opp.device)
            self._keep += [pos, tri, opp, opn, img, ti, rk, ds]
            self.images.append(img)
            self.rank.append(rk)
            self.true_distance.append(ds)
            arr[k] = MeshJob(_ptr(pos).value, pos.shape[0], _ptr(tri).value, tri.shape[0], _ptr(opp).value,
                             _ptr(opn).value, n, _ptr(img).value, _ptr(ti).value if ti is not None else None,
                             _ptr(rk).value if rk is not None else None, _ptr(ds).value if ds is not None else None)
        h = ctypes.c_void_p()
        check(ctx._lib.rici_batch_create(ctx._h, arr, len(jobs), float(support_radius), ctypes.byref(h)))
        self._h = h

    @property
    def scratch_bytes(self) -> int:
        return int(self._ctx._lib.rici_batch_scratch_bytes(self._h))

    def run(self, stream=None):
        check(self._ctx._lib.rici_batch_run(self._h, _stream_ptr(stream)))

    def kernel_ms(self, kernel: str) -> float:
        """Duration of the persistent "gen" or "search" kernel in the most recent
        run (HIP events recorded inside the graph; waits for that run)."""
        ms = ctypes.c_float()
        check(self._ctx._lib.rici_batch_kernel_ms(self._h, kernel.encode(), ctypes.byref(ms)))
        return float(ms.value)

    def close(self):
        if getattr(self, "_h", None):
            self._ctx._lib.rici_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
