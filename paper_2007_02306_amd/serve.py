"""Continuous-batching describe-and-match server over a device-resident RICI
database (control loop only: every device step is a librici call).

A request brings one mesh, the oriented points to describe (its needles) and
the database index of each needle's true match.  Its life:

  queued    waiting for a slot and for its HBM footprint to fit the budget;
  describe  on the describe stream: RICIs of the needles (rici_generate_noalloc:
            the library's static workspace, so no allocation or device-wide
            synchronisation in the loop), then
            rici_query_create (needle delta planes, exact true-match distances,
            exact counts of out-of-range images);
  scanning  joins the circular database scan at the next step once its
            describe work has completed; each scan step is one rici_db_scan
            over one slice of the database for every scanning request, so
            requests admitted while others are on the GPU share the same
            launches; after one full revolution (every slice once) its ranks
            are final (Sec. 4.1 step 6c, rank of the true match);
  done      ranks copied back, latency = completion - arrival.

Describe work (ALU bound) and scan work (MFMA bound) run on separate streams
and overlap on the device.  Each request's result is independent of what else
was in flight: ranks are integer sums over database slices.
"""

from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

from . import NOALLOC_MAX_TRIANGLES, NOALLOC_WORKSPACE_BYTES, Context, NBINS, _dev, _ptr, check
from . import roctx


def _torch():
    import torch
    return torch


def _to_dev(a, dtype, dev):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        return a.to(dev, dtype).contiguous()
    import numpy as np
    np_dtype = {torch.float32: np.float32, torch.int32: np.int32, torch.int64: np.int64}[dtype]
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(np_dtype))).to(dev)


class DescriptorDB:
    """A prepared, device-resident haystack (rici_db).  `images` is an int32
    [N, 64, 64] device tensor that must outlive the database."""

    def __init__(self, ctx: Context, images, stream=None):
        torch = _torch()
        self.ctx = ctx
        self.images = _dev(images, "images", torch.int32, (NBINS, NBINS), ctx.device)
        s = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        check(ctx._lib.rici_db_create(ctx._h, _ptr(self.images), self.images.shape[0], ctypes.c_void_p(s.cuda_stream),
                                      ctypes.byref(h)))
        self._h = h
        self.tiles = int(ctx._lib.rici_db_tiles(h))

    @property
    def size(self) -> int:
        return int(self.images.shape[0])

    @property
    def scratch_bytes(self) -> int:
        return int(self.ctx._lib.rici_db_scratch_bytes(self._h))

    def query_footprint(self, num_needles: int) -> int:
        return int(self.ctx._lib.rici_query_footprint(self._h, int(num_needles)))

    def close(self):
        if getattr(self, "_h", None):
            self.ctx._lib.rici_db_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Request:
    """positions [V,3] f32, triangles [T,3] u32-as-i32, normals [V,3] f32 (host
    numpy or device tensors), needle vertex ids [Q] and their true database
    indices [Q]."""
    rid: int
    positions: object
    triangles: object
    normals: object
    needle_ids: object
    true_index: object
    support_radius: float = 0.3
    arrival: float = 0.0
    admitted: float = 0.0
    finished: float = 0.0
    rank: object = None
    true_distance: object = None
    images: object = None
    # serving state
    _state: str = "queued"
    _dev: dict = field(default_factory=dict)
    _query: object = None
    _ready: object = None
    _done: object = None
    _slices_left: int = 0
    _footprint: int = 0

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Server:
    """Admission by HBM footprint, continuous batching of the database scan.

    budget_bytes: device memory the in-flight requests may hold (their
    tensors and query workspaces), plus the static generation workspace of the
    describe step, charged once.  max_active: at most this many
    requests scan at once (<= RICI_SCAN_MAX_QUERIES).  slices: the database is
    scanned in this many slices (one slice per step)."""

    def __init__(self, db: DescriptorDB, budget_bytes: int = 2 << 30, max_active: int = 8, slices: int = 16,
                 max_inflight_steps: int = 2, keep_images: bool = False):
        torch = _torch()
        self.db = db
        self.budget = int(budget_bytes)
        self.max_active = min(int(max_active), 24)
        self.slices = max(1, min(int(slices), db.tiles))
        self.bounds = [db.tiles * k // self.slices for k in range(self.slices + 1)]
        self.describe_ctx = Context(db.ctx.device)     # one handle per stream
        self.scan_ctx = db.ctx
        self.describe_stream = torch.cuda.Stream(device=db.ctx.device)
        self.scan_stream = torch.cuda.Stream(device=db.ctx.device)
        self.queue: list[Request] = []
        self.describing: list[Request] = []
        self.scanning: list[Request] = []
        self.finishing: list[Request] = []
        self.done: list[Request] = []
        # describe calls all use the GPU's static generation workspace; they are
        # serialised on the describe stream, so it is charged once
        self.used = NOALLOC_WORKSPACE_BYTES
        if self.used >= self.budget:
            raise ValueError("budget_bytes does not cover the describe workspace")
        self.cursor = 0
        self.steps_inflight: list = []
        self.max_inflight = int(max_inflight_steps)
        self.steps = 0
        self.keep_images = keep_images

    # ------------------------------------------------------------ footprint
    def footprint(self, req: Request) -> int:
        q = len(req.needle_ids)
        t = int(req.triangles.shape[0])
        v = int(req.positions.shape[0])
        images = q * NBINS * NBINS * 4
        inputs = v * 12 * 2 + t * 12 + q * (12 * 2 + 4 * 3 + 8)
        return images + inputs + self.db.query_footprint(q)

    def submit(self, req: Request, now: float | None = None):
        req.arrival = time.perf_counter() if now is None else now
        if int(req.triangles.shape[0]) > NOALLOC_MAX_TRIANGLES:
            raise ValueError(f"request {req.rid}: more than {NOALLOC_MAX_TRIANGLES} triangles")
        req._footprint = self.footprint(req)
        if req._footprint > self.budget - NOALLOC_WORKSPACE_BYTES:
            raise ValueError(f"request {req.rid} needs {req._footprint} bytes, above the whole budget")
        self.queue.append(req)

    # ---------------------------------------------------------------- steps
    def _admit(self):
        torch = _torch()
        while self.queue:
            req = self.queue[0]
            active = len(self.describing) + len(self.scanning) + len(self.finishing)
            if active >= self.max_active or self.used + req._footprint > self.budget:
                break
            self.queue.pop(0)
            self.used += req._footprint
            req.admitted = time.perf_counter()
            dev = torch.device("cuda", self.db.ctx.device)
            with roctx.range(f"admit+describe r{req.rid}"), torch.cuda.stream(self.describe_stream):
                t = lambda a, dt: _to_dev(a, dt, dev)
                pos = t(req.positions, torch.float32)
                tri = t(req.triangles, torch.int32)
                nrm = t(req.normals, torch.float32)
                ids = t(req.needle_ids, torch.int64)
                opp = pos.index_select(0, ids).contiguous()
                opn = nrm.index_select(0, ids).contiguous()
                ti = t(req.true_index, torch.int32)
                q = opp.shape[0]
                images = torch.empty((q, NBINS, NBINS), dtype=torch.int32, device=dev)
                rank = torch.empty(q, dtype=torch.int32, device=dev)
                dist = torch.empty(q, dtype=torch.int64, device=dev)
                ws = torch.empty(self.db.query_footprint(q), dtype=torch.uint8, device=dev)
                self.describe_ctx.generate_noalloc(pos, tri, opp, opn, req.support_radius, images,
                                                   stream=self.describe_stream)
                h = ctypes.c_void_p()
                lib = self.db.ctx._lib
                check(lib.rici_query_create(self.describe_ctx._h, self.db._h, _ptr(images), q, _ptr(ti), _ptr(rank),
                                            _ptr(dist), _ptr(ws), ws.numel(),
                                            ctypes.c_void_p(self.describe_stream.cuda_stream), ctypes.byref(h)))
                ev = torch.cuda.Event()
                ev.record(self.describe_stream)
            req._dev = dict(pos=pos, tri=tri, nrm=nrm, ids=ids, opp=opp, opn=opn, ti=ti, images=images, rank=rank,
                            dist=dist, ws=ws)
            req._query = h
            req._ready = ev
            req._state = "describe"
            self.describing.append(req)

    def _join(self):
        still = []
        for req in self.describing:
            if req._ready.query():
                req._state = "scanning"
                req._slices_left = self.slices
                self.scanning.append(req)
            else:
                still.append(req)
        self.describing = still

    def _scan_step(self):
        torch = _torch()
        self.steps_inflight = [e for e in self.steps_inflight if not e.query()]
        if not self.scanning or len(self.steps_inflight) >= self.max_inflight:
            return False
        k = self.cursor
        begin, count = self.bounds[k], self.bounds[k + 1] - self.bounds[k]
        arr = (ctypes.c_void_p * len(self.scanning))(*[r._query.value for r in self.scanning])
        with roctx.range(f"scan slice {k} x{len(self.scanning)}"):
            check(self.scan_ctx._lib.rici_db_scan(self.scan_ctx._h, self.db._h, arr, len(self.scanning), begin,
                                                  count, ctypes.c_void_p(self.scan_stream.cuda_stream)))
        ev = torch.cuda.Event()
        ev.record(self.scan_stream)
        self.steps_inflight.append(ev)
        self.cursor = (k + 1) % self.slices
        self.steps += 1
        still = []
        for req in self.scanning:
            req._slices_left -= 1
            if req._slices_left == 0:
                req._done = ev
                req._state = "finishing"
                self.finishing.append(req)
            else:
                still.append(req)
        self.scanning = still
        return True

    def _finish(self):
        lib = self.db.ctx._lib
        still = []
        for req in self.finishing:
            if req._done.query():
                roctx.push(f"finish r{req.rid}")
                req.finished = time.perf_counter()
                req.rank = req._dev["rank"].cpu().numpy().view("uint32")
                req.true_distance = req._dev["dist"].cpu().numpy()
                if self.keep_images:
                    req.images = req._dev["images"].cpu().numpy().view("uint32")
                lib.rici_query_destroy(req._query)   # caller workspace: no free, no wait
                req._query = None
                req._dev = {}
                req._state = "done"
                self.used -= req._footprint
                self.done.append(req)
                roctx.pop()
            else:
                still.append(req)
        self.finishing = still

    def poll(self) -> bool:
        """One pass of the loop; returns True while anything is in flight."""
        self._finish()
        self._join()
        self._admit()
        self._scan_step()
        return bool(self.queue or self.describing or self.scanning or self.finishing)

    def drain(self):
        while self.poll():
            time.sleep(0)

    def close(self):
        self.describe_ctx.close()


def serve_poisson(server: Server, requests, rate_hz: float, seed: int = 0):
    """Submit `requests` at Poisson arrival times of the given rate (wall
    clock) and serve them; returns the completed requests."""
    import numpy as np
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=len(requests))
    t0 = time.perf_counter()
    due = t0 + np.cumsum(gaps)
    i = 0
    while i < len(requests) or server.poll():
        now = time.perf_counter()
        while i < len(requests) and due[i] <= now:
            server.submit(requests[i], now=float(due[i]))
            i += 1
        server.poll()
    return server.done
