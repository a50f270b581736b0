"""Autotuner for the launch shapes of librici (rici_set_tuning knobs).

Knobs (results never depend on them, only speed):
    gen_images_per_group   images sharing a generation workgroup: 2 or 4
    gen_sort_triangles     triangle order for the generation culls: 0 mesh order, 1 Morton order
    search_tile_m          needles per search workgroup tile: 256 or 128

A choice is made per shape class by timing every candidate on a calibration
subset of the real inputs with the library's own HIP-event timers, and is kept
in a JSON cache keyed by the GPU architecture and the shape class, so a class
is measured once per machine:

    tuner = Tuner(ctx, cache_path)
    tuner.generate(positions, triangles, op_positions, op_normals, R)   # tuned rici_generate
    tuner.distance_rank(needles, haystack, true_index)                  # tuned rici_distance_rank
    plan = tuner.batch(jobs, R)                                         # tuned rici_batch_* plan

Shape classes:
    generation  log2 of the triangle count, log2 of the oriented-point count
                (both floored, capped) and the support radius relative to the
                mesh's bounding radius in half-octaves;
    search      needle tiles of 128 needed (1, 2, 3, ... capped at 16: the
                padding of the two tile heights differs only for small sets)
                and log2 of the haystack size;
    batch       mesh count, log2 of the total triangles and of the total
                oriented points.
"""

from __future__ import annotations

import json
import math
import os
import threading

GEN_CHOICES = (2, 4)
SORT_CHOICES = (0, 1)
SEARCH_CHOICES = (256, 128)

_lock = threading.Lock()


def _torch():
    import torch
    return torch


def _log2_bucket(x: int, cap: int = 40) -> int:
    return min(int(math.log2(max(int(x), 1))), cap)


class Tuner:
    """Picks knob values for one Context (they are set on its handle before
    each call).  cache_path None keeps the cache in memory only."""

    def __init__(self, ctx, cache_path: str | None = None, reps: int = 3, gen_sample: int = 1024,
                 search_haystack_sample: int = 32768, arch: str | None = None):
        torch = _torch()
        self.ctx = ctx
        self.cache_path = cache_path
        self.reps = int(reps)
        self.gen_sample = int(gen_sample)
        self.search_haystack_sample = int(search_haystack_sample)
        if arch is None:
            props = torch.cuda.get_device_properties(ctx.device)
            arch = getattr(props, "gcnArchName", props.name)
        self.arch = arch
        self.cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)
        self.measurements = []      # (key, choice, ms) of every timing taken

    # ------------------------------------------------------------ cache
    def _get(self, key):
        return self.cache.get(self.arch, {}).get(key)

    def _put(self, key, value):
        self.cache.setdefault(self.arch, {})[key] = value
        if self.cache_path:
            with _lock:
                os.makedirs(os.path.dirname(os.path.abspath(self.cache_path)), exist_ok=True)
                tmp = self.cache_path + ".tmp"
                with open(tmp, "w") as f:
                    json.dump(self.cache, f, indent=1, sort_keys=True)
                os.replace(tmp, self.cache_path)

    # ----------------------------------------------------------- timing
    def _time(self, kernel: str, fn) -> float:
        """Best of `reps` runs of fn, in ms of the named library kernel."""
        torch = _torch()
        ctx = self.ctx
        fn()                                   # warm up (workspace growth, code load)
        torch.cuda.synchronize()
        best = None
        for _ in range(self.reps):
            ctx.timing(True)
            ctx.timing_reset()
            fn()
            torch.cuda.synchronize()
            ms, n = ctx.timing_get(kernel)
            ctx.timing(False)
            best = ms if best is None else min(best, ms)
        return best

    # ------------------------------------------------------- generation
    @staticmethod
    def gen_class(positions, triangles, op_positions, R: float) -> str:
        torch = _torch()
        p = positions
        centre = (p.amax(0) + p.amin(0)) * 0.5
        radius = float(torch.linalg.vector_norm(p - centre, dim=1).max()) if p.shape[0] else 0.0
        rel = R / radius if radius > 0 else 1.0
        half_octaves = max(-12, min(12, int(math.floor(2 * math.log2(rel)))))
        return f"gen|t{_log2_bucket(triangles.shape[0], 30)}|n{_log2_bucket(op_positions.shape[0], 30)}|r{half_octaves}"

    def tune_generate(self, positions, triangles, op_positions, op_normals, R: float) -> tuple:
        """(gen_images_per_group, gen_sort_triangles) for this shape class."""
        key = self.gen_class(positions, triangles, op_positions, R)
        v = self._get(key)
        if v is not None:
            return (int(v), 2) if isinstance(v, int) else (int(v[0]), int(v[1]))
        torch = _torch()
        n = op_positions.shape[0]
        m = min(n, self.gen_sample)
        idx = torch.linspace(0, max(n - 1, 0), m, device=op_positions.device).round().long()
        opp = op_positions.index_select(0, idx).contiguous()
        opn = op_normals.index_select(0, idx).contiguous()
        out = torch.empty((m, 64, 64), dtype=torch.int32, device=opp.device)
        old = (self.ctx.get_tuning("gen_images_per_group"), self.ctx.get_tuning("gen_sort_triangles"))
        best, best_ms = None, None
        for g in GEN_CHOICES:
            for o in SORT_CHOICES:
                self.ctx.set_tuning("gen_images_per_group", g)
                self.ctx.set_tuning("gen_sort_triangles", o)
                # the triangle preparation is part of the cost of an order
                ms = sum(self._time(k, lambda: self.ctx.generate(positions, triangles, opp, opn, R, out=out))
                         for k in ("gen_prep", "gen"))
                self.measurements.append((key, (g, o), ms))
                if best_ms is None or ms < best_ms:
                    best, best_ms = (g, o), ms
        self.ctx.set_tuning("gen_images_per_group", old[0])
        self.ctx.set_tuning("gen_sort_triangles", old[1])
        self._put(key, list(best))
        return best

    def generate(self, positions, triangles, op_positions, op_normals, R: float, out=None, stream=None):
        g, o = self.tune_generate(positions, triangles, op_positions, op_normals, R)
        self.ctx.set_tuning("gen_images_per_group", g)
        self.ctx.set_tuning("gen_sort_triangles", o)
        return self.ctx.generate(positions, triangles, op_positions, op_normals, R, out=out, stream=stream)

    # ----------------------------------------------------------- search
    @staticmethod
    def search_class(num_needles: int, num_haystack: int) -> str:
        tiles128 = min(-(-int(num_needles) // 128), 16)
        return f"search|m{tiles128}|h{_log2_bucket(num_haystack, 40)}"

    def tune_search(self, needles, haystack, true_index) -> int:
        key = self.search_class(needles.shape[0], haystack.shape[0])
        v = self._get(key)
        if v is not None:
            return int(v)
        h = haystack[: min(haystack.shape[0], self.search_haystack_sample)]
        ti = true_index.clamp(max=h.shape[0] - 1) if h.shape[0] else true_index
        old = self.ctx.get_tuning("search_tile_m")
        best, best_ms = None, None
        for c in SEARCH_CHOICES:
            self.ctx.set_tuning("search_tile_m", c)
            ms = self._time("search", lambda: self.ctx.distance_rank(needles, h, ti))
            self.measurements.append((key, c, ms))
            if best_ms is None or ms < best_ms:
                best, best_ms = c, ms
        self.ctx.set_tuning("search_tile_m", old)
        self._put(key, best)
        return best

    def distance_rank(self, needles, haystack, true_index, **kw):
        c = self.tune_search(needles, haystack, true_index)
        self.ctx.set_tuning("search_tile_m", c)
        return self.ctx.distance_rank(needles, haystack, true_index, **kw)

    # ------------------------------------------------------------ batch
    @staticmethod
    def batch_class(jobs) -> str:
        tris = sum(int(j["triangles"].shape[0]) for j in jobs)
        pts = sum(int(j["op_positions"].shape[0]) for j in jobs)
        return f"batch|j{_log2_bucket(len(jobs), 20)}|t{_log2_bucket(tris, 40)}|n{_log2_bucket(pts, 40)}"

    def tune_batch(self, jobs, R: float, sample_jobs: int = 16):
        """(gen_images_per_group, search_tile_m, gen_sort_triangles) for a
        batched plan, timed as whole plan replays on an evenly spaced subset of
        the jobs (by size)."""
        key = self.batch_class(jobs)
        v = self._get(key)
        if v is not None:
            return tuple(v)
        torch = _torch()
        order = sorted(range(len(jobs)), key=lambda k: int(jobs[k]["triangles"].shape[0]))
        if len(order) > sample_jobs:
            order = [order[round(i * (len(order) - 1) / (sample_jobs - 1))] for i in range(sample_jobs)]
        sub = [jobs[k] for k in order]
        old = (self.ctx.get_tuning("gen_images_per_group"), self.ctx.get_tuning("search_tile_m"),
               self.ctx.get_tuning("gen_sort_triangles"))
        best, best_ms = None, None
        for g in GEN_CHOICES:
            for m in SEARCH_CHOICES:
                for srt in SORT_CHOICES:
                    self.ctx.set_tuning("gen_images_per_group", g)
                    self.ctx.set_tuning("search_tile_m", m)
                    self.ctx.set_tuning("gen_sort_triangles", srt)
                    plan = self.ctx.batch(sub, R)
                    ms = self._time("batch", plan.run)
                    plan.close()
                    self.measurements.append((key, (g, m, srt), ms))
                    if best_ms is None or ms < best_ms:
                        best, best_ms = (g, m, srt), ms
                    torch.cuda.synchronize()
        self.ctx.set_tuning("gen_images_per_group", old[0])
        self.ctx.set_tuning("search_tile_m", old[1])
        self.ctx.set_tuning("gen_sort_triangles", old[2])
        self._put(key, list(best))
        return best

    def batch(self, jobs, R: float):
        g, m, srt = self.tune_batch(jobs, R)
        self.ctx.set_tuning("gen_images_per_group", g)
        self.ctx.set_tuning("search_tile_m", m)
        self.ctx.set_tuning("gen_sort_triangles", srt)
        return self.ctx.batch(jobs, R)
