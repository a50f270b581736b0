#!/usr/bin/env python3
"""Benchmark of the whole RICI hot path on one MI355X.

One step = describe and rank one synthetic scene: every vertex of the union of
12 seeded superquadrics (23 352 oriented points, 46 656 triangles, support
radius 0.3, 64x64 images) gets its RICI (rici_generate), and every RICI is
ranked as a needle against all 23 352 RICIs as the haystack
(rici_distance_rank: column deltas, CRD contractions, true-match distance,
counts).  Inputs are resident in HBM before timing starts.

Prints one JSON line: throughput in RICIs described and ranked per second,
per-kernel roofline figures measured with HIP events on the library's stream,
and the CPU oracle timed on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0            # MI355X HBM3E
PEAK_INT8_TOPS = 5000.0          # MI355X dense int8 MFMA
PEAK_ALU_TOPS = 256 * 64 * 2.4e9 / 1e12   # 256 CUs x 64 lanes x 2.4 GHz, one op per lane per clock
OPS_PER_PAIR = 2 * 2 * 64 * 63   # two contractions over 4032 deltas, multiply + add


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-images", type=int, default=4096, help="oracle generation sample (images)")
    ap.add_argument("--cpu-needles", type=int, default=128, help="oracle rank sample (needles)")
    ap.add_argument("--workload", choices=["union12", "serving", "clutterbox"], default="union12",
                    help="union12: the describe-and-rank step (default); serving: Poisson request sweep; "
                         "clutterbox: the synthetic clutterbox experiment (rank-0 fractions at 1, 5, 10 objects)")
    ap.add_argument("--trials", type=int, default=30, help="clutterbox: trials")
    ap.add_argument("--batch-meshes", type=int, default=64,
                    help="meshes in the batched-vs-plain comparison (0 to skip)")
    ap.add_argument("--db-images", type=int, default=1_000_000, help="serving: database size")
    ap.add_argument("--requests", type=int, default=48, help="serving: requests per arrival rate")
    ap.add_argument("--no-other-configs", dest="other_configs", action="store_false",
                    help="skip the icosphere and clutter-scene figures")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy three times (scales the HBM byte counters)")
    return ap.parse_args()


KERNEL_SOURCES = {
    "k_gen": ["paper_2007_02306_amd/csrc/rici_gen.hip", "paper_2007_02306_amd/csrc/rici_internal.h"],
    "k_search": ["paper_2007_02306_amd/csrc/rici_search.hip", "paper_2007_02306_amd/csrc/rici_internal.h"],
}


def source_digest(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_record(kernel: str):
    """The committed counter record of `kernel` (see measured_traffic), or None
    when missing or taken from other sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_union12_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    return rec if rec.get("source_sha256") == source_digest(kernel) else None


def measured_busy(kernel: str):
    """Counter-derived VALU / MFMA busy fractions of `kernel` (rocprofv3 SQ
    counters on the same workload), or None."""
    rec = measured_record(kernel)
    if not rec or not rec.get("busy"):
        return None
    b = rec["busy"]
    key = "mfma_busy" if kernel == "k_search" else "valu_busy"
    return {key: b[key], "source": "profiles/union12_hbm_counters.md"}


def measured_traffic(kernel: str, launches_per_record: int = 1):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/<kernel>_union12_hbm_traffic.json: FETCH_SIZE and WRITE_SIZE per
    dispatch, each scaled by what the counter reads for a plain copy of known
    size), or None when the kernel's sources changed after the counters were
    taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_union12_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != source_digest(kernel):
        return None
    return rec["hbm_bytes_per_dispatch"] * launches_per_record


def copy_calibration():
    import torch
    n = 256 * 1024 * 1024                       # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": n * 4, "bytes_written": n * 4, "copies": 3}}), flush=True)


def cpu_baseline(scene, n_img, n_needles, gpu_images=None, gpu_rank=None):
    """The oracle, as it stands, on a bounded sample of the benchmark workload:
    generation of `n_img` seeded images and ranking of `n_needles` needles over
    a full-size haystack of oracle images; scaled to RICIs per second.  Also a
    1-thread figure on a smaller sample, and the parity verdict of the GPU's
    images (and ranks, against the GPU images as haystack) on the sample."""
    import numpy as np
    import oracle

    rng = np.random.default_rng(12345)
    n = scene.num_haystack
    sel = np.sort(rng.choice(n, min(n_img, n), replace=False))
    cores = oracle.threads(0)
    t0 = time.perf_counter()
    imgs, flags, work = oracle.rici_rowrange(scene.positions, scene.triangles, scene.op_positions[sel],
                                             scene.op_normals[sel], scene.support_radius, nthreads=cores)
    t_gen = (time.perf_counter() - t0) / len(sel)
    hay = np.resize(imgs, (n, 64, 64))          # full-size haystack of oracle images
    nsel = np.arange(min(n_needles, len(sel)))
    t0 = time.perf_counter()
    oracle.rank(imgs[nsel], hay, nsel.astype(np.uint32), nthreads=cores)
    t_rank = (time.perf_counter() - t0) / len(nsel)
    per_img = t_gen + t_rank
    # one thread, smaller sample
    s1 = sel[:64]
    t0 = time.perf_counter()
    oracle.rici_rowrange(scene.positions, scene.triangles, scene.op_positions[s1], scene.op_normals[s1],
                         scene.support_radius, nthreads=1)
    t_gen1 = (time.perf_counter() - t0) / len(s1)
    t0 = time.perf_counter()
    oracle.rank(imgs[:4], hay, np.arange(4, dtype=np.uint32), nthreads=1)
    t_rank1 = (time.perf_counter() - t0) / 4
    out = {
        "value": 1.0 / per_img,
        "unit": "RICIs/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"generation of {len(sel)} of {n} images + rank of {len(nsel)} needles against {n} "
                  f"haystack images; {t_gen * 1e3:.2f} ms/image + {t_rank * 1e3:.2f} ms/needle on {cores} threads",
        "single_thread": {"value": 1.0 / (t_gen1 + t_rank1), "unit": "RICIs/s",
                          "sample": f"generation of {len(s1)} images + rank of 4 needles on 1 thread"},
        "host": host_cpu(),
    }
    if gpu_images is not None:
        # parity of the GPU's images on the sample: equal at every pixel the
        # oracle does not flag; ranks of the sample needles against the GPU's
        # full haystack, true match = themselves shuffled
        g = gpu_images[sel]
        diff = (g != imgs)
        verdict = {"images": int(len(sel)), "pixels": int(diff.size), "flagged_pixels": int(flags.sum()),
                   "mismatches_outside_flags": int((diff & ~flags.astype(bool)).sum())}
        if gpu_rank is not None:
            ranks_gpu, needles_idx, true_idx = gpu_rank
            k = min(32, len(needles_idx))
            ork, _ = oracle.rank(gpu_images[needles_idx[:k]], gpu_images, true_idx[:k], nthreads=cores)
            verdict["ranks_checked"] = int(k)
            verdict["rank_mismatches"] = int((ork != ranks_gpu[:k]).sum())
        out["parity"] = verdict
    return out, work, sel


def host_cpu():
    """CPU model and logical CPU count of this host (the oracle's threads are
    capped separately by oracle.threads)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count()}


def value_distributions(images):
    """Statistics of a device image set (torch int32 [N,64,64]) that set the
    search's arithmetic paths: count histogram summary, needle-mask density
    (fraction of D != 0), per-image max |D| classes (<= 15: two contraction
    phases; 16..127: three; above: the exact int64 path)."""
    import torch
    x = images.to(torch.int64)
    d = x[:, :, 1:] - x[:, :, :-1]
    mx = d.abs().amax(dim=(1, 2))
    n = images.shape[0]
    hist = torch.bincount(images.clamp(max=16).flatten().to(torch.int64), minlength=17).cpu().tolist()
    return {
        "count_histogram_0_to_16plus": hist,
        "max_count": int(images.max()),
        "mask_density": float((d != 0).float().mean()),
        "max_abs_delta_share": {"le_15": float((mx <= 15).sum()) / n,
                                "16_to_127": float(((mx > 15) & (mx <= 127)).sum()) / n,
                                "gt_127": float((mx > 127).sum()) / n},
    }


def per_config(ctx, reps: int = 3):
    """Describe-and-rank figures of the icosphere (every image, full matrix)
    and of the clutter scene (haystack = every scene vertex, needles = object 0
    alone): best of `reps` runs each, HIP events for the kernels."""
    import numpy as np
    import torch
    import synth

    dev = torch.device("cuda:0")
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    i32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(dev)
    out = {}
    for name, make in (("icosphere", synth.config1_icosphere), ("clutter", synth.config3_clutter)):
        sc = make()
        hp, ht = f32(sc.positions), i32(sc.triangles)
        hop, hon = f32(sc.op_positions), f32(sc.op_normals)
        npos, ntri = f32(sc.needle_positions), i32(sc.needle_triangles)
        nop, non = f32(sc.needle_op_positions), f32(sc.needle_op_normals)
        ti = i32(sc.true_index)
        nh, nn = hop.shape[0], nop.shape[0]
        himg = torch.empty((nh, 64, 64), dtype=torch.int32, device=dev)
        nimg = himg if sc.needle_op_positions is sc.op_positions else torch.empty((nn, 64, 64), dtype=torch.int32,
                                                                                 device=dev)
        best = None
        for _ in range(reps + 1):
            ctx.timing(True)
            ctx.timing_reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.generate(hp, ht, hop, hon, sc.support_radius, out=himg)
            if nimg is not himg:
                ctx.generate(npos, ntri, nop, non, sc.support_radius, out=nimg)
            rank, dist = ctx.distance_rank(nimg, himg, ti)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            gen_ms = ctx.timing_get("gen")[0]
            search_ms = ctx.timing_get("search")[0]
            ctx.timing(False)
            if best is None or wall < best[0]:
                best = (wall, gen_ms, search_ms)
        wall, gen_ms, search_ms = best
        pairs_gen = nh * sc.triangles.shape[0] + (0 if nimg is himg else nn * sc.needle_triangles.shape[0])
        out[name] = {"images": int(nh + (0 if nimg is himg else nn)), "needles": int(nn), "haystack": int(nh),
                     "triangles": int(sc.triangles.shape[0]), "wall_ms": wall * 1e3, "gen_ms": gen_ms,
                     "search_ms": search_ms,
                     "rici_per_s": (nh + (0 if nimg is himg else nn)) / wall,
                     "image_triangle_pairs_per_s": pairs_gen / (gen_ms * 1e-3),
                     "distance_pairs_per_s": float(nn) * nh / (search_ms * 1e-3),
                     "search_int8_peak_frac": float(nn) * nh * OPS_PER_PAIR / (search_ms * 1e-3) / 1e12
                                              / PEAK_INT8_TOPS,
                     "ranks_per_s": nn / wall,
                     "max_rank": int(rank.max())}
        if name == "clutter":
            # the same ranks with the search's early exit (exact; off by default)
            ctx.set_tuning("search_early_exit", 1)
            best_e = None
            for _ in range(reps + 1):
                ctx.timing(True)
                ctx.timing_reset()
                rank_e, _ = ctx.distance_rank(nimg, himg, ti)
                torch.cuda.synchronize()
                ms = ctx.timing_get("search")[0]
                ctx.timing(False)
                best_e = ms if best_e is None else min(best_e, ms)
            ctx.set_tuning("search_early_exit", 0)
            out[name]["search_ms_early_exit"] = best_e
            out[name]["early_exit_ranks_equal"] = bool(torch.equal(rank_e, rank))
        if name == "icosphere":
            m = ctx.distance_matrix(nimg, himg)
            torch.cuda.synchronize()
            out[name]["matrix_checked_diagonal_zero"] = bool((torch.diagonal(m) == 0).all())
        del himg, nimg
    return out


def batched_vs_plain(ctx, meshes: int, seed: int = 4, reps: int = 3):
    """Describe-and-rank of `meshes` seeded meshes (log-uniform 1k-200k
    triangles, own frame, t(i) = i): one graph-replayed batched plan versus the
    plain per-mesh calls, on the same device buffers; both timed end to end."""
    import numpy as np
    import torch
    import synth

    rng = np.random.default_rng(seed)
    dev = torch.device("cuda:0")
    jobs, sizes = [], []
    for _ in range(meshes):
        t = int(round(np.exp(rng.uniform(np.log(1_000), np.log(200_000)))))
        m, _ = synth.configs.random_object(rng, t)
        pos = m.positions.astype(np.float32)
        nrm = synth.vertex_normals(pos, m.triangles)
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
        i = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(dev)
        jobs.append(dict(positions=f(pos), triangles=i(m.triangles), op_positions=f(pos), op_normals=f(nrm),
                         true_index=i(np.arange(pos.shape[0], dtype=np.uint32))))
        sizes.append((pos.shape[0], m.triangles.shape[0]))
    # batched form: knobs picked by the autotuner on a subset of the meshes
    # (not timed); plain form: a separate handle with the default knobs
    from paper_2007_02306_amd import Context
    from paper_2007_02306_amd.tune import Tuner
    tuner = Tuner(ctx, cache_path=None)
    t0 = time.perf_counter()
    knobs = tuner.tune_batch(jobs, 0.3)
    tune_s = time.perf_counter() - t0
    plan = tuner.batch(jobs, 0.3)
    plain_ctx = Context(0)

    def plain():
        for k, j in enumerate(jobs):
            img = plan.images[k]
            plain_ctx.generate(j["positions"], j["triangles"], j["op_positions"], j["op_normals"], 0.3, out=img)
            plain_ctx.distance_rank(img, img, j["true_index"], out_rank=plan.rank[k],
                                    out_true_distance=plan.true_distance[k])

    def timeit(fn):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return best

    def snapshot():
        """Per-image sums of the counts (int64), ranks and true distances of
        every mesh, as left in the plan's output buffers by the last run."""
        torch.cuda.synchronize()
        out = []
        for k in range(len(jobs)):
            im = plan.images[k]
            out.append((im.reshape(im.shape[0], -1).sum(dim=1, dtype=torch.int64).cpu(),
                        plan.rank[k].cpu().clone(), plan.true_distance[k].cpu().clone()))
        return out

    t_plain = timeit(plain)
    ref = snapshot()
    t_batch = timeit(plan.run)
    got = snapshot()
    ctx.sync()
    plain_ctx.sync()
    check = {"per_image_count_sums_equal": all(torch.equal(a[0], b[0]) for a, b in zip(ref, got)),
             "ranks_equal": all(torch.equal(a[1], b[1]) for a, b in zip(ref, got)),
             "true_distances_equal": all(torch.equal(a[2], b[2]) for a, b in zip(ref, got))}
    n_img = sum(v for v, _ in sizes)
    pairs = sum(v * v for v, _ in sizes)
    out = {"meshes": meshes, "images": n_img, "triangles": sum(t for _, t in sizes), "distance_pairs": pairs,
           "plain_s": t_plain, "batched_s": t_batch, "speedup": t_plain / t_batch,
           "batched_rici_per_s": n_img / t_batch, "plain_rici_per_s": n_img / t_plain,
           "plan_scratch_gb": plan.scratch_bytes / 1e9,
           "batched_equals_plain": check,
           "autotuned": {"gen_images_per_group": knobs[0], "search_tile_m": knobs[1], "tune_s": tune_s,
                         "candidates_ms": {f"{g}x{m}": ms for _, (g, m), ms in tuner.measurements}},
           "plain_knobs": {"gen_images_per_group": plain_ctx.get_tuning("gen_images_per_group"),
                           "search_tile_m": plain_ctx.get_tuning("search_tile_m")}}
    plan.close()
    plain_ctx.close()
    return out


def serving(args):
    """Poisson request sweep against a device-resident database of clutter-scene
    RICIs: p50/p99 latency and throughput per arrival rate."""
    import numpy as np
    import torch
    import synth
    from paper_2007_02306_amd import Context
    from paper_2007_02306_amd.serve import DescriptorDB, Request, Server, serve_poisson

    dev = torch.device("cuda:0")
    ctx = Context(0)
    rng = np.random.default_rng(5)
    chunks, objects, base = [], [], 0
    t0 = time.perf_counter()
    while base < args.db_images:
        mesh, canon, offsets, _ = synth.configs.clutter_scene(rng, 4, 1_000, 100_000, log_uniform=True)
        pos = mesh.positions.astype(np.float32)
        nrm = synth.vertex_normals(pos, mesh.triangles)
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
        i = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(dev)
        chunks.append(ctx.generate(f(pos), i(mesh.triangles), f(pos), f(nrm), 0.3))
        for o, m in enumerate(canon):
            objects.append((m, base + offsets[o]))
        base += pos.shape[0]
        print(f"# database: {base} images", file=sys.stderr, flush=True)
    images = torch.cat(chunks)[: args.db_images]
    del chunks
    objects = [(m, off) for m, off in objects if off + m.num_vertices <= images.shape[0]]
    db = DescriptorDB(ctx, images)
    ctx.sync()
    build_s = time.perf_counter() - t0

    def make_requests(n, seed):
        r = np.random.default_rng(seed)
        out = []
        for k in range(n):
            m, off = objects[int(r.integers(len(objects)))]
            pos = m.positions.astype(np.float32)
            nrm = synth.vertex_normals(pos, m.triangles)
            ids = np.sort(r.choice(pos.shape[0], min(1024, pos.shape[0]), replace=False))
            out.append(Request(k, pos, m.triangles, nrm, ids, (off + ids).astype(np.uint32)))
        return out

    # single-request service time (alone, sequential)
    srv = Server(db, max_active=1, slices=16)
    alone = make_requests(6, 1)
    t0 = time.perf_counter()
    for r in alone:
        srv.submit(r)
        srv.drain()
    mu = len(alone) / (time.perf_counter() - t0)
    srv.close()
    sweep = []
    for mult in (0.25, 0.5, 1.0, 2.0, 4.0):
        srv = Server(db, max_active=8, slices=16)
        reqs = make_requests(args.requests, int(mult * 100))
        t0 = time.perf_counter()
        done = serve_poisson(srv, reqs, rate_hz=mult * mu, seed=int(mult * 10))
        wall = time.perf_counter() - t0
        lat = np.array([r.latency for r in done]) * 1e3
        sweep.append({"rate_x_mu": mult, "rate_hz": mult * mu, "requests": len(done),
                      "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                      "throughput_rps": len(done) / wall, "scan_steps": srv.steps})
        print(f"# serving x{mult}: {sweep[-1]}", file=sys.stderr, flush=True)
        srv.close()
    out = {"metric": "serving latency and throughput (describe + rank against a device-resident RICI database)",
           "value": max(p["throughput_rps"] for p in sweep), "unit": "requests/s", "n_gpus": 1,
           "higher_is_better": True, "data": "synthetic (seeded clutter scenes; no dataset)",
           "config": {"workload": f"database of {images.shape[0]} clutter-scene RICIs, requests of up to 1024 "
                                  "needles from one canonical object of 1k-100k triangles, R=0.3",
                      "db_images": int(images.shape[0]), "db_tiles": db.tiles, "db_build_s": build_s},
           "single_request_rate_hz": mu, "sweep": sweep}
    print(json.dumps(out), flush=True)
    db.close()
    ctx.close()


def clutterbox(args):
    """The synthetic clutterbox experiment: per trial, objects of 1k-20k
    triangles (log-uniform) placed one by one into a cube of side 3; rank of
    every reference vertex's correct match at 1, 5 and 10 objects."""
    import numpy as np
    from paper_2007_02306_amd import Context
    from paper_2007_02306_amd.clutterbox import run_trial, summarise

    ctx = Context(0)
    rng = np.random.default_rng(2020)
    trials, gpu_s, searches = [], 0.0, 0
    t0 = time.perf_counter()
    for i in range(args.trials):
        r = run_trial(ctx, rng)
        trials.append(r)
        gpu_s += sum(v["gpu_s"] for v in r.values())
        searches += sum(v["reference_vertices"] * v["scene_vertices"] for v in r.values())
        print(f"# clutterbox trial {i + 1}/{args.trials}", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    summ = summarise(trials)
    out = {"metric": "clutterbox rank-0 fraction per clutter level (synthetic objects)",
           "value": summ[10]["rank0_fraction"], "unit": "fraction of searches with the correct match at rank 0",
           "higher_is_better": True, "n_gpus": 1, "data": "synthetic (seeded superquadrics and tori; no dataset)",
           "config": {"workload": "clutterbox, cube side 3, R = 0.3, objects of 1k-20k triangles, levels 1/5/10",
                      "trials": args.trials},
           "levels": {str(k): v for k, v in summ.items()},
           "gpu_describe_and_rank_s": gpu_s, "distance_pairs": searches, "wall_s": wall}
    print(json.dumps(out), flush=True)
    ctx.close()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2007_02306_amd import Context

    assert torch.cuda.is_available(), "bench.py needs the MI355X"
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "serving":
        serving(args)
        return
    if args.workload == "clutterbox":
        clutterbox(args)
        return
    dev = torch.device("cuda:0")
    scene = synth.config2_union12()
    N, T = scene.num_haystack, scene.triangles.shape[0]

    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    i32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(dev)
    pos, tri = f32(scene.positions), i32(scene.triangles)
    opp, opn = f32(scene.op_positions), f32(scene.op_normals)
    tidx = i32(scene.true_index)
    images = torch.empty((N, 64, 64), dtype=torch.int32, device=dev)
    rank = torch.empty(N, dtype=torch.int32, device=dev)
    dist = torch.empty(N, dtype=torch.int64, device=dev)

    ctx = Context(0)

    def step():
        ctx.generate(pos, tri, opp, opn, scene.support_radius, out=images)
        ctx.distance_rank(images, images, tidx, out_rank=rank, out_true_distance=dist)

    for _ in range(args.warmup):
        step()
    ctx.sync()
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.sync()
    ctx.timing(False)

    kernels = {}
    for k in ["gen_prep", "gen", "delta_needle", "delta_haystack", "true_distance", "search", "fallback"]:
        ms, n = ctx.timing_get(k)
        kernels[k] = {"avg_ms": ms / n if n else None, "launches": n}
    ms_step = elapsed * 1e3 / args.steps

    # roofline of the search contraction: exact algorithmic int8 ops per launch
    search_ms = kernels["search"]["avg_ms"]
    search_ops = float(N) * N * OPS_PER_PAIR
    search_achieved = search_ops / (search_ms * 1e-3) / 1e12
    roof_search = {"bound": "mfma", "achieved": search_achieved, "peak": PEAK_INT8_TOPS, "unit": "TFLOP/s",
                   "frac": search_achieved / PEAK_INT8_TOPS, "traffic": measured_traffic("k_search"),
                   "counters": measured_busy("k_search"), "kernel": "k_search",
                   "ops_per_launch": search_ops}

    cpu = None
    work = None
    if not args.no_cpu_baseline:
        # ranks of a seeded sample of needles against the GPU images with a
        # shuffled true-match map (non-trivial ranks) for the parity verdict
        rs = np.random.default_rng(7)
        nidx = np.sort(rs.choice(N, 32, replace=False))
        tmap = rs.permutation(N)[:32].astype(np.uint32)
        rk, _ = ctx.distance_rank(images[torch.from_numpy(nidx).to(dev)].contiguous(), images,
                                  i32(tmap))
        ctx.sync()
        host_images = images.cpu().numpy().view(np.uint32)
        cpu, work, _ = cpu_baseline(scene, args.cpu_images, args.cpu_needles, gpu_images=host_images,
                                    gpu_rank=(rk.cpu().numpy().view(np.uint32), nidx, tmap))
    dist = value_distributions(images)

    gen_ms = kernels["gen"]["avg_ms"]
    roof_gen = None
    if work is not None:
        # algorithmic ALU ops per image: 39 per triangle (projection of three
        # vertices + slab test), 40 per row slice, 1 per pixel update; slices and
        # updates per image averaged over the oracle's sample
        w = np.asarray(work, dtype=np.float64)
        per_img = 39.0 * T + 40.0 * w[:, 1].mean() + w[:, 2].mean()
        gen_ops = per_img * N
        gen_achieved = gen_ops / (gen_ms * 1e-3) / 1e12
        roof_gen = {"bound": "alu", "achieved": gen_achieved, "peak": PEAK_ALU_TOPS, "unit": "TFLOP/s",
                    "frac": gen_achieved / PEAK_ALU_TOPS, "traffic": measured_traffic("k_gen"),
                    "counters": measured_busy("k_gen"), "kernel": "k_gen", "ops_per_launch": gen_ops,
                    "ops_basis": "oracle work counters on the CPU-baseline sample",
                    "note": "the algorithmic count credits every (image, triangle) pair, as the method visits "
                            "all triangles per image; the kernel's exact bounding-sphere culls skip most of them, "
                            "so frac can exceed 1; counters.valu_busy is the hardware issue utilisation"}

    batched = batched_vs_plain(ctx, args.batch_meshes) if args.batch_meshes > 0 else None
    others = per_config(ctx) if args.other_configs else None

    dominant = "search" if (search_ms or 0) >= (gen_ms or 0) else "gen"
    roofline = roof_search if dominant == "search" or roof_gen is None else roof_gen
    value = N / (ms_step * 1e-3)
    out = {
        "metric": "RICIs generated/sec + needle x haystack distances/sec, batched vs plain, bit-exact",
        "value": value,
        "unit": "RICIs/s (described and ranked against the full haystack)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 geometry decisions, u32 counts, int8->int32 MFMA distances",
        "data": "synthetic (seeded superquadrics; no dataset)",
        "config": {"workload": "union of 12 seeded superquadrics, 23352 oriented points x 46656 triangles, "
                               "R=0.3, 64x64 u32 RICIs, all-vs-all CRD rank (23352 x 23352)",
                   "images": N, "triangles": T, "distance_pairs": N * N},
        "rates": {"rici_per_s": value, "distance_pairs_per_s": float(N) * N / (ms_step * 1e-3),
                  "ranks_per_s": value,
                  "gen_only_rici_per_s": N / (gen_ms * 1e-3) if gen_ms else None,
                  "image_triangle_pairs_per_s": float(N) * T / (gen_ms * 1e-3) if gen_ms else None,
                  "search_only_distance_pairs_per_s": float(N) * N / (search_ms * 1e-3) if search_ms else None},
        "value_distributions": dist,
        "roofline": roofline,
        "roofline_other": roof_gen if roofline is roof_search else roof_search,
        "kernels": kernels,
        "batched_vs_plain": batched,
        "other_configs": others,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
