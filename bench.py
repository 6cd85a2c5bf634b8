#!/usr/bin/env python3
"""Throughput of the NEB hot path on one MI355X.

A step is one progressive NEB iteration (one sample per pixel: view paths,
octree deposits, densities, NEE, photons from every NEE vertex with merges,
emission) over the room workload: a 10 x 10 x 3 m room (~2k triangles),
a 20k-triangle glass sphere (IOR 1.5) on a table and four emissive spheres,
512 x 512 pixels, path length 8, octree of 2^20 nodes, merge radius 0.02.
The 16 steps after the warm-up reproduce the workload's 16 spp.

Launch shapes are the library's defaults (tuned for this workload), or
tuned afresh with --autotune (they change the speed, not the result).  The
timed iterations are launched from the host, each forking the next one's
camera pass onto a third stream (--graph 1 replays the captured
iteration, --graph 2 launches the whole timed call as one captured graph;
HIP's graph replay runs these branches less concurrently); the per-kernel
passes launch eagerly too (their events need it).

Prints one JSON line with camera paths/s (value), photons/s, the roofline
of the dominant kernel (HIP-event durations on the launch stream, the
library's work counters for algorithmic bytes, HBM traffic from the
committed counter summary while the kernel source is unchanged), the FP64
oracle timed on the host cores over a bounded pixel window of the same
workload, the batched form (64 box rooms rendered in one context against
the same 64 scenes rendered one after another) and the learned-density form
(time to the plain form's RMSE at 64 spp).
"""
import hashlib
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "camera paths/s + photons/s at equal RMSE vs FP64 oracle; % of HBM roofline"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(stats, name, npix, vertices):
    """Bytes each kernel must move for the work it did (data layouts of the
    library: 16-byte float4 state words, 4-byte ints; the traversal kernels
    count every BVH node (64 bytes) and triangle (48 bytes) they fetch).
    Cache re-reads beyond that are excluded: this is the algorithmic
    minimum for the work the counters saw."""
    s = stats
    if name == "photon_merge":
        # photon state + U + hit in, two cell bounds per cell, one packed
        # (pos, id) per candidate, three vertex words + pixel and a 3-float
        # image atomic (read + write) per accepted merge
        return (s["photon_items"] * (48 + 4 + 8) + s["grid_cells"] * 8 +
                s["candidates"] * 16 + s["merges"] * (52 + 24))  # a merge reads 52 of its 64-byte record
    if name == "photon_scatter":
        # photon state + U + hit + the hit triangle's normal word in, next state out
        return s["photon_items"] * (48 + 4 + 8 + 16) + s["photon_continued"] * 52
    if name == "shade":
        rays = s["rays_camera"]
        return rays * (64 + 8) + vertices * 64 + s["continued_camera"] * 64 + s["events"] * 32
    if name == "nee":
        # light samples and shadow rays, their traversal (128-byte four-wide
        # nodes, 48-byte triangles), contributions and photons
        return (vertices * (64 + 4) + s["photons"] * 52 + s["nee_visible"] * 24 +
                s["bvh_nodes_shadow"] * 128 + s["bvh_tris_shadow"] * 48)
    if name in ("extend_camera", "extend_photon"):
        # ray in, hit out, and the traversal's node (128 B) and triangle (48 B) fetches
        kind = "camera" if name == "extend_camera" else "photon"
        rays = s["rays_camera"] if kind == "camera" else s["photon_items"]
        return rays * (16 + 16 + 8) + s["bvh_nodes_" + kind] * 128 + s["bvh_tris_" + kind] * 48
    if name == "density":
        return vertices * (16 + 16 + 4)
    if name == "octree_insert":
        return vertices * 16
    if name == "finalize":
        return s["events"] * (32 + 4 + 24)
    return None


def kernel_pass(R, stream, steps, npix):
    """Render `steps` iterations after a reset with an event pair around
    each launch (on the stream it runs on); returns the roofline of the
    kernel with the most time and every kernel's totals."""
    import torch
    R.reset()
    torch.cuda.synchronize()
    s1 = R.stats()
    R.profile_kernels(True)
    R.render(steps, stream=stream)
    torch.cuda.synchronize()
    prof = R.kernel_profile()
    R.profile_kernels(False)
    s2 = R.stats()
    d = {k: s2[k] - s1[k] for k in s2 if isinstance(s2[k], int)}
    d["rays_camera"] = d["camera_rays"]
    d["continued_camera"] = d["camera_rays"] - npix * steps  # every ray after the first bounce
    vertices = d["vertices"]
    kernels, best = {}, None
    for name, v in prof.items():
        nb = algorithmic_bytes(d, name, npix, vertices)
        kernels[name] = {"launches": v["launches"], "ms": round(v["total_ms"], 3),
                         "avg_us": round(1e3 * v["total_ms"] / max(1, v["launches"]), 2)}
        if nb is not None:
            kernels[name]["algorithmic_GBs"] = round(nb / (v["total_ms"] * 1e-3) / 1e9, 1)
            kernels[name]["algorithmic_bytes"] = int(nb)
            if best is None or v["total_ms"] > prof[best]["total_ms"]:
                best = name
    return roofline_of(kernels, best), kernels


def roofline_of(kernels, name):
    """The HBM roofline entry of kernel `name` from a kernel pass's totals:
    its algorithmic bytes per launch over its average launch duration."""
    if name is None or name not in kernels or "algorithmic_bytes" not in kernels[name]:
        return None
    v = kernels[name]
    per_launch = v["algorithmic_bytes"] / v["launches"]
    avg_s = v["ms"] * 1e-3 / v["launches"]
    achieved = per_launch / avg_s / 1e9
    traffic = committed_traffic(name)
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else int(traffic),
            "algorithmic_bytes_per_launch": int(per_launch),
            "avg_launch_us": round(1e6 * avg_s, 2)}


def cpu_baseline(target_s=11.0):
    """The oracle, untouched, on a window of the same workload (1 iteration):
    a 16x16 probe sizes a square window expected to take target_s."""
    from neb_inputs import room
    from oracle import oracle as O
    O.build()
    sc = room()
    osc = O.OracleScene(sc)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1

    def run(side):
        x0, y0 = 256 - side // 2, 256 - side // 2
        t0 = time.perf_counter()
        r = O.render(sc, n_iter=1, window=(x0, y0, x0 + side, y0 + side), n_threads=cores, oscene=osc)
        return r, time.perf_counter() - t0

    _, dt = run(16)
    side = int(max(16, min(256, 16 * (target_s / max(dt, 1e-3)) ** 0.5)))
    r, dt = run(side)
    paths = side * side
    host = ""
    try:
        with open("/proc/cpuinfo") as fh:
            host = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": paths / dt, "unit": "camera paths/s", "cores": cores, "kind": "oracle", "host_cpu": host,
            "sample": f"{side}x{side} pixel window at the centre of the 512x512 room, 1 iteration, full NEB "
                      f"(photons {int(r['stats']['photons'])}, merges {int(r['stats']['merges'])}) in {dt:.2f} s",
            "note": "the oracle's merge search is brute force over the window's view vertices, so its rate per "
                    "path falls as the window grows: the full image would run slower per path than this sample",
            "photons_per_s": r["stats"]["photons"] / dt}


def source_digest():
    """Digest of the sources that define the merge kernel's code, with
    comments and blank space removed (a comment edit keeps the counters)."""
    import re
    h = hashlib.sha256()
    for f in ("neb_render.hip", "neb_device.h", "neb_internal.h"):
        with open(os.path.join(ROOT, "paper_1909_00573_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def committed_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/<kernel>_room_counters.txt: 'key: value' lines), or None when
    the summary is missing or was taken from other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_room_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_digest") != source_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


MFMA_BF16_PEAK_TFLOPS = 2500.0
# multiply-adds of the model per sample, counted as 2 FLOP each: forward
# 80x64 + 64x64 + 64x64 + 64; training adds the backward data pass through
# W3 and W2 and the three weight-gradient products
MLP_FWD_FLOP = 2 * (80 * 64 + 64 * 64 + 64 * 64 + 64)
MLP_TRAIN_FLOP = MLP_FWD_FLOP + 2 * (64 * 64 + 64 * 64) + 2 * (80 * 64 + 64 * 64 + 64 * 64)


def mlp_roofline(stream, n_query=1835008, batch=65536, reps=20):
    """The learned density's kernels on the matrix cores: inference over
    n_query points (the room's NEE vertex slots of one iteration) and
    training steps (forward, backward, weight gradients, Adam) on batches of
    `batch`, each timed with HIP events on the launch stream; FLOPs count
    the model's multiply-adds, the peak is the dense bf16 one."""
    import numpy as np
    import torch
    from neb_inputs import query_points
    from paper_1909_00573_amd import neb
    q, nn = query_points(n_query, 5)
    Q = torch.from_numpy(q).cuda()
    N = torch.from_numpy(nn).cuda()
    T = torch.from_numpy(np.sin(7 * q[:batch, 0]).astype(np.float32) + 3.0).cuda()
    m = neb.Mlp(seed=1, max_batch=batch)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(k):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3 / k

    t_inf = timed(lambda: m.infer(Q, N, stream=stream), reps)
    Qb, Nb = Q[:batch].contiguous(), N[:batch].contiguous()
    t_trn = timed(lambda: m.train_step(Qb, Nb, T, lr=1e-3, stream=stream), reps)
    m.close()
    out = {}
    for name, t, flop in (("infer", t_inf, MLP_FWD_FLOP * n_query), ("train_step", t_trn, MLP_TRAIN_FLOP * batch)):
        ach = flop / t / 1e12
        out[name] = {"bound": "mfma", "achieved": round(ach, 2), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(ach / MFMA_BF16_PEAK_TFLOPS, 5), "us_per_call": round(1e6 * t, 1),
                     "flop_per_call": int(flop)}
    out["infer"]["queries"] = n_query
    out["train_step"]["batch"] = batch
    return out


def atomics_run(stream, blocks=2048, ops=16):
    """Device-scope atomic throughput (neb_atomic_probe): returning atomic
    adds and compare-and-swap increments over 2^20 words (4 MB, the room
    octree's node array) packed or one per 128-byte line, and on one word;
    G operations per second."""
    import torch
    from paper_1909_00573_amd import neb
    out = {}
    sink = torch.zeros(blocks * 256, dtype=torch.int32, device="cuda")
    for label, n_words, stride, nblk, k_ops in (("2^20 words packed", 1 << 20, 1, blocks, ops),
                                                 ("2^20 words, one per line", 1 << 20, 32, blocks, ops),
                                                 ("one word", 1, 1, 64, 4)):
        words = torch.zeros(n_words * stride, dtype=torch.int32, device="cuda")
        row = {}
        for kind, kname in ((0, "add"), (1, "cas")):
            neb.atomic_probe(words, n_words, stride, nblk, 1, kind, sink, stream=stream)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            neb.atomic_probe(words, n_words, stride, nblk, k_ops, kind, sink, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            t = a.elapsed_time(b) / 1e3
            n = nblk * 256 * k_ops
            row[kname + "_G_per_s"] = round(n / t / 1e9, 3)
        out[label] = row
        del words
    return out


def gather_run(stream, blocks=4096, ops=64):
    """Random-access read throughput (neb_gather_probe): 16- and 64-byte
    records at hashed indices over buffers of 32 MB (the room's merge cell
    table), 192 MB (the merge kernel's working set: table, sorted
    positions and merge records) and 1 GiB (beyond the chip's caches);
    G records and GB of records per second."""
    import torch
    from paper_1909_00573_amd import neb
    out = {}
    sink = torch.zeros(blocks * 256, dtype=torch.float32, device="cuda")
    for label, nbytes in (("32 MB", 32 << 20), ("192 MB", 192 << 20), ("1 GiB", 1 << 30)):
        buf = torch.rand(nbytes // 4, dtype=torch.float32, device="cuda")
        row = {}
        for width in (1, 4):
            neb.gather_probe(buf, width, blocks, 8, sink, stream=stream)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            neb.gather_probe(buf, width, blocks, ops, sink, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            t = a.elapsed_time(b) / 1e3
            n = blocks * 256 * ops
            row["%dB_G_per_s" % (16 * width)] = round(n / t / 1e9, 2)
            row["%dB_GB_per_s" % (16 * width)] = round(n * 16 * width / t / 1e9, 1)
        out[label] = row
        del buf
    return out


def octree_saturation(stream, steps=16):
    """How the room's octree capacity (2^20 nodes, which its first iteration
    fills) moves the density: the robust query of the default tree against
    the same workload's tree with 2^23 nodes after `steps` iterations, at
    the surface points of the first iteration's view vertices; and both
    against the k-nearest-neighbour estimate (k = 8) over those vertices
    (one iteration's worth, so noisier, but with no tree)."""
    import numpy as np
    import torch
    from neb_inputs import room
    from paper_1909_00573_amd import neb
    sc = room()
    dens, info = {}, {}
    pts = nrm = None
    for cap in (1 << 20, 1 << 23):
        R = neb.Renderer(sc.with_settings(octree_capacity=cap), flags=neb.FLAG_RECORD_PATHS)
        R.render(steps, stream=stream)
        st = R.stats()
        info[cap] = {"nodes": st["oct_allocated"], "split_failures": st["oct_overflow"], "depth": st["oct_depth"]}
        if pts is None:
            rec = R.records()
            live = (rec["type"] >= 1) & (rec["type"] <= 4)
            pos = rec["pos"][live].astype(np.float32)
            prim = rec["prim"][live]
            v = sc.vertices.astype(np.float64)
            t = sc.tris[prim]
            n = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
            n /= np.linalg.norm(n, axis=1, keepdims=True)
            pts = torch.from_numpy(pos).cuda()
            nrm = torch.from_numpy(n.astype(np.float32)).cuda()
        dens[cap] = R.query_density(pts, nrm, stream=stream).cpu().numpy().astype(np.float64)
        R.close()
    knn = neb.point_density(pts, pts, neb.DENSITY_KNN, 0.04, k=8, stream=stream).cpu().numpy().astype(np.float64)
    a, b = dens[1 << 20], dens[1 << 23]
    ok = (a > 0) & (b > 0) & (knn > 0)

    def rel(x, y):
        d = np.abs(x[ok] / y[ok] - 1)
        return {"median": round(float(np.median(d)), 4), "p90": round(float(np.quantile(d, 0.9)), 4),
                "over_10pct": round(float(np.mean(d > 0.1)), 4)}

    return {"points": int(len(a)), "trees": {str(k): v for k, v in info.items()},
            "default_vs_2^23": rel(a, b), "default_vs_knn": rel(a, knn), "2^23_vs_knn": rel(b, knn),
            "note": "relative differences of the robust octree density at the first iteration's view vertices "
                    "after %d iterations; knn over those vertices only (one iteration)" % steps}


def tiny_box_run(stream, reps=50):
    """The tiny box workload whole (64 x 64, its 4 spp, path length 5,
    octree capacity 4096, robust density): reset and render its 4
    iterations, `reps` times; inputs resident."""
    import torch
    from neb_inputs import tiny_box
    from paper_1909_00573_amd import neb
    sc = tiny_box()
    R = neb.Renderer(sc)
    secs = {}
    for graph in (0, 1, 2):
        # (a graph variant's first render captures its graphs, untimed)
        R.use_graph(graph)
        R.reset()
        R.render(sc.spp, stream=stream)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            R.reset()
            R.render(sc.spp, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        secs[graph] = a.elapsed_time(b) / 1e3
    sec = secs[0]
    st = R.stats()
    R.close()
    paths = sc.width * sc.height * sc.spp * reps
    return {"workload": "tiny box: unit box, %d triangles, mirror sphere, 0.1 m ceiling light; %dx%d, %d spp, "
                        "path length %d, octree capacity %d, robust octree density" %
                        (sc.n_tris, sc.width, sc.height, sc.spp, sc.max_path_len, sc.octree_capacity),
            "renders": reps, "ms_per_render": round(1e3 * sec / reps, 3),
            "camera_paths_per_s": round(paths / sec, 1),
            # launch-bound: replaying the captured iterations (graph) or the
            # captured render call (call_graph) instead of launching their
            # kernels one by one
            "ms_per_render_graph": round(1e3 * secs[1] / reps, 3),
            "graph_speedup": round(secs[0] / secs[1], 3),
            "ms_per_render_call_graph": round(1e3 * secs[2] / reps, 3),
            "call_graph_speedup": round(secs[0] / secs[2], 3),
            # the statistics restart at each reset: st holds the last render's work
            "photons_per_s": round(st["photons"] * reps / sec, 1),
            "work_per_render": {k: st[k] for k in ("vertices", "photons", "photon_segments", "merges")},
            "octree": {"nodes": st["oct_allocated"], "capacity": st["oct_capacity"], "overflow": st["oct_overflow"]},
            "note": "each render is the whole 4-spp job after a reset (the reset included)"}


def city_block_run(stream, graph, steps=8, warmup=2):
    """Throughput on the city block (288 x 288 lots of 2.1 m, one box each,
    ~1.05 M triangles, a 50k-triangle mirror torus, 1024 point lights
    sampled by power 150-250 m above the block, 1024 x 1024, path length
    10, octree 2^24 nodes, merge radius 0.2 m): the largest workload, timed
    like the room (inputs resident, warm-up, then a reset) with launch
    shapes the autotuner picks for it."""
    import torch
    from neb_inputs import city_block
    from paper_1909_00573_amd import neb
    t0 = time.perf_counter()
    sc = city_block()
    R = neb.Renderer(sc)
    setup = time.perf_counter() - t0
    # the library's defaults are tuned on the room; this workload is tuned
    # afresh (shapes change the speed, not the result)
    cfg = R.autotune(2, stream=stream)
    R.use_graph(graph)  # with graphs the warm-up captures the iteration
    R.render(warmup, stream=stream)
    if graph == 2:  # the timed call's own graph, captured untimed
        R.reset()
        R.render(steps, stream=stream)
    torch.cuda.synchronize()
    R.reset()
    s0 = R.stats()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    R.render(steps, stream=stream)
    b.record(stream)
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) / 1e3
    st = R.stats()
    R.close()
    npix = sc.width * sc.height
    return {"workload": "city block: 605x605 m of 2.1 m lots, one box per lot, %d triangles, mirror torus, %d point "
                        "lights 150-250 m up; %dx%d, path length %d, octree 2^24 nodes, merge radius %.2f m, robust "
                        "octree density" %
                        (sc.n_tris, len(sc.point_lights), sc.width, sc.height, sc.max_path_len, sc.merge_radius),
            "steps": steps, "ms_per_step": round(1e3 * sec / steps, 3),
            "camera_paths_per_s": round(npix * steps / sec, 1),
            "photons_per_s": round((st["photons"] - s0["photons"]) / sec, 1),
            "photon_segments_per_s": round((st["photon_segments"] - s0["photon_segments"]) / sec, 1),
            "work_per_step": {k: round((st[k] - s0[k]) / steps) for k in
                              ("vertices", "nee_visible", "photons", "photon_segments", "merges", "camera_rays",
                               "shadow_rays", "bvh_nodes")},
            "launch_config": cfg, "host_setup_s": round(setup, 1)}


def batch_comparison(stream, cfg_trials=1):
    """64 box rooms (batch recipe, seed 4) rendered to their own spp in one
    batched context, against the same scenes rendered one after another in
    single-scene contexts with the same launch shapes.  A batched scene
    renders the same estimator as alone (same paths and photons), so equal
    spp is equal RMSE and the time ratio is the time-to-equal-RMSE ratio."""
    import torch
    from neb_inputs import batch_rooms
    from paper_1909_00573_amd import neb
    t0 = time.perf_counter()
    scenes = batch_rooms()
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    B = neb.BatchRenderer(scenes, spp=[s.spp for s in scenes])
    t_build = time.perf_counter() - t0
    cfg = B.autotune(cfg_trials, stream=stream)
    n_iter = max(s.spp for s in scenes)
    paths = sum(s.width * s.height * s.spp for s in scenes)

    def timed(render):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        render()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3

    B.reset()
    t_batch = timed(lambda: B.render(n_iter, stream=stream))
    st = B.stats()
    # the same as graph replays of the captured iterations (captured by a
    # first untimed render), and as one launch of a graph holding the whole
    # call (captured by an untimed call of the same length); the
    # iterations' kernels are long, so launching them is not what limits a
    # graph here
    B.use_graph(1)
    B.reset()
    B.render(2, stream=stream)
    B.reset()
    t_graph = timed(lambda: B.render(n_iter, stream=stream))
    B.use_graph(2)
    B.reset()
    B.render(n_iter, stream=stream)
    B.reset()
    t_call = timed(lambda: B.render(n_iter, stream=stream))
    B.close()
    del B
    # the same scenes one after another (contexts built beforehand, not timed)
    ctxs = []
    t_seq = 0.0
    for sc in scenes:
        R = neb.Renderer(sc, spp=sc.spp)
        # the batch's stack is deeper than every scene's BVH
        R.set_launch_config(cfg["bvh_stack"], cfg["trace_blocks_per_cu"], cfg["photon_blocks_per_cu"],
                            cfg["photon_order"], cfg["nee_blocks_per_cu"])
        t_seq += timed(lambda: R.render(sc.spp, stream=stream))
        R.close()
    return {"scenes": len(scenes), "triangles": int(sum(s.n_tris for s in scenes)),
            "pixels": int(sum(s.width * s.height for s in scenes)), "camera_paths": int(paths),
            "photons": int(st["photons"]), "launch_config": cfg,
            "batched_s": round(t_batch, 4), "batched_graph_s": round(t_graph, 4),
            "batched_call_graph_s": round(t_call, 4), "sequential_s": round(t_seq, 4),
            "batched_paths_per_s": round(paths / t_batch, 1), "sequential_paths_per_s": round(paths / t_seq, 1),
            "speedup": round(t_seq / t_batch, 3), "speedup_graph": round(t_seq / t_graph, 3),
            "speedup_call_graph": round(t_seq / t_call, 3),
            "host_setup_s": {"generate": round(t_gen, 1), "bvh_and_pools": round(t_build, 1)}}


def rel_rmse(img, ref):
    import numpy as np
    return float(np.sqrt(np.mean((img.astype(np.float64) - ref) ** 2)) / np.mean(ref))


def block_rel_rmse(img, ref, k=8):
    """Relative RMSE of k x k pixel block means: insensitive to single bright
    pixels, sensitive to bias."""
    import numpy as np
    H, W = ref.shape[:2]
    a = img[:H - H % k, :W - W % k].astype(np.float64).reshape(H // k, k, W // k, k, -1).mean(axis=(1, 3))
    r = ref[:H - H % k, :W - W % k].reshape(H // k, k, W // k, k, -1).mean(axis=(1, 3))
    return float(np.sqrt(np.mean((a - r) ** 2)) / np.mean(r))


def quality_comparison(stream, spp=64, ref_spp=1024, target_spp=16, train_iterations=4, check_every=4):
    """Error against time on the room for several forms, each rendered to
    `spp` and checked every `check_every` iterations against a reference:
    - plain: NEB with the robust octree density (the headline form);
    - single_probe: NEB with the one-probe octree density;
    - light_photons: NEB plus one conventional light photon per pixel and
      iteration (the optional technique of Sec. 4);
    - learned: NEB with the learned density (trained on the octree for the
      first `train_iterations` iterations, then used with region-gated
      octree fallback);
    - fixed_radius, knn: NEB with the two estimators Sec. 5 tried before
      the octree (radius 0.04 m; k = 8 within 0.04 m);
    - path_tracing, path_tracing_recycled: no photons, NEE as usual or
      recycled from the NEE vertices within 0.02 m (Sec. 6's experiment).
    The reference is path tracing with NEE and light photons (no NEB
    photons, so no density estimate enters it) at `ref_spp`, seed + 1000;
    the same estimator equals the FP64 oracle element by element at a
    reduced size (tests/test_gpu_room_parity.py), and a second reference
    from seed + 2000 gives its own error.  Errors: relative RMSE (R22) and
    the same over 8 x 8 pixel block means.  The target is the plain form's
    error at `target_spp` (the workload's spp); each form reports the
    samples and the render time (GPU events around the render calls, the
    checks excluded) to reach it, by either measure."""
    import numpy as np
    import torch
    from neb_inputs import room
    from paper_1909_00573_amd import neb

    def timed(render):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        render()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3

    sc = room()
    nlp = sc.width * sc.height
    refs = []
    ref_s = 0.0
    for off in (1000, 2000):
        R = neb.Renderer(sc.with_settings(seed=sc.seed + off), flags=neb.FLAG_NO_PHOTONS, light_photons=nlp)
        ref_s += timed(lambda: R.render(ref_spp, stream=stream))
        refs.append(R.image_host().astype(np.float64))
        R.close()
    ref = refs[0]
    # two independent references: their difference has sqrt(2) x the error of one
    ref_err = rel_rmse(refs[1], ref) / np.sqrt(2.0)
    ref_err_block = block_rel_rmse(refs[1], ref) / np.sqrt(2.0)

    density_ms = {}

    def progression(name, R):
        t, curve = 0.0, []
        R.profile_kernels(True)
        for it in range(check_every, spp + 1, check_every):
            t += timed(lambda: R.render(check_every, stream=stream))
            img = R.image_host().astype(np.float64)
            curve.append((it, t, rel_rmse(img, ref), block_rel_rmse(img, ref), img.mean() / ref.mean() - 1))
        prof = R.kernel_profile()
        R.profile_kernels(False)
        density_ms[name] = round(sum(prof.get(k, {"total_ms": 0.0})["total_ms"]
                                     for k in ("octree_insert", "density", "density_grid", "nee_recycle")) / spp, 4)
        return curve

    curves = {}
    for name, kw in (("plain", {}), ("single_probe", {"density_mode": neb.DENSITY_OCTREE}),
                     ("light_photons", {"light_photons": nlp}),
                     ("fixed_radius", {"density_mode": neb.DENSITY_RADIUS, "density_radius": 0.04}),
                     ("knn", {"density_mode": neb.DENSITY_KNN, "density_radius": 0.04, "knn_k": 8}),
                     ("path_tracing", {"flags": neb.FLAG_NO_PHOTONS}),
                     ("path_tracing_recycled", {"flags": neb.FLAG_NO_PHOTONS, "nee_radius": 0.02})):
        P = neb.Renderer(sc, **kw)
        curves[name] = progression(name, P)
        P.close()
    M = neb.Renderer(sc, density_mode=neb.DENSITY_MLP)
    M.configure_mlp(train_iterations=train_iterations)
    curves["learned"] = progression("learned", M)
    status = M.mlp_status()
    M.close()
    at = next(r for r in curves["plain"] if r[0] == target_spp)
    target, target_block = at[2], at[3]
    # a second target the forms reach at different times: ten times the
    # reference's own block error (the plain form's drift keeps it above)
    target_ref = 10.0 * ref_err_block

    def time_to(curve, idx, tgt):
        for r in curve:
            if r[idx] <= tgt:
                return r[0], r[1]
        return None, None

    forms = {}
    for name, c in curves.items():
        it, t = time_to(c, 2, target)
        itb, tb = time_to(c, 3, target_block)
        itr, tr = time_to(c, 3, target_ref)
        forms[name] = {"rel_rmse": round(c[-1][2], 5), "block_rel_rmse": round(c[-1][3], 5),
                       "mean_deviation": round(c[-1][4], 5),
                       "s": round(c[-1][1], 4), "ms_per_spp": round(1e3 * c[-1][1] / spp, 3),
                       "density_ms_per_spp": density_ms[name],
                       "spp_to_target": it, "s_to_target": None if t is None else round(t, 4),
                       "speedup_to_target": None if t is None else round(at[1] / t, 3),
                       "spp_to_block_target": itb, "s_to_block_target": None if tb is None else round(tb, 4),
                       "speedup_to_block_target": None if tb is None else round(at[1] / tb, 3),
                       "spp_to_reference_target": itr, "s_to_reference_target": None if tr is None else round(tr, 4),
                       "curve": [[i, round(tt, 4), round(e, 5), round(eb, 5), round(md, 5)]
                                 for i, tt, e, eb, md in c]}
    return {"workload": "room 512x512, %d spp per form; light photons: %d per iteration; learned density "
                        "trained on the octree for %d iterations (250 Adam steps x 65536 each)" %
                        (spp, nlp, train_iterations),
            "reference": "path tracing with NEE and %d light photons per iteration, %d spp, seed %d (two references "
                         "%.1f s); its own relative RMSE %.5f, block %.5f" %
                         (nlp, ref_spp, sc.seed + 1000, ref_s, ref_err, ref_err_block),
            "reference_rel_rmse": round(ref_err, 5), "reference_block_rel_rmse": round(ref_err_block, 5),
            "target": "the plain form's error at %d spp: relative RMSE %.5f, block %.5f" %
                      (target_spp, target, target_block),
            "reference_target": "block error %.5f (10 x the reference's own)" % target_ref,
            "curve_columns": ["spp", "s", "rel_rmse", "block_rel_rmse", "mean_deviation"],
            "forms": forms,
            "learned_model": {k: status[k] for k in ("adam_steps", "last_loss", "probes", "probes_bad",
                                                     "regions_probed", "regions_disabled", "fallback_queries",
                                                     "probes_served", "probes_served_bad")}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel event pass")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-scene batching comparison")
    ap.add_argument("--no-quality", "--no-learned", dest="no_quality", action="store_true",
                    help="skip the error-against-time comparison (plain, light photons, learned density)")
    ap.add_argument("--no-city", action="store_true", help="skip the city-block throughput run")
    ap.add_argument("--no-tiny", action="store_true", help="skip the tiny-box throughput run")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned density's matrix-core roofline")
    ap.add_argument("--no-octree-extra", action="store_true",
                    help="skip the atomic-throughput probe and the octree capacity comparison")
    ap.add_argument("--graph", type=int, nargs="?", const=1, default=0, choices=(0, 1, 2),
                    help="1: replay the captured iteration as a HIP graph, 2: the whole timed call as one graph "
                         "(default 0: launch from the host)")
    ap.add_argument("--no-serialized", action="store_true",
                    help="skip the per-kernel pass with every launch on one stream")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the launch shapes on this workload first (default: the library's defaults)")
    ap.add_argument("--launch-config", default=None,
                    help="bvh_stack,trace_blocks_per_cu,photon_blocks_per_cu,photon_order[,nee_blocks_per_cu] "
                         "instead of autotuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 256 MiB device copy first (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the renderer runs on one GPU; --gpus {args.gpus} is not supported (several GPUs "
              "would each render their own iterations or scenes in a context of their own)", file=sys.stderr)
        sys.exit(2)

    import torch
    from neb_inputs import room
    from paper_1909_00573_amd import neb

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # one elementwise kernel that reads 256 MiB and writes 256 MiB
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b
    sc = room()
    npix = sc.width * sc.height
    R = neb.Renderer(sc)
    stream = torch.cuda.current_stream()
    if args.launch_config:
        R.set_launch_config(*[int(x) for x in args.launch_config.split(",")])
        launch_cfg = R.launch_config()
    elif args.autotune:
        launch_cfg = R.autotune(2, stream=stream)
    else:
        launch_cfg = R.launch_config()
    R.use_graph(args.graph)
    # warm-up on a throw-away progression (it captures the graph), then start
    # the 16-spp render afresh
    R.render(args.warmup, stream=stream)
    if args.graph == 2:
        # a whole-call graph is captured per iteration count: capture the
        # timed call's, untimed
        R.reset()
        R.render(args.steps, stream=stream)
    torch.cuda.synchronize()
    R.reset()
    s0 = R.stats()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    R.render(args.steps, stream=stream)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    st = R.stats()
    sec = ms / 1e3
    paths = npix * args.steps
    photons = st["photons"] - s0["photons"]

    # per-kernel pass: same steps again with an event pair around each launch
    roof, kernels, roof_ser, kernels_ser = None, {}, None, {}
    if not args.no_profile:
        roof, kernels = kernel_pass(R, stream, args.steps, npix)
    if not args.no_profile and not args.no_serialized:
        # the same once more with every launch on one stream: each kernel's
        # duration alone (the roofline above is the kernel as it runs,
        # beside the launches that overlap it)
        cfg = R.launch_config()
        R.set_launch_config(cfg["bvh_stack"], cfg["trace_blocks_per_cu"], cfg["photon_blocks_per_cu"],
                            cfg["photon_order"], cfg["nee_blocks_per_cu"], concurrent=0)
        roof_ser, kernels_ser = kernel_pass(R, stream, args.steps, npix)
        R.set_launch_config(cfg["bvh_stack"], cfg["trace_blocks_per_cu"], cfg["photon_blocks_per_cu"],
                            cfg["photon_order"], cfg["nee_blocks_per_cu"], concurrent=cfg["concurrent"])
        # the dominant kernel is the one with the most time alone (with
        # launches overlapping, a kernel's span also counts the time it
        # shares the chip); the roofline reports it as it runs
        if roof_ser is not None:
            roof = roofline_of(kernels, roof_ser["kernel"]) or roof

    out = {
        "metric": METRIC, "value": round(paths / sec, 1), "unit": "camera paths/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "photons_per_s": round(photons / sec, 1),
        "photon_segments_per_s": round((st["photon_segments"] - s0["photon_segments"]) / sec, 1),
        "config": {"workload": "room: 10x10x3 m, %d triangles, glass sphere IOR 1.5 on a table, 4 emissive "
                               "spheres r=0.02; 512x512, 1 spp per step, max path length 8, octree 2^20 nodes, "
                               "merge radius 0.02, robust octree density" % sc.n_tris,
                   "width": sc.width, "height": sc.height, "spp_per_step": 1, "max_path_len": sc.max_path_len,
                   "triangles": sc.n_tris, "octree_capacity": sc.octree_capacity, "merge_radius": sc.merge_radius},
        "octree": {"ledger": st["oct_ledger"], "deposits": st["oct_deposits"], "nodes": st["oct_allocated"],
                   "depth": st["oct_depth"], "overflow": st["oct_overflow"]},
        "work_per_step": {k: round((st[k] - s0[k]) / args.steps) for k in
                          ("vertices", "photons", "photon_segments", "merges", "candidates", "grid_cells",
                           "camera_rays", "shadow_rays", "bvh_nodes", "bvh_tris", "bvh_nodes_camera",
                           "bvh_nodes_photon", "bvh_nodes_shadow", "bvh_tris_camera", "bvh_tris_photon",
                           "bvh_tris_shadow")},
        "roofline": roof, "kernels": kernels, "launch_config": launch_cfg,
        "timed_launches": {0: "eager", 1: "graph replay per iteration", 2: "one graph per call"}[args.graph],
        "roofline_serialized": roof_ser, "kernels_serialized": kernels_ser,
    }
    R.close()
    if not args.no_mlp:
        out["roofline_mlp"] = mlp_roofline(stream)
    if not args.no_octree_extra:
        out["atomics"] = atomics_run(stream)
        ins = kernels_ser.get("octree_insert") if kernels_ser else None
        if ins:
            # deposits of the serialised pass over the same steps, per second of octree_insert alone
            rate = (st["oct_deposits"] - s0["oct_deposits"]) / (ins["ms"] * 1e-3) / 1e9
            cas = out["atomics"]["2^20 words packed"]["cas_G_per_s"]
            out["atomics"]["octree_insert_deposits_G_per_s"] = round(rate, 3)
            out["atomics"]["octree_insert_frac_of_cas"] = round(rate / cas, 4)
        out["octree_saturation"] = octree_saturation(stream)
        out["gather"] = gather_run(stream)
        pm = kernels_ser.get("photon_merge") if kernels_ser else None
        if pm:
            # the merge kernel's random reads: per cell lookup its row of the
            # start table and its run of candidates, per accepted merge its
            # record (photon state is read in queue order, not counted)
            work = {k: st[k] - s0[k] for k in ("grid_cells", "merges")}
            reads = 2 * work["grid_cells"] + work["merges"]
            rate = reads / (pm["ms"] * 1e-3) / 1e9
            ceil = out["gather"]["192 MB"]["64B_G_per_s"]
            out["gather"]["photon_merge_random_reads_G_per_s"] = round(rate, 2)
            out["gather"]["photon_merge_frac_of_64B_gather"] = round(rate / ceil, 4)
    if not args.no_tiny:
        out["tiny_box"] = tiny_box_run(stream)
    if not args.no_city:
        out["city_block"] = city_block_run(stream, args.graph)
    if not args.no_batch:
        out["batch"] = batch_comparison(stream)
    if not args.no_quality:
        out["quality"] = quality_comparison(stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
