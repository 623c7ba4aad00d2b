"""Benchmark of the gfx950 hierarchical slope-intercept Hough vote.

One step = one full detection (edge staging from a binary image resident in
HBM, then the level-synchronous vote of both passes down to the finest
level, with every detected cell's voters kept on the device) of the
1024x1024 segment workload: 32 segments of length U[200, 1000] px, 1-2 px
thick, 2% salt noise, seed 0, T = 120, depth 10, 4-bit corner code variant.

Prints one JSON line.  ``value`` is line-region code tests per second
(code tests = E + 4 * sum of the votes of the regions that split, summed
over both passes), timed over the steps with no per-launch events; images
per second is reported beside it.  ``roofline`` prices the dominant kernel
against MI355X HBM bandwidth: its algorithmic bytes per step divided by its
summed launch duration, measured with HIP events on the library's stream
over a second set of steps run with per-level events.  ``cpu_baseline``
times the CPU oracle on the same image.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(stats_by_pass, detected_votes_by_pass, E):
    """What the method must move per step, independent of this design: per
    pass 8 E (the points) + sum_{1<=l<D} 12 L_l (a 4-byte id and two 4-byte
    coordinates per candidate test) + sum_{1<=l<=D} 4 L_l (a 4-byte id per
    kept vote), with L_l the summed votes of the regions split at level l and
    L_D those of the detected cells.  The points are cache resident, so the
    HBM traffic measured can sit below it."""
    total = 0
    for p, st in stats_by_pass.items():
        D = len(st) - 1
        if D < 1 or st[0]["split"] == 0:
            continue
        L = [int(st[l]["entries"]) for l in range(D)] + [int(detected_votes_by_pass[p])]
        total += 8 * E + sum(12 * L[l] for l in range(1, D)) + sum(4 * L[l] for l in range(1, D + 1))
    return total


def kernel_bytes(timing, entry_bytes):
    """Algorithmic bytes per step of the two list kernels.  k_count reads
    every (parent, line) entry once; k_write reads it again and writes each
    vote for a kept child (the next level's lists, the voters of detected
    cells at the finest level).  Per-tile and per-region side arrays are
    below 1% and not counted."""
    n_in, n_out = timing["vote_entries"], timing["vote_written"]
    return {"count": entry_bytes * n_in, "write": entry_bytes * (n_in + n_out)}

def kernel_source_digest():
    """sha256 of the kernel source with comments and blank space removed, so
    that only a change of the code itself counts as a new kernel."""
    import hashlib
    import re
    src = open(os.path.join(ROOT, "paper_1007_0547_amd", "csrc", "hh_kernels.hip")).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return hashlib.sha256(" ".join(src.split()).encode()).hexdigest()


def measured_traffic(workload):
    """HBM bytes per step of the two list kernels (FETCH_SIZE and WRITE_SIZE
    from rocprofv3, scaled by a plain copy) from the committed summary for
    this workload, or None when the kernel code has changed since the
    counters were taken (or there is no summary)."""
    path = os.path.join(ROOT, "profiles", f"list_kernels_{workload}_hbm_traffic.md")
    try:
        text = open(path).read()
        sha = kernel_source_digest()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != sha:
        return None
    v = fields.get("traffic_bytes_per_step")
    return float(v) if v else None


def _quad_key(i, j, level):
    """Quad-digit key of region (level, i, j): NE=0, NW=1, SW=2, SE=3 from level 1 down."""
    k = 0
    for b in range(level - 1, -1, -1):
        e, n = (i >> b) & 1, (j >> b) & 1
        k = k * 4 + ((n ^ 1) << 1 | (e ^ n))
    return k


_CPU = {}


def _cpu_init(x, y, W, H, T, D, k, deadline):
    _CPU.update(x=x, y=y, W=W, H=H, T=T, D=D, k=k, deadline=deadline)


def _cpu_subtree(task):
    import oracle
    g = _CPU
    if time.time() > g["deadline"]:
        return 0
    p, i, j, key, cand = task
    r = oracle.detect_subtree(g["x"], g["y"], g["W"], g["H"], g["T"], g["D"], p, g["k"], i, j, key, cand,
                              keep_members=False)
    return int(r.stats[p][:, 4].sum())


def cpu_baseline(w, budget_s=10.0, split=4):
    """The CPU oracle (plain C, depth-first search) on a bounded sample of
    the benchmark image: the subtrees of level `split` of both passes, each
    searched from its parent's voters, in a seeded random order, as many as
    finish in `budget_s` -- once on one thread and once over the host's
    cores (a process pool, one subtree per task).  Rates are code tests per
    second over the subtrees that finished.  Runs before the GPU is touched
    (the pool forks)."""
    import multiprocessing as mp

    import numpy as np

    import oracle
    x, y = oracle.edge_points(w.image)
    W, H, T, D = w.width, w.height, w.threshold, w.max_depth
    tasks = []
    for p in (0, 1):
        level = {(0, 0): np.arange(len(x), dtype=np.int32)}
        for lev in range(1, split + 1):
            kids = {}
            for (i, j), v in sorted(level.items()):
                if len(v) > T:
                    for e in (0, 1):
                        for n in (0, 1):
                            kids[(2 * i + e, 2 * j + n)] = v
            if lev == split:
                tasks += [(p, i, j, _quad_key(i, j, split), v) for (i, j), v in sorted(kids.items())]
            else:
                level = {c: oracle.region_voters(x, y, W, H, p, lev, c[0], c[1]) for c in kids}
    order = np.random.default_rng(0).permutation(len(tasks))
    tasks = [tasks[k] for k in order]

    _cpu_init(x, y, W, H, T, D, split, float("inf"))
    t0 = time.perf_counter()
    tests1, n1 = 0, 0
    while n1 < len(tasks) and (n1 == 0 or time.perf_counter() - t0 < budget_s):
        tests1 += _cpu_subtree(tasks[n1])
        n1 += 1
    t1 = time.perf_counter() - t0

    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    with mp.get_context("fork").Pool(cores, initializer=_cpu_init,
                                     initargs=(x, y, W, H, T, D, split, time.time() + budget_s)) as pool:
        t0 = time.perf_counter()
        done = [v for v in pool.imap_unordered(_cpu_subtree, tasks, chunksize=1)]
        tn = time.perf_counter() - t0
    testsn = sum(done)
    nn = sum(1 for v in done if v)
    model = ""
    try:
        model = next(ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": testsn / tn, "unit": "code tests/s", "cores": cores, "kind": "oracle",
            "sample": f"{nn} of the {len(tasks)} level-{split} subtrees of the benchmark image (both passes), "
                      f"each searched from its parent's voters by the C oracle, {cores} processes for "
                      f"{tn:.1f} s; the same sample order on one thread: {n1} subtrees in {t1:.1f} s",
            "single_thread": {"value": tests1 / t1, "unit": "code tests/s", "cores": 1, "subtrees": n1,
                              "seconds": t1},
            "host_cpu": model, "host_threads": os.cpu_count()}


def bench_batched(seed, reps=3, arena_gb=160, variants=("pool", "tuned", "graph", "plain")):
    """The 512-image batch (sides log-uniform in 128..2048, Poisson(24)
    segments, noise U[0.5%, 3%], T = floor(side / 10), depth
    ceil(log2(side))), resident in HBM.  Per step one
    hough_hier_detect_batch call over all 512 images, against the same
    images in one hough_hier_detect call each.  Batched forms: the library's
    pool (the batch runs in groups under its memory budget), the launch
    shape from the autotuner, and one group in a caller arena of `arena_gb`
    GB with the level launches captured once into a HIP graph and replayed."""
    import numpy as np
    import torch

    import synth
    from paper_1007_0547_amd import HoughHier

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    ws = synth.batch_images(seed=seed, n=512)
    imgs = [torch.from_numpy(w.image).to(dev) for w in ws]
    inputs = [dict(image=d, width=w.width, height=w.height, threshold=w.threshold)
              for d, w in zip(imgs, ws)]

    def timed(ctx, warm=2):
        for _ in range(warm):   # the first calls learn the arena sizes and groups
            for r in ctx.detect_batch(inputs):
                r.free()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(reps):
            rs = ctx.detect_batch(inputs)
            for r in rs:
                r.free()
        torch.cuda.synchronize(dev)
        dt = (time.perf_counter() - t0) / reps
        rs = ctx.detect_batch(inputs)
        t = rs[0].timing()
        info = [r.info for r in rs]
        for r in rs:
            r.free()
        return dt, t, info

    ctx = HoughHier(threshold=0, membership=True, device=0, stream=stream)
    batch_s, tmb, info = timed(ctx)
    code_tests = sum(i["code_tests"] for i in info)
    points = sum(i["n_points"] for i in info)
    cells = sum(sum(i["n_cells"]) for i in info)
    ctx.close()

    ctx_t = HoughHier(threshold=0, membership=True, device=0, stream=stream, timing=True)
    _, kt, _ = timed(ctx_t, warm=2)
    ctx_t.close()
    out = {
        "workload": f"512 images, seed {seed}, sides log-uniform 128..2048 "
                    f"(max side {max(max(w.width, w.height) for w in ws)}), "
                    "Poisson(24) segments, noise U[0.5%,3%], T=floor(side/10), depth ceil(log2 side), "
                    "both passes, voters kept on device",
        "edge_points": points, "cells": cells, "code_tests": code_tests,
        "batched": {"ms_per_batch": batch_s * 1e3, "images_per_s": 512 / batch_s,
                    "code_tests_per_s": code_tests / batch_s, "groups": tmb["groups"],
                    "kernel_ms": {"count": kt["count_ms"], "write": kt["write_ms"],
                                  "decide": kt["decide_ms"], "extract": kt["extract_ms"]},
                    "vote_entries": kt["vote_entries"], "vote_written": kt["vote_written"]},
        "entry_bytes_model": {k: {"bytes": v, "GB/s": v / (kt[f"{k}_ms"] / 1e3) / 1e9,
                                  "frac": v / (kt[f"{k}_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS}
                              for k, v in kernel_bytes(kt, 4).items()},
    }
    if "tuned" not in variants:
        return out

    ctx_a = HoughHier(threshold=0, membership=True, device=0, stream=stream)
    tuned = ctx_a.autotune(inputs)
    tuned_s, _, _ = timed(ctx_a)
    ctx_a.close()

    graph = None
    arena = ctx_g = None
    try:
        arena = torch.empty(int(arena_gb * 1e9), dtype=torch.uint8, device=dev)
        side = torch.cuda.Stream(dev)
        torch.cuda.synchronize(dev)
        ctx_g = HoughHier(threshold=0, membership=True, device=0, stream=side, arena=arena, graph=True)
        ctx_g.set_launch(**{k: tuned[k] for k in ("task_steps", "queue_batch", "wg_per_cu")})
        graph_s, tg, _ = timed(ctx_g)
        graph = {"ms_per_batch": graph_s * 1e3, "images_per_s": 512 / graph_s,
                 "graph_replayed": tg["graph_replayed"], "arena_gb": arena_gb, "groups": tg["groups"]}
    except Exception as e:   # not enough device memory for one group: reported, not fatal
        graph = {"error": str(e)}
    finally:
        if ctx_g is not None:
            ctx_g.close()
    # the arena goes back to the device, not to torch's cache, for the blocks that follow
    arena = ctx_g = None
    torch.cuda.empty_cache()

    ctx = HoughHier(threshold=0, membership=True, device=0, stream=stream)
    for inp in inputs:   # one untimed pass: the arena reaches the sizes the largest images need
        ctx.detect(**inp).free()
    torch.cuda.synchronize(dev)
    lat = []
    t0 = time.perf_counter()
    for inp in inputs:
        t1 = time.perf_counter()
        ctx.detect(**inp).free()
        lat.append(time.perf_counter() - t1)
    torch.cuda.synchronize(dev)
    plain_s = time.perf_counter() - t0
    ctx.close()
    best = min(batch_s, tuned_s, graph.get("ms_per_batch", 1e30) / 1e3)
    out.update({
        "batched_autotuned": {"launch": tuned, "ms_per_batch": tuned_s * 1e3, "images_per_s": 512 / tuned_s},
        "batched_arena_graph": graph,
        "plain": {"s_per_512": plain_s, "images_per_s": 512 / plain_s,
                  "code_tests_per_s": code_tests / plain_s,
                  "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                                 "p99": float(np.percentile(lat, 99) * 1e3)}},
        "batched_over_plain": plain_s / best,
    })
    return out


def solution_bytes(r):
    """Algorithmic bytes of the removal walk over one result: every voter id
    read once (4 B), each cell's voter range read (12 B) and its keep flag
    written (1 B), one plotted flag per point and pass (1 B)."""
    cells = sum(r.info["n_cells"])
    passes = bin(r.info["passes"]).count("1")
    return 4 * r.info["member_slots"] + 13 * cells + passes * r.info["n_points"]


def bench_solution(seed, reps=5):
    """solution() with point removal (hough_hier_solution) on the 1024x1024
    image and on the 512-image batch: the walk's device time from HIP events
    in the library (its rounds of segment walks, the host's checks between
    them included), its algorithmic bandwidth, and the whole call (voter id
    conversion included) once the context has its buffers; beside it, the
    detection of the same image."""
    import numpy as np
    import torch

    import synth
    import paper_1007_0547_amd as hh

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    w = synth.workload("seg1024", seed)
    img = torch.from_numpy(w.image).to(dev)
    ctx = hh.HoughHier(threshold=w.threshold, max_depth=w.max_depth, device=0, stream=stream)
    ms, call, det = [], [], []
    for k in range(reps + 1):
        torch.cuda.synchronize(dev)
        td = time.perf_counter()
        r = ctx.detect(image=img, width=w.width, height=w.height)
        torch.cuda.synchronize(dev)
        det.append((time.perf_counter() - td) * 1e3)
        t0 = time.perf_counter()
        m = hh.solution(r)
        t1 = time.perf_counter()
        if k > 0:
            ms.append(m)
            call.append((t1 - t0) * 1e3)
        sol = [r.solution(p) for p in (0, 1)]
        nbytes = solution_bytes(r)
        members = r.info["member_slots"]
        r.free()
    ctx.close()
    walk = float(np.median(ms))
    one = {"workload": f"seg1024: 1024x1024, seed {seed}, T={w.threshold}, depth {w.max_depth}, both passes",
           "walk_ms": walk, "call_ms": float(np.median(call)), "rounds": sol[0]["rounds"],
           "detect_ms": float(np.median(det[1:])), "member_entries": members,
           "kept": [s["kept"] for s in sol], "plotted": [s["plotted_points"] for s in sol],
           "alg_bytes": nbytes, "GB/s": nbytes / (walk / 1e3) / 1e9,
           "frac": nbytes / (walk / 1e3) / 1e9 / HBM_PEAK_GBS, "workgroups": 2}

    ws = synth.batch_images(seed=seed, n=512)
    imgs = [torch.from_numpy(x.image).to(dev) for x in ws]
    inputs = [dict(image=d, width=x.width, height=x.height, threshold=x.threshold) for d, x in zip(imgs, ws)]
    ctx = hh.HoughHier(threshold=0, device=0, stream=stream)
    rs = ctx.detect_batch(inputs)   # learns the arena sizes
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    hh.solution(rs)                 # first call: maps the call's id buffer (then cached by the context)
    first_b = (time.perf_counter() - t0) * 1e3
    for r in rs:
        r.free()
    rs = ctx.detect_batch(inputs)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    walk_b = hh.solution(rs)
    call_b = (time.perf_counter() - t0) * 1e3
    nbytes_b = sum(solution_bytes(r) for r in rs)
    members_b = sum(r.info["member_slots"] for r in rs)
    kept_b = sum(r.solution(p)["kept"] for r in rs for p in (0, 1))
    for r in rs:
        r.free()
    ctx.close()
    batch = {"workload": "the 512-image batch (seed %d), all 1024 passes in one launch" % seed,
             "walk_ms": walk_b, "call_ms": call_b, "first_call_ms": first_b, "member_entries": members_b,
             "kept": kept_b, "alg_bytes": nbytes_b, "GB/s": nbytes_b / (walk_b / 1e3) / 1e9,
             "frac": nbytes_b / (walk_b / 1e3) / 1e9 / HBM_PEAK_GBS, "workgroups": 1024}
    return {"seg1024": one, "batch512": batch}


def level_footprint(stats, depth, entry_bytes=4):
    """Bytes of each level's lists and tables (both passes): the level's half
    of the arena holds the region table (24 B), task table (8 B per task of
    1024 entries) and child votes (16 B) per region, and the list."""
    levels = []
    for l in range(depth):
        regions = int(stats[0]["split"][l] + stats[1]["split"][l])
        entries = int(stats[0]["entries"][l] + stats[1]["entries"][l])
        tasks = entries // 1024 + regions
        levels.append({"level": l, "regions": regions, "list_entries": entries,
                       "bytes": regions * 40 + tasks * 8 + entries * entry_bytes})
    return levels


def bench_sweep(seed, reps=20):
    """Code test against the circle test (the comparison method) at the sizes
    of the paper's Table 1 (32..256, T = 40, both passes): total votes (sum
    over evaluated regions) and GPU time per image, their ratios C_v and C_t,
    and whether the GPU votes equal the oracle's.  Images: full-span lines
    with 1% noise (the paper's own images are not available)."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_1007_0547_amd import HoughHier

    dev = torch.device("cuda:0")
    out = []
    for n in (32, 64, 128, 256):
        img = synth.full_span_image(seed, n, n, 8, 0.01)
        x, y = oracle.edge_points(img)
        d_img = torch.from_numpy(img).to(dev)
        row = {"size": n, "edge_points": int(len(x))}
        for variant in ("code", "circle"):
            ctx = HoughHier(threshold=40, variant=variant, membership=True, device=0,
                            stream=torch.cuda.current_stream(dev))
            for _ in range(3):
                ctx.detect(image=d_img, width=n, height=n).free()
            torch.cuda.synchronize(dev)
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.detect(image=d_img, width=n, height=n).free()
            torch.cuda.synchronize(dev)
            ms = (time.perf_counter() - t0) / reps * 1e3
            r = ctx.detect(image=d_img, width=n, height=n)
            votes = int(sum(int(r.stats(p)["votes"].sum()) for p in (0, 1)))
            r.free()
            ctx.close()
            t0 = time.perf_counter()
            ref = oracle.detect(x, y, n, n, 40, 0, variant)
            row[f"oracle_ms_{variant}"] = (time.perf_counter() - t0) * 1e3
            ref_votes = int(sum(int(ref.stats[p][:, 1].sum()) for p in (0, 1)))
            row[f"votes_{variant}"] = votes
            row[f"ms_{variant}"] = ms
            row[f"oracle_votes_equal_{variant}"] = votes == ref_votes
        row["C_v"] = row["votes_circle"] / max(row["votes_code"], 1)
        row["C_t"] = row["ms_circle"] / row["ms_code"]
        row["C_t_oracle"] = row["oracle_ms_circle"] / row["oracle_ms_code"]
        out.append(row)
    return {"workload": f"full-span lines (8) with 1% noise, seed {seed}, T=40, default depth, both passes",
            "sizes": out,
            "paper_context": "the paper's Table 1 (FHT in floating point against the code test, Pentium IV): "
                             "C_v 7.5-7.7 and C_t 1340-1873 at 256x256; the circle test here is exact "
                             "integer arithmetic, so C_t reflects only the extra votes"}


def bench_gray(seed, reps=20):
    """The Sobel front end: a 1024x1024 gray image (32 bright segments of
    length U[200, 1000] on a noisy background, seed-fixed), edge threshold
    200, T = 120, depth 10, both passes on their own point sets."""
    import numpy as np
    import torch

    import synth
    from paper_1007_0547_amd import HoughHier

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    lines = synth.segment_image(rng, 1024, 1024, 32, 200.0, 1000.0, 0.0)
    g = (rng.integers(0, 40, (1024, 1024)) + lines.astype(np.int64) * 170).astype(np.uint8)
    d = torch.from_numpy(g).to(dev)
    stream = torch.cuda.current_stream(dev)
    ctx = HoughHier(threshold=120, max_depth=10, membership=True, device=0, stream=stream)
    for _ in range(3):
        ctx.detect(gray=d, edge_threshold=200, width=1024, height=1024).free()
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.detect(gray=d, edge_threshold=200, width=1024, height=1024).free()
    torch.cuda.synchronize(dev)
    ms = (time.perf_counter() - t0) / reps * 1e3
    r = ctx.detect(gray=d, edge_threshold=200, width=1024, height=1024)
    info = r.info
    n_alpha = int(r.stats(0)["votes"][0])
    r.free()
    ctx.close()
    ctx_t = HoughHier(threshold=120, max_depth=10, membership=True, device=0, stream=stream, timing=True)
    ctx_t.detect(gray=d, edge_threshold=200, width=1024, height=1024).free()
    r = ctx_t.detect(gray=d, edge_threshold=200, width=1024, height=1024)
    kt = r.timing()
    r.free()
    ctx_t.close()
    return {"workload": f"gray 1024x1024, seed {seed}, 32 segments, edge threshold 200, T=120, depth 10",
            "edge_points": info["n_points"], "alpha_points": n_alpha, "beta_points": info["n_points"] - n_alpha,
            "cells": sum(info["n_cells"]), "ms_per_image": ms, "front_end_ms": kt["extract_ms"],
            "code_tests_per_s": info["code_tests"] / (ms / 1e3)}


def bench_serving(seed, seconds, pool_size=384, lanes=3, max_batch=4):
    """Serving: a Poisson stream of requests for `seconds` seconds per rate,
    images drawn in turn from a pool of `pool_size` distinct images of the
    serving distribution (sides log-uniform 256..4096, Poisson(48) segments,
    1% noise, T = floor(side / 10), default depth) resident on the device.
    The capacity is measured first: a burst of requests through per-request
    launches (one lane, batches of one) until the queue drains.  Then, at
    0.9x and 1.5x that capacity, the same arrivals go through (a) continuous
    batching (`lanes` lanes, admission by predicted device memory) and (b)
    per-request launches.  Latency = arrival to cells and statistics on the
    host, measured inside the library; p50 / p99 over the requests of the
    stream."""
    import queue
    import threading

    import numpy as np
    import torch

    import synth
    from paper_1007_0547_amd import HoughHier

    dev = torch.device("cuda:0")
    trace = synth.serving_trace(seed=seed, rate_hz=1000.0, duration_s=1e9, max_requests=pool_size)
    pool = [w for _, w in trace]
    imgs = [torch.from_numpy(w.image).to(dev) for w in pool]
    torch.cuda.synchronize(dev)
    inputs = [dict(image=d, width=w.width, height=w.height, threshold=w.threshold) for d, w in zip(imgs, pool)]

    warm_failures = []

    def server(n_lanes, max_batch):
        srv = HoughHier(threshold=0, membership=True, device=0)
        srv.serve_start(lanes=n_lanes, max_batch=max_batch, queue_capacity=1 << 16)
        for _ in range(2):   # warm the lanes: arena sizes, group limits, the footprint model
            for k in range(0, len(inputs), 16):   # a window at a time: results are freed as they come
                for t in [srv.submit(**inp) for inp in inputs[k:k + 16]]:
                    try:
                        srv.poll(t).free()
                    except Exception as e:   # reported with the results, not raised
                        warm_failures.append(str(e))
        return srv

    def run(srv, arrivals):
        tickets = queue.Queue()
        lat, failed = [], []

        def collect():
            while True:
                t = tickets.get()
                if t is None:
                    return
                try:
                    r = srv.poll(t)
                except Exception as e:   # a failed request is reported, not timed
                    failed.append(str(e))
                    continue
                tm = r.timing()
                lat.append(tm["queue_ms"] + tm["service_ms"])
                r.free()

        th = threading.Thread(target=collect)
        th.start()
        t0 = time.perf_counter()
        for k, at in enumerate(arrivals):
            while True:
                d = at - (time.perf_counter() - t0)
                if d <= 0:
                    break
                time.sleep(min(d, 0.002))
            tickets.put(srv.submit(**inputs[k % len(inputs)]))
        tickets.put(None)
        th.join()
        wall = time.perf_counter() - t0
        res = {"requests": len(arrivals), "completed": len(lat), "images_per_s": len(lat) / wall,
               "wall_s": wall,
               "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}}
        if failed:
            res["failed"] = len(failed)
            res["first_failure"] = failed[0]
        return res

    plain = server(1, 1)
    burst = run(plain, np.zeros(2 * len(inputs)))
    capacity = burst["images_per_s"]
    batching = server(lanes, max_batch)
    out = {"workload": f"Poisson arrivals for {seconds:g} s per rate; images in turn from a pool of {len(pool)} "
                       f"distinct images (seed {seed}): sides log-uniform 256..4096, Poisson(48) segments, 1% noise, "
                       "T=floor(side/10), depth ceil(log2 side), both passes, voters kept on device",
           "mean_edge_points": float(np.mean([np.count_nonzero(w.image) for w in pool])),
           "capacity": {"what": "per-request launches (1 lane, batches of 1) under a burst of "
                                f"{2 * len(inputs)} requests", "images_per_s": capacity,
                        "latency_ms": burst["latency_ms"]},
           "continuous_batching_burst": run(batching, np.zeros(2 * len(inputs))),
           "rates": {}}
    for f in (0.9, 1.5):
        rate = f * capacity
        rng = np.random.default_rng(seed + 1)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * seconds * 1.2) + 16))
        arrivals = arrivals[arrivals < seconds]
        cb = run(batching, arrivals)
        note(f"serving {f}x capacity: continuous batching done")
        pr = run(plain, arrivals)
        note(f"serving {f}x capacity: per-request launches done")
        out["rates"][f"{f}x"] = {"arrival_rate_hz": rate, "continuous_batching": cb, "per_request": pr}
    out["slab"] = {"continuous_batching": batching.serve_stats(), "per_request": plain.serve_stats()}
    if warm_failures:
        out["warmup_failures"] = {"count": len(warm_failures), "first": warm_failures[0]}
    batching.close()
    plain.close()
    return out


def bench_single(name, seed, steps, warmup, variant="code", wide=False, kernel_steps=10):
    """One image of workload `name` per step (edge staging from the binary
    image resident in HBM, both passes to the finest level, voters kept on
    the device): wall time per step over `steps` steps with no per-launch
    events, then the count and compaction kernels' durations from HIP events
    on the library's stream over `kernel_steps` more steps, and the sizes the
    byte models need."""
    import numpy as np
    import torch

    import synth
    from paper_1007_0547_amd import HoughHier

    dev = torch.device("cuda:0")
    w = synth.workload(name, seed)
    img = torch.from_numpy(w.image).to(dev)
    stream = torch.cuda.current_stream(dev)

    def make(timing):
        return HoughHier(threshold=w.threshold, max_depth=w.max_depth, variant=variant, membership=True,
                         device=0, stream=stream, wide_compare=wide, timing=timing)

    def step(c):
        return c.detect(image=img, width=w.width, height=w.height)

    ctx = make(False)
    for _ in range(warmup):
        step(ctx).free()
    torch.cuda.synchronize(dev)
    lat = []
    info = None
    t_start = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        r = step(ctx)
        lat.append(time.perf_counter() - t0)
        info = r.info
        r.free()
    torch.cuda.synchronize(dev)
    elapsed = time.perf_counter() - t_start
    ctx.close()

    ctx_t = make(True)
    for _ in range(2):
        step(ctx_t).free()
    acc = {}
    for _ in range(kernel_steps):
        r = step(ctx_t)
        for k, v in r.timing().items():
            acc[k] = acc.get(k, 0) + v
        r.free()
    kt = {k: v / kernel_steps for k, v in acc.items()}
    r = step(ctx_t)
    stats = {p: r.stats(p) for p in (0, 1)}
    det_votes = {p: int(r.cells(p)["votes"].astype(np.int64).sum()) for p in (0, 1)}
    r.free()
    ctx_t.close()
    E = int(info["n_points"])
    return {"w": w, "info": info, "steps": steps, "elapsed": elapsed, "ms_per_step": elapsed / steps * 1e3,
            "lat": lat, "kt": kt, "stats": stats, "det_votes": det_votes, "E": E,
            "code_tests": int(info["code_tests"]),
            "alg_bytes": algorithmic_bytes(stats, det_votes, E)}


def bench_small_graph(seed, steps=300):
    """The launch-bound 256x256 image (line256: 8 full-span lines, 1% noise,
    T = 40, depth 8, both passes) one call per image, three ways: the
    library's pool; a caller arena; a caller arena with the level launches
    replayed from a captured HIP graph (HH_FLAG_GRAPH).  Wall time per image
    over `steps` calls (each result's cells brought to the host and freed)."""
    import torch

    import synth
    from paper_1007_0547_amd import HoughHier

    dev = torch.device("cuda:0")
    w = synth.workload("line256", seed)
    img = torch.from_numpy(w.image).to(dev)
    side = torch.cuda.Stream(dev)
    arena = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize(dev)
    out = {"workload": f"line256: 256x256, seed {seed}, T={w.threshold}, depth {w.max_depth}, both passes, "
                       "cells to the host per call"}
    for name, kw in (("pool", {}), ("arena", {"arena": arena}), ("arena_graph", {"arena": arena, "graph": True})):
        ctx = HoughHier(threshold=w.threshold, max_depth=w.max_depth, device=0, stream=side, **kw)
        replays = 0
        for k in range(steps + 5):
            if k == 5:
                torch.cuda.synchronize(dev)
                t0 = time.perf_counter()
                replays = 0
            r = ctx.detect(image=img, width=w.width, height=w.height)
            r.cells(0)
            replays += r.timing()["graph_replayed"]
            r.free()
        dt = (time.perf_counter() - t0) / steps
        out[name] = {"ms_per_image": dt * 1e3, "images_per_s": 1.0 / dt, "graph_replays": replays}
        ctx.close()
    return out


def single_summary(b):
    """The extra-block form of a bench_single run."""
    kt = b["kt"]
    pass_ms = kt["count_ms"] + kt["write_ms"]
    return {"workload": f"{b['w'].name}: {b['w'].width}x{b['w'].height}, T={b['w'].threshold}, "
                        f"depth {b['info']['depth']}, both passes, voters kept on device",
            "edge_points": b["E"], "cells": sum(b["info"]["n_cells"]), "code_tests": b["code_tests"],
            "ms_per_image": b["ms_per_step"], "images_per_s": 1e3 / b["ms_per_step"],
            "code_tests_per_s": b["code_tests"] / (b["ms_per_step"] / 1e3),
            "compare_bits": b["info"]["compare_bits"],
            "kernel_ms": {"count": kt["count_ms"], "write": kt["write_ms"], "decide": kt["decide_ms"],
                          "extract": kt["extract_ms"]},
            "vote_pass": {"alg_bytes": b["alg_bytes"], "ms": pass_ms,
                          "GB/s": b["alg_bytes"] / (pass_ms / 1e3) / 1e9,
                          "frac": b["alg_bytes"] / (pass_ms / 1e3) / 1e9 / HBM_PEAK_GBS}}


_T0 = time.time()


def note(what):
    """A progress line on stderr (the JSON result stays the only stdout line)."""
    print(f"bench: {what} ({time.time() - _T0:.0f} s)", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="seg4096", choices=["seg4096", "seg1024", "line256"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--variant", default="code", choices=["code", "circle"])
    ap.add_argument("--wide", action="store_true", help="64-bit corner compares")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the headline workload")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-image batch comparison")
    ap.add_argument("--no-sweep", action="store_true", help="skip the code/circle size sweep")
    ap.add_argument("--no-gray", action="store_true", help="skip the Sobel front-end image")
    ap.add_argument("--no-solution", action="store_true", help="skip solution() with point removal")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="arrival window per rate of the serving run (0 skips it)")
    ap.add_argument("--only", default="", choices=["", "batch512", "seg1024", "line256", "line256_graph", "serving",
                                                   "solution"],
                    help="run only this extra block (printed as its own JSON line), e.g. for a profiler")
    ap.add_argument("--batch-variants", default="pool,tuned,graph,plain",
                    help="with --only batch512: which batched forms to run (pool only for a profiler)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (3 times), the "
                         "reference kernel for scaling HBM byte counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import synth

    # the CPU baseline forks a process pool, so it runs before the GPU is touched
    cpu = None
    if not args.no_cpu_baseline and not args.calibrate_copy and not args.only:
        cpu = cpu_baseline(synth.workload(args.workload, args.seed))
        note("cpu baseline done")

    import torch

    if args.calibrate_copy:
        n = 1 << 30
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "copies": 3}), flush=True)
        return

    if args.only:
        fn = {"batch512": lambda: bench_batched(args.seed, variants=args.batch_variants.split(",")),
              "seg1024": lambda: single_summary(bench_single("seg1024", args.seed, args.steps, args.warmup)),
              "line256": lambda: single_summary(bench_single("line256", args.seed, args.steps, args.warmup)),
              "line256_graph": lambda: bench_small_graph(args.seed),
              "serving": lambda: bench_serving(args.seed, args.serve_seconds),
              "solution": lambda: bench_solution(args.seed)}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        return

    b = bench_single(args.workload, args.seed, args.steps, args.warmup, args.variant, args.wide)
    note(f"{args.workload}: {args.steps} timed steps done")
    info, kt, w = b["info"], b["kt"], b["w"]
    pass_ms = kt["count_ms"] + kt["write_ms"]
    achieved = b["alg_bytes"] / (pass_ms / 1e3) / 1e9
    kb = kernel_bytes(kt, 4)
    import numpy as np
    bits = info["compare_bits"]
    exact = (f"int32 corner compares, exact because S*2^depth = 2^{info['depth'] + int(info['side_pow2']).bit_length() - 1}"
             f" <= 2^28 keeps every scaled corner value below 2^31" if bits == 32 else
             "int64 corner compares")
    out = {
        "metric": "line-region code tests/s (plain, one image per call)",
        "value": b["code_tests"] * b["steps"] / b["elapsed"],
        "unit": "code tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": b["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"int{bits}",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: {w.width}x{w.height} binary image, seed {args.seed}, "
                        f"T={w.threshold}, depth {info['depth']}, both passes, {args.variant} variant, "
                        f"voters kept on device",
            "E": b["E"], "cells": sum(info["n_cells"]), "code_tests_per_image": b["code_tests"],
            "compares": exact,
        },
        "images_per_s": b["steps"] / b["elapsed"],
        "latency_ms": {"p50": float(np.percentile(b["lat"], 50) * 1e3),
                       "p99": float(np.percentile(b["lat"], 99) * 1e3)},
        "level_footprint": level_footprint(b["stats"], info["depth"]),
        "kernel_ms_per_step": {"count": kt["count_ms"], "write": kt["write_ms"],
                               "decide": kt["decide_ms"], "extract": kt["extract_ms"],
                               "device_total_with_events": kt["total_ms"]},
        "roofline": {"bound": "hbm", "kernel": "k_count+k_write (the vote and compaction pass, every level)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload),
                     "alg_bytes_per_step": b["alg_bytes"], "ms_per_step": pass_ms,
                     "other": {"entry_bytes_model": {
                         f"k_{k}": {"bytes_per_step": kb[k], "ms_per_step": kt[f"{k}_ms"],
                                    "GB/s": kb[k] / (kt[f"{k}_ms"] / 1e3) / 1e9 if kt[f"{k}_ms"] > 0 else 0.0}
                         for k in ("count", "write")}}},
    }
    def extra(key, fn, done):
        # an extra that fails is reported in its place; the headline stands
        try:
            out[key] = fn()
        except Exception as e:
            out[key] = {"error": f"{type(e).__name__}: {e}"}
        note(done)

    if not args.no_extras:
        if args.workload != "seg1024":
            extra("seg1024", lambda: single_summary(bench_single("seg1024", args.seed, 30, 3)), "seg1024 done")
        extra("line256", lambda: single_summary(bench_single("line256", args.seed, 100, 10)), "line256 done")
        extra("line256_graph", lambda: bench_small_graph(args.seed), "line256 graph done")
        if bits == 32:
            extra("wide_compares", lambda: single_summary(bench_single(args.workload, args.seed, 5, 2, wide=True)),
                  "wide compares done")
        if not args.no_batched:
            extra("batch512", lambda: bench_batched(args.seed), "batch512 done")
        if not args.no_sweep:
            extra("size_sweep", lambda: bench_sweep(args.seed), "size sweep done")
        if not args.no_gray:
            extra("gray1024", lambda: bench_gray(args.seed), "gray1024 done")
        if not args.no_solution:
            extra("solution", lambda: bench_solution(args.seed), "solution done")
        if args.serve_seconds > 0:
            extra("serving", lambda: bench_serving(args.seed, args.serve_seconds), "serving done")
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
