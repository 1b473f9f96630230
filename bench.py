"""Benchmark of the four-directional 5x5 Sobel operator on one MI355X.

Headline: uint8 8192x8192, magnitude only, replicate border -- Gpixel/s and
the achieved fraction of HBM peak, with inputs resident in HBM.  Launches
rotate over >= 1 GiB of distinct (src, mag) buffer sets so that the 256 MB
Infinity Cache cannot serve them.  Secondary results (mixed-size batch in one
persistent launch vs per-image launches, fp32 forward+backward, the size /
output-type sweep) are reported in extra keys of the same JSON line.

python bench.py [--gpus 1] [--steps K] [--warmup W]
                [--only u8,copy,sweep,ops,borders,batched,f32,weighted,pipe,mfma]
                [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "Gpixel/s + % of HBM peak, 4-dir 5x5 Sobel, uint8 8192² and mixed-size batch"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# Vector ALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.32e12 32-bit
# lane operations per second (one VALU instruction of a wave64 occupies a SIMD
# for 4 cycles).  Packed int16 instructions count once: they are one issue.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
N = 8192
ROTATE_BYTES = 2 << 30         # >= 1 GiB of distinct buffers (Infinity Cache is 256 MB)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    # the first ~200 launches run at lower clocks (measured: 62 us against 54 us
    # per 8192^2 launch), so the default warm-up covers them
    p.add_argument("--warmup", type=int, default=400)
    p.add_argument("--only", default=None,
                   help="comma-separated subset of: u8, copy, sweep, ops, borders, batched, f32, weighted, pipe, mfma")
    p.add_argument("--no-cpu-baseline", action="store_true")
    a = p.parse_args()
    if a.only is not None:
        a.only = set(x.strip() for x in a.only.split(",") if x.strip())
        bad = a.only - {"u8", "copy", "sweep", "ops", "borders", "batched", "f32", "weighted", "pipe", "mfma"}
        if bad:
            p.error("unknown --only part(s): %s" % ", ".join(sorted(bad)))
    return a


def time_launches(torch, fn, steps, warmup, first=0):
    """Average ms per call of fn(i) over `steps` calls (i counting from
    `first`), HIP events on the current stream, which is the stream the
    library's calls enqueue on."""
    for i in range(warmup):
        fn(first + i)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for i in range(steps):
        fn(first + warmup + i)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def clock_warmup(torch, fn, min_s=1.0, max_s=8.0, batch=50, tol=0.02):
    """Launch fn(i) in timed batches until the GPU clocks have settled: at
    least min_s seconds, and the last three batch averages within `tol` of
    each other (at most max_s seconds).  The first few hundred launches of a
    process run at ramp-up clocks; a fixed small --warmup would time those.
    Returns the number of launches made."""
    t0 = time.perf_counter()
    hist, n = [], 0
    while True:
        hist.append(time_launches(torch, fn, batch, 0, first=n))
        n += batch
        el = time.perf_counter() - t0
        if el >= max_s:
            break
        if el >= min_s and len(hist) >= 3 and max(hist[-3:]) <= (1 + tol) * min(hist[-3:]):
            break
    log("clock warm-up: %d launches in %.2f s; batch averages (ms) first %s, last %s" % (
        n, time.perf_counter() - t0, ["%.4f" % h for h in hist[:3]], ["%.4f" % h for h in hist[-3:]]))
    return n


def warm(torch, fn, n):
    """n untimed calls of fn(i), then a synchronisation."""
    for i in range(n):
        fn(i)
    torch.cuda.synchronize()


def per_launch_us(torch, fn, n):
    """Median and minimum of n single-launch times (an event pair around each
    launch, on the current stream), in microseconds."""
    s = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for i, (a, b) in enumerate(ev):
        a.record(s)
        fn(i)
        b.record(s)
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) * 1e3 for a, b in ev)
    return {"median": round(t[n // 2], 2), "min": round(t[0], 2), "launches": n}


def image_sets(torch, img, dev, nsets, pitch=None):
    h, w = img.shape
    base = torch.from_numpy(img).to(dev)
    srcs, mags = [], []
    for _ in range(nsets):
        s = torch.empty((h, w), dtype=torch.uint8, device=dev)
        s.copy_(base)
        srcs.append(s)
        mags.append(torch.empty((h, w), dtype=torch.uint8, device=dev))
    return srcs, mags


def bench_u8(torch, api, synth, dev, steps, warmup):
    img = synth.rect_image(N, N, 3)
    nsets = max(2, ROTATE_BYTES // (2 * N * N))
    srcs, mags = image_sets(torch, img, dev, nsets)

    def step(i):
        k = i % nsets
        api.sobel4x5_u8(srcs[k], mag=mags[k])

    nclock = clock_warmup(torch, step)
    ms = time_launches(torch, step, steps, warmup, first=nclock)
    per = per_launch_us(torch, step, 50)
    hot = time_launches(torch, lambda i: api.sobel4x5_u8(srcs[0], mag=mags[0]), steps, warmup)
    px = N * N
    res = {
        "ms": ms, "gpx": px / (ms * 1e-3) / 1e9, "alg_bytes": 2 * px, "clock_warmup_launches": nclock,
        "hot_ms": hot, "nsets": nsets, "rotating_gib": nsets * 2 * px / 2 ** 30, "per_launch_us": per,
    }
    del srcs, mags
    torch.cuda.empty_cache()
    return res, img


def bench_sweep(torch, api, synth, dev, steps, warmup):
    out = {}
    # the field images (1080p and 4K, rows pitched to 2048 / 3840 bytes), magnitude only
    for (h, w, pitch) in ((1080, 1920, 2048), (2160, 3840, 3840)):
        img = synth.field_image(h, w, 1)
        px = h * w
        nsets = max(2, ROTATE_BYTES // (2 * pitch * h))
        srcs = []
        for _ in range(nsets):
            flat = torch.empty((h * pitch,), dtype=torch.uint8, device=dev)
            v = flat.as_strided((h, w), (pitch, 1))
            v.copy_(torch.from_numpy(img))
            srcs.append(v)
        mags = [torch.empty((h, w), dtype=torch.uint8, device=dev) for _ in range(nsets)]
        fn = lambda i: api.sobel4x5_u8(srcs[i % nsets], mag=mags[i % nsets])
        warm(torch, fn, max(5, warmup))
        # a launch lasts a few microseconds, less than a host call: graph replay
        ms = time_graph(torch, fn, min(nsets, 200), max(2, steps // 20))
        out["field_%dx%d_mag_u8" % (w, h)] = {"ms": round(ms, 5), "gpx_per_s": round(px / (ms * 1e-3) / 1e9, 2),
                                             "timing": "graph replay"}
        del srcs, mags
        torch.cuda.empty_cache()
    for n in (4096, 8192, 16384):
        img = synth.rect_image(n, n, 3)
        px = n * n
        for mode in ("mag_u8", "dir_s16"):
            per = 2 * px if mode == "mag_u8" else 9 * px
            nsets = max(2, ROTATE_BYTES // per)
            base = torch.from_numpy(img).to(dev)
            srcs = [base.clone() for _ in range(nsets)]
            if mode == "mag_u8":
                outs = [torch.empty((n, n), dtype=torch.uint8, device=dev) for _ in range(nsets)]
                fn = lambda i: api.sobel4x5_u8(srcs[i % nsets], mag=outs[i % nsets])
            else:
                outs = [[torch.empty((n, n), dtype=torch.int16, device=dev) for _ in range(4)]
                        for _ in range(nsets)]
                fn = lambda i: api.sobel4x5_u8(srcs[i % nsets], want_mag=False, dir_type=api.DIR_S16,
                                               dirs=outs[i % nsets])
            k = max(10, steps // (1 if n <= 8192 else 4))
            if n <= 4096:
                # shorter than a host call: graph replay
                warm(torch, fn, max(3, warmup // 4))
                ms = time_graph(torch, fn, min(nsets, 100), max(2, steps // 20))
            else:
                ms = time_launches(torch, fn, k, max(3, warmup // 4))
            gbs = per / (ms * 1e-3) / 1e9
            out["%d_%s" % (n, mode)] = {"ms": round(ms, 5), "gpx_per_s": round(px / (ms * 1e-3) / 1e9, 2),
                                        "alg_GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                                        "bytes_per_px": per // px}
            del srcs, outs, base
            torch.cuda.empty_cache()
    return out


def bench_mfma(torch, api, synth, dev, steps, warmup):
    """The headline launch in its matrix-core form (SOBEL4X5_U8_MFMA=1, the
    5x5 responses as banded int8 products) beside the default form, on the
    same rotating buffers after the same clock warm-up; the matrix-core form
    at 1, 2 and 4 rounds of resident waves (SOBEL4X5_U8_WAVES)."""
    img = synth.rect_image(N, N, 3)
    nsets = max(2, ROTATE_BYTES // (2 * N * N))
    srcs, mags = image_sets(torch, img, dev, nsets)
    px = N * N
    out = {}
    saved = {k: os.environ.get(k) for k in ("SOBEL4X5_U8_MFMA", "SOBEL4X5_U8_WAVES")}
    try:
        for name, flag, waves in (("default", "0", None), ("matrix_cores_1_round", "1", 4096),
                                  ("matrix_cores_2_rounds", "1", 8192), ("matrix_cores_4_rounds", "1", 16384)):
            os.environ["SOBEL4X5_U8_MFMA"] = flag
            if waves is None:
                os.environ.pop("SOBEL4X5_U8_WAVES", None)
            else:
                os.environ["SOBEL4X5_U8_WAVES"] = str(waves)
            step = lambda i: api.sobel4x5_u8(srcs[i % nsets], mag=mags[i % nsets])
            clock_warmup(torch, step, max_s=3.0)
            ms = time_launches(torch, step, steps, warmup)
            out[name] = {"us": round(ms * 1e3, 2), "gpx_per_s": round(px / (ms * 1e-3) / 1e9, 2)}
        # both forms write the same bytes
        os.environ["SOBEL4X5_U8_MFMA"] = "1"
        api.sobel4x5_u8(srcs[0], mag=mags[0])
        os.environ["SOBEL4X5_U8_MFMA"] = "0"
        api.sobel4x5_u8(srcs[0], mag=mags[1])
        torch.cuda.synchronize()
        out["outputs_equal"] = bool(torch.equal(mags[0], mags[1]))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    del srcs, mags
    torch.cuda.empty_cache()
    return out


def time_graph(torch, fn, k, reps):
    """Average ms per launch of fn(i), i < k, captured once into a graph and
    replayed `reps` times: the device-side rate without the host's per-call
    cost (which exceeds the kernel time for small images)."""
    for i in range(min(k, 3)):
        fn(i)                      # per-kernel set-up (occupancy queries) outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for i in range(k):
            fn(i)
    g.replay()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        g.replay()
    e1.record(s)
    torch.cuda.synchronize()
    del g
    return e0.elapsed_time(e1) / (k * reps)


def bench_ops(torch, api, synth, dev, steps, warmup):
    """The paper's operator comparison (Sec. 5, Table 1: its four-directional
    5x5 kernel against the 3x3 operator) on this GPU: the four-directional
    5x5 operator, its 0 / 90 deg pair alone, and the two-directional 3x3
    Sobel pair, uint8 magnitude only, replicate border, at Table 1's sizes
    and at 8192^2.  Each entry: a graph of back-to-back launches over
    rotating buffers, replayed; `launch_us` is the same with one host call
    per launch."""
    names = {api.OP_4DIR_5X5: "4dir_5x5", api.OP_2DIR_5X5: "2dir_5x5", api.OP_2DIR_3X3: "2dir_3x3"}
    out = {}
    for n in (512, 1024, 2048, 8192):
        img = synth.rect_image(n, n, 3)
        px = n * n
        nsets = max(2, ROTATE_BYTES // (2 * px))
        base = torch.from_numpy(img).to(dev)
        srcs = [base.clone() for _ in range(nsets)]
        mags = [torch.empty((n, n), dtype=torch.uint8, device=dev) for _ in range(nsets)]
        row = {}
        for op, name in names.items():
            fn = lambda i, op=op: api.sobel4x5_u8_op(srcs[i % nsets], op, mag=mags[i % nsets])
            k = min(nsets, 200) if n <= 2048 else nsets
            reps = max(2, steps // 10) if n <= 2048 else max(2, steps // k)
            ms = time_graph(torch, fn, k, reps)
            launch_ms = time_launches(torch, fn, max(20, steps), max(5, warmup))
            gbs = 2 * px / (ms * 1e-3) / 1e9
            row[name] = {"us": round(ms * 1e3, 3), "gpx_per_s": round(px / (ms * 1e-3) / 1e9, 2),
                         "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "launch_us": round(launch_ms * 1e3, 3)}
        row["time_ratio_4dir5x5_over_2dir3x3"] = round(row["4dir_5x5"]["us"] / row["2dir_3x3"]["us"], 3)
        out["%d" % n] = row
        del srcs, mags, base
        torch.cuda.empty_cache()
    return out


def bench_batched(torch, api, synth, dev, steps, warmup):
    sizes = synth.batch_sizes(256, 77)
    imgs = [synth.rect_image(h, w, 1000 + i) for i, (h, w) in enumerate(sizes)]
    srcs, mags = [], []
    for m in imgs:
        h, w = m.shape
        pitch = synth.round_up(w, 256)
        flat = torch.empty(((h - 1) * pitch + w,), dtype=torch.uint8, device=dev)
        v = flat.as_strided((h, w), (pitch, 1))
        v.copy_(torch.from_numpy(m))
        srcs.append(v)
        mags.append(torch.empty((h, w), dtype=torch.uint8, device=dev))
    px = sum(h * w for h, w in sizes)
    # one launch of the batched kernel (autotuned tile shape and grid form:
    # one wave per tile, or a persistent grid on a work queue) in a hipGraph
    plan = api.Plan(srcs, mags, autotune=True)
    k = max(5, steps // 10)
    ms_plan = time_launches(torch, lambda i: plan.launch(), k, 20)

    def per_image(i):
        for s, m in zip(srcs, mags):
            api.sobel4x5_u8(s, mag=m)

    ms_eager = time_launches(torch, per_image, k, 2)
    # the same 256 launches captured in one graph (launch cost removed)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        per_image(0)
    ms_graph = time_launches(torch, lambda i: g.replay(), k, 2)
    info = plan.info()
    res = {"images": 256, "total_px": px, "bytes_per_px": 2,
           "one_launch_graph_ms": round(ms_plan, 4), "one_launch_gpx_per_s": round(px / ms_plan / 1e6, 2),
           "per_image_eager_ms": round(ms_eager, 4), "per_image_eager_gpx_per_s": round(px / ms_eager / 1e6, 2),
           "per_image_graph_ms": round(ms_graph, 4), "per_image_graph_gpx_per_s": round(px / ms_graph / 1e6, 2),
           "speedup_vs_eager": round(ms_eager / ms_plan, 3), "speedup_vs_graph": round(ms_graph / ms_plan, 3),
           "hbm_frac": round(2 * px / (ms_plan * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "tile": info}
    plan.close()
    del srcs, mags, g
    torch.cuda.empty_cache()
    return res


def bench_borders(torch, api, synth, dev, steps, warmup):
    """Border rules on the 8192^2 magnitude (replicate, zero, reflect-101),
    and the 256-image batch with int16 directional planes as well as
    magnitudes (2 + 8 = 10 B/px) in one persistent launch, per border."""
    out = {}
    img = synth.rect_image(N, N, 3)
    nsets = max(2, ROTATE_BYTES // (2 * N * N))
    base = torch.from_numpy(img).to(dev)
    srcs = [base.clone() for _ in range(nsets)]
    mags = [torch.empty((N, N), dtype=torch.uint8, device=dev) for _ in range(nsets)]
    names = {api.BORDER_REPLICATE: "replicate", api.BORDER_ZERO: "zero", api.BORDER_REFLECT101: "reflect101"}
    for b, name in names.items():
        fn = lambda i, b=b: api.sobel4x5_u8(srcs[i % nsets], b, mag=mags[i % nsets])
        ms = time_launches(torch, fn, steps, warmup)
        out["8192_mag_" + name] = {"ms": round(ms, 5), "gpx_per_s": round(N * N / (ms * 1e-3) / 1e9, 2)}
    del srcs, mags, base
    torch.cuda.empty_cache()
    sizes = synth.batch_sizes(256, 77)
    imgs = [synth.rect_image(h, w, 1000 + i) for i, (h, w) in enumerate(sizes)]
    px = sum(h * w for h, w in sizes)
    srcs = []
    for m in imgs:
        h, w = m.shape
        pitch = synth.round_up(w, 256)
        flat = torch.empty(((h - 1) * pitch + w,), dtype=torch.uint8, device=dev)
        v = flat.as_strided((h, w), (pitch, 1))
        v.copy_(torch.from_numpy(m))
        srcs.append(v)
    mags = [torch.empty(m.shape, dtype=torch.uint8, device=dev) for m in imgs]
    dirs = [[torch.empty(m.shape, dtype=torch.int16, device=dev) for _ in range(4)] for m in imgs]
    k = max(5, steps // 10)
    for b, name in names.items():
        plan = api.Plan(srcs, mags, b, dir_type=api.DIR_S16, dirs=dirs)
        ms = time_launches(torch, lambda i: plan.launch(), k, 20)
        gbs = 10 * px / (ms * 1e-3) / 1e9
        out["batch256_mag_dir_s16_" + name] = {"ms": round(ms, 4), "gpx_per_s": round(px / ms / 1e6, 2),
                                               "alg_GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                                               "tile": plan.info()}
        plan.close()
    del srcs, mags, dirs
    torch.cuda.empty_cache()
    return out


def bench_f32(torch, api, synth, dev, steps, warmup):
    B, H, W = 32, 1024, 1024
    x = torch.from_numpy(synth.float_batch(B, H, W)).to(dev)
    M = torch.empty_like(x)
    gm = torch.full_like(x, 1.0 / x.numel())
    dx = torch.empty_like(x)
    k = max(5, steps // 10)
    clock_warmup(torch, lambda i: api.sobel4x5_f32_bwd(x, gm, out=dx), max_s=4.0)
    ms_f = time_launches(torch, lambda i: api.sobel4x5_f32_fwd(x, out=M), k, max(3, warmup))
    ms_b = time_launches(torch, lambda i: api.sobel4x5_f32_bwd(x, gm, out=dx), k, max(3, warmup // 2))
    px = B * H * W
    res = {"batch": B, "H": H, "W": W, "fwd_ms": round(ms_f, 4), "bwd_ms": round(ms_b, 4),
           "fwd_bwd_gpx_per_s": round(px / ((ms_f + ms_b) * 1e-3) / 1e9, 2),
           "fwd_GBps": round(8 * px / (ms_f * 1e-3) / 1e9, 1), "bwd_GBps": round(12 * px / (ms_b * 1e-3) / 1e9, 1),
           "fwd_bwd_hbm_frac": round(20 * px / ((ms_f + ms_b) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del x, M, gm, dx
    torch.cuda.empty_cache()
    return res


def bench_weighted(torch, api, synth, dev, steps, warmup):
    """Run-time weights (the family K(a, b, n, m) at (1, 3, 5, 10)) on the
    8192x8192 image, magnitude only, rotating buffers as in the headline."""
    img = synth.rect_image(N, N, 3)
    nsets = max(2, ROTATE_BYTES // (2 * N * N))
    srcs, mags = image_sets(torch, img, dev, nsets)
    w = api.family_weights(*api.family_products(1, 3, 5, 10))
    k = max(10, steps // 4)
    ms = time_launches(torch, lambda i: api.sobel4x5_u8_weighted(srcs[i % nsets], w, mag=mags[i % nsets]), k,
                       max(3, warmup // 4))
    del srcs, mags
    torch.cuda.empty_cache()
    px = N * N
    return {"weights": "K(a,b,n,m) at (1,3,5,10)", "ms": round(ms, 5), "gpx_per_s": round(px / (ms * 1e-3) / 1e9, 2),
            "hbm_frac": round(2 * px / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def bench_pipe(torch, api, synth, dev, steps):
    """Host -> device -> host: 64 images of 3840x2160 in pinned host memory
    through the pipeline (copies overlapped with kernels over 3 slots),
    against one slot (copy in, kernel, copy out in sequence)."""
    h, w, n = 2160, 3840, 64
    base = [synth.field_image(h, w, 3000 + i) for i in range(4)]
    srcs = []
    for i in range(n):
        t = torch.empty((h, w), dtype=torch.uint8, pin_memory=True)
        t.copy_(torch.from_numpy(base[i % 4]))
        srcs.append(t)
    mags = [torch.empty((h, w), dtype=torch.uint8, pin_memory=True) for _ in range(n)]
    out = {"images": n, "shape": [h, w], "host_memory": "pinned"}
    for depth in (1, 3):
        p = api.Pipe(w, h, depth)
        p.run(srcs[:4], mags[:4])
        reps = max(1, steps // 100)
        t0 = time.perf_counter()
        for _ in range(reps):
            p.run(srcs, mags)
        dt = (time.perf_counter() - t0) / reps
        p.close()
        out["depth%d" % depth] = {"ms": round(dt * 1e3, 3), "gpx_per_s": round(n * h * w / dt / 1e9, 2),
                                  "pcie_GBps": round(2 * n * h * w / dt / 1e9, 2)}
    out["overlap_speedup"] = round(out["depth1"]["ms"] / out["depth3"]["ms"], 3)
    return out


def bench_copy(torch, api, dev, steps):
    """Achievable streaming bandwidth: a plain 128-bit copy of 1 GiB (2 GiB moved)."""
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device=dev)
    b = torch.empty(n, dtype=torch.uint8, device=dev)
    a.fill_(7)
    k = max(3, steps // 20)
    ms = time_launches(torch, lambda i: api.debug_copy(a, b) if i % 2 == 0 else api.debug_copy(b, a), k, 50)
    gbs = 2 * n / (ms * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_moved": 2 * n, "ms": round(ms, 4), "GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}


# Per-launch figures of the headline kernel read off its profile and its ISA,
# valid only for the kernel source they were taken on (the SHA-256 prefix of
# U8_KERNEL_SOURCES); reported as null for any other source.
#   traffic: HBM bytes per launch from rocprofv3 --pmc FETCH_SIZE and
#            WRITE_SIZE (KiB per dispatch), each scaled by what the same
#            counter reads for the plain copy kernel (sobel4x5_debug_copy) of
#            known size (profiles/k_u8_single_8192x8192_mag_u8.md);
#   valu:    VALU instructions per output pixel (SQ_INSTS_VALU x 64 / pixels
#            from the same profile; the kernel has no transcendental
#            instruction, so each is one issue slot).
U8_PROFILE = {"src_sha256": "5c30fa8417524d3a", "traffic_bytes": 145362304, "valu_slots_per_px": 21434880 * 64 / 8192.0 ** 2}


# Sources k_u8_single is compiled from (the hash covers them in this order);
# its launch code lives elsewhere (u8_launch.hpp, sobel4x5_u8.hip).
U8_KERNEL_SOURCES = ("u8_sweep.hpp", "load_columns.hpp", "internal.hpp")


def u8_source_hash():
    import hashlib
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2305_00515_amd", "csrc")
    h = hashlib.sha256()
    try:
        for name in U8_KERNEL_SOURCES:
            h.update(open(os.path.join(csrc, name), "rb").read())
    except OSError:
        return None
    return h.hexdigest()[:16]


def u8_profile(key):
    return U8_PROFILE[key] if u8_source_hash() == U8_PROFILE["src_sha256"] else None


def cpu_baseline(img):
    """The CPU oracle (as it stands) on the same 8192x8192 image, all cores."""
    import oracle
    oracle.build()
    cores = len(os.sched_getaffinity(0))
    runs = []
    t_total = 0.0
    while t_total < 10.0 and len(runs) < 200:
        t0 = time.perf_counter()
        oracle.sobel_u8(img, want_dir=False, nthreads=cores)
        dt = time.perf_counter() - t0
        runs.append(dt)
        t_total += dt
    best = min(runs)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    # single-thread references: the 512x512 parity image with every output,
    # and one 1024x1024 fp32 image forward + adjoint in fp64
    from paper_2305_00515_amd import synth
    small = synth.rect_image(512, 512, 0)
    t0 = time.perf_counter()
    oracle.sobel_u8(small, nthreads=1)
    t_small = time.perf_counter() - t0
    x = synth.float_batch(1, 1024, 1024).astype(np.float64)
    t0 = time.perf_counter()
    m, _ = oracle.sobel_f64_fwd(x, nthreads=1)
    oracle.sobel_f64_bwd(x, np.full(m.shape, 1.0 / m.size), nthreads=1)
    t_f64 = time.perf_counter() - t0
    return {"value": round(len(runs) * img.size / t_total / 1e9, 4), "unit": "Gpixel/s", "cores": cores,
            "kind": "oracle",
            "sample": "the full 8192x8192 uint8 image (magnitude only) repeated for >= 10 s: %d run(s), "
                      "best %.3f s; CPU %s" % (len(runs), best, model),
            "single_thread": {"u8_512x512_all_outputs_ms": round(t_small * 1e3, 2),
                              "f64_1024x1024_fwd_bwd_ms": round(t_f64 * 1e3, 1)}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from paper_2305_00515_amd import api, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    line = {"metric": METRIC, "unit": "Gpixel/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
            "data": "synthetic"}
    want = (lambda part: args.only is None or part in args.only)
    img = None
    if want("u8"):
        log("u8 8192x8192 magnitude: %d steps" % args.steps)
        r, img = bench_u8(torch, api, synth, dev, args.steps, args.warmup)
        # the dominant (and only) kernel of a step: algorithmic bytes per
        # launch (1 byte read + 1 written per pixel) over its average launch
        # time from the HIP events around the timed launches
        gbs = r["alg_bytes"] / (r["ms"] * 1e-3) / 1e9
        slots = u8_profile("valu_slots_per_px")
        valu = None
        if slots is not None:
            tops = slots * N * N / (r["ms"] * 1e-3) / 1e12
            valu = {"slots_per_px": round(slots, 3), "achieved_TOPs": round(tops, 2),
                    "peak_TOPs": round(VALU_PEAK_TOPS, 2), "issue_frac": round(tops / VALU_PEAK_TOPS, 4)}
        line.update({
            "value": round(r["gpx"], 2), "ms_per_step": round(r["ms"], 5),
            "config": {"workload": "uint8 8192x8192 four-directional 5x5 Sobel, uint8 magnitude only, "
                                   "replicate border, one image per step",
                       "image": "rect_image(8192, 8192, seed=3): uniform noise + 20 filled rectangles",
                       "bytes_per_px": 2, "rotating_buffers_gib": round(r["rotating_gib"], 2),
                       "clock_warmup_launches": r["clock_warmup_launches"],
                       "hot_same_buffer_ms": round(r["hot_ms"], 5), "per_launch_us": r["per_launch_us"]},
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": u8_profile("traffic_bytes"),
                         "kernel": "k_u8_single<8,replicate,aligned,mag-only>",
                         "alg_bytes_per_launch": r["alg_bytes"], "valu": valu},
        })
    if want("copy"):
        log("copy ceiling")
        line["copy_ceiling"] = bench_copy(torch, api, dev, args.steps)
    if want("sweep"):
        log("sweep")
        line["sweep"] = bench_sweep(torch, api, synth, dev, args.steps, args.warmup)
    if want("ops"):
        log("operator comparison (4-dir 5x5, 2-dir 5x5, 2-dir 3x3)")
        line["ops"] = bench_ops(torch, api, synth, dev, args.steps, args.warmup)
    if want("borders"):
        log("border rules 8192x8192; 256-image batch with directional planes")
        line["borders"] = bench_borders(torch, api, synth, dev, args.steps, args.warmup)
    if want("batched"):
        log("batched 256 images")
        line["batched"] = bench_batched(torch, api, synth, dev, args.steps, args.warmup)
    if want("weighted"):
        log("run-time weights 8192x8192")
        line["weighted"] = bench_weighted(torch, api, synth, dev, args.steps, args.warmup)
    if want("pipe"):
        log("host pipeline 64 x 3840x2160")
        line["pipe"] = bench_pipe(torch, api, synth, dev, args.steps)
    if want("mfma"):
        log("matrix-core form of the headline launch")
        line["mfma"] = bench_mfma(torch, api, synth, dev, args.steps, args.warmup)
    if want("f32"):
        log("fp32 32x1024^2 fwd+bwd")
        line["f32"] = bench_f32(torch, api, synth, dev, args.steps, args.warmup)
    if img is not None and not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(img)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
