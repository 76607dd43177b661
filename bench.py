#!/usr/bin/env python3
"""Benchmark of the EDGE pipeline on one MI355X.

One step = the whole hot path (blur, Laplacian, zero crossing, Sobel, max
reduction, threshold) over one batch of seeded synthetic images already
resident in HBM.  The default workload is 64 images of 1920x1080 (5x5
Gaussian, sigma 1), run as one batched graph launch; the same images are
also timed through the per-image forms (fused and one kernel per stage)
for the batched-vs-per-image comparison.  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# HIP gives a process 4 hardware queues unless told otherwise, and torch's
# own stream takes one: the batches bench.py keeps in flight on several
# streams then share queues and stop overlapping.  Ask for 8 (read when
# HIP initialises, which happens after this point).
if int(os.environ.get("GPU_MAX_HW_QUEUES", "0") or 0) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

METRIC = ("Mpixel/s and %HBM-roofline, batched vs per-image; "
          "p50/p99 latency at QPS")
HBM_PEAK_GBS = 8000.0
PATH_BYTES_PER_PX = 5.0    # input read once + mask written once
# Algorithmic bytes per pixel of each batched kernel, by pass structure:
# STORE's pass 1 reads the input (its 4 B/px code is an intermediate, not
# algorithmic) and its pass 2 writes the mask; RECOMPUTE's pass 1 reads the
# input for the maximum and its pass 2 reads it again and writes the mask.
# SPECULATE's pass 1 reads the input and writes the mask; its pass 2
# touches only the listed pixels.
KERNEL_BYTES_PER_PX = {1: {1: 4.0, 2: 1.0}, 2: {1: 4.0, 2: 5.0}, 3: {1: 5.0, 2: 0.0}}
BATCH_DEFAULT_PASS = 3    # the library's pass structure for batched calls
BATCH_TILE_W = 256        # batched sweep tiles: one wave, 4 columns per lane
BATCH_DEFAULT_TY = 64     # their height when neither tuned nor fixed
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_batch_64x1080p.json")
SWEEP_SOURCES = ["paper_2503_10855_amd/csrc/" + f for f in
                 ("sweep_impl.h", "hx_device.h", "hx_kernels.h", "k_batch.hip",
                  "thresh_impl.h")]


def workloads():
    from paper_2503_10855_amd import synth
    return {"batch-64x1080p": synth.batch_1080p, "uneven-512": synth.uneven_512,
            "single-8192-k7": synth.large_8192, "single-256": synth.single_256,
            "band-1024x8192-k7": synth.band_8192}


def srad_traffic_file(side):
    """The committed counter summary of SRAD on a side x side image."""
    return os.path.join(ROOT, "profiles", f"traffic_srad_{side}.json")


SRAD_SOURCES = ["paper_2503_10855_amd/csrc/" + f for f in ("k_srad.hip", "srad_kernels.h")]


def source_hash(sources=None):
    h = hashlib.sha256()
    for f in sources or SWEEP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, pixels, path=TRAFFIC_FILE, sources=None, tile_h=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when absent, taken on different kernel sources, or
    (for summaries taken per sweep tile height) not taken at `tile_h`."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash(sources) or t.get("pixels") != pixels:
        return None
    kernels = t.get("kernels", {})
    if "by_tile_h" in t:
        # Counters taken at several sweep tile heights: the one in use.
        kernels = t["by_tile_h"].get(str(tile_h), {}).get("kernels", {})
    k = kernels.get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(wl, images, budget_s=12.0):
    """The oracle (plain fp64 C) on a bounded sample of the workload: whole
    passes over its images, one image per thread, repeated to about
    `budget_s` seconds of wall time."""
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    oracle.edge_detect(images[0], wl.ksize, wl.sigma, wl.theta)
    one = time.perf_counter() - t0
    # Workloads with many large images are cut to a prefix of about the budget.
    n = int(max(1, min(len(images), budget_s * min(threads, len(images)) / max(one, 1e-6))))
    sample = images[:n]
    t0 = time.perf_counter()
    oracle.edge_detect_many(sample, wl.ksize, wl.sigma, wl.theta, nthreads=threads)
    first = time.perf_counter() - t0
    reps = int(max(1, budget_s / max(first, 1e-6)))
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.edge_detect_many(sample, wl.ksize, wl.sigma, wl.theta, nthreads=threads)
    dt = time.perf_counter() - t0
    px = reps * sum(a.shape[0] * a.shape[1] for a in sample)
    px0 = images[0].shape[0] * images[0].shape[1]
    return {"value": round(px / dt / 1e6, 3), "unit": "Mpixel/s", "cores": min(threads, n),
            "kind": "oracle",
            "sample": f"{reps} passes over {n} of {len(images)} images of the workload, "
                      f"one image per thread, fp64 C oracle, {dt:.2f} s wall",
            "one_core_value": round(px0 / one / 1e6, 3),
            "one_core_sample": f"image 0 alone on one core, {one:.3f} s",
            "host": host_info()}


def host_info():
    """The host's CPU model and the CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def cpu_tuned(wl, images, budget_s=5.0):
    """The tuned multi-core fp32 CPU implementation on the same images:
    whole passes over the workload, repeated to about budget_s seconds."""
    from paper_2503_10855_amd import cpu
    threads = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    cpu.edge_detect_many(images, wl.ksize, wl.sigma, wl.theta, nthreads=threads)
    first = time.perf_counter() - t0
    reps = int(max(1, budget_s / max(first, 1e-6)))
    t0 = time.perf_counter()
    for _ in range(reps):
        cpu.edge_detect_many(images, wl.ksize, wl.sigma, wl.theta, nthreads=threads)
    dt = time.perf_counter() - t0
    px = reps * sum(a.shape[0] * a.shape[1] for a in images)
    return {"value": round(px / dt / 1e6, 1), "unit": "Mpixel/s", "cores": threads,
            "kind": "tuned fp32 C++ (bands of 128 rows over std::threads)",
            "host": host_info(),
            "sample": f"{reps} passes over the {len(images)} images, {dt:.2f} s wall"}


def timed_streams(fns, streams, steps, warmup):
    """Step i runs fns[i % S](streams[i % S]); the K timed steps are
    bracketed by events on the current stream, which every stream waits on
    at the start and waits for at the end.  The warm-up runs at least three
    calls per stream whatever `warmup` says (the first builds a batch
    context's table, the second captures its graph, the third replays it),
    so every timed call replays a captured graph."""
    import torch
    S = len(streams)
    for i in range(max(warmup, 3 * S)):
        fns[i % S](streams[i % S])
    # Then keep the GPU busy for at least ~50 ms before the timed region, so
    # that a short run is not timed while the clocks ramp up.
    torch.cuda.synchronize()
    t_end = time.perf_counter() + 0.05
    i = 0
    while time.perf_counter() < t_end:
        for _ in range(S):
            fns[i % S](streams[i % S])
            i += 1
        torch.cuda.synchronize()
    torch.cuda.synchronize()
    cur = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    t0.record(cur)
    for st in streams:
        st.wait_event(t0)
    for i in range(steps):
        fns[i % S](streams[i % S])
    for st in streams:
        cur.wait_stream(st)
    t1.record(cur)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    return t0.elapsed_time(t1) / steps, wall


def timed(fn, steps, warmup, sync):
    import torch
    for _ in range(warmup):
        fn()
    sync()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    t0.record()
    for _ in range(steps):
        fn()
    t1.record()
    sync()
    wall = time.perf_counter() - w0
    return t0.elapsed_time(t1) / steps, wall


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 200 in batch mode, 20 otherwise)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default: 20 in batch mode, 5 otherwise)")

    ap.add_argument("--mode", default="batch",
                    choices=("batch", "serve", "reduce", "tune", "tune-batch", "srad"),
                    help="batch: the batched step (default); serve: the continuous-"
                         "batching server under Poisson arrivals; reduce: the "
                         "max-reduction ablation on the unfused per-image form; tune: "
                         "the autotuner's measurement of every schedule on the "
                         "workload's first image shape; tune-batch: the batch "
                         "autotuner's trials on the workload's whole batch; srad: the "
                         "second workload")
    ap.add_argument("--workload", default="batch-64x1080p", choices=sorted(workloads()))
    ap.add_argument("--requests", type=int, default=20000, help="serve: requests")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: arrivals per second")
    ap.add_argument("--budget-mb", type=int, default=32 * 1024, help="serve: HBM budget")
    ap.add_argument("--streams", type=int, default=None,
                    help="serve: compute streams (default 4); batch: consecutive batches go "
                         "to this many streams in turn, each with its own output buffers "
                         "(default 4; 1: one stream)")
    ap.add_argument("--max-batch", type=int, default=64, help="serve: images per batch")
    ap.add_argument("--zero-copy", action="store_true",
                    help="serve: requests go in through reserved pinned slots (the bench "
                         "copies each crop into its slot) and masks are read in place")
    ap.add_argument("--srad-side", type=int, default=4096, help="srad: image side")
    ap.add_argument("--srad-iters", type=int, default=100, help="srad: iterations per step")
    ap.add_argument("--images-reduce", type=int, default=8,
                    help="reduce: 1920x1080 images per step")
    ap.add_argument("--pass-mode", type=int, default=0, choices=(0, 1, 2, 3),
                    help="batched pass structure: 0 default, 1 STORE, 2 RECOMPUTE, "
                         "3 SPECULATE")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-tune", action="store_true",
                    help="batch: skip the batch autotuner (default tile height and pass)")
    ap.add_argument("--batch-tile-h", type=int, default=0, metavar="TY",
                    help="batch: fix the sweep tile height (16..256, a multiple of 8) "
                         "with --pass-mode's pass structure (SPECULATE if 0); skips "
                         "the batch autotuner")
    ap.add_argument("--no-serve", action="store_true",
                    help="batch: skip the short serving leg")
    ap.add_argument("--serve-requests", type=int, default=4000,
                    help="batch: requests of the serving leg (at --rate per second)")
    ap.add_argument("--no-per-image", action="store_true",
                    help="skip the per-image comparison forms")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device-to-device copy of MIB MiB, three "
                         "times (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 200 if args.mode == "batch" else 20
    if args.warmup is None:
        args.warmup = 20 if args.mode == "batch" else 5
    if args.streams is None:
        args.streams = 4
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}); "
              "images are independent, so several GPUs would each run their own "
              "batches with no communication", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2503_10855_amd.build import LIB
    if not os.path.exists(LIB):
        from paper_2503_10855_amd.build import build
        build()
    from paper_2503_10855_amd import hx

    if args.mode == "serve":
        return run_serve(args, hx)
    if args.mode == "reduce":
        return run_reduce(args, hx)
    if args.mode == "tune":
        return run_tune(args, hx)
    if args.mode == "tune-batch":
        return run_tune_batch(args, hx)
    if args.mode == "srad":
        return run_srad(args, hx)

    wl = workloads()[args.workload]()
    images = [wl.image(i) for i in range(len(wl.sizes))]
    srcs = [torch.from_numpy(a).cuda() for a in images]
    # One output set per stream: batches in flight on different streams
    # never share an output buffer.
    S = max(1, args.streams)
    mask_sets = [[torch.empty(s.shape, dtype=torch.uint8, device="cuda") for s in srcs]
                 for _ in range(S)]
    dmax_sets = [torch.zeros(len(srcs), device="cuda") for _ in range(S)]
    masks, dmax = mask_sets[0], dmax_sets[0]
    pixels = wl.pixels
    sync = torch.cuda.synchronize

    # One batch context per stream (at least the library's default 4), so
    # that each stream's output set keeps its own table and graph.
    with hx.Pipeline(ksize=wl.ksize, sigma=wl.sigma, theta=wl.theta,
                     max_pixels=pixels, max_images=max(len(srcs), 1),
                     pass_mode=args.pass_mode, batch_contexts=min(8, max(4, S))) as p:
        sched = p.schedule(*wl.sizes[0])
        # The batched launch's tile height and pass structure, chosen by the
        # batch autotuner on this batch (unless a pass structure is fixed).
        batch_sched = None
        if args.batch_tile_h:
            pm_fixed = args.pass_mode or BATCH_DEFAULT_PASS
            p.set_schedule(BATCH_TILE_W, args.batch_tile_h, 4, pm_fixed)
            batch_sched = {"tile_h": args.batch_tile_h,
                           "pass": {1: "store", 2: "recompute", 3: "speculate"}[pm_fixed],
                           "fixed": True}
        elif not args.no_tune and not args.pass_mode:
            t0 = time.perf_counter()
            th, pm = p.autotune_batch(srcs, mask_sets[0])
            batch_sched = {"tile_h": th, "pass": {1: "store", 2: "recompute",
                                                  3: "speculate"}[pm],
                           "tuner_s": round(time.perf_counter() - t0, 2)}

        preps = [p.prepare_batch(srcs, m, d) for m, d in zip(mask_sets, dmax_sets)]
        prepared = preps[0]
        batched = prepared.run

        streams = [torch.cuda.Stream() for _ in range(S)]
        ms_step, wall = timed_streams([q.run for q in preps], streams, args.steps,
                                      args.warmup)
        ms_step_1s, _ = timed_streams([prepared.run], streams[:1], args.steps, args.warmup)
        p.sync()
        same_sets = all(torch.equal(a, b) for ms in mask_sets[1:]
                        for a, b in zip(mask_sets[0], ms))
        value = pixels / (ms_step * 1e-3) / 1e6

        # The same kernels launched directly with events around each one
        # (timing mode): durations of the reset and the two passes.
        p.set_timing(True)
        for _ in range(args.warmup):
            batched()
        p.last_timing()
        acc = np.zeros(4)
        for _ in range(args.steps):
            batched()
            acc += np.array(p.last_timing())
        p.set_timing(False)
        ms_reset, ms_p1, ms_p2, ms_p0 = (acc / args.steps).tolist()
        p.set_schedule()

        per_image = None
        if not args.no_per_image:
            ref = [m.clone() for m in masks]

            def fused():
                for s, m in zip(srcs, masks):
                    p.edge_detect(s, m)
            ms_fused, _ = timed(fused, max(1, args.steps // 2), 1, sync)
            same = all(torch.equal(a, b) for a, b in zip(ref, masks))
            p.set_schedule(64, 16, 1)
            ms_plain, _ = timed(fused, max(1, args.steps // 4), 1, sync)
            p.set_schedule()
            per_image = {
                "fused_mpx_s": round(pixels / (ms_fused * 1e-3) / 1e6, 1),
                "plain_mpx_s": round(pixels / (ms_plain * 1e-3) / 1e6, 1),
                "fused_ms_per_step": round(ms_fused, 4),
                "plain_ms_per_step": round(ms_plain, 4),
                "batched_over_plain": round(ms_plain / ms_step, 2),
                "batched_over_fused": round(ms_fused / ms_step, 2),
                "masks_identical_to_batched": bool(same),
            }

        # Per-call latency of the per-image forms on the first image:
        # events around each single call, 200 calls after a warm-up.
        lat = {}
        for name, sch in (("fused", None), ("plain", (64, 16, 1))):
            if sch:
                p.set_schedule(*sch)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(200)]
            for _ in range(10):
                p.edge_detect(srcs[0], masks[0])
            sync()
            for a, b in ev:
                a.record()
                p.edge_detect(srcs[0], masks[0])
                b.record()
                sync()
            v = np.array([a.elapsed_time(b) for a, b in ev]) * 1e-3
            lat[name] = dict(percentiles(v), mean=round(float(v.mean()) * 1e3, 4),
                             shape=list(wl.sizes[0]))
        p.set_schedule()

    # The dominant kernel is the longer of the two passes.
    if batch_sched:
        pm = {"store": 1, "recompute": 2, "speculate": 3}[batch_sched["pass"]]
    else:
        pm = args.pass_mode or BATCH_DEFAULT_PASS
    dom = 1 if ms_p1 >= ms_p2 else 2
    ms_dom = ms_p1 if dom == 1 else ms_p2
    bpp = KERNEL_BYTES_PER_PX[pm][dom]
    kname = (f"k_batch_p1s<{wl.ksize}>" if (pm, dom) == (3, 1)
             else f"k_batch_p{dom}<{wl.ksize}, {pm}>")
    achieved = bpp * pixels / (ms_dom * 1e-3) / 1e9
    traffic = measured_traffic(kname, pixels,
                               tile_h=batch_sched["tile_h"] if batch_sched else BATCH_DEFAULT_TY)
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_one_stream": round(ms_step_1s, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "images": len(wl.sizes), "pixels": pixels,
                   "ksize": wl.ksize, "sigma": wl.sigma, "theta": wl.theta,
                   "form": f"batched graph launch, consecutive batches on {S} "
                           f"stream{'s' if S > 1 else ''} in turn",
                   "streams": S, "output_sets_identical": same_sets,
                   "pass_mode": {0: "batch default", 1: "store", 2: "recompute",
                                 3: "speculate"}[args.pass_mode],
                   "batch_schedule": batch_sched,
                   "per_image_schedule": list(sched)},
        "roofline": {"kernel": kname, "bound": "hbm",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "ms_per_launch": round(ms_dom, 4),
                     "bytes_per_px": bpp, "pixels_per_launch": pixels},
        "path_roofline": {"achieved": round(PATH_BYTES_PER_PX * pixels / (ms_step * 1e-3) / 1e9, 1),
                          "unit": "GB/s", "bytes_per_px": PATH_BYTES_PER_PX,
                          "frac": round(PATH_BYTES_PER_PX * pixels / (ms_step * 1e-3)
                                        / 1e9 / HBM_PEAK_GBS, 4)},
        "kernels_ms": {"reset": round(ms_reset, 4), "pass0": round(ms_p0, 4),
                       "pass1": round(ms_p1, 4), "pass2": round(ms_p2, 4)},
        "per_image": per_image,
        "per_call_latency_ms": lat,
        "wall_s": round(wall, 3),
    }
    # A plain 1 GiB device-to-device copy: the practical HBM ceiling.
    cb = 1 << 30
    ca = torch.ones(cb, dtype=torch.uint8, device="cuda")
    cbuf = torch.empty_like(ca)
    ms_copy, _ = timed(lambda: cbuf.copy_(ca), 10, 2, sync)
    line["copy_gbs"] = round(2 * cb / (ms_copy * 1e-3) / 1e9, 1)
    del ca, cbuf
    calib_copy(args, line)
    if not args.no_serve:
        # A short serving leg: continuous batching of Poisson arrivals, the
        # latency percentiles at that rate beside the batch throughput.
        del srcs, mask_sets, dmax_sets
        torch.cuda.empty_cache()
        line["serve"] = serve_leg(hx, args.serve_requests, args.rate, args.budget_mb,
                                  4, args.max_batch, pool_n=4)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wl, images)
        line["cpu_tuned"] = cpu_tuned(wl, images)
    print(json.dumps(line), flush=True)


def calib_copy(args, line):
    """With --calib-copy MIB: three device copies of that size, whose
    FETCH_SIZE / WRITE_SIZE readings scale the counters to bytes."""
    if not args.calib_copy:
        return
    import torch
    nbytes = args.calib_copy << 20
    a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    line["calib_copy_bytes"] = nbytes


def percentiles(v, qs=(50, 99)):
    import numpy as np
    return {f"p{q}": round(float(np.percentile(v, q)) * 1e3, 4) for q in qs}


def serve_leg(hx, n, rate, budget_mb, streams, max_batch, pool_n=None, verbose=True,
              zero_copy=False):
    """Continuous batching: n requests (crops of a pool of 4096x4096 images,
    sides log-uniform in [64, 4096]) arrive as a Poisson process at `rate`
    per second and are submitted at their scheduled times; latency runs from
    the scheduled arrival until the mask is in host memory.  Returns the
    measurements as a dict."""
    import numpy as np
    import torch
    from paper_2503_10855_amd import synth

    pool_n = pool_n or synth.SERVING_POOL
    if verbose:
        print(f"serve: generating the request pool ({pool_n} x "
              f"{synth.SERVING_POOL_SIDE}^2)", file=sys.stderr, flush=True)
    pool = synth.serving_pool(pool_n)
    reqs = synth.serving_requests(n, pool=pool_n)
    arrivals = synth.poisson_arrivals(n, rate)
    views = [pool[j][y0:y0 + h, x0:x0 + w] for j, y0, x0, h, w in reqs]
    total_px = sum(h * w for *_, h, w in reqs)
    budget = budget_mb << 20
    # A serving pipeline holds only the batched form's scratch, which counts
    # against the budget; the arena takes the rest.
    with hx.Pipeline(ksize=5, sigma=1.0, theta=0.1, max_pixels=1 << 25,
                     max_images=max_batch, forms=hx.FORM_BATCH,
                     batch_contexts=streams) as p:
        own = p.memory()[0]
        arena = torch.empty(max(budget - own, 1 << 12), dtype=torch.uint8, device="cuda")
        with hx.Server(p, hbm_budget=budget, streams=streams,
                       max_batch=max_batch, arena=arena) as srv:
            # Warm-up: every batch context captures its graph once.  A
            # full pinned pool is drained before the next submission.
            warm = []
            for i in range(min(64, n)):
                t = srv.try_submit(views[i])
                while t is None:
                    j, tj = warm.pop(0)
                    while srv.poll(tj, views[j].shape) is None:
                        time.sleep(1e-4)
                    t = srv.try_submit(views[i])
                warm.append((i, t))
            for i, t in warm:
                while srv.poll(t, views[i].shape) is None:
                    time.sleep(1e-4)
            st0 = srv.stats()
            if verbose:
                print(f"serve: {n} requests at {rate:g}/s, budget {budget_mb} MiB",
                      file=sys.stderr, flush=True)
            lat = np.zeros(n)
            svc = np.zeros(n)
            outs = {}
            pending = {}
            t0 = srv.now() + 0.05
            i = done = 0
            next_report = 1.0
            last_done, last_change = 0, srv.now()
            while done < n:
                now = srv.now()
                while i < n and t0 + arrivals[i] <= now:
                    if zero_copy:
                        # The caller writes the request into its pinned
                        # slot (here: copies the crop) and commits it.
                        rv = srv.reserve(views[i].shape)
                        if rv is None:
                            break
                        t, slot = rv
                        slot[...] = views[i]
                        srv.commit(t, arrival=t0 + arrivals[i])
                        pending[t] = (i, None)
                    else:
                        t = srv.try_submit(views[i], arrival=t0 + arrivals[i])
                        if t is None:
                            break  # pinned pool full until finished requests are polled
                        pending[t] = (i, np.empty(views[i].shape, np.uint8))
                    i += 1
                for t in list(pending):
                    k, buf = pending[t]
                    if zero_copy:
                        r = srv.view(t, views[k].shape)
                        if r is not None and k % 500 == 0:
                            outs[k] = r[0].copy()
                        if r is not None:
                            srv.release(t)
                    else:
                        r = srv.poll_timed(t, buf.shape, out=buf)
                        if r is not None and k % 500 == 0:
                            outs[k] = buf
                    if r is not None:
                        lat[k], svc[k] = r[1], r[2]
                        del pending[t]
                        done += 1
                if now - t0 > next_report:
                    if verbose:
                        print(f"serve: {now - t0:.1f} s, {done} done, {len(pending)} pending",
                              file=sys.stderr, flush=True)
                    next_report += 1.0
                if done != last_done:
                    last_done, last_change = done, now
                elif now - last_change > 30.0:
                    raise RuntimeError(f"serve: no request finished for 30 s "
                                       f"({done} done, {len(pending)} pending)")
                if i < n and not pending:
                    time.sleep(max(0.0, min(2e-4, t0 + arrivals[i] - srv.now())))
            t_end = srv.now()
            st = srv.stats()
        del arena
    # Served masks against the per-image call (bit-exact), on a sample.
    same = True
    with hx.Pipeline(ksize=5, sigma=1.0, theta=0.1, max_pixels=1 << 24) as q:
        for k, m in outs.items():
            ref = q.edge_detect(torch.from_numpy(np.ascontiguousarray(views[k])).cuda())
            same &= bool(np.array_equal(ref.cpu().numpy(), m))
    span = t_end - t0
    return {
        "workload": f"serve-{n}-poisson-{rate:g}-64..4096-k5",
        "mpx_s": round(total_px / span / 1e6, 1),
        "latency_ms": percentiles(lat),
        "latency_ms_mean": round(float(lat.mean()) * 1e3, 3),
        "service_ms": percentiles(svc),
        "offered_mpx_s": round(total_px / arrivals[-1] / 1e6, 1),
        "requests": n, "rate_per_s": rate, "pixels": total_px, "budget_mib": budget_mb,
        "streams": streams, "max_batch": max_batch, "pool_images": pool_n,
        "span_s": round(span, 3),
        "batches": st["batches"] - st0["batches"],
        "mean_batch": round(n / max(1, st["batches"] - st0["batches"]), 2),
        "peak_arena_mib": round(st["peak_bytes"] / 2**20, 1),
        "pipeline_scratch_mib": round(own / 2**20, 1),
        "sample_masks_identical_to_per_image": same,
        "sample": len(outs),
        "submission": "reserve/commit, view/release" if zero_copy else "submit/poll",
    }


def run_serve(args, hx):
    """The serving workload alone: its line carries throughput and the
    latency percentiles."""
    r = serve_leg(hx, args.requests, args.rate, args.budget_mb, args.streams,
                  args.max_batch, zero_copy=args.zero_copy)
    line = {
        "metric": METRIC,
        "value": r["mpx_s"],
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": r["workload"], "requests": r["requests"],
                   "rate_per_s": r["rate_per_s"], "pixels": r["pixels"],
                   "budget_mib": r["budget_mib"], "streams": r["streams"],
                   "max_batch": r["max_batch"], "submission": r["submission"]},
    }
    line.update({k: v for k, v in r.items() if k not in ("workload", "mpx_s", "requests",
                                                          "rate_per_s", "pixels",
                                                          "budget_mib", "streams",
                                                          "max_batch")})
    print(json.dumps(line), flush=True)


def run_reduce(args, hx):
    """The max-reduction ablation: the unfused per-image form (one kernel
    per stage) with three reductions of the gradient magnitude: the wave64
    shuffle tree with one atomic per wave, a two-level tree (per-thread
    partials, then one thread over them), and one thread scanning every
    value."""
    import numpy as np
    import torch
    from paper_2503_10855_amd import synth

    wl = synth.batch_1080p(args.images_reduce)
    imgs = [torch.from_numpy(wl.image(i)).cuda() for i in range(len(wl.sizes))]
    masks = [torch.empty(a.shape, dtype=torch.uint8, device="cuda") for a in imgs]
    sync = torch.cuda.synchronize
    out = {}
    ref = None
    with hx.Pipeline(ksize=5, sigma=1.0, theta=0.1, max_pixels=wl.pixels,
                     max_images=len(imgs)) as p:
        for name, mode in (("tree", hx.REDUCE_TREE), ("two_level", hx.REDUCE_TWO_LEVEL),
                           ("sequential", hx.REDUCE_SEQUENTIAL)):
            p.set_schedule(64, 16, 1, hx.PASS_STORE, mode)
            print(f"reduce: {name}", file=sys.stderr, flush=True)

            def step():
                for s, m in zip(imgs, masks):
                    p.edge_detect(s, m)
            steps = args.steps if mode != hx.REDUCE_SEQUENTIAL else max(1, args.steps // 10)
            ms, _ = timed(step, steps, 1, sync)
            got = [m.cpu() for m in masks]
            if ref is None:
                ref = got
            out[name] = {"ms_per_step": round(ms, 4),
                         "mpx_s": round(wl.pixels / (ms * 1e-3) / 1e6, 1),
                         "same_masks": all(torch.equal(a, b) for a, b in zip(ref, got))}
        p.set_schedule()
    for v in out.values():
        v["speedup_vs_sequential"] = round(out["sequential"]["ms_per_step"] / v["ms_per_step"], 2)
    line = {"metric": "max-reduction ablation (unfused per-image EDGE)", "unit": "Mpixel/s",
            "value": out["tree"]["mpx_s"], "n_gpus": 1, "higher_is_better": True,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": wl.name, "images": len(imgs), "pixels": wl.pixels,
                       "schedule": "64x16 tiles, fusion depth 1"},
            "variants": out}
    print(json.dumps(line), flush=True)


SRAD_BYTES_PER_PX = 8.0   # fused: J read once and written once per iteration
MALL_BYTES = 256e6        # the MI355X's last-level cache (Infinity Cache)


def run_srad(args, hx):
    """SRAD on one square speckle image (default 4096x4096), 100 iterations
    per step: the fused form (timed) and the unfused form, the oracle on a
    bounded number of iterations of the same image.  A step restores the
    input (a device copy, timed separately and subtracted); the per-launch
    time of the fused kernel is the step's time less that of a
    zero-iteration step (copy + the initial sums), over the iterations.
    The fused kernel reads J and writes the next J (8 B/px per iteration);
    when those two planes fit in the 256 MB MALL (4096^2: 134 MB) the
    iterations run out of it, and the line says so: only a size whose planes
    exceed it (8192^2: 537 MB) measures HBM."""
    import torch
    from paper_2503_10855_amd import synth

    H = W = args.srad_side
    niter = args.srad_iters
    lam = 0.5
    img = synth.speckle(H, W)
    J0 = torch.from_numpy(img).cuda()
    J = torch.empty_like(J0)
    sync = torch.cuda.synchronize
    out = {}
    with hx.Pipeline(max_pixels=H * W) as p:
        for fused in (True, False):
            def run(n):
                J.copy_(J0)
                p.srad(J, n, lam, fused=fused)
            ms_zero, _ = timed(lambda: run(0), args.steps, args.warmup, sync)
            ms_full, _ = timed(lambda: run(niter), args.steps, args.warmup, sync)
            out["fused" if fused else "unfused"] = (ms_full, (ms_full - ms_zero) / niter,
                                                    J.clone())
        ms_copy, _ = timed(lambda: J.copy_(J0), args.steps, args.warmup, sync)
    same = bool(torch.equal(out["fused"][2], out["unfused"][2]))
    ms_step = out["fused"][0] - ms_copy
    ms_launch = out["fused"][1]
    mpx_it = H * W * niter / (ms_step * 1e-3) / 1e6
    achieved = SRAD_BYTES_PER_PX * H * W / (ms_launch * 1e-3) / 1e9
    traffic = measured_traffic("k_srad_sweep<0>", H * W, srad_traffic_file(H), SRAD_SOURCES)
    working_set = SRAD_BYTES_PER_PX * H * W
    mall = working_set <= MALL_BYTES
    line = {"metric": "SRAD Mpixel-iterations/s", "value": round(mpx_it, 1),
            "unit": "Mpixel*iter/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "higher_is_better": True, "dtype": "f32",
            "data": "synthetic", "vs_baseline": None,
            "config": {"workload": f"srad-{H}x{W}-{niter}iter", "lambda": lam,
                       "form": "fused (c in registers)",
                       "working_set_mb": round(working_set / 1e6, 1),
                       "resident": "MALL (256 MB)" if mall else "HBM"},
            "ms_per_step": round(ms_step, 4),
            # Priced against the HBM peak either way; a MALL-resident
            # working set (config.resident) makes that an upper bound on
            # what HBM delivered, not a measurement of it.
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                         "kernel": "k_srad_sweep<0>", "ms_per_launch": round(ms_launch, 5),
                         "bytes_per_px": SRAD_BYTES_PER_PX},
            "copy_gbs": round(2 * 4 * H * W / (ms_copy * 1e-3) / 1e9, 1),
            "unfused_ms_per_iteration": round(out["unfused"][1], 5),
            "fused_over_unfused": round(out["unfused"][1] / ms_launch, 2),
            "fused_equals_unfused": same}
    if not args.no_cpu:
        import oracle
        # The oracle on the same image for as many of the iterations as fit
        # in about 10 s on one core (all 100 at 4096^2).
        t0 = time.perf_counter()
        oracle.srad(img, 1, lam)
        one = time.perf_counter() - t0
        n_or = int(max(1, min(niter, 10.0 / max(one, 1e-6))))
        t0 = time.perf_counter()
        oracle.srad(img, n_or, lam)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": round(H * W * n_or / dt / 1e6, 2),
                                "unit": "Mpixel*iter/s", "cores": 1, "kind": "oracle",
                                "host": host_info(),
                                "sample": f"{n_or} of the {niter} iterations on the "
                                          f"{H}x{W} image, {dt:.2f} s"}
    calib_copy(args, line)
    print(json.dumps(line), flush=True)


def run_tune(args, hx):
    """Every candidate schedule (tile x fusion depth x pass structure) timed
    by hx_autotune on one image of the workload's shape (per-image form)."""
    import tempfile
    from paper_2503_10855_amd import synth
    wl = workloads()[args.workload]()
    H, W = wl.sizes[0]
    with tempfile.TemporaryDirectory() as td:
        cache = os.path.join(td, "tune.jsonl")
        with hx.Pipeline(ksize=wl.ksize, sigma=wl.sigma, theta=wl.theta,
                         max_pixels=H * W, max_images=1) as p:
            print(f"tune: {H}x{W} k{wl.ksize}", file=sys.stderr, flush=True)
            chosen = p.autotune(H, W, cache)
        lines = [json.loads(x) for x in open(cache)]
    rows = []
    for x in lines:
        if "trial" not in x:
            continue
        t = x["trial"]
        ms = t["ms"]
        rows.append({"schedule": t["schedule"], "text": t.get("text"), "ms": round(ms, 4),
                     "mpx_s": round(H * W / (ms * 1e-3) / 1e6, 1),
                     "effective_gbs": round(PATH_BYTES_PER_PX * H * W / (ms * 1e-3) / 1e9, 1)})
    rows.sort(key=lambda r: r["ms"])
    line = {"metric": "autotuner sweep (per-image form)", "unit": "Mpixel/s",
            "value": rows[0]["mpx_s"], "n_gpus": 1, "higher_is_better": True,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": wl.name, "height": H, "width": W, "ksize": wl.ksize,
                       "sigma": wl.sigma, "schedule_fields": "tile_w, tile_h, fusion_depth, "
                       "pass_mode (1 store, 2 recompute, 3 speculate), reduce_mode"},
            "chosen": list(chosen), "trials": rows}
    print(json.dumps(line), flush=True)


def run_tune_batch(args, hx):
    """The batch autotuner on the workload's whole batch: every (tile height,
    pass structure) candidate's median time per batched call, and the
    choice."""
    import tempfile
    import torch
    wl = workloads()[args.workload]()
    srcs = [torch.from_numpy(wl.image(i)).cuda() for i in range(len(wl.sizes))]
    with tempfile.TemporaryDirectory() as td:
        cache = os.path.join(td, "tune_batch.jsonl")
        with hx.Pipeline(ksize=wl.ksize, sigma=wl.sigma, theta=wl.theta,
                         max_pixels=wl.pixels, max_images=len(srcs),
                         batch_contexts=min(8, max(1, args.streams))) as p:
            print(f"tune-batch: {wl.name}", file=sys.stderr, flush=True)
            th, pm = p.autotune_batch(srcs, cache_path=cache)
        lines = [json.loads(x) for x in open(cache)]
    names = {1: "store", 2: "recompute", 3: "speculate"}
    rows = [{"tile_h": t["tile_h"], "pass": names[t["pass"]], "ms": round(t["ms"], 4),
             "tput_ms": round(t["tput_ms"], 4), "in_flight": t["in_flight"],
             "mpx_s": round(wl.pixels / (t["tput_ms"] * 1e-3) / 1e6, 1),
             "path_frac": round(PATH_BYTES_PER_PX * wl.pixels / (t["tput_ms"] * 1e-3) / 1e9
                                / HBM_PEAK_GBS, 4)}
            for x in lines if "batch_trial" in x for t in [x["batch_trial"]]]
    rows.sort(key=lambda r: r["tput_ms"])
    line = {"metric": "batch autotuner sweep (time per batched call with calls in flight on "
                      "several streams; ms: one call alone)",
            "unit": "Mpixel/s", "value": rows[0]["mpx_s"], "n_gpus": 1,
            "higher_is_better": True, "dtype": "f32", "data": "synthetic",
            "config": {"workload": wl.name, "images": len(srcs), "pixels": wl.pixels,
                       "ksize": wl.ksize},
            "chosen": {"tile_h": th, "pass": names[pm]}, "trials": rows}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
