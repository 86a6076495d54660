"""Benchmark: shaded rays/s of the KiloNeuS hot path on one MI355X.

Workload (C3): a 16^3 grid over [-1,1]^3 of per-cell MLPs (SDF: 39 -> 2x64
softplus -> 16; color: 48 -> 32 ReLU -> 3 sigmoid), seeded geometric
initialisation toward a sphere of radius 0.6 with N(0, 0.02^2) noise,
1920x1080 primary rays per frame, 8 seeded orbit views cycled, at most 128
sphere-tracing steps, eps 1e-4.  One step = one frame (2,073,600 rays)
through every stage: ray generation and box clip, per-round cell binning,
the march (bfloat16 MLP on MFMA, float32 positions and cell stepping), hit
binning, then refinement and shading with float32 weights and arithmetic.

The same frames are then timed for the variants: split-bfloat16 refinement
and shading (faster, ~2^-16 relative per product), the fp8 e4m3 march and
the float32 march.  A separate pass of 56 frames (8 views x 7, after 16
warm-up frames) gives the frame latency p50 / p99.  Then C5 (path tracing,
32^3, 4 spp, 3 bounces, FP8 vs BF16) and C4 (serving: 8 resident scenes,
Poisson arrivals at 200 requests/s, 2000 measured requests) unless skipped,
and the FP64 oracle on the host's cores.

Prints one JSON line: metric, value, unit, timing, dtype, config, the
roofline of the dominant kernel and the oracle's CPU rate.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "shaded rays/sec at 1920×1080 (BF16/FP8 vs FP32) + p50/p99 frame latency"
# Peaks (MI355X): dense float32 MFMA 157.3 TFLOP/s; transcendentals (exp2,
# log2, sin, cos, rcp) issue at a quarter of the float32 FMA rate of 128
# lanes/clock per CU: 256 CU x 32 /clock x 2.4 GHz = 19.7 T/s.
PEAK_FP32_MFMA = 157.3e12
PEAK_TRANS = 256 * 32 * 2.4e9
PEAK_HBM = 8.0e12

# HBM bytes per launch of the bfloat16 march kernel on this workload, from
# two hardware-counter runs (FETCH_SIZE, then WRITE_SIZE, averaged over the
# launches of 10 frames), each scaled by what the same counter reads for a
# 1 GiB device copy in the same run (fetch x2.0, write x1.0); summary and
# commands in profiles/k_march_bf16_c3_1080p.md.  Valid only for the kernel
# sources they were taken on (the device code's files, KERNEL_SOURCES): any
# change to them makes the figure null.
MARCH_TRAFFIC = dict(sources_sha256="e9d7a0b903a2f4cc314e2c072179353ed7f549c31b28449e94d0d175b81f5b23",
                     bytes_per_launch=68644227.5, fetch_kib=25295.14, write_kib=16446.92,
                     fetch_factor=2.0, write_factor=1.0)


# the files the device code is compiled from (the host runtime is not)
KERNEL_SOURCES = ("kn_device.h", "kn_internal.h", "kn_kernels.hip", "kn_launch.h")


def kernel_sources_sha256() -> str:
    import hashlib
    root = os.path.join(ROOT, "paper_2206_10885_amd", "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(f.encode())
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def march_work(H: int) -> dict:
    """Algorithmic work of one SDF evaluation in the march (per point): the
    dense MLP's FLOPs (39 -> H -> H -> the SDF row) and its transcendental
    operations: an exponential and a logarithm per softplus unit (2H units)
    and the encoding's sines and cosines at the lowest frequency of each axis
    (3 sin + 3 cos; the higher frequencies follow by the double-angle
    identities with multiply-adds), 4H + 6 x 2 = 268 for H = 64, whatever
    the kernel itself issues."""
    flop = 2 * (39 * H + H * H + H)
    trans = 2 * (2 * H) + 12
    return dict(flop=flop, trans=trans)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=56, help="timed frames")
    ap.add_argument("--warmup", type=int, default=16, help="untimed frames")
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32"])
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the split-bf16-shading, fp8 and float32 runs on the same frames")
    ap.add_argument("--latency-frames", type=int, default=56, help="frames of the latency pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target CPU-oracle time (all threads)")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving workload (8 resident scenes, Poisson arrivals)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--no-pathtrace", action="store_true",
                    help="skip the path-tracing workload (32^3, 4 spp, 3 bounces, FP8 vs BF16)")
    ap.add_argument("--no-query", action="store_true",
                    help="skip the point-query workloads (512^3 lattice, eikonal term, random points)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after timing, run one plain float32 device copy of this many MiB "
                         "(a kernel of known HBM traffic, used to scale hardware byte counters)")
    return ap.parse_args()


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return 0.0
    k = (len(xs) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def timed_frames(ctx, sid, cams, out, steps, warmup, torch):
    """Two passes over the same `steps` frames.  The first, with no per-launch
    events, gives the throughput and the frame latencies; the second records
    HIP events around every march and shading launch (on the render stream),
    which costs about 0.3 ms per 1080p frame, and gives the kernel times that
    the roofline uses."""
    for i in range(warmup):
        ctx.render_into(sid, cams[i % len(cams)], out)
    torch.cuda.synchronize()
    gpu_ms, wall_ms, evals, hits, tiles, chunks = [], [], 0, 0, 0, 0
    t0 = time.perf_counter()
    for i in range(steps):
        w0 = time.perf_counter()
        st = ctx.render_into(sid, cams[i % len(cams)], out)
        wall_ms.append((time.perf_counter() - w0) * 1e3)
        gpu_ms.append(st["gpu_ms"])
        evals += st["evals"]
        hits += st["hits"]
        tiles += st["march_tiles"]
        chunks += st["march_chunks"]
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    march_ms, launches, evals_timed, shade_ms = [], 0, 0, []
    for i in range(steps):
        st = ctx.render_into(sid, cams[i % len(cams)], out, kernel_times=True)
        march_ms.append(st["march_ms"])
        launches += st["march_launches"]
        evals_timed += st["evals"]
        shade_ms.append(st["shade_ms"])
    torch.cuda.synchronize()
    return dict(total_s=total, gpu_ms=gpu_ms, wall_ms=wall_ms, evals=evals, hits=hits, tiles=tiles,
                chunks=chunks, march_ms=sum(march_ms), march_launches=launches, evals_timed=evals_timed,
                shade_ms=shade_ms)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, views, W, H, S, eps, target_s):
    """The FP64 oracle, as committed, on seeded pixel samples of the same
    frames: once with every thread the job may use (OMP_NUM_THREADS, else all
    cores), sized to about target_s seconds, then with one thread on a sample
    a tenth that size."""
    from oracle import oracle as O
    from paper_2206_10885_amd import synth
    nproc = os.cpu_count() or 1
    threads = min(nproc, int(os.environ.get("OMP_NUM_THREADS") or nproc))
    os_ = O.OracleScene.from_scene(scene)
    pix = synth.sample_pixels(W, H, 2000, seed=77)
    t = time.perf_counter()
    os_.render(views[0], W, H, S, eps, pixels=pix, nthreads=threads)
    dt = time.perf_counter() - t
    n = int(min(W * H, max(2000, 2000 * target_s / max(dt, 1e-3) / len(views))))

    def run(nthreads, per_view):
        px, tt = 0, 0.0
        for vi, v in enumerate(views):
            p = synth.sample_pixels(W, H, per_view, seed=77 + vi)
            t0 = time.perf_counter()
            os_.render(v, W, H, S, eps, pixels=p, nthreads=nthreads)
            tt += time.perf_counter() - t0
            px += len(p)
        return px, tt

    px, tt = run(threads, n)
    n1 = max(200, n // 10 // max(1, threads // 4))
    px1, tt1 = run(1, n1)
    return dict(value=px / tt, unit="rays/s", cores=threads, kind="oracle",
                sample=f"{px} seeded pixels ({n} per view) of the 8 C3 views, FP64, {tt:.1f} s on {threads} "
                       f"threads; {px1} pixels ({n1} per view) in {tt1:.1f} s on 1 thread",
                value_1_thread=px1 / tt1, nproc=nproc, cpu_model=cpu_model())


def serve_bench(n_req: int, torch) -> dict:
    """8 resident scenes (grids 16^3-32^3, H 32 / 64), requests at Poisson
    arrivals of 200/s with seeded orbit views at resolutions drawn from
    {256^2, 512^2, 800^2, 1920x1080}, 256 steps, bfloat16 march, float32
    refinement and shading; 200 warm-up requests, then n_req measured;
    latency = submission to completion on the host clock."""
    import threading
    from paper_2206_10885_amd import kn, synth
    Ns = [16, 16, 20, 24, 24, 28, 32, 32]
    scenes = [synth.sphere_scene(Ns[k], 32 if k % 2 == 0 else 64, 0.5 + 0.02 * k, 0.02, 4000 + k)
              for k in range(8)]
    sizes = [(256, 256), (512, 512), (800, 800), (1920, 1080)]
    print("serving: scenes generated", file=sys.stderr, flush=True)
    ctx = kn.Context(0, hbm_budget_bytes=(sum(sc.sdf.nbytes for sc in scenes) * 3) + (16 << 30))
    sids = [ctx.scene_create(sc, precisions=("bf16",)) for sc in scenes]
    del scenes
    print("serving: scenes resident", file=sys.stderr, flush=True)
    warm = 200
    total = warm + n_req
    rng = np.random.default_rng(4004)
    gaps = rng.exponential(1.0 / 200.0, total)
    which = rng.integers(0, 8, total)
    res = rng.integers(0, 4, total)
    views = [synth.orbit_views(64, 4000 + k + 500) for k in range(8)]
    ring = 40
    outs = {i: [dict(rgb=torch.empty((h, w, 3), dtype=torch.float32, device="cuda")) for _ in range(ring)]
            for i, (w, h) in enumerate(sizes)}
    torch.cuda.synchronize()
    ctx.serve_start(max_inflight=32, precision="bf16")
    ids = [None] * total
    submitted = threading.Semaphore(0)
    t0 = time.perf_counter()
    arrivals = t0 + np.cumsum(gaps)

    def submitter():
        for i in range(total):
            dt = arrivals[i] - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            w, h = sizes[res[i]]
            cam = kn.make_camera(views[which[i]][i % 64], w, h, 256, 1e-4, "bf16")
            ids[i] = ctx.serve_submit(sids[which[i]], cam, outs[res[i]][i % ring])
            submitted.release()

    th = threading.Thread(target=submitter)
    th.start()
    lat, rays, done_t = [], 0, []
    for i in range(total):
        submitted.acquire()
        st = ctx.serve_poll(ids[i], timeout_us=120_000_000)
        if i % 500 == 499:
            print(f"serving: {i + 1} requests done", file=sys.stderr, flush=True)
        if i >= warm:
            lat.append(st["wall_ms"])
            rays += st["rays"]
            done_t.append(time.perf_counter())
    th.join()
    t_meas0 = arrivals[warm]
    span = max(done_t) - t_meas0
    ctx.serve_stop()
    ctx.close()
    return dict(requests=n_req, warmup=warm, arrival_rate=200.0, latency_ms_p50=pct(lat, 50),
                latency_ms_p99=pct(lat, 99), latency_ms_max=max(lat), rays_per_s=rays / span,
                offered_rays_per_s=rays / (arrivals[-1] - t_meas0), precision="bf16 march, fp32 shading",
                max_steps=256, loop="host-driven rounds (groups of 4 rounds and a shading pass)",
                scenes="8 resident: N=16,16,20,24,24,28,32,32; H=32 (even k) / 64 (odd k); r=0.5+0.02k")


def pathtrace_bench(torch, frames: int = 3) -> dict:
    """32^3 grid, H=64, 1920x1080, 4 spp, 3 Lambertian bounces, 512x256
    environment; FP8 e4m3 march against bfloat16 (refinement and shading with
    float32 weights in both)."""
    from paper_2206_10885_amd import kn, synth
    c = synth.CONFIGS["c5"]
    sc = synth.config_scene("c5")
    env = torch.tensor(synth.env_map(512, 256, seed=c["env_seed"]), device="cuda")
    view = synth.orbit_views(1, c["seed"] + 500)[0]
    W, H = c["width"], c["height"]
    ctx = kn.Context(0)
    sid = ctx.scene_create(sc, precisions=("bf16", "fp8"))
    del sc
    print("pathtrace: scene resident", file=sys.stderr, flush=True)
    out = ctx.alloc_frame(W, H)
    res = {}
    for prec in ("fp8", "bf16"):
        cam = kn.make_camera(view, W, H, c["max_steps"], c["eps"], prec, spp=c["spp"],
                             bounces=c["bounces"], seed=c["path_seed"], env=env)
        ctx.render_into(sid, cam, out)
        torch.cuda.synchronize()
        ms, evals, hits = [], 0, 0
        t = time.perf_counter()
        for _ in range(frames):
            st = ctx.render_into(sid, cam, out)
            ms.append(st["gpu_ms"])
            evals += st["evals"]
            hits += st["hits"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        paths = W * H * c["spp"] * frames
        print(f"pathtrace: {prec} done", file=sys.stderr, flush=True)
        res[prec] = dict(paths_per_s=paths / dt, frame_ms_p50=pct(ms, 50), evals_per_path=evals / paths,
                         hit_segments_per_path=hits / paths, segments_per_s=(hits + paths) / dt)
    ctx.close()
    res["fp8_over_bf16"] = res["fp8"]["paths_per_s"] / res["bf16"]["paths_per_s"]
    res["workload"] = ("32^3 grid, SDF 39->2x64->16, 1920x1080, 4 spp, 3 bounces, 512x256 environment, "
                       "256 steps; segments = primary paths + hit segments")
    return res


def query_bench(torch, reps: int = 3) -> dict:
    """Point-query workloads on the C3 scene (16^3, H=64): dense lattice
    sampling at 512^3 (the mesh-extraction input; 134 M points) in float32,
    bfloat16 and fp8, and with world gradients (float32); the finite-
    difference eikonal term over the paper's M = 16384 uniform points
    (6 stencil evaluations each, delta 1e-3); random points through the
    binned query (1 M points).  Times: HIP events on the call's stream."""
    from paper_2206_10885_amd import kn, synth
    sc = synth.config_scene("c3")
    ctx = kn.Context(0)
    sid = ctx.scene_create(sc, precisions=("bf16", "fp8"))
    R = 512
    d = torch.empty((R, R, R), dtype=torch.float32, device="cuda")
    g = torch.empty((R, R, R, 3), dtype=torch.float32, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        ms = []
        for _ in range(reps):
            ev0.record()
            fn()
            ev1.record()
            torch.cuda.synchronize()
            ms.append(ev0.elapsed_time(ev1))
        return min(ms)

    res = {}
    for prec in ("fp32", "bf16", "fp8"):
        ms = timed(lambda: ctx.grid_sample(sid, R, prec, out=dict(d=d)))
        res[f"grid512_{prec}"] = dict(ms=ms, points_per_s=R ** 3 / (ms / 1e3))
        print(f"query: grid 512 {prec} done", file=sys.stderr, flush=True)
    ms = timed(lambda: ctx.grid_sample(sid, R, "fp32", out=dict(d=d, grad=g)))
    res["grid512_fp32_grad"] = dict(ms=ms, points_per_s=R ** 3 / (ms / 1e3))
    del d, g
    rng = np.random.default_rng(4242)
    pts = torch.tensor(rng.uniform(-1, 1, (16384, 3)).astype(np.float32), device="cuda")
    for prec in ("fp32", "bf16"):
        ms = timed(lambda: ctx.eikonal_fd(sid, pts, 1e-3, prec))
        res[f"eikonal_16384_{prec}"] = dict(ms=ms, points_per_s=16384 / (ms / 1e3))
    pts = torch.tensor(rng.uniform(-1, 1, (1 << 20, 3)).astype(np.float32), device="cuda")
    for prec in ("fp32", "bf16"):
        ms = timed(lambda: ctx.query(sid, pts, prec))
        res[f"query_1M_{prec}"] = dict(ms=ms, points_per_s=(1 << 20) / (ms / 1e3))
    ctx.close()
    res["workload"] = ("C3 scene (16^3, SDF 39->2x64->16): 512^3 lattice (kn_grid_sample); eikonal term by "
                       "central differences at 16384 uniform points, delta 1e-3 (kn_eikonal_fd); "
                       "2^20 uniform random points (kn_query, d only)")
    print("query: done", file=sys.stderr, flush=True)
    return res


def variant(ctx, sid, views, W, H, S, eps, prec, split, out, steps, warmup, torch, kn):
    cams = [kn.make_camera(v, W, H, S, eps, prec, split_shading=split) for v in views]
    r = timed_frames(ctx, sid, cams, out, steps, warmup, torch)
    return r, steps * W * H / r["total_s"]


def latency_pass(ctx, sid, cams, out, frames, torch) -> dict:
    """Frame latency over `frames` frames (the views cycled) after two
    warm-up passes over the views: GPU time first to last kernel (HIP
    events) and host wall time of each kn_render call."""
    for i in range(2 * len(cams)):
        ctx.render_into(sid, cams[i % len(cams)], out)
    torch.cuda.synchronize()
    g, w = [], []
    for i in range(frames):
        t = time.perf_counter()
        st = ctx.render_into(sid, cams[i % len(cams)], out)
        w.append((time.perf_counter() - t) * 1e3)
        g.append(st["gpu_ms"])
    return dict(frames=frames, frame_ms_p50=pct(g, 50), frame_ms_p99=pct(g, 99),
                frame_wall_ms_p50=pct(w, 50), frame_wall_ms_p99=pct(w, 99))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the renderer runs on one GPU per process; "
                                   "--gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2206_10885_amd import kn, synth

    c = synth.CONFIGS["c3"]
    W, H, S, eps = c["width"], c["height"], c["max_steps"], c["eps"]
    scene = synth.config_scene("c3")
    views = synth.config_views("c3")
    ctx = kn.Context(0)
    sid = ctx.scene_create(scene, precisions=("bf16", "fp8"))
    out = ctx.alloc_frame(W, H)
    rays = W * H

    cams = [kn.make_camera(v, W, H, S, eps, args.precision) for v in views]
    r = timed_frames(ctx, sid, cams, out, args.steps, args.warmup, torch)
    value = args.steps * rays / r["total_s"]
    print(f"bench: headline {args.precision} done", file=sys.stderr, flush=True)
    lat = latency_pass(ctx, sid, cams, out, max(args.latency_frames, args.steps), torch)
    work = march_work(scene.H)
    avg_launch_s = r["march_ms"] / 1e3 / max(1, r["march_launches"])
    evals_per_launch = r["evals_timed"] / max(1, r["march_launches"])
    if args.precision == "bf16":
        achieved = evals_per_launch * work["trans"] / avg_launch_s
        traffic = None
        if kernel_sources_sha256() == MARCH_TRAFFIC["sources_sha256"]:
            traffic = MARCH_TRAFFIC["bytes_per_launch"]
        roofline = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_TRANS / 1e12,
                        unit="Tops/s transcendental", frac=achieved / PEAK_TRANS, traffic=traffic,
                        traffic_unit="bytes per launch",
                        traffic_frac_of_hbm=(None if traffic is None else
                                             traffic / avg_launch_s / PEAK_HBM),
                        kernel="k_march<64,bf16>", avg_launch_ms=avg_launch_s * 1e3,
                        evals_per_launch=evals_per_launch, trans_per_eval=work["trans"],
                        timed_over="a second pass over the same frames with HIP events around "
                                   "every march launch on the render stream")
    else:
        achieved = evals_per_launch * work["flop"] / avg_launch_s
        roofline = dict(bound="mfma", achieved=achieved / 1e12, peak=PEAK_FP32_MFMA / 1e12,
                        unit="TFLOP/s", frac=achieved / PEAK_FP32_MFMA, traffic=None,
                        kernel="k_march<64,fp32>", avg_launch_ms=avg_launch_s * 1e3,
                        evals_per_launch=evals_per_launch)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["total_s"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": "C3: 16^3 grid of per-cell SDF MLPs (39->2x64 softplus->16) and "
                               "color MLPs (48->32->3), 1920x1080, 8 seeded orbit views, "
                               "<=128 steps, eps 1e-4; march in " + args.precision +
                               " (float32 ray positions and cell stepping), refinement and shading "
                               "with float32 weights and arithmetic",
                   "rays_per_frame": rays, "views": len(views)},
        "frame_ms_p50": lat["frame_ms_p50"],
        "frame_ms_p99": lat["frame_ms_p99"],
        "frame_wall_ms_p50": lat["frame_wall_ms_p50"],
        "frame_wall_ms_p99": lat["frame_wall_ms_p99"],
        "latency_frames": lat["frames"],
        "evals_per_ray": r["evals"] / (args.steps * rays),
        "march_ms_per_frame": r["march_ms"] / args.steps,
        "shade_ms_per_frame": sum(r["shade_ms"]) / args.steps,
        "march_launches_per_frame": r["march_launches"] / args.steps,
        "march_chunks_per_frame": r["chunks"] / args.steps,
        "evals_per_tile": r["evals"] / max(1, r["tiles"]),
        "hit_fraction": r["hits"] / (args.steps * rays),
        "roofline": roofline,
    }
    if not args.no_variants and args.precision != "fp32":
        vs = {}
        for name, prec, split in (("bf16_split_shading", "bf16", True), ("fp8", "fp8", False),
                                  ("fp8_split_shading", "fp8", True), ("fp32", "fp32", False)):
            rv, vv = variant(ctx, sid, views, W, H, S, eps, prec, split, out, args.steps, args.warmup // 2,
                             torch, kn)
            vs[name] = dict(value=vv, frame_ms_p50=pct(rv["gpu_ms"], 50), frame_ms_p99=pct(rv["gpu_ms"], 99),
                            frames=args.steps, march_ms_per_frame=rv["march_ms"] / args.steps,
                            shade_ms_per_frame=sum(rv["shade_ms"]) / args.steps)
            if prec == "fp32":
                a32 = (rv["evals_timed"] / max(1, rv["march_launches"])) * work["flop"] / (
                    rv["march_ms"] / 1e3 / max(1, rv["march_launches"]))
                vs[name]["march_roofline"] = dict(bound="mfma", achieved=a32 / 1e12, peak=PEAK_FP32_MFMA / 1e12,
                                                  unit="TFLOP/s", frac=a32 / PEAK_FP32_MFMA)
            print(f"bench: variant {name} done", file=sys.stderr, flush=True)
        line["variants"] = vs
        line["fp32_value"] = vs["fp32"]["value"]
        line["bf16_over_fp32"] = value / vs["fp32"]["value"]
        line["fp8_over_fp32"] = vs["fp8"]["value"] / vs["fp32"]["value"]
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx.close()
    if not args.no_pathtrace:
        line["pathtrace"] = pathtrace_bench(torch)
    if not args.no_serve:
        line["serving"] = serve_bench(args.serve_requests, torch)
    if not args.no_query:
        line["point_query"] = query_bench(torch)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(scene, views, W, H, S, eps, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
