"""Benchmark of the AAA-Gaussians rasterisation path on one MI355X.

Workload: 1,000,000 Gaussians of the seeded cluster generator (SH degree 3,
float32), 1920x1080, 60 deg horizontal field of view, 16x16 tiles, per-ray
window K = 16, the 32 poses on a sphere of radius 12 (one pose per step,
cycled).  A step is one full forward frame: preprocess, pair count, scan,
pair write, radix sort, tile ranges and blend.  The scene is resident in HBM
before the timed region starts.

Prints one JSON line with the throughput (frames/s), the roofline of the
dominant kernel (the blend, VALU-bound) measured with HIP events on the
render stream, and the FP64 CPU oracle timed on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic FP32 work of the blend (FMA = 2 flops), per unit:
#   every evaluation (pixel x list entry, prefilter path): 2 offsets, line
#   direction 3x2 FMA, o_g x r 3x2 FMA, two squared norms (1 mul + 2 FMA
#   each), prefilter product                                          -> 37
#   every evaluation that passes the prefilter: reciprocal, rho^2, scale,
#   exp2, amplitude, clamp, depth numerator (2 FMA), depth, 2 compares -> 13
#   every contributor: K window compares + blend (1 sub, 2 mul,
#   1 compare, 3 FMA)                                                 -> K + 10
FLOPS_EVAL = 37
FLOPS_NEAR = 13
FLOPS_CONTRIB_BASE = 10
# FP32 vector peak without packed FP32 (disabled in every build here):
# 256 CUs x 64 lanes x 2 flops (FMA) x 2.4 GHz.
PEAK_VALU_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12   # 78.6
PEAK_HBM_GBS = 8000.0
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_blend_1M_1080p_counters.txt")
BLEND_SRC = os.path.join(ROOT, "paper_2504_12811_amd", "csrc", "blend.hip")


def blend_counters():
    """key: value lines of the committed counter summary, or {} when it is
    missing or belongs to a different blend source."""
    import hashlib
    try:
        kv = {}
        with open(COUNTERS_FILE) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        with open(BLEND_SRC, "rb") as f:
            sha = hashlib.sha1(f.read()).hexdigest()
        return kv if kv.get("source_sha1") == sha else {}
    except OSError:
        return {}


def blend_traffic_bytes():
    """HBM bytes per blend launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the same
    counter reads for a copy of known size), or None when the summary is
    missing or was taken on a different blend source."""
    import hashlib
    try:
        kv = {}
        with open(COUNTERS_FILE) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        with open(BLEND_SRC, "rb") as f:
            sha = hashlib.sha1(f.read()).hexdigest()
        if kv.get("source_sha1") != sha:
            return None
        probe = float(kv["copy_probe_bytes"])
        f_scale = probe / (float(kv["copy_fetch_kib"]) * 1024.0)
        w_scale = probe / (float(kv["copy_write_kib"]) * 1024.0)
        return (float(kv["fetch_kib_per_dispatch"]) * 1024.0 * f_scale
                + float(kv["write_kib_per_dispatch"]) * 1024.0 * w_scale)
    except (OSError, KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=128)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--window", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-poses", type=int, default=12)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed region, copy this many MiB once (counter calibration)")
    ap.add_argument("--bwd-steps", type=int, default=32)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="seconds of Poisson arrivals per rate and mode (60 for the full protocol)")
    ap.add_argument("--serve-rates", type=str, default="50,100,200,400,800")
    ap.add_argument("--serve-rates-single", type=str, default="50,100,200,400,800",
                    help="rates for the one-request-at-a-time baseline")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the other workloads (500k 1080p, 3M 2064x2208 120deg and its zoom sweep, the "
                         "1M 720p 16-view training step) and the Tab. 5 ablations")
    ap.add_argument("--frames-3m", type=int, default=0,
                    help="only render the 3M 2064x2208 120deg primary view this many times (for kernel profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_12811_amd import scenes as S
    from paper_2504_12811_amd.render import DeviceScene, Rasterizer

    if args.frames_3m > 0:
        scene, cam, _ = S.ood_scene()
        ds = DeviceScene.from_host(scene, "cuda:0")
        ras = Rasterizer(0)
        st = S.Settings(ray_window=args.window)
        r = _time_frames(ras, ds, [cam], st, steps=args.frames_3m, warmup=2)
        print(json.dumps({"workload": "3M 2064x2208 120deg primary view", **r}), flush=True)
        return

    t0 = time.time()
    scene, cams = S.headline(n=args.n)
    gen_s = time.time() - t0
    print(f"# scene generated in {gen_s:.1f}s", file=sys.stderr, flush=True)
    st = S.Settings(ray_window=args.window)
    ds = DeviceScene.from_host(scene, "cuda:0")
    ras = Rasterizer(0)
    torch.cuda.synchronize()

    # per-pose counters (untimed): pairs, evaluations, contributors
    counts = []
    for cam in cams:
        _, _, s = ras.render(ds, cam, st, stats=True)
        counts.append((s.pairs, s.evaluations, s.near, s.contributors, s.visible, s.wave_steps, s.wave_near_steps,
                       s.wave_contrib_steps))
    torch.cuda.synchronize()
    for k in range(args.warmup):
        ras.render(ds, cams[k % len(cams)], st)
    torch.cuda.synchronize()
    ras.stage_times(reset=True)

    # timed region (HIP events around every frame on the render stream give
    # the per-frame times; the wall clock gives the throughput).  The frames
    # carry no per-stage events: those stall the stream at every stage
    # boundary (~40 us per frame) and are taken on a separate run below.
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record()
        ras.render(ds, cams[k % len(cams)], st)
        evs[k][1].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    frame_ms = np.array([a.elapsed_time(b) for a, b in evs])
    # per-stage times (HIP events between the stages, on the render stream)
    stage_frames = min(args.steps, 64)
    for k in range(stage_frames):
        ras.render(ds, cams[k % len(cams)], st, timing=True)
    torch.cuda.synchronize()
    stage_ms, frames = ras.stage_times(reset=True)
    assert frames == stage_frames, (frames, stage_frames)

    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        a = torch.empty(nb // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()

    # measured machine rates beside the spec peaks (FMA and exp rates,
    # copy bandwidth over a 1 GiB buffer)
    import ctypes
    from paper_2504_12811_amd import _lib as L
    pk_buf = torch.empty((1 << 30) + 256, dtype=torch.uint8, device="cuda:0")
    pk = (ctypes.c_double * 3)()
    L.check(L.lib().aaa_measure_peaks(pk_buf.data_ptr() + (-pk_buf.data_ptr()) % 256, 1 << 30, 5,
                                      torch.cuda.current_stream().cuda_stream, pk))
    del pk_buf
    peaks_measured = {"fp32_fma_tflops": round(pk[0], 2), "exp_g_per_s": round(pk[1], 1),
                      "copy_gbps": round(pk[2], 1),
                      "spec": {"fp32_vector_tflops_nonpacked": round(PEAK_VALU_TFLOPS, 1),
                               "fp32_vector_tflops_packed": 157.3, "hbm_gbps": PEAK_HBM_GBS}}

    fps = args.steps / elapsed
    ms_step = 1000.0 * elapsed / args.steps
    # algorithmic work of the timed frames (same pose cycle as the counters)
    used = [counts[k % len(cams)] for k in range(args.steps)]
    P = np.array([u[0] for u in used], np.float64)
    E = np.array([u[1] for u in used], np.float64)
    NE = np.array([u[2] for u in used], np.float64)
    CT = np.array([u[3] for u in used], np.float64)
    VIS = np.array([u[4] for u in used], np.float64)
    blend_ms = stage_ms["blend"] / frames
    flops = FLOPS_EVAL * E.mean() + FLOPS_NEAR * NE.mean() + (args.window + FLOPS_CONTRIB_BASE) * CT.mean()
    achieved = flops / (blend_ms * 1e-3) / 1e12
    # HBM-bound stages, algorithmic bytes: the preprocess reads the 12
    # non-SH floats of every Gaussian and writes its status, and reads the SH
    # coefficients and writes a ~96-byte render record only for the visible
    # ones; the sort's passes over the list bits read every key for the
    # histogram (8 B) and read and write key and value (24 B), then the
    # per-list sort reads and writes each pair once more (24 B)
    n = ds.n
    sh_floats = 3 * (scene.sh_degree + 1) ** 2
    pre_bytes = n * (4 * 12 + 4) + VIS.mean() * (4 * sh_floats + 96)
    ntiles = cams[0].tiles[0] * cams[0].tiles[1]
    passes = (int(np.ceil(np.log2(ntiles))) + 7) // 8
    sort_bytes = P.mean() * (32 * passes + 24)
    pre_ms = stage_ms["preprocess"] / frames
    sort_ms = stage_ms["sort"] / frames

    res = {
        "metric": "frames/s @1080p 1M Gaussians (forward)",
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded cluster scene; datasets and trained scenes not available)",
        "config": {"workload": f"forward render, {n} Gaussians SH3, 1920x1080, 60deg FoV, 16x16 tiles, "
                               f"K={args.window}, 32 poses r=12", "n_gaussians": n, "width": 1920,
                   "height": 1080, "fov_deg": 60, "sh_degree": 3, "ray_window": args.window},
        "mpix_per_s": round(fps * 1920 * 1080 / 1e6, 2),
        "frame_ms": {"median": round(float(np.median(frame_ms)), 4), "p99": round(float(np.percentile(frame_ms, 99)), 4),
                     "frames": int(len(frame_ms)), "timer": "HIP events around each frame on the render stream (no per-stage events)"},
        "roofline": {
            "kernel": "k_blend<16>",
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": round(PEAK_VALU_TFLOPS, 1),
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_VALU_TFLOPS, 4),
            "traffic": (lambda b: None if b is None else round(b))(blend_traffic_bytes()),
            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "valu_busy": (lambda kv: float(kv["valu_busy"]) if "valu_busy" in kv else None)(blend_counters()),
            "avg_ms": round(blend_ms, 4),
            "flops_per_launch": flops,
            "frac_of_measured_fma_rate": round(achieved / peaks_measured["fp32_fma_tflops"], 4)
            if peaks_measured["fp32_fma_tflops"] > 0 else None,
        },
        "peaks_measured": peaks_measured,
        "stages_ms": {k: round(v / frames, 4) for k, v in stage_ms.items()},
        "stages_timer": f"HIP events between the stages, {frames} further frames",
        "hbm_stages": {
            "preprocess": {"bytes": round(pre_bytes), "GBps": round(pre_bytes / (pre_ms * 1e-3) / 1e9, 1),
                           "frac": round(pre_bytes / (pre_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
            "sort": {"bytes": round(sort_bytes), "passes": passes, "GBps": round(sort_bytes / (sort_ms * 1e-3) / 1e9, 1),
                     "frac": round(sort_bytes / (sort_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
        },
        "per_frame": {"pairs": P.mean(), "visible": VIS.mean(), "evaluations": E.mean(),
                      "prefilter_passes": NE.mean(), "contributors": CT.mean(),
                      "wave_steps": float(np.mean([u[5] for u in used])),
                      "wave_steps_prefilter": float(np.mean([u[6] for u in used])),
                      "wave_steps_contributor": float(np.mean([u[7] for u in used]))},
    }

    # forward + backward: L1 loss against a seeded noise target, one pose per step
    if args.bwd_steps > 0:
        target = torch.from_numpy(S.noise_target(1080, 1920)).to("cuda:0")
        for k in range(4):
            rgb, T, _ = ras.render(ds, cams[k % len(cams)], st)
            g = torch.sign(rgb - target) / rgb.numel()
            ras.backward(ds, cams[k % len(cams)], st, ras.last_ws, rgb, g)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        bwd_ms = 0.0
        t0 = time.perf_counter()
        for k in range(args.bwd_steps):
            cam = cams[k % len(cams)]
            rgb, T, _ = ras.render(ds, cam, st)
            g = torch.sign(rgb - target) / rgb.numel()
            ev0.record()
            ras.backward(ds, cam, st, ras.last_ws, rgb, g)
            ev1.record()
            ev1.synchronize()
            bwd_ms += ev0.elapsed_time(ev1)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res["fwd_bwd"] = {"value": round(args.bwd_steps / el, 3), "unit": "frames/s", "steps": args.bwd_steps,
                          "ms_per_step": round(1000 * el / args.bwd_steps, 4),
                          "backward_ms": round(bwd_ms / args.bwd_steps, 4),
                          "loss": "L1 vs seeded U[0,1] noise image"}

    # serving: Poisson arrivals, mixed resolution / FoV / zoom, 1M resident scene
    if not args.no_serving:
        from paper_2504_12811_amd.serve import Server, gpu_render_batch, run_load
        serving = {}
        cap = 16 << 30
        for mode, (workers, maxb) in {"batched": (2, 8), "one_at_a_time": (1, 1)}.items():
            # each worker's workspace (its share of the cap) is allocated here,
            # before any request arrives
            fn = gpu_render_batch(ds, st, n_workers=workers, worker_bytes=cap // workers)
            rates = args.serve_rates if mode == "batched" else args.serve_rates_single
            for rate in [float(r) for r in rates.split(",")]:
                with Server(fn, n_gaussians=ds.n, mem_cap=cap, max_batch=maxb, n_workers=workers) as srv:
                    run_load(srv, rate, 0.5, seed=99)  # warm-up (allocations, code paths)
                    lat, frames, wall, rej = run_load(srv, rate, args.serve_seconds, seed=int(rate))
                    batches = list(srv.batches)
                serving[f"{mode}@{int(rate)}"] = {
                    "rate_req_s": rate, "requests": int(len(lat)), "rejected": rej,
                    "p50_ms": round(1000 * float(np.percentile(lat, 50)), 2) if len(lat) else None,
                    "p99_ms": round(1000 * float(np.percentile(lat, 99)), 2) if len(lat) else None,
                    "frames_per_s": round(frames / wall, 2), "mean_batch": round(float(np.mean(batches)), 2),
                    "seconds": args.serve_seconds}
                print(f"# serving {mode} {rate}: {serving[f'{mode}@{int(rate)}']}", file=sys.stderr, flush=True)
            del fn
            torch.cuda.empty_cache()
        res["serving"] = serving

    if not args.no_workloads:
        res["workloads"] = run_workloads(ras, st, args)

    if not args.no_cpu_baseline:
        from oracle import oracle as O
        k = max(1, args.cpu_poses)
        t0 = time.perf_counter()
        for p in range(k):
            O.render(scene, cams[p], st)
        cpu_s = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(k / cpu_s, 4), "unit": "frames/s", "cores": O.num_threads(),
                               "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": f"{k} full 1920x1080 frames (poses 0..{k - 1}) of the same 1M scene, "
                                         f"FP64 oracle, {cpu_s:.1f}s wall"}
    print(json.dumps(res), flush=True)


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_frames(ras, ds, cams, st, steps, warmup):
    """Forward frames over `cams` (cycled): frames/s, median and p99 frame
    time (HIP events around each frame), then per-stage ms (HIP events
    between the stages) on up to 32 further frames."""
    import torch
    for k in range(warmup):
        ras.render(ds, cams[k % len(cams)], st)
    torch.cuda.synchronize()
    ras.stage_times(reset=True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        evs[k][0].record()
        ras.render(ds, cams[k % len(cams)], st)
        evs[k][1].record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    fm = np.array([a.elapsed_time(b) for a, b in evs])
    for k in range(min(steps, 32)):
        ras.render(ds, cams[k % len(cams)], st, timing=True)
    torch.cuda.synchronize()
    ms, frames = ras.stage_times(reset=True)
    _, _, s0 = ras.render(ds, cams[0], st, stats=True)
    c = cams[0]
    return {"frames_per_s": round(steps / el, 3), "ms_per_frame": round(1000 * el / steps, 4),
            "median_ms": round(float(np.median(fm)), 4), "p99_ms": round(float(np.percentile(fm, 99)), 4),
            "frames": steps, "mpix_per_s": round(steps / el * c.width * c.height / 1e6, 2),
            "stages_ms": {k: round(v / frames, 4) for k, v in ms.items()},
            "pairs": int(s0.pairs), "evaluations": int(s0.evaluations), "contributors": int(s0.contributors)}


def run_workloads(ras, st, args):
    """The other workloads of the benchmark family, each timed on its own."""
    import torch
    from paper_2504_12811_amd import scenes as S
    from paper_2504_12811_amd.render import DeviceScene
    out = {}
    # ablations of Tab. 5 on the headline scene: without 3D tile culling
    # (rectangles only) and without the per-ray window (K = 0: tile order)
    scene, cams = S.headline()
    ds = DeviceScene.from_host(scene, "cuda:0")
    full = _time_frames(ras, ds, cams, st, steps=64, warmup=8)
    no_cull = _time_frames(ras, ds, cams, S.Settings(ray_window=st.ray_window, tile_cull=False), steps=64, warmup=8)
    no_sort = _time_frames(ras, ds, cams, S.Settings(ray_window=0), steps=64, warmup=8)
    # the three-level hierarchy: tile culling, the exact per-8x8 sub-tile
    # re-sort and the per-ray window
    three = _time_frames(ras, ds, cams, S.Settings(ray_window=st.ray_window, subtile_sort=True), steps=64, warmup=8)
    out["ablation_1M_1080p"] = {
        "full_ms": full["ms_per_frame"], "no_tile_cull_ms": no_cull["ms_per_frame"],
        "no_ray_window_ms": no_sort["ms_per_frame"], "three_level_ms": three["ms_per_frame"],
        "culling_speedup": round(no_cull["ms_per_frame"] / full["ms_per_frame"], 3),
        "ray_window_cost": round(full["ms_per_frame"] / no_sort["ms_per_frame"], 3),
        "hier_sort_cost_three_level": round(three["ms_per_frame"] / no_sort["ms_per_frame"], 3),
        "pairs": {"full": full["pairs"], "no_tile_cull": no_cull["pairs"], "three_level": three["pairs"]},
        "stages_ms": {"full": full["stages_ms"], "no_tile_cull": no_cull["stages_ms"],
                      "no_ray_window": no_sort["stages_ms"], "three_level": three["stages_ms"]},
        "paper_tab5_ratios": {"culling_speedup": [1.87, 2.16, 1.82, 1.53], "hier_sort_cost": [1.88, 1.69, 1.91, 1.67],
                              "hardware": "RTX 4090, trained scenes"}}
    print(f"# workload ablation: {out['ablation_1M_1080p']}", file=sys.stderr, flush=True)
    del ds
    # 500k Gaussians, 1920x1080, 60 deg, the 32 poses
    scene, cams = S.medium()
    ds = DeviceScene.from_host(scene, "cuda:0")
    out["500k_1080p"] = _time_frames(ras, ds, cams, st, steps=128, warmup=16)
    print(f"# workload 500k: {out['500k_1080p']}", file=sys.stderr, flush=True)
    del ds
    # 3M Gaussians (10% straddling the near plane), 2064x2208, 120 deg; zoom sweep 2x..64x scene radius
    scene, cam, zoom = S.ood_scene()
    ds = DeviceScene.from_host(scene, "cuda:0")
    out["3M_2064x2208_120deg"] = _time_frames(ras, ds, [cam], st, steps=100, warmup=4)
    print(f"# workload 3M primary: {out['3M_2064x2208_120deg']}", file=sys.stderr, flush=True)
    sweep = []
    for z in zoom:
        r = _time_frames(ras, ds, [z], st, steps=100, warmup=4)
        sweep.append({"distance": round(float(np.linalg.norm(z.position)), 2), **r})
        print(f"# workload 3M zoom {sweep[-1]['distance']}: {r['frames_per_s']} fps", file=sys.stderr, flush=True)
    out["3M_zoom_sweep"] = sweep
    del ds
    # 1M Gaussians, 1280x720, 70 deg: one training step = 16 views forward
    # (one batch), L1 loss, 16 views backward, Adam update of every parameter
    from paper_2504_12811_amd.train import Adam, train_step
    scene, cams = S.fwd_bwd_scene()
    ds = DeviceScene.from_host(scene, "cuda:0")
    target = torch.from_numpy(S.noise_target(720, 1280)).to("cuda:0")
    opt = Adam(ds)

    def step():
        return train_step(ras, ds, cams, [target] * len(cams), st, opt)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    n_steps = 6
    t0 = time.perf_counter()
    for _ in range(n_steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["1M_720p_16view_fwd_bwd"] = {"steps_per_s": round(n_steps / el, 3), "ms_per_step": round(1000 * el / n_steps, 3),
                                     "views_per_s": round(16 * n_steps / el, 2), "views_per_step": 16,
                                     "loss": "L1 vs seeded U[0,1] noise image", "optimizer": "Adam (fused kernel)"}
    print(f"# workload 720p fwd+bwd: {out['1M_720p_16view_fwd_bwd']}", file=sys.stderr, flush=True)
    return out


if __name__ == "__main__":
    main()
