"""Benchmark: frames/s of the motion-focus path (pose + focus + map) on one MI355X.

One step = one synthetic stream of the small workload (64 frames 3x280x504, windows of 16 frames
sharing 8, 12-layer D=384 ViT in BF16) pushed from device memory: every window's forward in one
fused batch, FP64 anchoring, focus and focus maps, all 64 results polled (maps into device
memory).  Prints one JSON line.
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
sys.path.insert(0, ROOT)

import mf_synth  # noqa: E402

PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "attn_global_small_traffic.md")
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_2601_07154_amd", "csrc", f) for f in ("attention.hip", "device.h")]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per global-attention launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, if it was taken on this workload and the current kernel source (else None)."""
    import re
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    src = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    val = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    wl = re.search(r"workload:\s*(\S+)", text)
    if not src or not val or not wl or src.group(1) != kernel_source_hash() or wl.group(1) != workload:
        return None
    return float(val.group(1))


def window_sizes(n_frames: int, window: int, overlap: int) -> list:
    """Frames per window of one stream: windows start every window - overlap frames, plus a tail
    window ending at the last frame when the stride does not land there (Sec. 2.2's sliding window)."""
    if n_frames <= window:
        return [n_frames] if n_frames > 0 else []
    starts = list(range(0, n_frames - window + 1, window - overlap))
    if starts[-1] + window < n_frames:
        starts.append(n_frames - window)
    return [window] * len(starts)


def global_attention_flops(wl) -> float:
    """Algorithmic flops of one global-attention launch: every window of the stream, 4 T^2 D each
    (QK^T and PV, 2 flops per multiply-add), T = frames per window x tokens per frame."""
    n = wl.tokens_per_frame
    return sum(4.0 * (S * n) ** 2 * wl.model.dim for S in window_sizes(wl.frames, wl.window, wl.overlap))


def gemm_flops(wl) -> float:
    """Algorithmic flops of the transformer GEMMs (QKV, out-projection, fc1, fc2) of one step."""
    n, D, F, L = wl.tokens_per_frame, wl.model.dim, wl.model.mlp, wl.model.depth
    return sum(L * 2.0 * S * n * D * (3 * D + D + 2 * F) for S in window_sizes(wl.frames, wl.window, wl.overlap))


def path_flops(wl) -> float:
    n, D, F, L = wl.tokens_per_frame, wl.model.dim, wl.model.mlp, wl.model.depth
    tot = 0.0
    for S in window_sizes(wl.frames, wl.window, wl.overlap):
        T = S * n
        gemm = 2.0 * T * D * (3 * D + D + 2 * F)
        tot += L * gemm + (L // 2) * 4.0 * T * T * D + (L - L // 2) * 4.0 * T * n * D
        tot += 2.0 * S * (wl.height // 14) * (wl.width // 14) * 588 * D
    return tot


def run_gpu(wl, precision: str, steps: int, warmup: int, sigma: float, profile: bool = True, graphs: bool = True):
    import torch
    import paper_2601_07154_amd as mfp
    blob = mf_synth.make_weights(wl.model, wl.seed_weights)
    frames = torch.from_numpy(mf_synth.workload_frames(wl)).cuda()
    rows = mfp.rows_per_frame(wl.height, wl.width)
    sched_frames = sum(window_sizes(wl.frames, wl.window, wl.overlap))
    eng = mfp.Engine.from_model(wl.model, blob, precision=precision, max_tokens=sched_frames * rows + 64,
                                graphs=graphs)
    K = (wl.fx, wl.fy, wl.cx, wl.cy)
    maps = torch.empty((wl.frames, wl.height, wl.width), device="cuda", dtype=torch.float32)
    sids = [eng.open_stream(wl.height, wl.width, wl.window, wl.overlap, K, sigma=sigma, ring_frames=wl.frames,
                            result_frames=wl.frames) for _ in range(steps + warmup)]
    recs_all = []

    def step(sid):
        eng.push_frames(sid, frames, eos=True)
        eng.sync()
        got = 0
        while got < wl.frames:
            r, st = eng.poll(sid, wl.frames - got, maps[got:])
            got += len(r)
            recs_all.append(r)
            if st != 0 and got < wl.frames:
                raise RuntimeError("stream ended early")
        return got

    for i in range(warmup):
        step(sids[i])
    recs_all.clear()
    if profile:
        eng.profile(1)   # HIP events around every GEMM and attention launch (eager launches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = 0
    for i in range(steps):
        n += step(sids[warmup + i])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = eng.profile(0)
    stats = eng.stats()
    recs = np.concatenate(recs_all)
    lat = (recs["t_ready"] - recs["t_push"]) * 1e3
    for sid in sids:   # drain: releases the streams
        eng.poll(sid, 1)
    first = recs[:wl.frames]
    eng.close()
    return dict(frames=n, seconds=dt, prof=prof, stats=stats, lat=lat, first=first)


def cpu_baseline(wl, sigma: float):
    """The FP64 oracle on a bounded sample: window 0 (all layers) plus chaining, focus and maps of
    its frames; frames/s extrapolated to the whole stream (its windows per its frames)."""
    from oracle import pipeline, vit
    blob = mf_synth.make_weights(wl.model, wl.seed_weights)
    w = vit.unpack_weights(blob, wl.model.depth, wl.model.dim, wl.model.mlp)
    frames = mf_synth.workload_frames(wl, wl.window)
    t0 = time.perf_counter()
    out = pipeline.run_stream(frames, w, wl.model.heads, wl.window, wl.overlap, (wl.fx, wl.fy, wl.cx, wl.cy),
                              sigma=sigma)
    dt = time.perf_counter() - t0
    nwin = len(window_sizes(wl.frames, wl.window, wl.overlap))
    fps = wl.frames / (nwin * dt)
    return fps, dt, out


def run_serve(args):
    """Serving workload: streams of uneven lengths and resolutions ({280, 378, 504} x 504), Poisson
    arrivals, window 16 stride 8, the 24-layer D=1024 model in BF16 on the threaded engine, against
    the plain FP32 single-stream path (one stream at a time, one window per batch)."""
    import torch
    import paper_2601_07154_amd as mfp
    from paper_2601_07154_amd import serving
    model = mf_synth.SERVE_MODEL
    blob = mf_synth.make_weights(model, 0)
    raw = mf_synth.serve_streams(args.serve_streams, seed=5, min_len=60, max_len=args.serve_max_len,
                                 rate=args.serve_rate)
    specs = [serving.StreamSpec(a if args.serve_paced else 0.0, n, H, W, seed) for (a, n, H, W, seed) in raw]
    pools = {}

    def pool(H, W):
        if (H, W) not in pools:
            pools[(H, W)] = torch.from_numpy(mf_synth.make_frames(16, H, W, 7000 + H)).cuda()
        return pools[(H, W)]

    K = lambda H, W: (0.8 * W, 0.8 * W, W / 2.0, H / 2.0)
    rows = mfp.rows_per_frame(504, 504)
    eng = mfp.Engine.from_model(model, blob, precision="bf16", threaded=True, max_tokens=6 * 16 * rows)
    out = serving.serve(eng, specs, pool, 16, 8, K, fps=30.0, paced=args.serve_paced, time_limit=900)
    st = eng.stats()
    eng.close()
    lat = serving.latency_summary(out["records"])
    frames = lat["frames"]
    res = {"metric": "serving frames/sec and per-frame latency (BF16, continuous batching) vs FP32 single-stream",
           "value": frames / out["wall"], "unit": "frames/s", "n_gpus": 1, "dtype": "bf16",
           "regime": "paced 30 fps, Poisson arrivals" if args.serve_paced else "throughput (all frames available)",
           "streams": len(specs), "frames": frames, "wall_s": out["wall"], "latency_ms": lat,
           "batches": st["batches_run"], "windows": st["windows_run"], "gpu_ms": st["gpu_ms"],
           "config": {"workload": "serving", "model": "24L D1024 16 heads MLP 4096", "window": 16, "overlap": 8,
                      "lengths": f"U[60, {args.serve_max_len}]", "resolutions": "{280,378,504}x504",
                      "rate_per_s": args.serve_rate}}
    if args.serve_fp32_streams:
        eng = mfp.Engine.from_model(model, blob, precision="fp32", threaded=True, max_tokens=16 * rows)
        sub = [serving.StreamSpec(0.0, sp.length, sp.height, sp.width) for sp in specs[:args.serve_fp32_streams]]
        t_frames, t_wall, lats = 0, 0.0, []
        for sp in sub:                      # one stream at a time, one window per batch
            o = serving.serve(eng, [sp], pool, 16, 8, K, paced=False, time_limit=900)
            t_frames += len(o["records"][0])
            t_wall += o["wall"]
            lats.append(o["records"][0])
        eng.close()
        fl = serving.latency_summary(lats)
        res["fp32_single_stream"] = {"value": t_frames / t_wall, "unit": "frames/s", "streams": len(sub),
                                     "latency_ms": fl}
        res["speedup_vs_fp32_single_stream"] = res["value"] / res["fp32_single_stream"]["value"]
    print(json.dumps(res))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-fp8", action="store_true")
    ap.add_argument("--workload", default="small", choices=["small", "large", "fp8"],
                    help="small (the headline line) or one of the larger configurations (no FP32 leg, no CPU baseline)")
    ap.add_argument("--sigma", type=float, default=1000.0)
    ap.add_argument("--source-hash", action="store_true", help="print the attention source hash and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 256 MiB device copy (an elementwise torch kernel) so that HBM counters "
                         "of the same profiler run can be scaled by a transfer of known size")
    ap.add_argument("--serve", action="store_true", help="run the serving workload instead (separate JSON line)")
    ap.add_argument("--serve-streams", type=int, default=8)
    ap.add_argument("--serve-max-len", type=int, default=160)
    ap.add_argument("--serve-rate", type=float, default=0.4)
    ap.add_argument("--serve-paced", action="store_true")
    ap.add_argument("--serve-fp32-streams", type=int, default=2)
    args = ap.parse_args()
    if args.source_hash:
        print(kernel_source_hash())
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported"}))
        sys.exit(2)
    if args.serve:
        run_serve(args)
        return
    wl = {"small": mf_synth.SMALL, "large": mf_synth.LARGE, "fp8": mf_synth.FP8}[args.workload]
    if args.workload != "small":
        args.no_fp32 = True
        args.no_cpu_baseline = True
    if args.copy_calibration:
        # a plain copy of known size for the HBM counters: 1 GiB read and 1 GiB written by one
        # kernel, after 1 GiB of other writes has pushed the source out of the caches
        import torch
        src = torch.ones(256 << 20, device="cuda", dtype=torch.float32)
        flush = torch.zeros(256 << 20, device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, flush, dst
    r = run_gpu(wl, args.precision, args.steps, args.warmup, args.sigma)
    fps = r["frames"] / r["seconds"]
    rg = run_gpu(wl, args.precision, args.steps, args.warmup, args.sigma, profile=False, graphs=True)
    ms_step = r["seconds"] * 1e3 / args.steps
    res = {
        "metric": "frames/sec pose+focus (BF16/FP8 vs FP32 at stated pose error); p50/p99 latency",
        "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic (seeded uniform pixels, seeded N(0,0.02) random-init weights)",
        "config": {"workload": wl.name, "frames": wl.frames, "height": wl.height, "width": wl.width,
                   "window": wl.window, "overlap": wl.overlap, "layers": wl.model.depth, "dim": wl.model.dim,
                   "heads": wl.model.heads, "mlp": wl.model.mlp,
                   "windows_per_step": len(window_sizes(wl.frames, wl.window, wl.overlap)),
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": float(np.percentile(r["lat"], 50)), "p99": float(np.percentile(r["lat"], 99))},
        "path_tflops": path_flops(wl) * args.steps / r["seconds"] / 1e12,
        "value_graphs_unprofiled": rg["frames"] / rg["seconds"],
    }
    prof = r["prof"]
    calls = max(1, prof["attn_global_calls"])
    avg_ms = prof["attn_global_ms"] / calls
    flops = global_attention_flops(wl)
    ach = flops / (avg_ms * 1e-3) / 1e12
    res["roofline"] = {"kernel": "global flash attention (attn_kernel_v3, bf16, hd 64)", "bound": "mfma",
                       "achieved": ach, "peak": PEAK_TFLOPS[args.precision], "unit": "TFLOP/s",
                       "frac": ach / PEAK_TFLOPS[args.precision],
                       "traffic": measured_traffic(wl.name) if args.precision == "bf16" else None,
                       "avg_launch_ms": avg_ms, "launches": prof["attn_global_calls"],
                       "flops_per_launch": flops}
    res["stage_ms_per_step"] = {"attn_global": prof["attn_global_ms"] / args.steps,
                                "attn_frame": prof["attn_frame_ms"] / args.steps,
                                "gemm": prof["gemm_ms"] / args.steps}
    if prof["gemm_ms"] > 0:
        gt = gemm_flops(wl) / (prof["gemm_ms"] / args.steps * 1e-3) / 1e12
        res["gemm_tflops"] = gt
        res["gemm_mfma_frac"] = gt / PEAK_TFLOPS[args.precision]
    if not args.no_fp32 and args.precision != "fp32":
        f = run_gpu(wl, "fp32", 2, 1, args.sigma)
        res["fp32_value"] = f["frames"] / f["seconds"]
        res["speedup_vs_fp32"] = fps / res["fp32_value"]
    f8 = None
    if not args.no_fp8 and args.precision == "bf16":
        f8 = run_gpu(wl, "fp8", args.steps, args.warmup, args.sigma, profile=False, graphs=True)
        res["fp8_value"] = f8["frames"] / f8["seconds"]
        res["speedup_fp8_vs_bf16_graphs"] = res["fp8_value"] / res["value_graphs_unprofiled"]
    if not args.no_cpu_baseline:
        cfps, cdt, out = cpu_baseline(wl, args.sigma)
        nwin = len(window_sizes(wl.frames, wl.window, wl.overlap))
        res["cpu_baseline"] = {"value": cfps, "unit": "frames/s", "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                               "kind": "oracle",
                               "sample": f"window 0 of the workload ({wl.window} frames, all {wl.model.depth} layers, FP64) + "
                                         f"anchoring/focus/maps: {cdt:.1f} s, scaled to {nwin} windows per {wl.frames} frames"}
        # pose error of the timed GPU run against the FP64 oracle on window 0
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from gpu_util import dir_err_deg, rot_err_deg
        Tg = r["first"]["T_w2c"].reshape(-1, 4, 4)[:wl.window]
        Tr = out["T_w"][:wl.window]
        res["pose_error_window0"] = {"rot_deg_max": float(rot_err_deg(Tg[:, :3, :3], Tr[:, :3, :3]).max()),
                                     "tdir_deg_max": float(dir_err_deg(Tg[:, :3, 3], Tr[:, :3, 3]).max())}
        if f8 is not None:
            T8 = f8["first"]["T_w2c"].reshape(-1, 4, 4)[:wl.window]
            res["pose_error_window0_fp8"] = {"rot_deg_max": float(rot_err_deg(T8[:, :3, :3], Tr[:, :3, :3]).max()),
                                             "tdir_deg_max": float(dir_err_deg(T8[:, :3, 3], Tr[:, :3, 3]).max())}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
