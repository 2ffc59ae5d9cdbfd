"""Benchmark: frames/s of the motion-focus path (pose + focus + map) on one MI355X.

One step = one synthetic stream of the large workload (256 frames 3x378x504, windows of 32 frames
sharing 16, 24-layer D=1024 ViT with 16 heads, MLP 4096, BF16) pushed from device memory: every
window's forward in one fused batch (15 windows, 31 136 tokens each in global attention), FP64
anchoring, focus and focus maps, all 256 results polled (maps into device memory).  Prints one
JSON line.  --workload small|fp8 runs the other configurations.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import mf_synth  # noqa: E402

PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3, "fp8": 5000.0}
HBM_GBPS = 8000.0
TRAFFIC_FILES = {mf_synth.SMALL.name: os.path.join(ROOT, "profiles", "attn_global_small_traffic.md"),
                 mf_synth.LARGE.name: os.path.join(ROOT, "profiles", "attn_global_large_traffic.md")}
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_2601_07154_amd", "csrc", f) for f in ("attention.hip", "device.h")]
GOLDEN = {mf_synth.SMALL.name: "small_fp64_w01", mf_synth.LARGE.name: "large_fp64_w01",
          mf_synth.FP8.name: "fp8_fp64_w0"}
SIGMA = 1000.0   # focus-map spread per unit of |a_w|, the value the stored oracle outputs use
GEMM_STAGES = ("qkv", "out_proj", "fc1", "fc2")


def progress(msg: str) -> None:
    """A line on stderr per finished leg (the JSON result stays the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per global-attention launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary of this workload, if it was taken on the current kernel source (else None)."""
    import re
    path = TRAFFIC_FILES.get(workload)
    if path is None:
        return None
    try:
        text = open(path).read()
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


def global_attention_bytes(wl) -> float:
    """Algorithmic HBM bytes of one global-attention launch: Q, K, V read once and O written once,
    bf16, T x D each per window."""
    n = wl.tokens_per_frame
    return sum(4 * 2.0 * S * n * wl.model.dim for S in window_sizes(wl.frames, wl.window, wl.overlap))


def gemm_stage_flops(wl) -> dict:
    """Algorithmic flops per launch of each transformer GEMM (all windows of the step): 2 T D x out."""
    n, D, F = wl.tokens_per_frame, wl.model.dim, wl.model.mlp
    T = sum(S * n for S in window_sizes(wl.frames, wl.window, wl.overlap))
    return {"qkv": 2.0 * T * D * 3 * D, "out_proj": 2.0 * T * D * D, "fc1": 2.0 * T * D * F, "fc2": 2.0 * T * F * D}


def gemm_flops(wl) -> float:
    """Algorithmic flops of the transformer GEMMs (QKV, out-projection, fc1, fc2) of one step."""
    return wl.model.depth * sum(gemm_stage_flops(wl).values())


def path_flops(wl) -> float:
    n, D, F, L = wl.tokens_per_frame, wl.model.dim, wl.model.mlp, wl.model.depth
    tot = 0.0
    for S in window_sizes(wl.frames, wl.window, wl.overlap):
        T = S * n
        gemm = 2.0 * T * D * (3 * D + D + 2 * F)
        tot += L * gemm + (L // 2) * 4.0 * T * T * D + (L - L // 2) * 4.0 * T * n * D
        tot += 2.0 * S * (wl.height // 14) * (wl.width // 14) * 588 * D
    return tot


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class Inputs:
    """The workload's seeded weight blob and frames (host and device), made once per run."""

    def __init__(self, wl):
        import torch
        self.wl = wl
        self.blob = mf_synth.make_weights(wl.model, wl.seed_weights)
        self.frames_np = mf_synth.workload_frames(wl)
        self.frames = torch.from_numpy(self.frames_np).cuda()


def run_gpu(inp: Inputs, precision: str, steps: int, warmup: int, profile: bool = True, graphs: bool = True):
    """steps + warmup streams of the workload, each pushed whole (MF_EOS) and drained; every window
    of a stream runs in one fused batch.  Returns frames, seconds, timing and the first stream's records."""
    import torch
    import paper_2601_07154_amd as mfp
    wl = inp.wl
    rows = mfp.rows_per_frame(wl.height, wl.width)
    sched_frames = sum(window_sizes(wl.frames, wl.window, wl.overlap))
    eng = mfp.Engine.from_model(wl.model, inp.blob, precision=precision, max_tokens=sched_frames * rows + 64,
                                graphs=graphs)
    K = (wl.fx, wl.fy, wl.cx, wl.cy)
    maps = torch.empty((wl.frames, wl.height, wl.width), device="cuda", dtype=torch.float32)
    sids = [eng.open_stream(wl.height, wl.width, wl.window, wl.overlap, K, sigma=SIGMA, ring_frames=wl.frames,
                            result_frames=wl.frames) for _ in range(steps + warmup)]
    recs_all = []

    def step(sid):
        eng.push_frames(sid, inp.frames, eos=True)
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
    prof = eng.profile(-1)
    stages = eng.profile_stages()
    eng.profile(0)
    recs = np.concatenate(recs_all)
    for sid in sids:   # drain: releases the streams
        eng.poll(sid, 1)
    first = recs[:wl.frames]
    shared = eng.stats()["frames_embed_shared"] / (steps + warmup)
    eng.close()
    return dict(frames=n, seconds=dt, prof=prof, stages=stages, first=first, shared_per_step=shared,
                batch_ms=(recs["t_ready"] - recs["t_push"]).max() * 1e3)


def run_fp32_single_stream(inp: Inputs):
    """The plain FP32 path: the same kernels instantiated for fp32 operands, one window per batch
    (one stream, no batching of windows), no hipGraphs; one whole stream after a one-window warm-up."""
    import torch
    import paper_2601_07154_amd as mfp
    wl = inp.wl
    rows = mfp.rows_per_frame(wl.height, wl.width)
    eng = mfp.Engine.from_model(wl.model, inp.blob, precision="fp32", max_tokens=wl.window * rows + 64, graphs=False)
    K = (wl.fx, wl.fy, wl.cx, wl.cy)
    maps = torch.empty((wl.frames, wl.height, wl.width), device="cuda", dtype=torch.float32)

    def stream(nf):
        sid = eng.open_stream(wl.height, wl.width, wl.window, wl.overlap, K, sigma=SIGMA, ring_frames=wl.frames,
                              result_frames=wl.frames)
        eng.push_frames(sid, inp.frames[:nf], eos=True)
        got = 0
        while got < nf:
            eng.sync()
            r, _ = eng.poll(sid, nf - got, maps[got:])
            got += len(r)
        eng.poll(sid, 1)
        return got

    stream(wl.window)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = stream(wl.frames)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = eng.stats()
    eng.close()
    return n / dt, dt, st


def cpu_baseline(wl, blob):
    """The FP64 oracle on a bounded sample of window 0: its forward with 0 and with 2 transformer
    blocks (one frame-wise, one global), each with the pose head, anchoring, focus and maps of its
    frames.  A window's time is extrapolated as t0 + (depth / 2)(t2 - t0); frames/s = frames per
    stream / (windows per stream x that time)."""
    from oracle import pipeline, vit
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    w = vit.unpack_weights(blob, wl.model.depth, wl.model.dim, wl.model.mlp)
    frames = mf_synth.workload_frames(wl, wl.window)
    K = (wl.fx, wl.fy, wl.cx, wl.cy)
    times = {}
    for nl in (0, 2):
        wt = dict(w)
        wt["layers"] = w["layers"][:nl]
        t0 = time.perf_counter()
        pipeline.run_stream(frames, wt, wl.model.heads, wl.window, wl.overlap, K, sigma=SIGMA, windows=1,
                            workers=threads)
        times[nl] = time.perf_counter() - t0
    t_win = times[0] + (wl.model.depth / 2.0) * (times[2] - times[0])
    nwin = len(window_sizes(wl.frames, wl.window, wl.overlap))
    fps = wl.frames / (nwin * t_win)
    sample = (f"window 0 ({wl.window} frames) through the FP64 oracle with 0 and with 2 of its {wl.model.depth} "
              f"blocks (+ pose head, anchoring, focus, maps): {times[0]:.1f} s and {times[2]:.1f} s; a window "
              f"extrapolated to {t_win:.0f} s, {nwin} windows per {wl.frames} frames; {threads} threads over "
              f"attention heads and BLAS")
    return {"value": fps, "unit": "frames/s", "cores": threads, "kind": "oracle", "sample": sample,
            "cpu_model": cpu_model(), "seconds": times[0] + times[2]}


def golden_errors(wl, inp: Inputs, recs):
    """Errors of a GPU run's first windows against the stored FP64 oracle outputs of this workload
    (rotation and translation-direction degrees; acceleration direction degrees over the frames with
    a focus; focus-pixel L2 over the frames whose acceleration points within 60 deg of the optical
    axis, |a_z| >= 0.5 |a|).  None when no stored output exists for this workload and these inputs."""
    name = GOLDEN.get(wl.name)
    path = os.path.join(ROOT, "tests", "golden", (name or "") + ".json")
    if not name or not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    k = g["key"]
    sha = lambda a: hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
    if k["weights_sha256"] != sha(inp.blob) or k["frames_sha256"] != sha(inp.frames_np[:k["frames_read"]]):
        return None
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_util import dir_err_deg, rot_err_deg
    Tr = np.array(g["T_w"]).reshape(-1, 4, 4)
    n = Tr.shape[0]
    T = recs["T_w2c"][:n].reshape(-1, 4, 4)
    tr = g["track"]
    a_w = np.array(tr["a_w"]).reshape(-1, 3)
    a_c = np.array(tr["a_c"]).reshape(-1, 3)
    uv = np.array(tr["uv"]).reshape(-1, 2)
    valid = np.array(tr["valid"], bool) & ((recs["valid"][:n] & 1) == 1)
    cond = valid & (np.abs(a_c[:, 2]) >= 0.5 * np.linalg.norm(a_c, axis=1))
    adir = dir_err_deg(recs["a_world"][:n][valid], a_w[valid])
    px = np.hypot(recs["u"][:n][cond] - uv[cond, 0], recs["v"][:n][cond] - uv[cond, 1])
    pct = lambda a, q: float(np.percentile(a, q)) if a.size else None
    return {"windows": k["windows"], "frames": n,
            "rot_deg_max": float(rot_err_deg(T[:, :3, :3], Tr[:, :3, :3]).max()),
            "tdir_deg_max": float(dir_err_deg(T[:, :3, 3], Tr[:, :3, 3]).max()),
            "accel_dir_deg_p50": pct(adir, 50), "accel_dir_deg_p99": pct(adir, 99),
            "focus_px_p50": pct(px, 50), "focus_px_p99": pct(px, 99), "focus_frames": int(cond.sum())}


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
    report = lambda d: print(f"[serve] {d['t']:.0f} s: {d['admitted']} admitted, {d['active']} active, "
                             f"{d['done']} done, {d['frames']} frames", file=sys.stderr, flush=True)
    out = serving.serve(eng, specs, pool, 16, 8, K, fps=30.0, paced=args.serve_paced, time_limit=args.serve_time_limit,
                        progress=report)
    st = eng.stats()
    eng.close()
    # paced: latency from each frame's capture time (admission wait included); unpaced: from its push
    lat = serving.latency_summary(out["records"], out["waits"] if args.serve_paced else None)
    frames = lat["frames"]
    res = {"metric": "serving frames/sec and per-frame latency (BF16, continuous batching) vs FP32 single-stream",
           "value": frames / out["wall"], "unit": "frames/s", "n_gpus": 1, "dtype": "bf16",
           "regime": "paced 30 fps, Poisson arrivals" if args.serve_paced else "throughput (all frames available)",
           "streams": len(specs), "frames": frames, "wall_s": out["wall"], "latency_ms": lat,
           "batches": st["batches_run"], "windows": st["windows_run"], "gpu_ms": st["gpu_ms"],
           "admission_refusals": int(sum(out["refused"])), "max_streams_open": out["max_active"],
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
    ap.add_argument("--no-graphs", action="store_true", help="skip the hipGraph replay leg")
    ap.add_argument("--workload", default="large", choices=["large", "small", "fp8"],
                    help="large (the headline line: the largest single-GPU configuration), small or fp8")
    ap.add_argument("--source-hash", action="store_true", help="print the attention source hash and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy (an elementwise torch kernel) so that HBM counters "
                         "of the same profiler run can be scaled by a transfer of known size")
    ap.add_argument("--serve", action="store_true", help="run the serving workload instead (separate JSON line)")
    ap.add_argument("--serve-streams", type=int, default=8)
    ap.add_argument("--serve-max-len", type=int, default=160)
    ap.add_argument("--serve-rate", type=float, default=0.4)
    ap.add_argument("--serve-paced", action="store_true")
    ap.add_argument("--serve-fp32-streams", type=int, default=2)
    ap.add_argument("--serve-time-limit", type=float, default=900.0)
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
    inp = Inputs(wl)
    progress(f"inputs ready: {wl.name}")
    r = run_gpu(inp, args.precision, args.steps, args.warmup)
    fps = r["frames"] / r["seconds"]
    progress(f"{args.precision} eager leg: {fps:.1f} frames/s")
    ms_step = r["seconds"] * 1e3 / args.steps
    nwin = len(window_sizes(wl.frames, wl.window, wl.overlap))
    res = {
        "metric": "frames/sec pose+focus (BF16/FP8 vs FP32 at stated pose error); p50/p99 latency",
        "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic (seeded uniform pixels, seeded N(0,0.02) random-init weights)",
        "config": {"workload": wl.name, "frames": wl.frames, "height": wl.height, "width": wl.width,
                   "window": wl.window, "overlap": wl.overlap, "layers": wl.model.depth, "dim": wl.model.dim,
                   "heads": wl.model.heads, "mlp": wl.model.mlp, "windows_per_step": nwin,
                   "parallelism": "single GPU"},
        # a step pushes a whole stream at once: this is the time from that push to its last result
        # (per-frame serving latency is the --serve line's)
        "stream_batch_latency_ms": float(r["batch_ms"]),
        # overlap frames of consecutive windows whose patch embedding is taken from the earlier window
        "patch_embedding_shared_frames_per_step": r["shared_per_step"],
        "path_tflops": path_flops(wl) * args.steps / r["seconds"] / 1e12,
    }
    if not args.no_graphs:
        rg = run_gpu(inp, args.precision, args.steps, args.warmup, profile=False, graphs=True)
        res["value_graphs_unprofiled"] = rg["frames"] / rg["seconds"]
        progress(f"{args.precision} graph leg: {res['value_graphs_unprofiled']:.1f} frames/s")
    prof, stages = r["prof"], r["stages"]
    calls = max(1, prof["attn_global_calls"])
    avg_ms = prof["attn_global_ms"] / calls
    flops = global_attention_flops(wl)
    ach = flops / (avg_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    res["roofline"] = {"kernel": "global flash attention (attn_kernel_v3, hd 64)", "bound": "mfma",
                       "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                       "traffic": measured_traffic(wl.name) if args.precision == "bf16" else None,
                       "algorithmic_bytes_per_launch": global_attention_bytes(wl),
                       "avg_launch_ms": avg_ms, "launches": prof["attn_global_calls"], "flops_per_launch": flops}
    res["stage_ms_per_step"] = {k: v[0] / args.steps for k, v in stages.items() if v[1]}
    sf = gemm_stage_flops(wl)
    per = {}
    for k in GEMM_STAGES:
        ms, n = stages[k]
        if n:
            t = sf[k] / (ms / n * 1e-3) / 1e12
            per[k] = {"tflops": t, "frac": t / peak, "avg_launch_ms": ms / n}
    gms = sum(stages[k][0] for k in GEMM_STAGES)
    if gms > 0:
        gt = gemm_flops(wl) / (gms / args.steps * 1e-3) / 1e12
        res["gemm"] = {"tflops": gt, "frac": gt / peak, "per_gemm": per,
                       "what": "QKV, out-projection, fc1 (GELU) and fc2 with their fused epilogues; algorithmic "
                               "flops over HIP-event launch times"}
    err = golden_errors(wl, inp, r["first"])
    if err is not None:
        res["error_vs_fp64_oracle"] = err
    if not args.no_fp8 and args.precision == "bf16":
        f8 = run_gpu(inp, "fp8", args.steps, args.warmup, profile=False, graphs=not args.no_graphs)
        res["fp8_value"] = f8["frames"] / f8["seconds"]
        if "value_graphs_unprofiled" in res:
            res["speedup_fp8_vs_bf16_graphs"] = res["fp8_value"] / res["value_graphs_unprofiled"]
        e8 = golden_errors(wl, inp, f8["first"])
        if e8 is not None:
            res["error_vs_fp64_oracle_fp8"] = e8
        # stage timing of the fp8 precision (a short eager run with events)
        p8 = run_gpu(inp, "fp8", 2, 1, profile=True, graphs=False)
        st8 = p8["stages"]
        res["fp8_stage_ms_per_step"] = {k: v[0] / 2 for k, v in st8.items() if v[1]}
        g8 = sum(st8[k][0] for k in GEMM_STAGES) / 2
        gb = sum(stages[k][0] for k in GEMM_STAGES) / args.steps
        if g8 > 0 and gb > 0:
            res["fp8_gemm_speedup_vs_bf16"] = gb / g8
        progress(f"fp8 legs: {res['fp8_value']:.1f} frames/s")
    if not args.no_fp32 and args.precision != "fp32":
        v32, dt32, st32 = run_fp32_single_stream(inp)
        res["fp32_single_stream"] = {"value": v32, "unit": "frames/s", "seconds": dt32,
                                     "batches": st32["batches_run"],
                                     "what": "plain FP32 path: fp32 operands on fp32 MFMA, one window per batch, "
                                             "one stream, no hipGraphs"}
        res["speedup_vs_fp32_single_stream"] = fps / v32
        progress(f"fp32 single-stream leg: {v32:.1f} frames/s")
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl, inp.blob)
        progress("cpu baseline done")
    print(json.dumps(res))


if __name__ == "__main__":
    main()
