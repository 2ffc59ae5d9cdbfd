"""Write the stored FP64 (and emulated-precision) oracle outputs that the full-size GPU parity tests
compare against.  Calls only the oracle and the seeded input generators; run on a CPU:

    python tests/golden/make_golden.py <fixture> [--workers N]
    python tests/golden/make_golden.py --list

Each fixture is one JSON file next to this script holding, for the first windows of one workload
stream (Sec. 2.2's sliding windows, anchoring and emission; Sec. 2.3's Eq. 1-7 focus and map):
the window schedule, every window's pose9, the chained world poses of the emitted frames, the focus
track (camera centres, world and camera motion vectors, (u, v), |a_w|, validity) and the map
normaliser Z and argmax of each emitted frame.  It is keyed by the workload's parameters and the
SHA-256 of the fp32 weight blob and of the fp32 frames it read, which the tests recompute before
they trust the file.  Floats are written with Python's repr (exact round trip).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import mf_synth  # noqa: E402

SIGMA = 1000.0      # focus-map spread per unit of |a_w| used by every full-size test
N_POINTS = 15

# name -> (workload, number of windows, oracle precision)
FIXTURES = {
    "small_fp64_w01": (mf_synth.SMALL, 2, "fp64"),
    "small_bf16emu_w01": (mf_synth.SMALL, 2, "bf16"),
    "large_fp64_w01": (mf_synth.LARGE, 2, "fp64"),
    "large_bf16emu_w01": (mf_synth.LARGE, 2, "bf16"),
    "fp8_fp64_w0": (mf_synth.FP8, 1, "fp64"),
    "fp8_fp8emu_w0": (mf_synth.FP8, 1, "fp8"),
    "fp8_bf16emu_w0": (mf_synth.FP8, 1, "bf16"),
}


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def frames_needed(wl, nwin: int) -> int:
    """Frames the first nwin windows read (their last window's end)."""
    from oracle import motion
    sched = motion.window_schedule(wl.frames, wl.window, wl.overlap)[:nwin]
    return max(w["start"] + w["size"] for w in sched)


def key(wl, nwin: int, precision: str) -> dict:
    """What a fixture depends on besides the oracle's code: the workload, the windows, the precision
    and the checksums of the inputs (recomputed by the tests)."""
    n = frames_needed(wl, nwin)
    blob = mf_synth.make_weights(wl.model, wl.seed_weights)
    frames = mf_synth.workload_frames(wl, n)
    return {"workload": wl.name, "model": [wl.model.depth, wl.model.dim, wl.model.heads, wl.model.mlp],
            "frames_total": wl.frames, "frames_read": n, "height": wl.height, "width": wl.width,
            "window": wl.window, "overlap": wl.overlap, "K": [wl.fx, wl.fy, wl.cx, wl.cy],
            "seed_weights": wl.seed_weights, "seed_pixels": wl.seed_pixels, "windows": nwin,
            "precision": precision, "sigma": SIGMA, "n_points": N_POINTS,
            "weights_sha256": sha256(blob), "frames_sha256": sha256(frames)}


def make(name: str, workers: int) -> dict:
    from oracle import pipeline, vit
    wl, nwin, precision = FIXTURES[name]
    k = key(wl, nwin, precision)
    blob = mf_synth.make_weights(wl.model, wl.seed_weights)
    w = vit.unpack_weights(blob, wl.model.depth, wl.model.dim, wl.model.mlp)
    frames = mf_synth.workload_frames(wl, k["frames_read"])
    del blob
    t0 = time.time()
    out = pipeline.run_stream(frames, w, wl.model.heads, wl.window, wl.overlap, tuple(k["K"]),
                              n_points=N_POINTS, sigma=SIGMA, precision=precision, windows=nwin,
                              workers=workers)
    dt = time.time() - t0
    tr = out["track"]
    rec = {"key": k, "oracle_seconds": dt, "workers": workers,
           "schedule": out["schedule"],
           "pose9": [p.tolist() for p in out["pose9"]],
           "T_w": out["T_w"].reshape(-1, 16).tolist(),
           "track": {"p": tr["p"].tolist(), "a_w": tr["a_w"].tolist(), "a_c": tr["a_c"].tolist(),
                     "uv": tr["uv"].tolist(), "s": tr["s"].tolist(),
                     "valid": tr["valid"].astype(int).tolist()},
           "Z": out["Z"].tolist(), "argmax": out["argmax"].tolist()}
    return rec


def path(name: str) -> str:
    return os.path.join(HERE, name + ".json")


def load(name: str, check_inputs: bool = True) -> dict:
    """Read a fixture as numpy arrays; with check_inputs, recompute its key from the generators and
    refuse a file written for other inputs."""
    with open(path(name)) as f:
        rec = json.load(f)
    if check_inputs:
        wl, nwin, precision = FIXTURES[name]
        k = key(wl, nwin, precision)
        if k != rec["key"]:
            diff = {kk: (rec["key"].get(kk), v) for kk, v in k.items() if rec["key"].get(kk) != v}
            raise ValueError(f"golden {name} was written for other inputs: {diff}")
    tr = rec["track"]
    return {"key": rec["key"], "schedule": rec["schedule"],
            "pose9": [np.array(p) for p in rec["pose9"]],
            "T_w": np.array(rec["T_w"]).reshape(-1, 4, 4),
            "track": {"p": np.array(tr["p"]).reshape(-1, 3), "a_w": np.array(tr["a_w"]).reshape(-1, 3),
                      "a_c": np.array(tr["a_c"]).reshape(-1, 3), "uv": np.array(tr["uv"]).reshape(-1, 2),
                      "s": np.array(tr["s"]), "valid": np.array(tr["valid"], dtype=bool)},
            "Z": np.array(rec["Z"]), "argmax": np.array(rec["argmax"], dtype=np.int64)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fixtures", nargs="*")
    ap.add_argument("--workers", type=int, default=1, help="threads over attention heads")
    ap.add_argument("--list", action="store_true")
    args = ap.parse_args()
    if args.list or not args.fixtures:
        for n, (wl, nwin, p) in FIXTURES.items():
            print(f"{n}: {wl.name}, windows 0..{nwin - 1}, {p}, exists={os.path.exists(path(n))}")
        return
    for name in args.fixtures:
        if name not in FIXTURES:
            raise SystemExit(f"unknown fixture {name}")
        print(f"[golden] {name}: start", flush=True)
        rec = make(name, args.workers)
        tmp = path(name) + ".tmp"
        with open(tmp, "w") as f:
            json.dump(rec, f)
        os.replace(tmp, path(name))
        print(f"[golden] {name}: {rec['oracle_seconds']:.0f} s -> {path(name)}", flush=True)


if __name__ == "__main__":
    main()
