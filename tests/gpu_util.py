"""Helpers of the GPU parity tests: device access, the library handle, error measures."""
import math
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def mf():
    """The library binding; fails loudly when the library is missing (no fallback)."""
    import paper_2601_07154_amd as m
    m._lib.lib()
    return m


def rot_err_deg(R1, R2):
    """Angle of R1^T R2 in degrees, 2 asin(|R1 - R2|_F / sqrt 8): well conditioned near 0."""
    d = np.linalg.norm(np.asarray(R1) - np.asarray(R2), axis=(-2, -1)) / math.sqrt(8.0)
    return np.degrees(2.0 * np.arcsin(np.minimum(1.0, d)))


def dir_err_deg(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    na, nb = np.linalg.norm(a, axis=-1), np.linalg.norm(b, axis=-1)
    c = np.sum(a * b, axis=-1) / np.maximum(na * nb, 1e-300)
    s = np.linalg.norm(np.cross(a, b), axis=-1) / np.maximum(na * nb, 1e-300)
    return np.degrees(np.arctan2(s, c))


def round_bf16(x):
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def golden(name):
    """A stored oracle output (tests/golden), its input checksums verified against the generators."""
    import sys
    here = os.path.join(ROOT, "tests", "golden")
    if here not in sys.path:
        sys.path.insert(0, here)
    import make_golden
    if not os.path.exists(make_golden.path(name)):
        pytest.fail(f"stored oracle output {name} is missing: python tests/golden/make_golden.py {name}")
    return make_golden.load(name)


def track_errors(T, a_w, uv, valid, ref):
    """Errors of a pose/focus track against a stored FP64 oracle output over its frames.

    rot, tdir: per frame, rotation angle of R^T R_ref and the angle between the translations (deg);
    adir: angle between the acceleration vectors where both have a focus (deg);
    px: focus-point distance (pixels) where both have a focus and the oracle's acceleration is
    within 60 deg of the optical axis (|a_z| >= 0.5 |a|; near a_z = 0 the projection diverges)."""
    n = ref["T_w"].shape[0]
    T = np.asarray(T)[:n].reshape(-1, 4, 4)
    tr = ref["track"]
    v = tr["valid"] & np.asarray(valid[:n], bool)
    cond = v & (np.abs(tr["a_c"][:, 2]) >= 0.5 * np.linalg.norm(tr["a_c"], axis=1))
    uv = np.asarray(uv)[:n]
    return dict(rot=rot_err_deg(T[:, :3, :3], ref["T_w"][:, :3, :3]),
                tdir=dir_err_deg(T[:, :3, 3], ref["T_w"][:, :3, 3]),
                adir=dir_err_deg(np.asarray(a_w)[:n][v], tr["a_w"][v]),
                px=np.hypot(uv[cond, 0] - tr["uv"][cond, 0], uv[cond, 1] - tr["uv"][cond, 1]))


def record_errors(recs, ref):
    """track_errors of the library's result records."""
    return track_errors(recs["T_w2c"], recs["a_world"], np.stack([recs["u"], recs["v"]], axis=1),
                        (recs["valid"] & 1) == 1, ref)


def golden_errors(emu, ref):
    """track_errors of one stored oracle output (an emulated precision) against another (FP64)."""
    return track_errors(emu["T_w"], emu["track"]["a_w"], emu["track"]["uv"], emu["track"]["valid"], ref)


def summary(e):
    q = lambda a, p: float(np.percentile(a, p)) if a.size else 0.0
    return (f"rot max {e['rot'].max():.3f} deg, tdir max {e['tdir'].max():.3f} deg, accel dir p50/p99 "
            f"{q(e['adir'], 50):.2f}/{q(e['adir'], 99):.2f} deg, focus px p50/p99 {q(e['px'], 50):.1f}/"
            f"{q(e['px'], 99):.1f} ({e['px'].size} frames)")


def run_stream_fused(wl, precision, blob, frames_dev, graphs=True):
    """One whole stream of a workload pushed from device memory with every window in one fused batch
    (the benchmark's launch configuration); returns the result records of all frames."""
    from oracle import motion
    m = mf()
    rows = m.rows_per_frame(wl.height, wl.width)
    nwin = len(motion.window_schedule(wl.frames, wl.window, wl.overlap))
    eng = m.Engine.from_model(wl.model, blob, precision=precision, max_tokens=nwin * wl.window * rows + 64,
                              graphs=graphs)
    sid = eng.open_stream(wl.height, wl.width, wl.window, wl.overlap, (wl.fx, wl.fy, wl.cx, wl.cy), sigma=1000.0,
                          ring_frames=wl.frames, result_frames=wl.frames)
    eng.push_frames(sid, frames_dev, eos=True)
    eng.sync()
    st = eng.stats()
    recs, _ = eng.poll(sid, wl.frames)
    eng.close()
    assert st["batches_run"] == 1 and st["windows_run"] == nwin
    assert list(recs["frame"]) == list(range(wl.frames))
    return recs


def check_emulation_gates(e, emu, factor=3.0, pose_floor=2.0, pose_add=0.0):
    """Precision gates calibrated by the oracle's emulation of the same precision on the same inputs:
    rotation and translation direction within max(pose_floor, factor x emulated + pose_add) degrees;
    acceleration-direction and focus-pixel errors at their median and 99th percentile within factor
    x the emulation's.  Returns the limits."""
    lim = {"pose": max(pose_floor, factor * max(emu["rot"].max(), emu["tdir"].max()) + pose_add)}
    assert e["rot"].max() <= lim["pose"] and e["tdir"].max() <= lim["pose"], (e["rot"].max(), e["tdir"].max(), lim)
    for key in ("adir", "px"):
        for q in (50, 99):
            lim[f"{key}_p{q}"] = factor * float(np.percentile(emu[key], q)) if emu[key].size else 0.0
            got = float(np.percentile(e[key], q)) if e[key].size else 0.0
            assert got <= lim[f"{key}_p{q}"], (key, q, got, lim)
    return lim
