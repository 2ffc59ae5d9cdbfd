"""The whole stream through the oracle: windows -> pose forward -> anchoring -> focus -> maps
(test infrastructure only).  See oracle.vit and oracle.motion for the steps."""
from __future__ import annotations

import numpy as np

from . import motion, vit


def run_stream(frames: np.ndarray, weights: dict, heads: int, window: int, overlap: int,
               K, n_points: int = 15, sigma: float = 1.0, sigma_min: float = 0.5,
               sigma_max: float | None = None, anchor_mode: int = motion.ANCHOR_YAW,
               precision: str = "fp64", windows=None, maps: bool = True, patch: int = 14,
               focus_mode: int = motion.FOCUS_ACCEL, stride: int = 1, workers: int = 1,
               map_mode: int = motion.MAP_MAX, depth: bool = False):
    """Run the oracle on one stream of frames [N,3,H,W].

    windows: optionally restrict to the first `windows` windows (large configs).
    workers: threads over the attention heads of the forward (same values for any count).
    depth: the weights carry a depth head; also return the emitted frames' depth maps [N, H, W]
    (each from the window that emits the frame, times that window's scale: 1 under rigid
    anchoring, the anchoring's scale factor in ANCHOR_YAW_SCALE; depth is camera-relative, so a
    rigid change of world frame leaves it unchanged).
    Returns dict(schedule, pose9 [per window], T_loc [per window], T_w, track, sigma_px, maps, Z,
    argmax[, depth]); sigma_px is each frame's own Eq. 7 spread (0 where it has no focus point).
    """
    fx, fy, cx, cy = K
    N, _, H, W = frames.shape
    if sigma_max is None:
        sigma_max = 4.0 * max(H, W)
    sched = motion.window_schedule(N, window, overlap)
    if windows is not None:
        sched = sched[:windows]
    p9s, Tls, dls = [], [], []
    for win in sched:
        r = vit.forward_window(frames[win["start"]:win["start"] + win["size"]], weights, heads,
                               patch, precision, workers=workers, depth=depth)
        p9 = r[0] if depth else r
        if depth:
            dls.append(r[1])
        p9s.append(p9)
        Tls.append(np.stack([vit.pose9_to_T(q) for q in p9]))
    T_w, scales = motion.chain_windows(sched, Tls, anchor_mode, return_scales=True)
    track = motion.focus_track(T_w, fx, fy, cx, cy, focus_mode, stride)
    out = dict(schedule=sched, pose9=p9s, T_loc=Tls, T_w=T_w, track=track,
               sigma_px=_sigma_px(track, sigma, sigma_min, sigma_max))
    if depth:
        dep = np.zeros((T_w.shape[0], H, W))
        for win, d, rho in zip(sched, dls, scales):
            for t in range(win["emit_begin"], win["emit_end"]):
                dep[t] = rho * d[t - win["start"]]
        out.update(depth=dep, window_scale=np.array(scales))
    if maps:
        Ms, Zs, am = [], [], []
        for t in range(T_w.shape[0]):
            pts = motion.map_points(t, T_w, track, n_points, fx, fy, cx, cy, sigma, sigma_min,
                                    sigma_max)
            M, Z, a = motion.focus_map(pts, H, W, map_mode)
            Ms.append(M.astype(np.float32))
            Zs.append(Z)
            am.append(a)
        out.update(maps=np.stack(Ms) if Ms else np.zeros((0, H, W), np.float32),
                   Z=np.array(Zs), argmax=np.array(am))
    return out


def _sigma_px(track: dict, sigma: float, sigma_min: float, sigma_max: float) -> np.ndarray:
    """Each frame's own spread in pixels (Eq. 7), 0 for frames without a focus point."""
    return np.array([motion.spread(s, sigma, sigma_min, sigma_max) if ok else 0.0
                     for s, ok in zip(track["s"], track["valid"])])


def run_poses(T_w2c: np.ndarray, K, height: int, width: int, n_points: int = 15,
              sigma: float = 1.0, sigma_min: float = 0.5, sigma_max: float | None = None,
              maps: bool = True, focus_mode: int = motion.FOCUS_ACCEL, stride: int = 1,
              map_mode: int = motion.MAP_MAX):
    """Focus and maps for world poses given directly (the 'any pose estimator' entry)."""
    fx, fy, cx, cy = K
    if sigma_max is None:
        sigma_max = 4.0 * max(height, width)
    track = motion.focus_track(T_w2c, fx, fy, cx, cy, focus_mode, stride)
    out = dict(T_w=T_w2c, track=track, sigma_px=_sigma_px(track, sigma, sigma_min, sigma_max))
    if maps:
        Ms, Zs, am = [], [], []
        for t in range(T_w2c.shape[0]):
            pts = motion.map_points(t, T_w2c, track, n_points, fx, fy, cx, cy, sigma, sigma_min,
                                    sigma_max)
            M, Z, a = motion.focus_map(pts, height, width, map_mode)
            Ms.append(M.astype(np.float32))
            Zs.append(Z)
            am.append(a)
        out.update(maps=np.stack(Ms) if Ms else np.zeros((0, height, width), np.float32),
                   Z=np.array(Zs), argmax=np.array(am))
    return out
