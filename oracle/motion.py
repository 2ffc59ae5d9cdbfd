"""Sliding windows, incremental anchoring, motion focus and the focus map, FP64
(oracle; test infrastructure only).

Sources: the sliding-window / anchoring paragraph of Sec. 2.2 (window length L,
overlap O, anchor frame shared by consecutive windows, pitch and roll locked,
yaw and translation propagated, only new frames emitted) and Sec. 2.3, Eq. 1-7
(camera centre, discrete acceleration, rotation into the current camera,
pinhole projection, Gaussian focus map).

Readings of points the paper leaves open (each is a project decision):
  * tail window [N-L, N) when the regular windows stop short of the stream's
    end; one window of all frames when N <= L;
  * the anchor is the last frame the previous window emitted (it is shared by
    both windows);
  * gravity is the world y axis (OpenCV camera axes, first camera upright); the
    yaw of the alignment is atan2(A[0,2], A[2,2]) of its rotation;
  * the alignment translation keeps the anchor's camera centre continuous;
  * an option rescales each window's translations first, by the ratio of its
    shared frames' centre distances to the anchor in the world and in the window
    (the paper chains rigidly, keeping each window's scale);
  * the difference step is one frame (a stride s >= 1 is an option); frames before
    the first full difference (0 and 1 at stride 1) carry no focus; the first
    difference of Eq. 2 alone gives the velocity-based projection the paper
    contrasts its focus with (Sec. 2.3), as a second mode;
  * a focus is valid iff |a_w| > 1e-12 max(1, |p_t|) and |a_c,z| > 1e-6 |a_c|;
  * map points are the last N valid accelerations rotated by the current
    camera's rotation; spread clip(sigma*s_i, sigma_min, sigma_max) pixels with
    s_i = |a_w,i|; Z = max of the unnormalised map (peak 1), or as an option Z = its sum
    over the pixel grid (a probability map); 0 map if Z < 1e-30 in either mode.
"""
from __future__ import annotations

import math

import numpy as np

ANCHOR_YAW = 0        # lock pitch and roll, propagate yaw and translation (the paper's anchoring)
ANCHOR_SE3 = 1        # full rigid alignment (no lock), used to pin the chaining algebra
ANCHOR_YAW_SCALE = 2  # the paper's anchoring after rescaling the window's translations (see below)


# ----------------------------------------------------------------------------- schedule
def window_schedule(n_frames: int, window: int, overlap: int):
    """Windows of a stream of n_frames frames.

    Returns a list of dicts {start, size, emit_begin, emit_end}: window k covers frames
    [start, start+size) and emits frames [emit_begin, emit_end), consecutive windows
    sharing `overlap` frames.
    """
    if window < 1 or overlap < 0 or overlap >= window:
        raise ValueError("need window >= 1 and 0 <= overlap < window")
    if n_frames <= 0:
        return []
    if n_frames <= window:
        return [dict(start=0, size=n_frames, emit_begin=0, emit_end=n_frames)]
    stride = window - overlap
    starts = list(range(0, n_frames - window + 1, stride))
    if starts[-1] + window < n_frames:
        starts.append(n_frames - window)
    out, prev_end = [], 0
    for s in starts:
        e = s + window
        out.append(dict(start=s, size=window, emit_begin=prev_end, emit_end=e))
        prev_end = e
    return out


# ----------------------------------------------------------------------------- poses
def invert(T: np.ndarray) -> np.ndarray:
    """Inverse of a rigid 4x4 transform."""
    R, t = T[:3, :3], T[:3, 3]
    Ti = np.eye(4)
    Ti[:3, :3] = R.T
    Ti[:3, 3] = -R.T @ t
    return Ti


def camera_centre(T_w2c: np.ndarray) -> np.ndarray:
    """Eq. 1: p = (T^{w->c})^{-1}[1:3, 4], the camera position in world coordinates."""
    return invert(T_w2c)[:3, 3]


def rot_y(psi: float) -> np.ndarray:
    c, s = math.cos(psi), math.sin(psi)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def alignment(T_loc_anchor: np.ndarray, T_w_anchor: np.ndarray, mode: int = ANCHOR_YAW) -> np.ndarray:
    """Rigid world->window-local transform A with T_w = T_loc A at the anchor frame.

    SE3 mode: the exact A = T_loc(a)^{-1} T_w(a).  Yaw mode: the rotation of that A
    reduced to its yaw about the gravity (y) axis, and the translation chosen so the
    anchor's camera centre is the same in both windows.
    """
    A_full = invert(T_loc_anchor) @ T_w_anchor
    if mode == ANCHOR_SE3:
        return A_full
    s, c = A_full[0, 2], A_full[2, 2]
    psi = math.atan2(s, c) if s * s + c * c >= 1e-24 else 0.0
    R_A = rot_y(psi)
    c_loc = camera_centre(T_loc_anchor)
    c_w = camera_centre(T_w_anchor)
    A = np.eye(4)
    A[:3, :3] = R_A
    A[:3, 3] = c_loc - R_A @ c_w
    return A


def window_scale(win, Tl: np.ndarray, T_w: np.ndarray) -> float:
    """Scale of window `win`'s local frame relative to the world chain, from the frames it shares
    with the windows before it (start .. emit_begin - 1, already in T_w): the summed distances of
    their camera centres to the anchor's (the last shared frame) in the world, over the same sum
    in the window's frame.  1 when the shared centres do not move (nothing to measure)."""
    a = win["emit_begin"] - 1
    shared = range(win["start"], win["emit_begin"])
    cw_a, cl_a = camera_centre(T_w[a]), camera_centre(Tl[a - win["start"]])
    num = sum(np.linalg.norm(camera_centre(T_w[i]) - cw_a) for i in shared)
    den = sum(np.linalg.norm(camera_centre(Tl[i - win["start"]]) - cl_a) for i in shared)
    return num / den if den > 1e-12 else 1.0


def scale_translation(Tl: np.ndarray, rho: float) -> np.ndarray:
    """[R | rho t]: every camera centre of the frame scaled by rho about its origin."""
    out = np.array(Tl, dtype=np.float64, copy=True)
    out[..., :3, 3] *= rho
    return out


def chain_windows(schedule, local_poses, mode: int = ANCHOR_YAW, return_scales: bool = False):
    """Stitch per-window local poses into world poses of every emitted frame.

    schedule: output of window_schedule; local_poses[k]: [size_k, 4, 4] world(window-local)
    -> camera poses of window k.  Window 0 defines the world frame.  Returns [N, 4, 4].
    ANCHOR_YAW_SCALE first rescales window k's translations by window_scale (monocular windows
    carry independent scale; the paper's rigid chaining keeps each window's), then anchors as
    ANCHOR_YAW.
    return_scales: also return each window's scale factor (1 except in ANCHOR_YAW_SCALE), by which
    the window's depth maps are multiplied to live in the world's units.
    """
    n = schedule[-1]["emit_end"] if schedule else 0
    T_w = np.zeros((n, 4, 4))
    scales = []
    for k, win in enumerate(schedule):
        Tl = local_poses[k]
        rho = 1.0
        if k == 0:
            A = np.eye(4)
        else:
            a = win["emit_begin"] - 1
            if a < win["start"]:
                raise ValueError("consecutive windows share no frame (overlap 0)")
            if mode == ANCHOR_YAW_SCALE:
                rho = window_scale(win, Tl, T_w)
                Tl = scale_translation(Tl, rho)
            A = alignment(Tl[a - win["start"]], T_w[a], ANCHOR_YAW if mode == ANCHOR_YAW_SCALE else mode)
        scales.append(rho)
        for t in range(win["emit_begin"], win["emit_end"]):
            T_w[t] = Tl[t - win["start"]] @ A
    return (T_w, scales) if return_scales else T_w


# ----------------------------------------------------------------------------- focus
def project(a_c: np.ndarray, fx: float, fy: float, cx: float, cy: float):
    """Eq. 6: pinhole projection of a camera-frame direction (a_x, a_y, a_z)."""
    return cx + fx * a_c[0] / a_c[2], cy + fy * a_c[1] / a_c[2]


FOCUS_ACCEL = 0      # Eq. 3: second difference of the camera centres (the paper's focus)
FOCUS_VELOCITY = 1   # Eq. 2: first difference, the velocity-based projection the paper contrasts


def focus_track(T_w: np.ndarray, fx: float, fy: float, cx: float, cy: float, mode: int = FOCUS_ACCEL,
                stride: int = 1):
    """Per-frame motion focus from world poses [N,4,4] (Eq. 1-6).

    The motion vector m_t is the acceleration a_w of Eq. 2-3 (mode FOCUS_ACCEL) or the velocity
    v_t of Eq. 2 (mode FOCUS_VELOCITY), with the differences taken over `stride` frames:
    a = p_t - 2 p_{t-s} + p_{t-2s}, v = p_t - p_{t-s} (stride 1 is the paper's).  It is rotated
    into the camera (Eq. 4) and projected (Eq. 5-6) in either mode.

    Returns a dict of arrays: p [N,3] camera centres, a_w [N,3] the world motion vector,
    a_c [N,3] the camera-frame motion vector, uv [N,2], s [N] = |a_w|, valid [N] bool.
    Frames before the first full difference (t < 2 stride, or t < stride for velocity) have no
    motion vector (valid = False, zeros).
    """
    if mode not in (FOCUS_ACCEL, FOCUS_VELOCITY) or stride < 1:
        raise ValueError("mode must be FOCUS_ACCEL or FOCUS_VELOCITY and stride >= 1")
    N = T_w.shape[0]
    p = np.stack([camera_centre(T) for T in T_w]) if N else np.zeros((0, 3))
    a_w = np.zeros((N, 3))
    a_c = np.zeros((N, 3))
    uv = np.zeros((N, 2))
    s = np.zeros(N)
    valid = np.zeros(N, dtype=bool)
    first = stride if mode == FOCUS_VELOCITY else 2 * stride
    for t in range(first, N):
        v_t = p[t] - p[t - stride]                       # Eq. 2
        if mode == FOCUS_VELOCITY:
            a_w[t] = v_t
        else:
            v_tm1 = p[t - stride] - p[t - 2 * stride]
            a_w[t] = v_t - v_tm1                         # Eq. 3
        a_c[t] = T_w[t, :3, :3] @ a_w[t]                 # Eq. 4
        s[t] = np.linalg.norm(a_w[t])
        na_c = np.linalg.norm(a_c[t])
        ok = s[t] > 1e-12 * max(1.0, np.linalg.norm(p[t])) and abs(a_c[t, 2]) > 1e-6 * na_c
        valid[t] = ok
        if ok:
            uv[t] = project(a_c[t], fx, fy, cx, cy)
    return dict(p=p, a_w=a_w, a_c=a_c, uv=uv, s=s, valid=valid)


def map_points(t: int, T_w: np.ndarray, track: dict, n_points: int, fx, fy, cx, cy,
               sigma: float, sigma_min: float, sigma_max: float):
    """The motion points of frame t's map: the last n_points valid accelerations, each
    rotated into frame t and projected (Fig. 4), with spread clip(sigma * s_i)."""
    R_t = T_w[t, :3, :3]
    pts = []
    for i in range(max(0, t - n_points + 1), t + 1):
        if not track["valid"][i]:
            continue
        a = R_t @ track["a_w"][i]
        if not abs(a[2]) > 1e-6 * np.linalg.norm(a):
            continue
        u, v = project(a, fx, fy, cx, cy)
        pts.append((u, v, spread(track["s"][i], sigma, sigma_min, sigma_max)))
    return pts


MAP_MAX = 0   # Z = the largest value of the unnormalised map: the peak of M is 1
MAP_SUM = 1   # Z = the sum of the unnormalised map over the pixel grid: M sums to 1


def spread(s: float, sigma: float, sigma_min: float, sigma_max: float) -> float:
    """Eq. 7's spread of a motion point in pixels: sigma times its magnitude s, clipped."""
    return min(max(sigma * s, sigma_min), sigma_max)


def focus_map(points, height: int, width: int, z_mode: int = MAP_MAX):
    """Eq. 7: M(x, y) = (1/Z) sum_i exp(-((x-u_i)^2 + (y-v_i)^2) / (2 sigma_i^2)) on the
    integer pixel grid; Z = the map's maximum (MAP_MAX) or its sum over the grid (MAP_SUM).
    Returns (M [H,W], Z, argmax index); the argmax does not depend on the mode."""
    if z_mode not in (MAP_MAX, MAP_SUM):
        raise ValueError("z_mode must be MAP_MAX or MAP_SUM")
    ys = np.arange(height, dtype=np.float64)[:, None]
    xs = np.arange(width, dtype=np.float64)[None, :]
    G = np.zeros((height, width))
    for (u, v, sig) in points:
        G += np.exp(-((xs - u) ** 2 + (ys - v) ** 2) / (2.0 * sig * sig))
    if not G.size:
        Z = 0.0
    else:
        Z = float(G.max()) if z_mode == MAP_MAX else float(G.sum())
    if Z < 1e-30:
        return np.zeros_like(G), Z, 0
    M = G / Z
    return M, Z, int(np.argmax(M))
