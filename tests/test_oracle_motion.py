"""Pins of the oracle's windowing, anchoring, focus and map stages (closed forms,
brute-force enumeration, invariants)."""
import math

import numpy as np
import pytest
from scipy.stats import norm

import mf_synth
from oracle import motion

K = (400.0, 380.0, 252.0, 140.0)


# ----------------------------------------------------------------------------- schedule
@pytest.mark.parametrize("L,O", [(8, 0), (16, 8), (32, 16), (48, 24), (5, 4), (7, 1), (1, 0)])
def test_schedule_enumeration(L, O):
    for N in list(range(1, 130)) + [255, 256, 257, 1000, 1999, 2000]:
        sched = motion.window_schedule(N, L, O)
        emitted = [t for w in sched for t in range(w["emit_begin"], w["emit_end"])]
        assert emitted == list(range(N))                                   # once each, in order
        for k, w in enumerate(sched):
            assert w["size"] == min(L, N)
            assert 0 <= w["start"] and w["start"] + w["size"] <= N
            assert w["start"] <= w["emit_begin"] < w["emit_end"] == w["start"] + w["size"]
            if k:
                prev = sched[k - 1]
                a = w["emit_begin"] - 1                                     # anchor frame
                assert prev["start"] <= a < prev["start"] + prev["size"]
                if O == 0:
                    continue                                                # no shared frame
                assert w["start"] <= a
                shared = prev["start"] + prev["size"] - w["start"]
                assert shared >= O                                          # tail may share more
                if w["start"] - prev["start"] == L - O:
                    assert shared == O
        # the regular starts are multiples of the stride
        reg = [w["start"] for w in sched if w["start"] % (L - O) == 0]
        assert reg[:len(reg)] == [k * (L - O) for k in range(len(reg))]


def test_schedule_examples():
    s = motion.window_schedule(64, 16, 8)
    assert [w["start"] for w in s] == [0, 8, 16, 24, 32, 40, 48]
    s = motion.window_schedule(256, 32, 16)
    assert [w["start"] for w in s] == list(range(0, 225, 16))
    s = motion.window_schedule(128, 48, 24)
    assert [w["start"] for w in s] == [0, 24, 48, 72, 80]                  # tail window
    assert (s[-1]["emit_begin"], s[-1]["emit_end"]) == (120, 128)
    with pytest.raises(ValueError):
        motion.window_schedule(10, 4, 4)


# ----------------------------------------------------------------------------- chaining
def _trajectory(n, rng):
    return np.stack([mf_synth.random_rigid(rng, 0.8, 3.0) for _ in range(n)])


@pytest.mark.parametrize("N,L,O", [(64, 16, 8), (50, 12, 3), (33, 8, 1)])
def test_se3_chaining_recovers_trajectory(N, L, O):
    rng = np.random.default_rng(7)
    T_w = _trajectory(N, rng)
    sched = motion.window_schedule(N, L, O)
    G = [mf_synth.random_rigid(rng, 3.0, 10.0) for _ in sched]     # arbitrary window-local frames
    local = [np.stack([T_w[t] @ np.linalg.inv(G[k]) for t in range(w["start"], w["start"] + w["size"])])
             for k, w in enumerate(sched)]
    got = motion.chain_windows(sched, local, motion.ANCHOR_SE3)
    want = np.stack([T_w[t] @ np.linalg.inv(G[0]) for t in range(N)])   # world = window 0's frame
    np.testing.assert_allclose(got, want, atol=1e-11)


def test_yaw_lock_exact_for_yaw_only_frames():
    """Window frames that differ from the world by a yaw about gravity and a shift: exact."""
    rng = np.random.default_rng(8)
    N, L, O = 64, 16, 8
    T_w = _trajectory(N, rng)
    sched = motion.window_schedule(N, L, O)
    G = []
    for k in range(len(sched)):
        g = np.eye(4)
        g[:3, :3] = mf_synth.rot_y(rng.uniform(-3, 3))
        g[:3, 3] = rng.uniform(-5, 5, size=3)
        G.append(g if k else np.eye(4))
    local = [np.stack([T_w[t] @ np.linalg.inv(G[k]) for t in range(w["start"], w["start"] + w["size"])])
             for k, w in enumerate(sched)]
    got = motion.chain_windows(sched, local, motion.ANCHOR_YAW)
    np.testing.assert_allclose(got, T_w, atol=1e-11)


def test_scale_aware_chaining_undoes_per_window_scale():
    """Windows whose frames are a yaw plus shift of the world with their own scale (translations,
    hence centres, times lambda_k; window 0 at the world's): the scale-aware chaining recovers the
    trajectory exactly; the rigid one does not; with all lambda = 1 both agree."""
    rng = np.random.default_rng(9)
    N, L, O = 64, 16, 8
    T_w = _trajectory(N, rng)
    sched = motion.window_schedule(N, L, O)

    def locals_(lams):
        out = []
        for k, w in enumerate(sched):
            g = np.eye(4)
            if k:
                g[:3, :3] = mf_synth.rot_y(rng.uniform(-3, 3))
                g[:3, 3] = rng.uniform(-5, 5, size=3)
            Tl = np.stack([T_w[t] @ np.linalg.inv(g) for t in range(w["start"], w["start"] + w["size"])])
            Tl[:, :3, 3] *= lams[k]
            out.append(Tl)
        return out

    lams = [1.0] + list(rng.uniform(0.5, 2.0, len(sched) - 1))
    loc = locals_(lams)
    got = motion.chain_windows(sched, loc, motion.ANCHOR_YAW_SCALE)
    np.testing.assert_allclose(got, T_w, atol=1e-10)
    rigid = motion.chain_windows(sched, loc, motion.ANCHOR_YAW)
    assert np.abs(rigid - T_w).max() > 1e-2
    loc1 = locals_([1.0] * len(sched))
    np.testing.assert_allclose(motion.chain_windows(sched, loc1, motion.ANCHOR_YAW_SCALE),
                               motion.chain_windows(sched, loc1, motion.ANCHOR_YAW), atol=1e-11)


def test_window_scale_is_one_without_motion():
    T = np.tile(np.eye(4), (6, 1, 1))
    win = dict(start=0, size=6, emit_begin=3, emit_end=6)
    assert motion.window_scale(win, T, T) == 1.0


def test_yaw_lock_drops_pitch_and_keeps_anchor_centre():
    """A local frame with yaw psi then pitch theta (Y-X order): the alignment keeps exactly R_y(psi),
    and the anchor camera's centre is continuous across the boundary."""
    rng = np.random.default_rng(9)
    Tl_a = mf_synth.random_rigid(rng, 1.0, 2.0)
    psi, theta = 0.4, 0.15
    A_true = np.eye(4)
    A_true[:3, :3] = mf_synth.rot_y(psi) @ mf_synth.rot_x(theta)
    A_true[:3, 3] = [0.3, -0.2, 1.0]
    T_w_a = Tl_a @ A_true
    A = motion.alignment(Tl_a, T_w_a, motion.ANCHOR_YAW)
    np.testing.assert_allclose(A[:3, :3], mf_synth.rot_y(psi), atol=1e-14)
    np.testing.assert_allclose(motion.camera_centre(Tl_a @ A), motion.camera_centre(T_w_a), atol=1e-13)
    # the locked pitch shows up as a rotation error of exactly theta on the anchor frame
    Rerr = (Tl_a @ A)[:3, :3] @ T_w_a[:3, :3].T
    assert abs(math.acos((np.trace(Rerr) - 1) / 2) - theta) < 1e-9
    # full SE3 mode reproduces the anchor exactly
    np.testing.assert_allclose(Tl_a @ motion.alignment(Tl_a, T_w_a, motion.ANCHOR_SE3), T_w_a, atol=1e-13)


def test_camera_centre_is_inverse_translation():
    T = mf_synth.pose_from_center([1.0, -2.0, 3.0], mf_synth.rot_y(0.3) @ mf_synth.rot_x(-0.2))
    np.testing.assert_allclose(motion.camera_centre(T), [1.0, -2.0, 3.0], atol=1e-15)
    np.testing.assert_allclose(motion.invert(T) @ T, np.eye(4), atol=1e-15)


# ----------------------------------------------------------------------------- focus
def test_constant_acceleration_closed_form():
    fps, acc = 30.0, (0.1, -0.05, 0.5)
    path = mf_synth.CameraPath(fps=fps, velocity=(0.2, 0.0, 1.5), accel=acc, sway_deg=0.0)
    tr = motion.focus_track(path.poses(20), *K)
    dt2 = 1.0 / fps ** 2
    np.testing.assert_allclose(tr["a_w"][2:], np.tile(np.array(acc) * dt2, (18, 1)), rtol=1e-9, atol=1e-15)
    fx, fy, cx, cy = K
    np.testing.assert_allclose(tr["uv"][2:, 0], cx + fx * 0.1 / 0.5, rtol=1e-9)
    np.testing.assert_allclose(tr["uv"][2:, 1], cy + fy * -0.05 / 0.5, rtol=1e-9)
    assert not tr["valid"][:2].any() and tr["valid"][2:].all()
    np.testing.assert_allclose(tr["s"][2:], np.linalg.norm(acc) * dt2, rtol=1e-9)


def test_optical_axis_acceleration_hits_principal_point():
    path = mf_synth.CameraPath(velocity=(0, 0, 1.5), accel=(0, 0, 0.5), sway_deg=0.0)
    tr = motion.focus_track(path.poses(10), *K)
    np.testing.assert_allclose(tr["uv"][2:], np.tile([K[2], K[3]], (8, 1)), atol=1e-9)


@pytest.mark.parametrize("psi_deg", [-30.0, -5.0, 10.0, 25.0])
def test_forward_acceleration_with_head_yaw(psi_deg):
    """Torso accelerates along world z while the head is turned by psi: u = cx - fx tan(psi), v = cy."""
    path = mf_synth.CameraPath(velocity=(0, 0, 1.0), accel=(0, 0, 0.8), sway_deg=0.0, yaw0_deg=psi_deg)
    tr = motion.focus_track(path.poses(8), *K)
    psi = math.radians(psi_deg)
    np.testing.assert_allclose(tr["uv"][2:, 0], K[2] - K[0] * math.tan(psi), rtol=1e-9)
    np.testing.assert_allclose(tr["uv"][2:, 1], K[3], atol=1e-9)


@pytest.mark.parametrize("lam", [3.0, -1.0, -0.25, 1e-3])
def test_focus_invariant_to_acceleration_scale_and_sign(lam):
    base = mf_synth.CameraPath(velocity=(0.1, 0.2, 1.0), accel=(0.3, 0.1, 0.6), sway_deg=4.0)
    scaled = mf_synth.CameraPath(velocity=(0.1, 0.2, 1.0), accel=tuple(lam * a for a in (0.3, 0.1, 0.6)),
                                 sway_deg=4.0)
    # remove the velocity contribution difference: second differences of the velocity part vanish
    t1, t2 = motion.focus_track(base.poses(12), *K), motion.focus_track(scaled.poses(12), *K)
    np.testing.assert_allclose(t2["uv"][2:], t1["uv"][2:], rtol=1e-6)


def test_constant_velocity_is_invalid():
    path = mf_synth.CameraPath(velocity=(0.3, 0, 1.5), accel=(0, 0, 0), sway_deg=5.0)
    tr = motion.focus_track(path.poses(30), *K)
    assert not tr["valid"].any()


def test_sway_path_of_the_workload_has_zero_acceleration():
    """The 1.5 m/s + 2 Hz sway path moves its centre linearly: Eq. 3 gives zero, the focus is invalid."""
    tr = motion.focus_track(mf_synth.CameraPath().poses(64), *K)
    assert np.abs(tr["a_w"]).max() < 1e-13 and not tr["valid"].any()


@pytest.mark.parametrize("stride", [1, 2, 5])
def test_strided_acceleration_closed_form(stride):
    """A quadratic path's second difference over s frames is exactly a (s dt)^2: the focus is the
    stride-1 focus, and the first 2 s frames have none."""
    fps, acc = 30.0, (0.1, -0.05, 0.5)
    path = mf_synth.CameraPath(fps=fps, velocity=(0.2, 0.0, 1.5), accel=acc, sway_deg=0.0)
    tr = motion.focus_track(path.poses(24), *K, mode=motion.FOCUS_ACCEL, stride=stride)
    f = 2 * stride
    np.testing.assert_allclose(tr["a_w"][f:], np.tile(np.array(acc) * (stride / fps) ** 2, (24 - f, 1)),
                               rtol=1e-9, atol=1e-15)
    fx, fy, cx, cy = K
    np.testing.assert_allclose(tr["uv"][f:, 0], cx + fx * 0.1 / 0.5, rtol=1e-9)
    assert not tr["valid"][:f].any() and tr["valid"][f:].all() and not tr["a_w"][:f].any()


@pytest.mark.parametrize("stride", [1, 3])
def test_velocity_mode_is_the_focus_of_expansion(stride):
    """Velocity mode on a straight constant-velocity path: m = v s dt exactly, and the point is
    the focus of expansion, the projection of the direction of travel: the principal point for
    motion along the optical axis; cx - fx tan(psi) with the head turned by psi."""
    fx, fy, cx, cy = K
    fwd = mf_synth.CameraPath(velocity=(0, 0, 1.5), accel=(0, 0, 0), sway_deg=0.0)
    tr = motion.focus_track(fwd.poses(12), *K, mode=motion.FOCUS_VELOCITY, stride=stride)
    np.testing.assert_allclose(tr["a_w"][stride:], np.tile([0, 0, 1.5 * stride / 30.0], (12 - stride, 1)),
                               atol=1e-12)
    np.testing.assert_allclose(tr["uv"][stride:], np.tile([cx, cy], (12 - stride, 1)), atol=1e-9)
    assert not tr["valid"][:stride].any() and tr["valid"][stride:].all()
    psi = 17.0
    turned = mf_synth.CameraPath(velocity=(0, 0, 1.0), accel=(0, 0, 0), sway_deg=0.0, yaw0_deg=psi)
    tr = motion.focus_track(turned.poses(10), *K, mode=motion.FOCUS_VELOCITY, stride=stride)
    np.testing.assert_allclose(tr["uv"][stride:, 0], cx - fx * math.tan(math.radians(psi)), rtol=1e-9)


def test_velocity_and_acceleration_differ_when_turning():
    """Braking while moving forward and sideways: velocity mode points along the travel direction,
    acceleration mode along the (opposite, braking) acceleration, on the other side of the image."""
    fx, fy, cx, cy = K
    path = mf_synth.CameraPath(velocity=(0.5, 0, 1.5), accel=(-0.6, 0, 0.4), sway_deg=0.0)
    T = path.poses(6)
    vel = motion.focus_track(T, *K, mode=motion.FOCUS_VELOCITY)
    acc = motion.focus_track(T, *K, mode=motion.FOCUS_ACCEL)
    t = 5
    p = [motion.camera_centre(T[i]) for i in range(6)]
    np.testing.assert_allclose(vel["a_w"][t], p[t] - p[t - 1], atol=1e-15)
    np.testing.assert_allclose(acc["a_w"][t], p[t] - 2 * p[t - 1] + p[t - 2], atol=1e-15)
    assert vel["uv"][t, 0] > cx > acc["uv"][t, 0]


def test_focus_track_rejects_bad_mode_and_stride():
    T = mf_synth.CameraPath().poses(4)
    with pytest.raises(ValueError):
        motion.focus_track(T, *K, mode=2)
    with pytest.raises(ValueError):
        motion.focus_track(T, *K, stride=0)


# ----------------------------------------------------------------------------- map
def test_single_point_map():
    H, W, u, v, sig = 40, 60, 23.0, 17.0, 4.0
    M, Z, am = motion.focus_map([(u, v, sig)], H, W)
    assert M[17, 23] == 1.0 and am == 17 * W + 23 and Z == 1.0
    for dx, dy in [(3, 0), (0, -5), (2, 2), (-7, 4)]:
        ref = norm.pdf(math.hypot(dx, dy), scale=sig) / norm.pdf(0, scale=sig)
        assert abs(M[17 + dy, 23 + dx] - ref) < 1e-14
    np.testing.assert_allclose(M[17, 23 - 6:23], M[17, 23 + 6:23:-1], atol=1e-15)   # symmetric
    np.testing.assert_allclose(M[17 - 6:17, 23], M[17 + 6:17:-1, 23], atol=1e-15)


def test_map_is_linear_before_normalisation_and_ties_go_low():
    H, W = 30, 30
    p1, p2 = (8.0, 10.0, 3.0), (20.0, 10.0, 3.0)
    M1, Z1, _ = motion.focus_map([p1], H, W)
    M2, Z2, _ = motion.focus_map([p2], H, W)
    M12, Z12, am = motion.focus_map([p1, p2], H, W)
    np.testing.assert_allclose(M12 * Z12, M1 * Z1 + M2 * Z2, atol=1e-14)
    assert am == 10 * W + 8                                     # symmetric peaks: smallest index
    M0, Z0, a0 = motion.focus_map([], H, W)
    assert Z0 == 0 and not M0.any() and a0 == 0
    far, Zf, _ = motion.focus_map([(1e6, 1e6, 1.0)], H, W)     # Z underflows: zero map
    assert Zf < 1e-30 and not far.any()


def test_sum_normalised_map_single_point():
    """Z = the sum over the grid: a single Gaussian is separable, so the normalised value at (x, y) is
    the product of the two 1-D normal densities at x - u and y - v, each divided by its own sum over
    the grid's columns / rows (scipy's density, independent of the oracle's formula); M sums to 1."""
    H, W, u, v, sig = 36, 50, 21.3, 14.6, 3.5
    M, Z, am = motion.focus_map([(u, v, sig)], H, W, motion.MAP_SUM)
    px = norm.pdf(np.arange(W) - u, scale=sig)
    py = norm.pdf(np.arange(H) - v, scale=sig)
    ref = np.outer(py / py.sum(), px / px.sum())
    np.testing.assert_allclose(M, ref, rtol=1e-12, atol=1e-18)
    assert abs(M.sum() - 1.0) < 1e-12
    assert am == int(np.argmax(ref))


def test_sum_and_max_normalisations_differ_by_one_factor():
    """The two normalisers of Eq. 7 give the same map up to Z_max / Z_sum, the same argmax, and the
    same zero map when nothing projects."""
    H, W = 30, 44
    pts = [(8.0, 10.0, 3.0), (20.5, 12.25, 5.0), (35.0, 4.0, 1.5)]
    Mm, Zm, am_m = motion.focus_map(pts, H, W, motion.MAP_MAX)
    Ms, Zs, am_s = motion.focus_map(pts, H, W, motion.MAP_SUM)
    np.testing.assert_allclose(Ms * (Zs / Zm), Mm, rtol=1e-13, atol=1e-16)
    assert am_m == am_s and Ms.max() < 1.0 and abs(Ms.sum() - 1.0) < 1e-12
    M0, Z0, a0 = motion.focus_map([], H, W, motion.MAP_SUM)
    assert Z0 == 0 and not M0.any() and a0 == 0
    with pytest.raises(ValueError):
        motion.focus_map(pts, H, W, 2)


def test_sigma_px_closed_form():
    """Each frame's own spread (Eq. 7) on a constant-acceleration path: the second difference of the
    centres is a dt^2 exactly, so sigma_px = clip(sigma |a| dt^2, sigma_min, sigma_max) from frame 2 on
    and 0 on frames 0 and 1 (no focus point)."""
    from oracle import pipeline
    fps, acc = 30.0, (0.3, 0.0, 0.8)
    T_w = mf_synth.CameraPath(accel=acc, sway_deg=0.0).poses(12)
    s_ref = np.linalg.norm(acc) / fps ** 2
    for sigma, lo, hi in ((1e4, 0.5, 2000.0), (1.0, 0.5, 2000.0), (1e9, 0.5, 40.0)):
        out = pipeline.run_poses(T_w, K, 40, 60, sigma=sigma, sigma_min=lo, sigma_max=hi, maps=False)
        sp = out["sigma_px"]
        assert sp[0] == 0.0 and sp[1] == 0.0
        np.testing.assert_allclose(sp[2:], min(max(sigma * s_ref, lo), hi), rtol=1e-9)


def test_map_points_use_current_rotation():
    """Constant world acceleration along z and a camera whose yaw changes per frame: every point of
    frame t projects to cx - fx tan(yaw_t)."""
    fps = 30.0
    poses = []
    for i in range(20):
        yaw = math.radians(2.0 * i)
        c = np.array([0, 0, 1.0 * i / fps + 0.5 * 0.8 * (i / fps) ** 2])
        poses.append(mf_synth.pose_from_center(c, mf_synth.rot_y(yaw)))
    T_w = np.stack(poses)
    tr = motion.focus_track(T_w, *K)
    for t in (5, 14, 19):
        pts = motion.map_points(t, T_w, tr, 15, *K, 1e4, 0.5, 2000.0)
        assert len(pts) == min(15, t - 1)
        for (u, v, s) in pts:
            assert abs(u - (K[2] - K[0] * math.tan(math.radians(2.0 * t)))) < 1e-7
            assert abs(v - K[3]) < 1e-7
            assert abs(s - min(max(1e4 * 0.8 / fps ** 2, 0.5), 2000.0)) < 1e-9
