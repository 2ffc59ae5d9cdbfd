"""End-to-end parity through the stream C ABI: push frames (or poses) -> windows -> forward ->
anchoring -> focus -> maps, against the oracle pipeline."""
import math

import numpy as np
import pytest

import mf_synth
from gpu_util import mf, torch_cuda
from oracle import motion, pipeline, vit

pytestmark = pytest.mark.gpu


def _drain(eng, sid, H, W, cap=4096):
    recs, maps = [], []
    while True:
        buf = np.zeros((cap, H, W), np.float32)
        r, st = eng.poll(sid, cap, buf)
        if len(r):
            recs.append(r)
            maps.append(buf[:len(r)])
        if st != 0:
            break
    return np.concatenate(recs), np.concatenate(maps)


def _run_poses_engine(m, T, K, H, W, sigma, n_points=15, local_windows=None, focus_mode=0, diff_stride=1,
                      anchor_mode=0, map_mode=0):
    eng = m.Engine(1, 128, 4, 128, np.zeros(mf_synth.weight_count(mf_synth.ModelConfig(1, 128, 4, 128)),
                                            np.float32), precision="fp32", max_tokens=16384)
    n = len(T) if T is not None else sum(len(t) for _, t in local_windows)
    sid = eng.open_stream(H, W, 16, 8, K, n_points=n_points, sigma=sigma, result_frames=max(64, n),
                          focus_mode=focus_mode, diff_stride=diff_stride, anchor_mode=anchor_mode, map_mode=map_mode)
    if local_windows is None:
        eng.push_poses(sid, T, 0, eos=True)
    else:
        for (start, Tl) in local_windows:
            eng.push_poses(sid, Tl, start, local=True)
        eng.close_stream(sid)
    eng.sync()
    recs, maps = _drain(eng, sid, H, W)
    eng.close()
    return recs, maps


def test_world_poses_closed_form_head_yaw():
    """Forward acceleration with the head turned by psi: u = cx - fx tan(psi), v = cy."""
    torch_cuda()
    m = mf()
    K = (400.0, 400.0, 252.0, 140.0)
    psi = 12.0
    path = mf_synth.CameraPath(velocity=(0, 0, 1.0), accel=(0, 0, 0.8), sway_deg=0.0, yaw0_deg=psi)
    T = path.poses(40)
    recs, maps = _run_poses_engine(m, T, K, 280, 504, sigma=2e4)
    assert list(recs["frame"]) == list(range(40))
    assert not recs["valid"][:2].any() and (recs["valid"][2:] & 1).all()
    np.testing.assert_allclose(recs["u"][2:], K[2] - K[0] * math.tan(math.radians(psi)), rtol=1e-9)
    np.testing.assert_allclose(recs["v"][2:], K[3], atol=1e-9)


def test_world_poses_match_oracle_track_and_maps():
    torch_cuda()
    m = mf()
    K = (400.0, 380.0, 252.0, 140.0)
    H, W = 140, 252
    path = mf_synth.CameraPath(velocity=(0.2, 0.0, 1.5), accel=(0.3, -0.1, 0.5), sway_deg=3.0)
    T = path.poses(50)
    sigma = 3e4
    recs, maps = _run_poses_engine(m, T, K, H, W, sigma)
    ref = pipeline.run_poses(T, K, H, W, sigma=sigma)
    tr = ref["track"]
    np.testing.assert_array_equal(recs["valid"] & 1, tr["valid"].astype(np.int32))
    v = tr["valid"]
    np.testing.assert_allclose(recs["a_world"], tr["a_w"], rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(recs["a_cam"], tr["a_c"], rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(recs["u"][v], tr["uv"][v, 0], rtol=1e-9)
    np.testing.assert_allclose(recs["v"][v], tr["uv"][v, 1], rtol=1e-9)
    np.testing.assert_allclose(maps, ref["maps"], atol=1e-5)
    for i, r in enumerate(recs):
        if ref["Z"][i] >= 1e-30:
            assert r["valid"] & 2
            am = r["peak_y"] * W + r["peak_x"]
            assert ref["maps"][i].ravel()[am] >= 1.0 - 1e-5
        else:
            assert not (r["valid"] & 2) and not maps[i].any()


def test_sum_normalised_maps_and_sigma_px_match_oracle():
    """Eq. 7 with Z = the map's sum over the pixel grid (MF_MAP_SUM), and each record's own spread
    sigma_px, against the oracle; a frame whose normaliser underflows gives the zero map in both."""
    torch_cuda()
    m = mf()
    K = (400.0, 380.0, 252.0, 140.0)
    H, W = 154, 266     # not a multiple of the render workgroup's 8 rows
    path = mf_synth.CameraPath(velocity=(0.2, 0.0, 1.5), accel=(0.3, -0.1, 0.5), sway_deg=3.0)
    T = path.poses(44)
    sigma = 3e4
    recs, maps = _run_poses_engine(m, T, K, H, W, sigma, map_mode=m.MF_MAP_SUM)
    ref = pipeline.run_poses(T, K, H, W, sigma=sigma, map_mode=motion.MAP_SUM)
    np.testing.assert_allclose(recs["sigma_px"], ref["sigma_px"], rtol=1e-6, atol=0)
    assert (recs["sigma_px"][:2] == 0).all()
    for i, r in enumerate(recs):
        if ref["Z"][i] >= 1e-30:
            # every value within 1e-5 of the map's peak (fp32 Gaussians, a double-precision sum)
            np.testing.assert_allclose(maps[i], ref["maps"][i], atol=1e-5 * ref["maps"][i].max(), rtol=0)
            assert abs(float(maps[i].astype(np.float64).sum()) - 1.0) < 1e-4
            assert r["valid"] & 2
            # the peak (fp32 values on the device): the oracle's map is maximal there up to fp32 rounding
            am = r["peak_y"] * W + r["peak_x"]
            assert ref["maps"][i].ravel()[am] >= ref["maps"][i].max() * (1.0 - 1e-5)
        else:
            assert not (r["valid"] & 2) and not maps[i].any()


@pytest.mark.parametrize("focus_mode,stride", [(0, 3), (1, 1), (1, 4)])
def test_focus_modes_and_strides_match_oracle(focus_mode, stride):
    """Velocity-based projection and strided differences: motion vectors, focus points, validity
    and maps against the oracle (FP64 on both sides)."""
    torch_cuda()
    m = mf()
    K = (400.0, 380.0, 252.0, 140.0)
    H, W = 140, 252
    path = mf_synth.CameraPath(velocity=(0.2, 0.0, 1.5), accel=(0.3, -0.1, 0.5), sway_deg=3.0)
    T = path.poses(60)
    sigma = 3e4 if focus_mode == 0 else 300.0
    recs, maps = _run_poses_engine(m, T, K, H, W, sigma, focus_mode=focus_mode, diff_stride=stride)
    ref = pipeline.run_poses(T, K, H, W, sigma=sigma, focus_mode=focus_mode, stride=stride)
    tr = ref["track"]
    first = stride if focus_mode == 1 else 2 * stride
    assert not (recs["valid"][:first] & 1).any()
    np.testing.assert_array_equal(recs["valid"] & 1, tr["valid"].astype(np.int32))
    v = tr["valid"]
    np.testing.assert_allclose(recs["a_world"], tr["a_w"], rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(recs["a_cam"], tr["a_c"], rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(recs["u"][v], tr["uv"][v, 0], rtol=1e-9)
    np.testing.assert_allclose(recs["v"][v], tr["uv"][v, 1], rtol=1e-9)
    np.testing.assert_allclose(maps, ref["maps"], atol=1e-5)


def test_scale_aware_anchoring_matches_oracle():
    """Window-local poses with a per-window scale (translations times lambda_k) chained with
    MF_ANCHOR_YAW_SCALE: equal to the oracle's scale-aware chaining and to the true trajectory."""
    torch_cuda()
    m = mf()
    rng = np.random.default_rng(12)
    N, L, O = 56, 16, 8
    path = mf_synth.CameraPath(velocity=(0.1, 0, 1.2), accel=(0, 0.05, 0.4), sway_deg=4.0)
    T_w = path.poses(N)
    sched = motion.window_schedule(N, L, O)
    wins, locs = [], []
    for k, w in enumerate(sched):
        G = np.eye(4)
        lam = 1.0
        if k:
            G[:3, :3] = mf_synth.rot_y(rng.uniform(-2, 2))
            G[:3, 3] = rng.uniform(-3, 3, 3)
            lam = rng.uniform(0.5, 2.0)
        Tl = np.stack([T_w[t] @ np.linalg.inv(G) for t in range(w["start"], w["start"] + w["size"])])
        Tl[:, :3, 3] *= lam
        wins.append((w["start"], Tl))
        locs.append(Tl)
    K = (400.0, 400.0, 126.0, 70.0)
    recs, _ = _run_poses_engine(m, None, K, 140, 252, 1e4, local_windows=wins, anchor_mode=m.MF_ANCHOR_YAW_SCALE)
    chained = motion.chain_windows(sched, locs, motion.ANCHOR_YAW_SCALE)
    got = recs["T_w2c"].reshape(-1, 4, 4)
    np.testing.assert_allclose(got, chained, atol=1e-12)
    np.testing.assert_allclose(got, T_w, atol=1e-9)


def test_local_poses_anchoring_matches_oracle():
    """Window-local poses (arbitrary yaw-plus-shift frames per window) chained by the library in
    FP64 reproduce the oracle's chaining exactly (and the true trajectory)."""
    torch_cuda()
    m = mf()
    rng = np.random.default_rng(11)
    N, L, O = 48, 16, 8
    path = mf_synth.CameraPath(velocity=(0.1, 0, 1.2), accel=(0, 0.05, 0.4), sway_deg=4.0)
    T_w = path.poses(N)
    sched = motion.window_schedule(N, L, O)
    wins, locs = [], []
    for k, w in enumerate(sched):
        G = np.eye(4)
        if k:
            G[:3, :3] = mf_synth.rot_y(rng.uniform(-2, 2))
            G[:3, 3] = rng.uniform(-3, 3, 3)
        Tl = np.stack([T_w[t] @ np.linalg.inv(G) for t in range(w["start"], w["start"] + w["size"])])
        wins.append((w["start"], Tl))
        locs.append(Tl)
    K = (400.0, 400.0, 126.0, 70.0)
    recs, _ = _run_poses_engine(m, None, K, 140, 252, 1e4, local_windows=wins)
    chained = motion.chain_windows(sched, locs, motion.ANCHOR_YAW)
    got = recs["T_w2c"].reshape(-1, 4, 4)
    np.testing.assert_allclose(got, chained, atol=1e-12)
    np.testing.assert_allclose(got, T_w, atol=1e-10)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_tiny_stream_end_to_end(prec):
    torch = torch_cuda()
    m = mf()
    wl = mf_synth.TINY
    blob = mf_synth.make_weights(wl.model, wl.seed_weights)
    frames = mf_synth.workload_frames(wl)
    K = (wl.fx, wl.fy, wl.cx, wl.cy)
    eng = m.Engine.from_model(wl.model, blob, precision=prec, max_tokens=4096)
    sid = eng.open_stream(wl.height, wl.width, wl.window, wl.overlap, K, sigma=50.0)
    eng.push_frames(sid, torch.from_numpy(frames).cuda(), eos=True)
    eng.sync()
    recs, maps = _drain(eng, sid, wl.height, wl.width)
    w = vit.unpack_weights(blob, wl.model.depth, wl.model.dim, wl.model.mlp)
    ref = pipeline.run_stream(frames, w, wl.model.heads, wl.window, wl.overlap, K, sigma=50.0)
    assert list(recs["frame"]) == list(range(wl.frames))
    got_T = recs["T_w2c"].reshape(-1, 4, 4)
    err_T = np.abs(got_T - ref["T_w"]).max()
    print(f"{prec}: max |T - T_ref| = {err_T:.3e}")
    if prec == "fp32":
        assert err_T < 1e-4
        np.testing.assert_array_equal(recs["valid"] & 1, ref["track"]["valid"].astype(np.int32))
    else:
        assert err_T < 0.05


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_graph_replays_match_eager(precision):
    """A batch shape is captured once as a hipGraph and replayed: every replay (with unrelated eager
    work and synchronisation in between) equals the eager launch sequence bit for bit (fp8: the
    per-window amax buffers are cleared by a kernel inside the graph on every replay)."""
    torch = torch_cuda()
    m = mf()
    model = mf_synth.ModelConfig(4, 384, 6, 1536)
    blob = mf_synth.make_weights(model, 3)
    H, W, L, O, N = 112, 168, 8, 4, 20
    K = (120.0, 120.0, W / 2, H / 2)
    frames = torch.from_numpy(mf_synth.make_frames(N, H, W, 9)).cuda()

    def run(eng):
        sid = eng.open_stream(H, W, L, O, K, sigma=300.0, ring_frames=N, result_frames=N)
        eng.push_frames(sid, frames, eos=True)
        eng.sync()
        mp = np.zeros((N, H, W), np.float32)
        r, _ = eng.poll(sid, N, mp)
        eng.poll(sid, 1)
        return r, mp

    eager = m.Engine.from_model(model, blob, precision=precision, max_tokens=8192, graphs=False)
    ref, ref_maps = run(eager)
    eager.close()
    eng = m.Engine.from_model(model, blob, precision=precision, max_tokens=8192, graphs=True)
    x = torch.randn(64, 384, device="cuda")
    for rep in range(4):
        got, maps = run(eng)
        for f in ("T_w2c", "pose9", "a_world", "u", "v", "valid", "peak_x", "peak_y", "frame", "window"):
            np.testing.assert_array_equal(got[f], ref[f], err_msg=f"replay {rep} field {f}")
        np.testing.assert_array_equal(maps, ref_maps)
        y = torch.empty(64, 384, device="cuda")           # eager work between replays
        m.op_layernorm("fp32", x, y, torch.ones(384, device="cuda"), torch.zeros(384, device="cuda"))
        torch.cuda.synchronize()
    eng.close()


def test_graph_key_separates_batches_with_equal_counts():
    """Two batch compositions with the same token rows, frames and attention work items but different
    windows (short streams of 14 + 10 frames, then of 16 + 8, at 720 patches per frame): the fp8
    window quantiser's grid follows the largest window, so the second batch must not replay the
    graph captured for the first.  Results equal the eager launch sequence bit for bit."""
    torch = torch_cuda()
    m = mf()
    model = mf_synth.ModelConfig(2, 384, 6, 1536)
    blob = mf_synth.make_weights(model, 4)
    H, W, L, O = 280, 504, 16, 8
    rows = m.rows_per_frame(H, W)
    assert rows == 728
    K = (400.0, 400.0, W / 2, H / 2)
    frames = torch.from_numpy(mf_synth.make_frames(16, H, W, 21)).cuda()

    def batch(eng, lengths):
        sids = [eng.open_stream(H, W, L, O, K, sigma=300.0, ring_frames=L, result_frames=L) for _ in lengths]
        for sid, n in zip(sids, lengths):
            eng.push_frames(sid, frames[:n], eos=True)
        eng.sync()
        out = []
        for sid, n in zip(sids, lengths):
            mp = np.zeros((n, H, W), np.float32)
            r, _ = eng.poll(sid, n, mp)
            eng.poll(sid, 1)
            out.append((r, mp))
        return out

    eager = m.Engine.from_model(model, blob, precision="fp8", max_tokens=24 * rows + 64, graphs=False)
    ref = batch(eager, [16, 8])
    eager.close()
    eng = m.Engine.from_model(model, blob, precision="fp8", max_tokens=24 * rows + 64, graphs=True)
    batch(eng, [14, 10])                 # captured first
    got = batch(eng, [16, 8])
    st = eng.stats()
    eng.close()
    assert st["batches_run"] == 2
    for (r, mp), (rr, rmp) in zip(got, ref):
        for f in ("T_w2c", "pose9", "a_world", "u", "v", "valid", "peak_x", "peak_y", "frame"):
            np.testing.assert_array_equal(r[f], rr[f], err_msg=f)
        np.testing.assert_array_equal(mp, rmp)


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
@pytest.mark.parametrize("H,W", [(112, 168), (14, 28)])
def test_shared_frame_embedding_equals_separate_batches(precision, H, W):
    """Consecutive windows share their overlap frames (Sec. 2.2).  A stream pushed whole runs its four
    windows in one batch, where every overlap frame takes the earlier window's patch embedding (12
    frames); pushed a stride at a time, each window runs in a batch of its own and embeds all its
    frames.  The records and maps are the same bit for bit.  14 x 28 frames: 2 patches, 8 token rows
    per frame (fewer rows than one 32-key attention step)."""
    torch = torch_cuda()
    m = mf()
    model = mf_synth.ModelConfig(4, 384, 6, 1536)
    blob = mf_synth.make_weights(model, 5)
    L, O, N = 8, 4, 20
    K = (120.0, 120.0, W / 2, H / 2)
    frames = torch.from_numpy(mf_synth.make_frames(N, H, W, 17)).cuda()

    def run(pieces):
        eng = m.Engine.from_model(model, blob, precision=precision, max_tokens=8192, graphs=False)
        sid = eng.open_stream(H, W, L, O, K, sigma=300.0, ring_frames=N, result_frames=N)
        for i, (a, b) in enumerate(pieces):
            eng.push_frames(sid, frames[a:b], eos=i == len(pieces) - 1)
            eng.sync()
        mp = np.zeros((N, H, W), np.float32)
        r, _ = eng.poll(sid, N, mp)
        eng.poll(sid, 1)
        st = eng.stats()
        eng.close()
        assert list(r["frame"]) == list(range(N))
        return r, mp, st

    whole, whole_maps, st_whole = run([(0, N)])
    apart, apart_maps, st_apart = run([(0, L)] + [(a, a + L - O) for a in range(L, N, L - O)])
    assert st_whole["batches_run"] == 1 and st_whole["frames_embed_shared"] == 3 * O
    assert st_apart["batches_run"] == 4 and st_apart["frames_embed_shared"] == 0
    for f in ("T_w2c", "pose9", "a_world", "u", "v", "valid", "peak_x", "peak_y", "window"):
        np.testing.assert_array_equal(whole[f], apart[f], err_msg=f)
    np.testing.assert_array_equal(whole_maps, apart_maps)


@pytest.mark.parametrize("threaded", [False, True])
def test_torch_allocator_matches_default(threaded):
    """With allocator="torch" every device buffer of the engine comes from torch's caching
    allocator (through the C ABI's dev_alloc / dev_free); the results are bitwise those of the
    engine's own hipMalloc path, and closing the engine hands every buffer back."""
    torch = torch_cuda()
    m = mf()
    wl = mf_synth.TINY
    blob = mf_synth.make_weights(wl.model, wl.seed_weights)
    frames = torch.from_numpy(mf_synth.workload_frames(wl)).cuda()
    K = (wl.fx, wl.fy, wl.cx, wl.cy)

    def run(alloc):
        eng = m.Engine.from_model(wl.model, blob, precision="bf16", max_tokens=4096, threaded=threaded,
                                  allocator=alloc)
        held = len(eng._alloc.live) if alloc else 0
        sid = eng.open_stream(wl.height, wl.width, wl.window, wl.overlap, K, sigma=50.0)
        eng.push_frames(sid, frames, eos=True)
        eng.sync()
        recs, maps = _drain(eng, sid, wl.height, wl.width)
        a = eng._alloc
        eng.close()
        return recs, maps, held, a

    torch.cuda.synchronize()
    base_mem = torch.cuda.memory_allocated()
    r0, m0, _, _ = run(None)
    r1, m1, held, alloc = run("torch")
    assert held > 10                                   # weights and workspace came from torch
    assert len(alloc.live) == 0                        # ... and all went back on close
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base_mem
    for f in ("frame", "T_w2c", "pose9", "a_world", "u", "v", "valid", "peak_x", "peak_y"):
        np.testing.assert_array_equal(r0[f], r1[f], err_msg=f)
    np.testing.assert_array_equal(m0, m1)
