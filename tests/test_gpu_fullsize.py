"""Parity at the small workload's full size (64 frames 280x504, 12 layers, D=384), in the launch
configuration the benchmark times (all 7 windows of the stream in one fused batch): windows 0-1
against the FP64 oracle; and serving invariance (a stream alone and in a mix of streams)."""
import numpy as np
import pytest

import mf_synth
from gpu_util import dir_err_deg, mf, rot_err_deg, torch_cuda
from oracle import motion, pipeline, vit

pytestmark = pytest.mark.gpu

WL = mf_synth.SMALL
K = (WL.fx, WL.fy, WL.cx, WL.cy)
SIGMA = 1000.0


@pytest.fixture(scope="module")
def oracle_w01():
    blob = mf_synth.make_weights(WL.model, WL.seed_weights)
    w = vit.unpack_weights(blob, WL.model.depth, WL.model.dim, WL.model.mlp)
    frames = mf_synth.workload_frames(WL, 24)          # windows 0 and 1 cover frames 0..23
    return pipeline.run_stream(frames, w, WL.model.heads, WL.window, WL.overlap, K, sigma=SIGMA, windows=2)


def _run_engine(precision):
    torch = torch_cuda()
    m = mf()
    blob = mf_synth.make_weights(WL.model, WL.seed_weights)
    rows = m.rows_per_frame(WL.height, WL.width)
    nwin = len(motion.window_schedule(WL.frames, WL.window, WL.overlap))
    eng = m.Engine.from_model(WL.model, blob, precision=precision, max_tokens=nwin * WL.window * rows + 64)
    sid = eng.open_stream(WL.height, WL.width, WL.window, WL.overlap, K, sigma=SIGMA, ring_frames=WL.frames,
                          result_frames=WL.frames)
    frames = torch.from_numpy(mf_synth.workload_frames(WL)).cuda()
    eng.push_frames(sid, frames, eos=True)
    eng.sync()
    st = eng.stats()
    maps = np.zeros((WL.frames, WL.height, WL.width), np.float32)
    recs, _ = eng.poll(sid, WL.frames, maps)
    eng.close()
    assert st["batches_run"] == 1 and st["windows_run"] == nwin      # one fused batch
    return recs, maps


def _errors(recs, ref):
    """Pose errors, and the focus errors next to the bounds their conditioning allows.

    The acceleration is a second difference of camera centres, so an error dp in the centres moves
    a_w by up to 4 max|dp| and its direction by up to 4 max|dp| / |a_w| rad; where the oracle has
    |a_z| >= 0.5 |a| the pixel moves by at most 4 f times that angle (d tan / d angle <= 4 there).
    """
    n = ref["T_w"].shape[0]
    T = recs["T_w2c"][:n].reshape(-1, 4, 4)
    Tr = ref["T_w"]
    rot = rot_err_deg(T[:, :3, :3], Tr[:, :3, :3])
    tdir = dir_err_deg(T[:, :3, 3], Tr[:, :3, 3])
    tr = ref["track"]
    cg = -np.einsum("nji,nj->ni", T[:, :3, :3], T[:, :3, 3])
    dp = np.linalg.norm(cg - tr["p"], axis=1)
    dp3 = np.maximum(dp, np.maximum(np.r_[0, dp[:-1]], np.r_[0, 0, dp[:-2]]))
    v = tr["valid"] & ((recs["valid"][:n] & 1) == 1)
    adir = dir_err_deg(recs["a_world"][:n][v], tr["a_w"][v])
    abound = np.degrees(4 * dp3[v] / np.linalg.norm(tr["a_w"][v], axis=1))
    cond = v & (np.abs(tr["a_c"][:, 2]) >= 0.5 * np.linalg.norm(tr["a_c"], axis=1))
    px = np.hypot(recs["u"][:n][cond] - tr["uv"][cond, 0], recs["v"][:n][cond] - tr["uv"][cond, 1])
    pbound = 4 * max(K[0], K[1]) * 4 * dp3[cond] / np.linalg.norm(tr["a_w"][cond], axis=1)
    return rot, tdir, adir, abound, px, pbound


def test_small_fp32_windows01(oracle_w01):
    recs, maps = _run_engine("fp32")
    assert list(recs["frame"]) == list(range(WL.frames))
    rot, tdir, adir, abound, px, pbound = _errors(recs, oracle_w01)
    print(f"fp32: rot {rot.max():.2e} deg, tdir {tdir.max():.2e} deg, accel dir {adir.max() if adir.size else 0:.2e} "
          f"deg (bound {abound.max() if abound.size else 0:.2e}), focus px {px.max() if px.size else 0:.2e} "
          f"(bound {pbound.max() if pbound.size else 0:.2e})")
    assert rot.max() < 1e-3 and tdir.max() < 1e-3
    assert (adir <= abound + 1e-9).all()
    assert (px <= pbound + 1e-9).all()
    n = oracle_w01["T_w"].shape[0]
    np.testing.assert_array_equal(recs["valid"][:n] & 1, oracle_w01["track"]["valid"].astype(np.int32))


def test_small_bf16_windows01(oracle_w01):
    recs, maps = _run_engine("bf16")
    assert list(recs["frame"]) == list(range(WL.frames))
    rot, tdir, adir, abound, px, pbound = _errors(recs, oracle_w01)
    print(f"bf16: rot {rot.max():.3f} deg, tdir {tdir.max():.3f} deg, accel dir p99 "
          f"{np.percentile(adir, 99) if adir.size else 0:.2f} deg, focus px p50 {np.median(px) if px.size else 0:.1f}")
    assert rot.max() < 2.0 and tdir.max() < 2.0
    assert (adir <= np.minimum(abound, 180.0) + 1e-9).all()
    # every map is a valid normalised map: peak 1 at the reported argmax, values in [0, 1]
    for r, mp in zip(recs, maps):
        if r["valid"] & 2:
            assert abs(mp[r["peak_y"], r["peak_x"]] - 1.0) < 1e-6 and mp.max() <= 1.0 + 1e-6 and mp.min() >= 0.0


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_stream_alone_equals_stream_in_mix(precision):
    """Continuous batching does not change a stream's results: rows and segments are computed
    independently of what else shares the batch (fp8 activation scales are per window), so the
    outputs are bitwise equal."""
    torch = torch_cuda()
    m = mf()
    model = mf_synth.ModelConfig(4, 384, 6, 1536)
    blob = mf_synth.make_weights(model, 5)
    geo = [(112, 168, 8, 4, 21), (140, 252, 8, 4, 13), (112, 112, 6, 2, 17)]
    frames = [torch.from_numpy(mf_synth.make_frames(n, H, W, 40 + i)).cuda() for i, (H, W, L, O, n) in enumerate(geo)]

    def run(which):
        eng = m.Engine.from_model(model, blob, precision=precision, max_tokens=65536)
        sids = {}
        for i in which:
            H, W, L, O, n = geo[i]
            sids[i] = eng.open_stream(H, W, L, O, (100.0, 100.0, W / 2, H / 2), sigma=200.0, ring_frames=n + L,
                                      result_frames=n + L)
        for i in which:
            eng.push_frames(sids[i], frames[i], eos=True)
        eng.sync()
        out = {}
        for i in which:
            H, W, L, O, n = geo[i]
            mp = np.zeros((n, H, W), np.float32)
            out[i] = (eng.poll(sids[i], n, mp)[0], mp)
        st = eng.stats()
        eng.close()
        return out, st

    mix, st = run([0, 1, 2])
    assert st["batches_run"] == 1
    for i in range(3):
        alone, _ = run([i])
        a, b = alone[i][0], mix[i][0]
        assert list(a["frame"]) == list(range(geo[i][4]))
        for f in ("T_w2c", "pose9", "a_world", "u", "v", "valid", "peak_x", "peak_y"):
            np.testing.assert_array_equal(a[f], b[f], err_msg=f"stream {i} field {f}")
        np.testing.assert_array_equal(alone[i][1], mix[i][1])
