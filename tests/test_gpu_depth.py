"""Depth maps of the window forward (Sec. 2.2: each window predicts depth maps beside the poses; only
frames not emitted before are emitted) through the stream API, against the oracle's depth head on
the same seeded weights and frames: a 20-frame stream of four overlapping windows, rigid and
scale-aware anchoring (the depth of a scale-anchored window is multiplied by its scale factor)."""
import numpy as np
import pytest

import mf_synth
from gpu_util import mf, torch_cuda
from oracle import motion, pipeline, vit

pytestmark = pytest.mark.gpu

MODEL = mf_synth.ModelConfig(4, 128, 4, 512, depth_head=True)
N, H, W, L, O = 20, 56, 84, 8, 4
K = (60.0, 60.0, 42.0, 28.0)
# BF16: the depth error (relative) within BF16_EMU_FACTOR x the oracle's emulated-bf16 depth error
BF16_EMU_FACTOR = 3.0


@pytest.fixture(scope="module")
def inputs():
    blob = mf_synth.make_weights(MODEL, 4, std=0.05)
    w = vit.unpack_weights(blob, MODEL.depth, MODEL.dim, MODEL.mlp, depth_head=True)
    frames = mf_synth.make_frames(N, H, W, 31)
    return blob, w, frames


def _run(blob, frames, precision, mode, graphs=False, extra=False):
    torch = torch_cuda()
    m = mf()
    eng = m.Engine.from_model(MODEL, blob, precision=precision, max_tokens=65536, graphs=graphs)
    sid = eng.open_stream(H, W, L, O, K, sigma=50.0, anchor_mode=mode, emit_depth=True, result_frames=N)
    other = None
    if extra:   # a second stream without depth shares the batch
        other = eng.open_stream(H, W, L, O, K, sigma=50.0, result_frames=N)
        eng.push_frames(other, torch.from_numpy(frames[::-1].copy()).cuda(), eos=True)
    eng.push_frames(sid, torch.from_numpy(frames).cuda(), eos=True)
    eng.sync()
    depth = np.zeros((N, H, W), np.float32)
    maps = np.zeros((N, H, W), np.float32)
    recs, _ = eng.poll(sid, N, maps, depth)
    st = eng.stats()
    eng.close()
    assert list(recs["frame"]) == list(range(N))
    return recs, depth, st


@pytest.mark.parametrize("mode", [motion.ANCHOR_YAW, motion.ANCHOR_YAW_SCALE])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_stream_depth_matches_oracle(inputs, precision, mode):
    blob, w, frames = inputs
    recs, depth, _ = _run(blob, frames, precision, mode)
    ref = pipeline.run_stream(frames, w, MODEL.heads, L, O, K, sigma=50.0, anchor_mode=mode, depth=True, maps=False)
    rel = np.abs(depth - ref["depth"]) / ref["depth"]
    assert (depth > 0).all()
    if precision == "fp32":
        tol = 1e-4
    else:
        emu = pipeline.run_stream(frames, w, MODEL.heads, L, O, K, sigma=50.0, anchor_mode=mode, depth=True,
                                  maps=False, precision="bf16")
        tol = BF16_EMU_FACTOR * float((np.abs(emu["depth"] - ref["depth"]) / ref["depth"]).max())
    print(f"{precision} mode {mode}: depth max rel err {rel.max():.3e} (tolerance {tol:.3e}), window scales "
          f"{np.round(ref['window_scale'], 4).tolist()}")
    assert rel.max() <= tol


def test_depth_alone_equals_depth_in_a_mixed_batch(inputs):
    """A depth stream batched with a stream that keeps no depth: bitwise the same depth and poses."""
    blob, _, frames = inputs
    a, da, _ = _run(blob, frames, "bf16", motion.ANCHOR_YAW_SCALE)
    b, db, st = _run(blob, frames, "bf16", motion.ANCHOR_YAW_SCALE, extra=True)
    assert st["batches_run"] >= 1
    np.testing.assert_array_equal(da, db)
    np.testing.assert_array_equal(a["T_w2c"], b["T_w2c"])


def test_depth_replayed_from_graphs_equals_eager(inputs):
    """The same stream three times on one engine with hipGraphs (captured by the first, replayed by
    the others), with eager work and synchronisation between them: every run equals the eager one."""
    torch = torch_cuda()
    m = mf()
    blob, _, frames = inputs
    _, d_eager, _ = _run(blob, frames, "bf16", motion.ANCHOR_YAW_SCALE, graphs=False)
    eng = m.Engine.from_model(MODEL, blob, precision="bf16", max_tokens=65536, graphs=True)
    dfr = torch.from_numpy(frames).cuda()
    for _ in range(3):
        sid = eng.open_stream(H, W, L, O, K, sigma=50.0, anchor_mode=motion.ANCHOR_YAW_SCALE, emit_depth=True,
                              result_frames=N)
        eng.push_frames(sid, dfr, eos=True)
        eng.sync()
        d = np.zeros((N, H, W), np.float32)
        recs, _ = eng.poll(sid, N, None, d)
        eng.poll(sid, 1)
        assert len(recs) == N
        np.testing.assert_array_equal(d, d_eager)
        torch.cuda.synchronize()
    eng.close()


def test_emit_depth_needs_a_depth_head():
    torch_cuda()
    m = mf()
    plain = mf_synth.ModelConfig(2, 128, 4, 256)
    eng = m.Engine.from_model(plain, mf_synth.make_weights(plain, 0), precision="bf16", max_tokens=8192)
    with pytest.raises(m.MfError):
        eng.open_stream(H, W, L, O, K, emit_depth=True)
    sid = eng.open_stream(H, W, L, O, K)
    with pytest.raises(m.MfError):          # depth asked of a stream that keeps none
        eng.poll(sid, 4, depth=np.zeros((4, H, W), np.float32))
    eng.close()
