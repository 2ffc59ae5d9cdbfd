"""Pins of the oracle's depth head (the window forward's depth maps of Sec. 2.2) and of their
emission and scale through the anchoring: an independent torch formulation (layer_norm, linear,
exp, pixel_shuffle), the closed form of a zero weight matrix, patch locality, and the anchoring's
scale factors undoing known per-window scales exactly."""
import numpy as np
import pytest

import mf_synth
from oracle import motion, pipeline, vit

RNG = np.random.default_rng(23)


def _head_weights(D, std=0.05):
    return {"lnd_g": 1.0 + RNG.normal(0, std, D), "lnd_b": RNG.normal(0, std, D),
            "W_d": RNG.normal(0, std, (D, 196)), "b_d": RNG.normal(0, std, 196)}


def test_depth_head_matches_torch_pixel_shuffle():
    import torch
    import torch.nn.functional as F
    S, H, W, D = 2, 56, 84, 64
    gh, gw = H // 14, W // 14
    n = gh * gw + 1
    x = RNG.normal(0, 1, (S * n, D))
    w = _head_weights(D)
    got = vit.depth_head(x, w, S, H, W)
    t = torch.from_numpy(x).reshape(S, n, D)[:, 1:, :]
    z = F.linear(F.layer_norm(t, (D,), torch.from_numpy(w["lnd_g"]), torch.from_numpy(w["lnd_b"]), eps=1e-6),
                 torch.from_numpy(w["W_d"].T.copy()), torch.from_numpy(w["b_d"]))
    img = F.pixel_shuffle(torch.exp(z).reshape(S, gh, gw, 196).permute(0, 3, 1, 2), 14)   # [S, 1, H, W]
    assert got.shape == (S, H, W)
    np.testing.assert_allclose(got, img[:, 0].numpy(), rtol=1e-12, atol=0)


def test_zero_weights_give_the_bias_pattern_in_every_patch():
    S, H, W, D = 1, 28, 42, 32
    n = (H // 14) * (W // 14) + 1
    w = _head_weights(D)
    w["W_d"] = np.zeros((D, 196))
    d = vit.depth_head(RNG.normal(0, 1, (S * n, D)), w, S, H, W)
    yy, xx = np.mgrid[0:H, 0:W]
    np.testing.assert_array_equal(d[0], np.exp(w["b_d"])[(yy % 14) * 14 + xx % 14])


def test_a_patch_token_moves_only_its_own_pixels():
    S, H, W, D = 2, 42, 56, 48
    gh, gw = H // 14, W // 14
    n = gh * gw + 1
    x = RNG.normal(0, 1, (S * n, D))
    w = _head_weights(D)
    base = vit.depth_head(x, w, S, H, W)
    f, py, px = 1, 2, 1
    x2 = x.copy()
    x2[f * n + 1 + py * gw + px] += RNG.normal(0, 1, D)
    x2[f * n] += 5.0                      # the camera token does not enter the depth head
    diff = vit.depth_head(x2, w, S, H, W) != base
    want = np.zeros_like(diff)
    want[f, py * 14:(py + 1) * 14, px * 14:(px + 1) * 14] = True
    np.testing.assert_array_equal(diff, want)


def test_unpack_with_and_without_the_depth_head():
    m = mf_synth.ModelConfig(2, 64, 2, 128, depth_head=True)
    blob = mf_synth.make_weights(m, 3)
    w = vit.unpack_weights(blob, 2, 64, 128, depth_head=True)
    assert w["W_d"].shape == (64, 196) and w["b_d"].shape == (196,)
    np.testing.assert_array_equal(w["b_d"], blob[-196:].astype(np.float64))
    with pytest.raises(ValueError):
        vit.unpack_weights(blob, 2, 64, 128)          # trailing depth-head values
    plain = mf_synth.make_weights(mf_synth.ModelConfig(2, 64, 2, 128), 3)
    np.testing.assert_array_equal(plain, blob[:plain.size])   # the head is appended, nothing else moves


def test_chain_scales_undo_known_window_scales():
    """Window-local poses made from a world trajectory and multiplied in translation by a known
    scale s_k per window: the scale-aware anchoring returns 1/s_k for every later window (the
    factor the window's depth is multiplied by), and 1 everywhere under rigid anchoring."""
    N, L, O = 40, 12, 5
    T = mf_synth.CameraPath(velocity=(0.2, 0.0, 1.5), accel=(0.0, 0.1, 0.5)).poses(N)
    sched = motion.window_schedule(N, L, O)
    s = [1.0] + list(RNG.uniform(0.5, 2.0, len(sched) - 1))
    loc = []
    for k, win in enumerate(sched):
        g = np.eye(4)                     # each window's own frame: a yaw and a shift of the world
        if k:
            g[:3, :3] = mf_synth.rot_y(RNG.uniform(-3, 3))
            g[:3, 3] = RNG.uniform(-5, 5, size=3)
        Tl = np.stack([T[t] @ np.linalg.inv(g) for t in range(win["start"], win["start"] + win["size"])])
        Tl[:, :3, 3] *= s[k]
        loc.append(Tl)
    _, sc = motion.chain_windows(sched, loc, motion.ANCHOR_YAW_SCALE, return_scales=True)
    np.testing.assert_allclose(sc, [1.0 / v for v in s], rtol=1e-10)
    _, sc_rigid = motion.chain_windows(sched, loc, motion.ANCHOR_YAW, return_scales=True)
    assert sc_rigid == [1.0] * len(sched)


@pytest.mark.parametrize("mode", [motion.ANCHOR_YAW, motion.ANCHOR_YAW_SCALE])
def test_stream_depth_comes_from_the_emitting_window(mode):
    """Each emitted frame's depth map is the depth of the window that emits it, times that window's
    scale factor (1 under the paper's rigid anchoring)."""
    m = mf_synth.ModelConfig(2, 64, 2, 128, depth_head=True)
    w = vit.unpack_weights(mf_synth.make_weights(m, 1, std=0.05), 2, 64, 128, depth_head=True)
    frames = mf_synth.make_frames(11, 28, 42, 5)
    out = pipeline.run_stream(frames, w, 2, 6, 3, (40.0, 40.0, 21.0, 14.0), anchor_mode=mode, depth=True,
                              maps=False)
    assert out["depth"].shape == (11, 28, 42)
    for k, win in enumerate(out["schedule"]):
        _, d = vit.forward_window(frames[win["start"]:win["start"] + win["size"]], w, 2, depth=True)
        rho = out["window_scale"][k]
        if mode == motion.ANCHOR_YAW:
            assert rho == 1.0
        for t in range(win["emit_begin"], win["emit_end"]):
            np.testing.assert_array_equal(out["depth"][t], rho * d[t - win["start"]])
    assert (out["depth"] > 0).all()
