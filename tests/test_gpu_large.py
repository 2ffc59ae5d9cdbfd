"""Parity at the large workload's full size (32-frame windows of 378x504 = 31 136 tokens, 24 layers,
D=1024, 16 heads, BF16).

End to end: the benchmark's launch configuration (the whole 256-frame stream, 15 windows in one
fused batch) against the stored FP64 oracle outputs of windows 0-1 (tests/golden), with the BF16
gates calibrated by the stored emulated-bf16 oracle outputs of the same windows.

Step-local: each stage is fed the library's own previous output and checked against the FP64 oracle
on sampled token rows (the oracle computes all keys/values, but only the sampled queries)."""
import numpy as np
import pytest

import mf_synth
from gpu_util import (check_emulation_gates, golden, golden_errors, mf, record_errors, run_stream_fused, summary,
                      torch_cuda)
from oracle import vit

pytestmark = pytest.mark.gpu

WL = mf_synth.LARGE
S = WL.window
RNG = np.random.default_rng(7)


@pytest.fixture(scope="module")
def setup():
    torch = torch_cuda()
    m = mf()
    blob = mf_synth.make_weights(WL.model, WL.seed_weights)
    w = vit.unpack_weights(blob, WL.model.depth, WL.model.dim, WL.model.mlp)
    frames = mf_synth.workload_frames(WL, S)
    rows = m.rows_per_frame(WL.height, WL.width)
    eng = m.Engine.from_model(WL.model, blob, precision="bf16", max_tokens=S * rows + 64)
    dfr = torch.from_numpy(frames).cuda()
    n = (WL.height // 14) * (WL.width // 14) + 1
    valid = np.concatenate([np.arange(f * rows, f * rows + n) for f in range(S)])
    yield dict(m=m, eng=eng, w=w, frames=frames, dfr=dfr, n=n, rows=rows, valid=valid)
    eng.close()


def tokens(s, layers):
    _, _, tok = s["eng"].forward_window(s["dfr"], max_layers=layers, want_tokens=True)
    return tok[s["valid"]].astype(np.float64)


def block_rows(x, lw, heads, groups, sample):
    """One pre-LN block for the rows `sample` of x (all rows feed keys and values)."""
    D = x.shape[1]
    hd = D // heads
    xn = vit.layer_norm(x, lw["ln1_g"], lw["ln1_b"])
    qkv = xn @ lw["W_qkv"] + lw["b_qkv"]
    q, k, v = qkv[:, :D], qkv[:, D:2 * D], qkv[:, 2 * D:]
    o = np.zeros((len(sample), D))
    for i, r in enumerate(sample):
        s0, ln = next((g0, gl) for g0, gl in groups if g0 <= r < g0 + gl)
        for h in range(heads):
            c = slice(h * hd, (h + 1) * hd)
            o[i, c] = vit.attention(q[r:r + 1, c], k[s0:s0 + ln, c], v[s0:s0 + ln, c])[0]
    y = x[sample] + o @ lw["W_o"] + lw["b_o"]
    hmid = vit.gelu(vit.layer_norm(y, lw["ln2_g"], lw["ln2_b"]) @ lw["W_1"] + lw["b_1"])
    return y + hmid @ lw["W_2"] + lw["b_2"]


def test_patch_embedding_full_size(setup):
    s = setup
    x0 = tokens(s, 0)
    sample = np.unique(np.r_[RNG.integers(0, x0.shape[0], 200), np.arange(0, x0.shape[0], s["n"])])
    ref = vit.embed(s["frames"][:, :, :, :], s["w"])[sample]
    err = np.abs(x0[sample] - ref).max() / np.abs(ref).max()
    print(f"embedding rel err {err:.2e}")
    assert err < 1e-2          # bf16 patch operands, fp32 accumulation over 588 terms


@pytest.mark.parametrize("layer", [0, 1, 9])
def test_block_full_size(setup, layer):
    s = setup
    n = s["n"]
    xl = tokens(s, layer)
    xn1 = tokens(s, layer + 1)
    groups = [(f * n, n) for f in range(S)] if layer % 2 == 0 else [(0, S * n)]
    sample = np.unique(np.r_[RNG.integers(0, xl.shape[0], 48), [0, n, 5 * n + 7]])
    ref = block_rows(xl, s["w"]["layers"][layer], WL.model.heads, groups, sample)
    err = np.abs(xn1[sample] - ref).max() / np.abs(ref).max()
    print(f"layer {layer} ({'global' if layer % 2 else 'frame-wise'}) rel err {err:.2e}")
    assert err < 2e-2          # one block of bf16 operands: ~2^-8 per rounding, fp32 accumulation


def test_pose_head_full_size(setup):
    s = setup
    p9, T, tok = s["eng"].forward_window(s["dfr"], max_layers=-1, want_tokens=True)
    cam = tok[np.arange(S) * s["rows"]].astype(np.float64)
    ref = vit.pose_head(cam, s["w"])
    err = np.abs(p9 - ref).max() / np.abs(ref).max()
    print(f"pose head rel err {err:.2e}")
    assert err < 1e-4          # the head runs in fp32 from the same tokens
    Tref = np.stack([vit.pose9_to_T(r) for r in p9.astype(np.float64)])
    np.testing.assert_allclose(T, Tref, atol=1e-12)   # quaternion -> rotation in FP64


BF16_EMU_FACTOR = 3.0   # the gate rule of the small workload's end-to-end test


def test_large_bf16_windows01_against_fp64():
    torch = torch_cuda()
    ref = golden("large_fp64_w01")
    emu = golden_errors(golden("large_bf16emu_w01"), ref)
    blob = mf_synth.make_weights(WL.model, WL.seed_weights)
    frames = torch.from_numpy(mf_synth.workload_frames(WL)).cuda()
    recs = run_stream_fused(WL, "bf16", blob, frames)
    del frames
    e = record_errors(recs, ref)
    print("large bf16 vs FP64, windows 0-1: " + summary(e))
    print("emulated bf16 vs FP64: " + summary(emu))
    lim = check_emulation_gates(e, emu, BF16_EMU_FACTOR, pose_floor=2.0)
    print("limits: " + ", ".join(f"{k} {v:.2f}" for k, v in lim.items()))
