"""Window forward parity (patch embedding, blocks, pose head) of the HIP path against the FP64
oracle on the same seeded weights and pixels."""
import math

import numpy as np
import pytest

import mf_synth
from gpu_util import dir_err_deg, mf, rot_err_deg, torch_cuda
from oracle import vit

pytestmark = pytest.mark.gpu

# FP32 operands on fp32 MFMA: per-element relative error ~1e-6 per layer.
FP32_TOK_TOL = 2e-4
# BF16 operands: the tolerance is BF16_EMU_FACTOR times the error of the oracle's emulated-bf16
# forward on the same inputs (operands rounded to bf16 where the device rounds them, FP64 elsewhere),
# so a kernel mistake worth more than a few bf16 roundings fails.
BF16_EMU_FACTOR = 3.0


def _setup(model, S, H, W, seed_w=0, seed_px=1, std=0.02):
    blob = mf_synth.make_weights(model, seed_w, std=std)
    frames = mf_synth.make_frames(S, H, W, seed_px)
    w = vit.unpack_weights(blob, model.depth, model.dim, model.mlp)
    return blob, frames, w


def _oracle_tokens(frames, w, heads, layers, precision="fp64"):
    S, _, H, W = frames.shape
    n = (H // 14) * (W // 14) + 1
    prec = vit.Prec(precision)
    x = vit.embed(frames, w, prec=prec)
    for l in range(layers):
        groups = [(f * n, n) for f in range(S)] if l % 2 == 0 else [(0, S * n)]
        x = vit.block(x, w["layers"][l], heads, groups, prec)
    return x


def _valid_rows(S, n, npad):
    return np.concatenate([np.arange(f * npad, f * npad + n) for f in range(S)])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("layers", [0, 1, 2])
def test_tokens_after_layers(prec, layers):
    torch = torch_cuda()
    m = mf()
    model = mf_synth.ModelConfig(4, 128, 4, 512)
    S, H, W = 3, 56, 84
    blob, frames, w = _setup(model, S, H, W, std=0.05)
    eng = m.Engine.from_model(model, blob, precision=prec, max_tokens=4096)
    _, _, tok = eng.forward_window(torch.from_numpy(frames).cuda(), max_layers=layers, want_tokens=True)
    n = (H // 14) * (W // 14) + 1
    npad = m.rows_per_frame(H, W)
    ref = _oracle_tokens(frames.astype(np.float64), w, model.heads, layers)
    got = tok[_valid_rows(S, n, npad)]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    if prec == "fp32":
        tol = FP32_TOK_TOL
    else:
        emu = _oracle_tokens(frames.astype(np.float64), w, model.heads, layers, "bf16")
        tol = BF16_EMU_FACTOR * np.abs(emu - ref).max() / np.abs(ref).max()
    print(f"{prec} layers={layers} max rel token error {err:.3e} (tolerance {tol:.3e})")
    assert err < tol


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_tiny_workload_poses(prec):
    """The tiny workload (8 frames 112x112, 4 layers, D=128): pose9 and T against the oracle."""
    torch = torch_cuda()
    m = mf()
    wl = mf_synth.TINY
    blob, frames, w = _setup(wl.model, wl.frames, wl.height, wl.width, wl.seed_weights, wl.seed_pixels)
    eng = m.Engine.from_model(wl.model, blob, precision=prec, max_tokens=4096)
    p9, T, _ = eng.forward_window(torch.from_numpy(frames).cuda())
    ref = vit.forward_window(frames, w, wl.model.heads)
    Tref = np.stack([vit.pose9_to_T(r) for r in ref])
    rot = rot_err_deg(T[:, :3, :3], Tref[:, :3, :3]).max()
    tdir = dir_err_deg(T[:, :3, 3], Tref[:, :3, 3]).max()
    p9err = np.abs(p9 - ref).max()
    print(f"{prec}: pose9 max abs err {p9err:.3e} rot {rot:.3e} deg tdir {tdir:.3e} deg")
    if prec == "fp32":
        assert rot < 1e-3 and tdir < 1e-3 and p9err < 1e-5
    else:
        assert rot < 2.0 and tdir < 2.0
    # the pose is a proper rigid transform
    R = T[:, :3, :3]
    np.testing.assert_allclose(R @ R.transpose(0, 2, 1), np.tile(np.eye(3), (wl.frames, 1, 1)), atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-12)


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-5), ("bf16", 2e-2)])
def test_qkv_scatter_layouts(prec, tol):
    """Step-local: the QKV GEMM's epilogue writes Q and K head-major and V transposed exactly
    as the oracle's q, k, v of the first block (from the same embedded tokens); Q is stored
    multiplied by log2(e)/sqrt(hd), the form the attention kernels take."""
    torch = torch_cuda()
    m = mf()
    model = mf_synth.ModelConfig(2, 128, 4, 256)
    S, H, W = 3, 56, 84
    blob, frames, w = _setup(model, S, H, W, std=0.05)
    eng = m.Engine.from_model(model, blob, precision=prec, max_tokens=4096)
    eng.forward_window(torch.from_numpy(frames).cuda(), max_layers=1)
    mpad = 4096 + 256
    dt = np.float32 if prec == "fp32" else np.uint16
    def fetch(which, shape):
        a = eng.debug_copy(which, shape, dt)
        if prec == "bf16":
            a = (a.astype(np.uint32) << 16).view(np.float32)
        return a.astype(np.float64)
    hd = model.head_dim
    Q = fetch(2, (model.heads, mpad, hd)) * (math.sqrt(hd) / math.log2(math.e))   # stored scaled
    Kb = fetch(3, (model.heads, mpad, hd))
    Vt = fetch(4, (model.heads, hd, mpad))
    n = (H // 14) * (W // 14) + 1
    npad = m.rows_per_frame(H, W)
    valid = _valid_rows(S, n, npad)
    x0 = vit.embed(frames.astype(np.float64), w)
    lw = w["layers"][0]
    qkv = vit.layer_norm(x0, lw["ln1_g"], lw["ln1_b"]) @ lw["W_qkv"] + lw["b_qkv"]
    D = model.dim
    scale = np.abs(qkv).max()
    for h in range(model.heads):
        c = slice(h * hd, (h + 1) * hd)
        assert np.abs(Q[h][valid] - qkv[:, :D][:, c]).max() < tol * scale
        assert np.abs(Kb[h][valid] - qkv[:, D:2 * D][:, c]).max() < tol * scale
        assert np.abs(Vt[h][:, valid].T - qkv[:, 2 * D:][:, c]).max() < tol * scale
