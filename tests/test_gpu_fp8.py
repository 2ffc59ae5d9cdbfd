"""FP8 (OCP E4M3) path: the quantiser against the oracle's E4M3 rounding, the E4M3 MFMA GEMM on
exactly representable inputs, and the fp8 engine (QKV / fc1 / fc2 on E4M3 operands with per-tensor
weight scales and per-window activation scales) against the oracle's fp8 emulation and FP64."""
import math

import numpy as np
import pytest

import mf_synth
from gpu_util import dir_err_deg, mf, rot_err_deg, torch_cuda
from oracle import vit

pytestmark = pytest.mark.gpu


def e4m3_decode(codes):
    """Values of E4M3 byte codes from their bit fields (bias 7; exponent 0 subnormal; S.1111.111 NaN)."""
    c = np.asarray(codes, dtype=np.int64)
    s, e, m = c >> 7, (c >> 3) & 15, c & 7
    mag = np.where(e == 0, (m / 8.0) * 2.0 ** -6, (1.0 + m / 8.0) * 2.0 ** (e - 7.0))
    mag = np.where((e == 15) & (m == 7), np.nan, mag)
    return np.where(s == 1, -mag, mag)


def e4m3_encode(values):
    """Byte codes of exactly representable values (inverse of the decode table)."""
    table = {}
    for code in range(256):
        v = float(e4m3_decode(code))
        if not np.isnan(v):
            table.setdefault(v, code)
    return np.array([table[float(v)] for v in np.ravel(values)], dtype=np.uint8).reshape(np.shape(values))


def test_decode_table_matches_oracle_rounding():
    v = e4m3_decode(np.arange(256))
    fin = v[~np.isnan(v)]
    assert np.array_equal(vit.round_e4m3(fin), fin) and np.nanmax(v) == 448.0


@pytest.mark.parametrize("scale", [1.0, 0.37, 1.0 / 448.0 * 5.0, 3.0e-3])
def test_quantize_fp8_matches_oracle_rounding(scale):
    """Device E4M3(x / scale) against the oracle's round-to-nearest-even with saturation: the
    device scales in fp32 (x * (1/scale)), so the oracle rounds that same fp32 product."""
    torch = torch_cuda()
    m = mf()
    rng = np.random.default_rng(7)
    fin = e4m3_decode(np.arange(256))
    fin = np.unique(fin[~np.isnan(fin)])
    mids = 0.5 * (fin[1:] + fin[:-1])                              # every tie between neighbours
    x = np.concatenate([
        rng.standard_normal(40000) * np.exp(rng.uniform(-12, 7, 40000)),
        fin, mids, -mids, [0.0, -0.0, 447.9, 448.0, 460.0, 464.0, 470.0, 1e30, -1e30, 2.0 ** -10, 2.0 ** -9 * 1.5]])
    x = (x * scale).astype(np.float32)
    x = x[: len(x) // 4 * 4]
    dx = torch.from_numpy(x).cuda()
    dq = torch.zeros(x.size, dtype=torch.uint8, device="cuda")
    m.op_quantize_fp8(dx, scale, dq)
    got = e4m3_decode(dq.cpu().numpy())
    inv = np.float32(1.0) / np.float32(scale)
    want = vit.round_e4m3((x * inv).astype(np.float32).astype(np.float64))
    assert not np.isnan(got).any()
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, f"{bad.size} mismatches, first x={x[bad[:5]]} got={got[bad[:5]]} want={want[bad[:5]]}"


@pytest.mark.parametrize("M,N,K", [(300, 256, 256), (1, 128, 640), (517, 384, 1536), (16400, 1024, 256)])
def test_gemm_fp8_representable_inputs_exact(M, N, K):
    """Integers in [-8, 8] are exact in E4M3; with power-of-two scales and integer biases every
    partial sum is exact in fp32, so C must equal the integer product bit for bit.  The last
    shape takes the 256 x 128 tile path."""
    torch = torch_cuda()
    m = mf()
    rng = np.random.default_rng(M + 3 * N + K)
    A = rng.integers(-8, 9, size=(M, K))
    B = rng.integers(-8, 9, size=(N, K))
    bias = rng.integers(-5, 6, size=N).astype(np.float32)
    asc = (2.0 ** rng.integers(-3, 4, size=M)).astype(np.float32)
    bsc = np.array([0.5], np.float32)
    ref = (A @ B.T).astype(np.float64) * asc[:, None].astype(np.float64) * 0.5 + bias[None, :]
    dA = torch.from_numpy(e4m3_encode(A)).cuda()
    dB = torch.from_numpy(e4m3_encode(B)).cuda()
    dC = torch.full((M, N), 7.0, device="cuda")
    m.op_gemm_fp8(dA, dB, torch.from_numpy(asc).cuda(), torch.from_numpy(bsc).cuda(), torch.from_numpy(bias).cuda(),
                  dC)
    got = dC.cpu().numpy().astype(np.float64)
    assert np.array_equal(got, ref)


def test_gemm_fp8_random_codes_within_fp32_accumulation_bound():
    """Arbitrary E4M3 operands (every finite code) with random scales: the device result equals the
    FP64 product of the decoded values to within fp32 accumulation rounding, (K + 2) u |A||B|^T."""
    torch = torch_cuda()
    m = mf()
    rng = np.random.default_rng(11)
    M, N, K = 333, 256, 1024
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], dtype=np.uint8)
    A8 = rng.choice(codes, size=(M, K))
    B8 = rng.choice(codes, size=(N, K))
    A, B = e4m3_decode(A8), e4m3_decode(B8)
    asc = rng.uniform(0.5, 2.0, M).astype(np.float32)
    bsc = np.array([0.013], np.float32)
    bias = rng.standard_normal(N).astype(np.float32)
    sc = asc.astype(np.float64)[:, None] * np.float64(bsc[0])
    ref = (A @ B.T) * sc + bias[None, :]
    bound = (K + 2) * 2.0 ** -24 * ((np.abs(A) @ np.abs(B).T) * sc + np.abs(bias)[None, :]) + 1e-30
    dC = torch.zeros((M, N), device="cuda")
    m.op_gemm_fp8(torch.from_numpy(A8).cuda(), torch.from_numpy(B8).cuda(), torch.from_numpy(asc).cuda(),
                  torch.from_numpy(bsc).cuda(), torch.from_numpy(bias).cuda(), dC)
    err = np.abs(dC.cpu().numpy().astype(np.float64) - ref)
    print(f"fp8 gemm random codes: max err / bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)


def test_quantize_fp8_windows_scales_and_codes():
    """Per-window dynamic scaling: the scale is amax/448 over the valid rows only (padding rows
    hold large values that must not count), every row of a window (padding too) is quantised with
    its window's scale, and an all-zero window gets scale 1.  Codes are compared with the oracle's
    E4M3 rounding of the same fp32 products y * (1/s)."""
    torch = torch_cuda()
    m = mf()
    rng = np.random.default_rng(3)
    Cdim = 400
    segs = np.array([[0, 3, 50, 56], [168, 1, 200, 200], [368, 2, 9, 16], [400, 1, 24, 24]], np.int32)
    rows = 424
    y = (rng.standard_normal((rows, Cdim)) * np.exp(rng.uniform(-3, 3, (rows, 1)))).astype(np.float32)
    valid = np.zeros(rows, bool)
    for base, nf, n, npad in segs:
        for f in range(nf):
            valid[base + f * npad: base + f * npad + n] = True
    y[~valid] *= 1e3
    y[400:424] = 0.0
    yb = torch.from_numpy(y).to(torch.bfloat16)
    ybf = yb.float().numpy()
    dq = torch.zeros((rows, Cdim), dtype=torch.uint8, device="cuda")
    ds = torch.zeros(rows, device="cuda")
    m.op_quantize_fp8_windows(yb.cuda(), segs, dq, ds)
    got_q, got_s = e4m3_decode(dq.cpu().numpy()), ds.cpu().numpy()
    for base, nf, n, npad in segs:
        r = slice(base, base + nf * npad)
        amax = np.float32(np.max(np.abs(ybf[r][valid[r]])))
        s = np.float32(amax / np.float32(448.0)) if amax > 0 else np.float32(1.0)
        assert np.all(got_s[r] == s), (base, got_s[r][:3], s)
        inv = np.float32(1.0) / s
        want = vit.round_e4m3((ybf[r] * inv).astype(np.float32).astype(np.float64))
        assert np.array_equal(got_q[r], want)
        assert np.max(np.abs(got_q[r][valid[r]])) == (448.0 if amax > 0 else 0.0)


def test_gemm_fp8_rejects_bad_shapes():
    torch = torch_cuda()
    m = mf()
    dA = torch.zeros((64, 96), dtype=torch.uint8, device="cuda")       # K % 128 != 0
    dB = torch.zeros((128, 96), dtype=torch.uint8, device="cuda")
    s = torch.ones(128, device="cuda")
    dC = torch.zeros((64, 128), device="cuda")
    with pytest.raises(m.MfError):
        m.op_gemm_fp8(dA, dB, s, s, None, dC)


MODEL = mf_synth.ModelConfig(4, 256, 4, 1024)


def _oracle_tokens(frames, w, heads, layers, precision):
    S, _, H, W = frames.shape
    n = (H // 14) * (W // 14) + 1
    prec = vit.Prec(precision)
    x = vit.embed(frames, w, prec=prec)
    for l in range(layers):
        groups = [(f * n, n) for f in range(S)] if l % 2 == 0 else [(0, S * n)]
        x = vit.block(x, w["layers"][l], heads, groups, prec)
    return x


@pytest.mark.parametrize("layers", [1, 2])
def test_fp8_tokens_track_the_fp8_emulation(layers):
    """Tokens after 1-2 blocks against FP64: the device fp8 error is of the size the oracle's fp8
    emulation predicts (within 1.5x of it), and the device sits nearer the emulation than the
    emulation sits to FP64.  The two cannot agree more closely: E4M3 has a 2^-3 relative step, so
    a last-bit difference of a bf16 activation flips its E4M3 rounding with probability ~1/32 and
    each flip moves a product term by a full E4M3 step."""
    torch = torch_cuda()
    m = mf()
    S, H, W = 4, 56, 112
    blob = mf_synth.make_weights(MODEL, 0, std=0.05)
    frames = mf_synth.make_frames(S, H, W, 1)
    w = vit.unpack_weights(blob, MODEL.depth, MODEL.dim, MODEL.mlp)
    eng = m.Engine.from_model(MODEL, blob, precision="fp8", max_tokens=4096)
    _, _, tok = eng.forward_window(torch.from_numpy(frames).cuda(), max_layers=layers, want_tokens=True)
    eng.close()
    n = (H // 14) * (W // 14) + 1
    npad = m.rows_per_frame(H, W)
    got = tok[np.concatenate([np.arange(f * npad, f * npad + n) for f in range(S)])]
    f64 = frames.astype(np.float64)
    ref64 = _oracle_tokens(f64, w, MODEL.heads, layers, "fp64")
    emu = _oracle_tokens(f64, w, MODEL.heads, layers, "fp8")
    scale = np.abs(ref64).max()
    e_emu = np.abs(got - emu).max() / scale
    e_64 = np.abs(got - ref64).max() / scale
    emu_64 = np.abs(emu - ref64).max() / scale
    print(f"fp8 layers={layers}: vs emulation {e_emu:.3e}, vs fp64 {e_64:.3e}, emulation vs fp64 {emu_64:.3e}")
    assert e_emu < emu_64
    assert e_64 < 1.5 * emu_64


def test_fp8_tiny_poses_within_emulated_error():
    """Poses of the tiny geometry (8 frames 112x112, 4 layers) with a D=256 model: the device fp8
    error against FP64 stays within 3x the emulated-fp8 error (random weights make the pose
    ill-conditioned, so the emulation itself sets the scale), and T is a rigid transform."""
    torch = torch_cuda()
    m = mf()
    wl = mf_synth.TINY
    blob = mf_synth.make_weights(MODEL, wl.seed_weights)
    frames = mf_synth.make_frames(wl.frames, wl.height, wl.width, wl.seed_pixels)
    w = vit.unpack_weights(blob, MODEL.depth, MODEL.dim, MODEL.mlp)
    eng = m.Engine.from_model(MODEL, blob, precision="fp8", max_tokens=4096)
    p9, T, _ = eng.forward_window(torch.from_numpy(frames).cuda())
    eng.close()
    ref = np.stack([vit.pose9_to_T(r) for r in vit.forward_window(frames, w, MODEL.heads)])
    emu = np.stack([vit.pose9_to_T(r) for r in vit.forward_window(frames, w, MODEL.heads, precision="fp8")])
    rot = rot_err_deg(T[:, :3, :3], ref[:, :3, :3]).max()
    tdir = dir_err_deg(T[:, :3, 3], ref[:, :3, 3]).max()
    rot_e = rot_err_deg(emu[:, :3, :3], ref[:, :3, :3]).max()
    tdir_e = dir_err_deg(emu[:, :3, 3], ref[:, :3, 3]).max()
    print(f"fp8 tiny: rot {rot:.2f} deg (emulated {rot_e:.2f}), tdir {tdir:.2f} deg (emulated {tdir_e:.2f})")
    assert rot <= 3 * rot_e + 0.5 and tdir <= 3 * tdir_e + 0.5
    R = T[:, :3, :3]
    np.testing.assert_allclose(R @ R.transpose(0, 2, 1), np.tile(np.eye(3), (wl.frames, 1, 1)), atol=1e-12)



def _fp8_attention_case(torch, frames, n, heads=2, seed=41):
    """E4M3 query and key rows with per-row power-of-two scales (the oracle's row quantiser applied
    to queries already multiplied by log2(e)/sqrt(64) in fp32), bf16 V, in the library layouts."""
    rng = np.random.default_rng(seed)
    hd = 64
    npad = (n + 7) // 8 * 8
    mpad = frames * npad + 256 + 64
    c = np.float32(math.log2(math.e) / math.sqrt(hd))
    q = (rng.normal(0, 1.5, (heads, mpad, hd)).astype(np.float32) * c).astype(np.float64)
    k = rng.normal(0, 1.5, (heads, mpad, hd)).astype(np.float32).astype(np.float64)
    v = vit.round_bf16(rng.normal(0, 1, (heads, mpad, hd)))
    q8, eq = vit.quantise_rows_e4m3(q)
    k8, ek = vit.quantise_rows_e4m3(k)
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt).contiguous()
    d = dict(q8=dev(e4m3_encode(q8), torch.uint8), k8=dev(e4m3_encode(k8), torch.uint8),
             qe=dev((eq + 127).astype(np.uint8), torch.uint8), ke=dev((ek + 127).astype(np.uint8), torch.uint8),
             vt=dev(v.transpose(0, 2, 1).astype(np.float32), torch.bfloat16))
    qd, kd = q8 * 2.0 ** eq[..., None], k8 * 2.0 ** ek[..., None]     # the decoded operands
    return d, qd, kd, v, npad, mpad


def _softmax2_attention(qd, kd, v):
    s = qd @ kd.T                                 # base-2 exponent units
    p = np.exp2(s - s.max(axis=1, keepdims=True))
    return (p @ v) / p.sum(axis=1, keepdims=True)


@pytest.mark.parametrize("n,frames", [(145, 3), (300, 2), (65, 4)])
def test_attention_fp8_scores_match_fp64_on_decoded_operands(n, frames):
    """The attention with E4M3 scores (MF_FP8, head dim 64) against FP64 on the decoded E4M3 operands:
    the scores are exact products of representable values accumulated in fp32, so only the bf16
    rounding of the probabilities separates the two (the bf16 attention test's 1.5e-2); frame-wise
    segments and one global segment with the padding keys masked."""
    torch = torch_cuda()
    m = mf()
    heads, D = 2, 128
    d, qd, kd, v, npad, mpad = _fp8_attention_case(torch, frames, n, heads)
    o = torch.zeros((mpad, D), device="cuda", dtype=torch.bfloat16)
    m.op_attention_fp8(heads, D, d["q8"], d["qe"], d["k8"], d["ke"], d["vt"], o, mpad,
                       [[f * npad, 1, n, npad] for f in range(frames)])
    got = o.float().cpu().numpy()
    for f in range(frames):
        r = slice(f * npad, f * npad + n)
        for h in range(heads):
            ref = _softmax2_attention(qd[h, r], kd[h, r], v[h, r])
            np.testing.assert_allclose(got[r, h * 64:(h + 1) * 64], ref, atol=1.5e-2, rtol=1.5e-2)
    o.zero_()
    m.op_attention_fp8(heads, D, d["q8"], d["qe"], d["k8"], d["ke"], d["vt"], o, mpad, [[0, frames, n, npad]])
    got = o.float().cpu().numpy()
    valid = np.concatenate([np.arange(f * npad, f * npad + n) for f in range(frames)])
    for h in range(heads):
        ref = _softmax2_attention(qd[h, valid], kd[h, valid], v[h, valid])
        np.testing.assert_allclose(got[valid, h * 64:(h + 1) * 64], ref, atol=1.5e-2, rtol=1.5e-2)


def test_qkv_epilogue_writes_e4m3_rows_with_least_power_of_two_scales():
    """In an fp8 engine (head dim 64) the QKV projection writes every query and key row of every head
    as E4M3 with an E8M0 exponent (and no bf16 copy).  Decoded, they match the oracle's E4M3
    emulation of the same projection on the device's layer-0 tokens (LayerNorm in FP64 rounded to
    bf16, the window's amax/448 activation scale and the weight's amax/448 scale, E4M3 operands,
    FP64 products; queries times log2(e)/sqrt(hd)) within one E4M3 rounding of the output plus the
    bf16 rounding (a few activations whose bf16 LayerNorm output differs in the last bit round to
    another E4M3 code: at most 1 in 200), and each non-zero row reaches the top binade (|code| max in
    [224, 448]), which makes its exponent the least that fits."""
    torch = torch_cuda()
    m = mf()
    S, H, W = 3, 56, 84
    blob = mf_synth.make_weights(MODEL, 2, std=0.05)
    frames = mf_synth.make_frames(S, H, W, 6)
    eng = m.Engine.from_model(MODEL, blob, precision="fp8", max_tokens=2048)
    dfr = torch.from_numpy(frames).cuda()
    _, _, tok0 = eng.forward_window(dfr, max_layers=0, want_tokens=True)
    eng.forward_window(dfr, max_layers=1)
    D, heads = MODEL.dim, MODEL.heads
    hd = D // heads
    assert hd == 64
    mpad = (2048 + 7) // 8 * 8 + 256
    n = (H // 14) * (W // 14) + 1
    npad = m.rows_per_frame(H, W)
    rows = np.concatenate([np.arange(f * npad, f * npad + n) for f in range(S)])
    lw = vit.unpack_weights(blob, MODEL.depth, MODEL.dim, MODEL.mlp)["layers"][0]
    f32 = lambda x: np.asarray(x, dtype=np.float32)
    y = vit.round_bf16(vit.layer_norm(tok0[rows].astype(np.float64), lw["ln1_g"], lw["ln1_b"])).astype(np.float32)
    sa = f32(f32(np.max(np.abs(y))) / f32(448.0))
    qa = vit.round_e4m3(f32(y * (f32(1.0) / sa)).astype(np.float64))
    Wq = f32(lw["W_qkv"])
    sw = f32(f32(np.max(np.abs(Wq))) / f32(448.0))
    qw = vit.round_e4m3(f32(Wq * (f32(1.0) / sw)).astype(np.float64))
    ref = (qa @ qw) * np.float64(f32(sa * sw)) + lw["b_qkv"]
    c = np.float64(np.float32(math.log2(math.e) / math.sqrt(hd)))
    for block, w8, we in ((0, 7, 9), (1, 8, 10)):
        want = ref[:, block * D:(block + 1) * D].reshape(len(rows), heads, hd).transpose(1, 0, 2)
        if block == 0:
            want = want * c
        codes = eng.debug_copy(w8, (heads, mpad, hd), np.uint8)[:, rows]
        e = eng.debug_copy(we, (heads, mpad), np.uint8)[:, rows].astype(np.float64) - 127.0
        dec = e4m3_decode(codes) * 2.0 ** e[..., None]
        tol = 2.0 ** -4 * np.abs(want) + 2.0 ** -7 * np.abs(want) + 2.0 ** (e[..., None] - 8)
        bad = np.abs(dec - want) > tol
        print(f"block {block}: max |dec - ref| / |ref|max {np.abs(dec - want).max() / np.abs(want).max():.3e}, "
              f"beyond one E4M3 rounding {bad.sum()} of {bad.size}")
        assert bad.sum() <= bad.size // 200
        top = np.abs(e4m3_decode(codes)).max(axis=-1)
        assert ((top >= 224.0) & (top <= 448.0)).all()
    eng.close()
