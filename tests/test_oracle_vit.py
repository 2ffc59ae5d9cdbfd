"""Pins of the oracle's network stage against brute force, library routines and invariants.

Nothing here compares the oracle with itself: each check is a pure-Python brute force,
an independent PyTorch-float64 library formulation, a closed form or an invariance.
"""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F
from scipy.spatial.transform import Rotation

import mf_synth
from oracle import vit

RNG = np.random.default_rng(1234)


def brute_attention(q, k, v):
    """Triple loop over queries, keys and channels with math.exp."""
    Tq, hd = q.shape
    Tk = k.shape[0]
    out = np.zeros((Tq, v.shape[1]))
    for i in range(Tq):
        s = [sum(q[i, c] * k[j, c] for c in range(hd)) / math.sqrt(hd) for j in range(Tk)]
        m = max(s)
        e = [math.exp(x - m) for x in s]
        z = sum(e)
        for c in range(v.shape[1]):
            out[i, c] = sum(e[j] * v[j, c] for j in range(Tk)) / z
    return out


def test_attention_brute_force():
    q, k, v = RNG.normal(size=(5, 3)), RNG.normal(size=(7, 3)), RNG.normal(size=(7, 4))
    np.testing.assert_allclose(vit.attention(q, k, v), brute_attention(q, k, v), rtol=1e-13, atol=1e-14)


def test_attention_chunking_is_exact():
    q, k, v = RNG.normal(size=(37, 8)), RNG.normal(size=(41, 8)), RNG.normal(size=(41, 8))
    np.testing.assert_allclose(vit.attention(q, k, v, chunk=5), vit.attention(q, k, v, chunk=1000),
                               rtol=1e-14, atol=1e-15)


def test_attention_rows_sum_to_one():
    q, k = RNG.normal(size=(9, 4)) * 3, RNG.normal(size=(11, 4)) * 3
    ones = np.ones((11, 2))
    np.testing.assert_allclose(vit.attention(q, k, ones), 1.0, rtol=0, atol=1e-14)
    # with V = identity the output rows are the softmax weights themselves
    P = vit.attention(q, k, np.eye(11))
    assert (P >= 0).all()
    np.testing.assert_allclose(P.sum(1), 1.0, atol=1e-14)


def test_attention_vs_torch_sdpa():
    q, k, v = RNG.normal(size=(33, 16)), RNG.normal(size=(33, 16)), RNG.normal(size=(33, 16))
    ref = F.scaled_dot_product_attention(*(torch.from_numpy(a)[None, None] for a in (q, k, v)))[0, 0]
    np.testing.assert_allclose(vit.attention(q, k, v), ref.numpy(), rtol=1e-12, atol=1e-13)


def test_layer_norm_stats_and_library():
    x = RNG.normal(size=(6, 48)) * 5 + 3
    y = vit.layer_norm(x, np.ones(48), np.zeros(48))
    np.testing.assert_allclose(y.mean(1), 0, atol=1e-13)
    np.testing.assert_allclose((y ** 2).mean(1), 1 / (1 + 1e-6 / x.var(1)), rtol=1e-12)
    g, b = RNG.normal(size=48), RNG.normal(size=48)
    ref = F.layer_norm(torch.from_numpy(x), (48,), torch.from_numpy(g), torch.from_numpy(b), eps=1e-6)
    np.testing.assert_allclose(vit.layer_norm(x, g, b), ref.numpy(), rtol=1e-12, atol=1e-12)


def test_gelu_erf():
    z = np.linspace(-6, 6, 101)
    ref = np.array([0.5 * t * (1 + math.erf(t / math.sqrt(2))) for t in z])
    np.testing.assert_allclose(vit.gelu(z), ref, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(vit.gelu(z), F.gelu(torch.from_numpy(z)).numpy(), rtol=1e-14, atol=1e-16)


def test_normalise_imagenet():
    mean, std = np.array([0.485, 0.456, 0.406]), np.array([0.229, 0.224, 0.225])
    px = np.zeros((1, 3, 14, 14))
    px[0, :, 0, 0] = mean
    px[0, :, 0, 1] = mean + std
    y = vit.normalise(px)
    np.testing.assert_allclose(y[0, :, 0, 0], 0, atol=1e-15)
    np.testing.assert_allclose(y[0, :, 0, 1], 1, atol=1e-14)


def test_patch_embedding_is_a_stride14_convolution():
    S, H, W, D = 2, 28, 42, 8
    x = RNG.random((S, 3, H, W))
    Wp = RNG.normal(size=(588, D))
    got = vit.patchify(x) @ Wp
    conv = F.conv2d(torch.from_numpy(x), torch.from_numpy(Wp.T.reshape(D, 3, 14, 14).copy()), stride=14)
    ref = conv.permute(0, 2, 3, 1).reshape(S, -1, D).numpy()   # grid row-major
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_sincos_pe_structure():
    gh, gw, D = 3, 5, 16
    pe = vit.sincos_pe(gh, gw, D)
    q = D // 4
    np.testing.assert_array_equal(pe[0], np.r_[np.zeros(q), np.ones(q), np.zeros(q), np.ones(q)])
    # rows are row-major over the grid: the first half depends only on the row, the second on the column
    for y in range(gh):
        for x in range(gw):
            np.testing.assert_array_equal(pe[y * gw + x, :2 * q], pe[y * gw, :2 * q])
            np.testing.assert_array_equal(pe[y * gw + x, 2 * q:], pe[x, 2 * q:])
    # dot products depend on displacements only: sum_i cos(dy w_i) + cos(dx w_i)
    a, b, c, d = pe[1 * gw + 4], pe[2 * gw + 1], pe[0 * gw + 3], pe[1 * gw + 0]
    assert abs(a @ b - c @ d) < 1e-12                 # both displacements are (+1, -3)
    assert pe[:, :q].max() <= 1 and pe[:, q:2 * q].min() >= -1
    # lowest frequency is 1 rad per patch: sin(y * 1) for y = 2
    assert abs(pe[2 * gw, 0] - math.sin(2.0)) < 1e-15


def test_quaternion_rotation():
    for _ in range(20):
        q = RNG.normal(size=4) * RNG.uniform(0.1, 10)
        R = vit.quat_to_rot(q)
        np.testing.assert_allclose(R, Rotation.from_quat(q).as_matrix(), atol=1e-13)   # scalar-last
        np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(R) - 1) < 1e-12
    th = 0.7
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    np.testing.assert_allclose(vit.quat_to_rot(np.array([0, 0, math.sin(th / 2), math.cos(th / 2)])), Rz,
                               atol=1e-15)
    np.testing.assert_array_equal(vit.quat_to_rot(np.zeros(4)), np.eye(3))


# ------------------------------------------------------------------------- whole network
def torch_forward(frames, blob, cfg):
    """Independent float64 formulation of the same network with torch library ops."""
    t = lambda a: torch.from_numpy(np.asarray(a, dtype=np.float64))
    names = [n for n, _ in mf_synth.weight_spec(cfg)]
    shapes = [s for _, s in mf_synth.weight_spec(cfg)]
    off, P = 0, {}
    flat = np.asarray(blob, np.float32).astype(np.float64)
    for n, s in zip(names, shapes):
        k = int(np.prod(s))
        P[n] = t(flat[off:off + k].reshape(s))
        off += k
    S, _, H, W = frames.shape
    D, nh = cfg.dim, cfg.heads
    hd = D // nh
    gh, gw = H // 14, W // 14
    mean = torch.tensor([0.485, 0.456, 0.406], dtype=torch.float64).view(1, 3, 1, 1)
    std = torch.tensor([0.229, 0.224, 0.225], dtype=torch.float64).view(1, 3, 1, 1)
    x = (t(frames) - mean) / std
    emb = F.conv2d(x, P["W_p"].T.reshape(D, 3, 14, 14), P["b_p"], stride=14)   # [S,D,gh,gw]
    emb = emb.flatten(2).transpose(1, 2)                                         # [S,P,D]
    om = 10000.0 ** (-torch.arange(D // 4, dtype=torch.float64) / (D // 4))
    yy, xx = torch.meshgrid(torch.arange(gh, dtype=torch.float64), torch.arange(gw, dtype=torch.float64),
                            indexing="ij")
    ay, ax = yy.reshape(-1, 1) * om, xx.reshape(-1, 1) * om
    emb = emb + torch.cat([ay.sin(), ay.cos(), ax.sin(), ax.cos()], 1)
    cam = torch.stack([P["c_ref"]] + [P["c_other"]] * (S - 1))[:, None]
    X = torch.cat([cam, emb], 1)                                                  # [S,n,D]
    n = X.shape[1]
    for l in range(cfg.depth):
        p = f"l{l}."
        h = F.layer_norm(X, (D,), P[p + "ln1.g"], P[p + "ln1.b"], eps=1e-6)
        if l % 2 == 1:
            h = h.reshape(1, S * n, D)
        qkv = F.linear(h, P[p + "W_qkv"].T, P[p + "b_qkv"])
        B, T = qkv.shape[:2]
        q, k, v = (qkv[..., i * D:(i + 1) * D].reshape(B, T, nh, hd).transpose(1, 2) for i in range(3))
        o = F.scaled_dot_product_attention(q, k, v).transpose(1, 2).reshape(B, T, D)
        X = X + F.linear(o, P[p + "W_o"].T, P[p + "b_o"]).reshape(S, n, D)
        h = F.layer_norm(X, (D,), P[p + "ln2.g"], P[p + "ln2.b"], eps=1e-6)
        X = X + F.linear(F.gelu(F.linear(h, P[p + "W_1"].T, P[p + "b_1"])), P[p + "W_2"].T, P[p + "b_2"])
    c = F.layer_norm(X[:, 0], (D,), P["lnf.g"], P["lnf.b"], eps=1e-6)
    return F.linear(F.gelu(F.linear(c, P["H_1"].T, P["h_1"])), P["H_2"].T, P["h_2"]).numpy()


def tiny_setup(S=4, H=42, W=56, depth=4, dim=32, heads=2, mlp=64, seed=3):
    cfg = mf_synth.ModelConfig(depth, dim, heads, mlp)
    blob = mf_synth.make_weights(cfg, seed, std=0.2)   # large std so every term matters
    frames = mf_synth.make_frames(S, H, W, seed + 1)
    return cfg, blob, frames, vit.unpack_weights(blob, depth, dim, mlp)


def test_forward_vs_torch_library_formulation():
    cfg, blob, frames, w = tiny_setup()
    got = vit.forward_window(frames.astype(np.float64), w, cfg.heads)
    ref = torch_forward(frames, blob, cfg)
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-12)


def test_forward_tiny_workload_vs_torch():
    w = mf_synth.TINY
    blob = mf_synth.make_weights(w.model, w.seed_weights)
    frames = mf_synth.workload_frames(w)
    got = vit.forward_window(frames, vit.unpack_weights(blob, w.model.depth, w.model.dim, w.model.mlp),
                             w.model.heads)
    np.testing.assert_allclose(got, torch_forward(frames, blob, w.model), rtol=1e-10, atol=1e-13)


def test_frame_permutation_equivariance():
    """No frame-index embedding: permuting frames 1..S-1 permutes the poses; frame 0 is special."""
    cfg, blob, frames, w = tiny_setup(S=5)
    base = vit.forward_window(frames, w, cfg.heads)
    perm = np.array([0, 3, 1, 4, 2])
    got = vit.forward_window(frames[perm], w, cfg.heads)
    np.testing.assert_allclose(got, base[perm], rtol=1e-11, atol=1e-13)
    swapped = vit.forward_window(frames[[1, 0, 2, 3, 4]], w, cfg.heads)
    assert np.abs(swapped[0] - base[1]).max() > 1e-6      # c_ref vs c_other matters


def test_framewise_block_is_per_frame():
    """An even (frame-wise) block on the whole window equals the block applied frame by frame."""
    cfg, blob, frames, w = tiny_setup(S=3, depth=1)
    x = vit.embed(frames, w)
    n = x.shape[0] // 3
    prec = vit.Prec()
    whole = vit.block(x, w["layers"][0], cfg.heads, [(f * n, n) for f in range(3)], prec)
    for f in range(3):
        one = vit.block(x[f * n:(f + 1) * n], w["layers"][0], cfg.heads, [(0, n)], prec)
        np.testing.assert_allclose(whole[f * n:(f + 1) * n], one, rtol=1e-12, atol=1e-13)


def test_bf16_rounding_emulation():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -3.140625, 1e-3])
    r = vit.round_bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0                          # tie to even
    assert r[2] == 1.0 + 2 ** -6                                # tie to even (odd lower neighbour)
    assert r[3] == -3.140625
    assert torch.tensor(x).to(torch.bfloat16).double().numpy().tolist() == r.tolist()


def e4m3_table():
    """All finite OCP E4M3 values, decoded from the bit fields of the 8-bit codes:
    sign s, exponent e (4 bits, bias 7), mantissa m (3 bits); e = 0 is subnormal
    (m/8 * 2^-6); S.1111.111 is NaN (the only non-finite code)."""
    vals = {}
    for code in range(256):
        s, e, m = code >> 7, (code >> 3) & 15, code & 7
        if e == 15 and m == 7:
            continue
        mag = (m / 8.0) * 2.0 ** -6 if e == 0 else (1.0 + m / 8.0) * 2.0 ** (e - 7)
        vals[code] = -mag if s else mag
    return vals


def test_e4m3_table_facts():
    t = e4m3_table()
    assert len(t) == 254
    pos = sorted({v for v in t.values() if v >= 0})
    assert pos[-1] == 448.0 == vit.E4M3_MAX
    assert pos[1] == 2.0 ** -9                      # smallest subnormal
    assert min(v for v in pos if v >= 2.0 ** -6) == vit.E4M3_MIN_NORMAL


def test_round_e4m3_representables_and_ties():
    """Brute force over the decoded code table: every finite value rounds to itself; every
    midpoint between neighbours rounds to the neighbour with the even mantissa code; points
    just off the midpoint go to the nearer neighbour; beyond 448 saturates."""
    t = e4m3_table()
    vals = np.array(sorted(set(t.values())))
    assert np.array_equal(vit.round_e4m3(vals), vals)
    pos = sorted((v, c) for c, v in t.items() if v > 0 or (v == 0 and c == 0))
    for (lo, clo), (hi, chi) in zip(pos[:-1], pos[1:]):
        mid = 0.5 * (lo + hi)
        even = lo if (clo & 1) == 0 else hi
        assert (chi & 1) != (clo & 1)
        assert vit.round_e4m3(np.array([mid]))[0] == even
        assert vit.round_e4m3(np.array([-mid]))[0] == -even
        eps = (hi - lo) * 1e-6
        assert vit.round_e4m3(np.array([mid - eps]))[0] == lo
        assert vit.round_e4m3(np.array([mid + eps]))[0] == hi
    assert vit.round_e4m3(np.array([449.0, 1e6, -500.0])).tolist() == [448.0, 448.0, -448.0]
    assert vit.round_e4m3(np.array([2.0 ** -11]))[0] == 0.0      # below half the smallest subnormal


def test_round_e4m3_is_nearest():
    """For random inputs within range, no table value is strictly nearer than the result."""
    vals = np.array(sorted(set(e4m3_table().values())))
    x = RNG.standard_normal(2000) * np.exp(RNG.uniform(-8, 6, 2000))
    x = x[np.abs(x) <= 448.0]
    r = vit.round_e4m3(x)
    best = np.min(np.abs(x[:, None] - vals[None, :]), axis=1)
    assert np.all(np.isin(r, vals))
    assert np.allclose(np.abs(x - r), best, rtol=0, atol=0)


def test_quantise_e4m3_scale():
    x = RNG.standard_normal((17, 33)) * 3.0
    q, s = vit.quantise_e4m3(x)
    assert s == np.max(np.abs(x)) / 448.0
    assert np.max(np.abs(q)) == 448.0
    assert np.max(np.abs(q * s - x) / np.maximum(np.abs(x), 2.0 ** -6 * s)) <= 2.0 ** -4 + 1e-12
    assert vit.quantise_e4m3(np.zeros((3, 3)))[1] == 1.0


def test_fp8_mode_only_changes_qkv_and_mlp():
    """In fp8 mode matmul_q differs from the bf16 product by at most the E4M3 rounding of both
    operands (relative 2^-4 each), and the plain matmul is unchanged."""
    a = RNG.standard_normal((40, 64))
    b = RNG.standard_normal((64, 48)) * 0.02
    p8, pb = vit.Prec("fp8"), vit.Prec("bf16")
    assert np.array_equal(p8.matmul(a, b), pb.matmul(a, b))
    ref = a @ b
    sa, sb = np.max(np.abs(a)) / 448.0, np.max(np.abs(b)) / 448.0
    sub = 2.0 ** -10                                 # half the subnormal spacing, in units of the scale
    bound = ((2 * 2.0 ** -4 + 2.0 ** -8) * (np.abs(a) @ np.abs(b))
             + sub * sa * 1.1 * np.abs(b).sum(0)[None, :] + sub * sb * 1.1 * np.abs(a).sum(1)[:, None]
             + sub * sub * sa * sb * a.shape[1] + 1e-12)
    assert np.all(np.abs(p8.matmul_q(a, b) - ref) <= bound)
    assert not np.array_equal(p8.matmul_q(a, b), pb.matmul(a, b))


def test_pow2_row_scale_is_the_smallest_power_of_two_that_fits():
    """e is the least integer with 448 * 2^e >= amax: brute force over exponents, including amax on
    and next to the boundaries 448 * 2^k and the zero row."""
    rng = np.random.default_rng(31)
    amax = np.concatenate([np.exp(rng.uniform(-40, 40, 500)),
                           448.0 * 2.0 ** np.arange(-20, 21, dtype=np.float64),
                           np.nextafter(448.0 * 2.0 ** np.arange(-20, 21, dtype=np.float64), np.inf),
                           np.nextafter(448.0 * 2.0 ** np.arange(-20, 21, dtype=np.float64), 0.0)])
    e = vit.pow2_row_scale(amax)
    for a, ei in zip(amax, e):
        ks = [k for k in range(-200, 200) if 448.0 * 2.0 ** k >= a]
        assert ei == min(ks), (a, ei)
    assert vit.pow2_row_scale(np.array([0.0]))[0] == 0.0


def test_row_quantisation_decodes_within_e4m3_rounding():
    """q * 2^e is x to within half an E4M3 quantum of x / 2^e, every |q| <= 448, and each non-zero row
    reaches its top binade: max |x| / 2^e lies in (224, 448], so after rounding (quantum 16 below 256)
    |q|max lies in [224, 448]."""
    rng = np.random.default_rng(32)
    x = rng.normal(0, 1, (64, 64)) * np.exp(rng.uniform(-8, 8, (64, 1)))
    q, e = vit.quantise_rows_e4m3(x)
    assert np.abs(q).max() <= 448.0
    rowmax = np.abs(q).max(axis=1)
    assert ((rowmax >= 224.0) & (rowmax <= 448.0)).all()
    ratio = np.abs(x).max(axis=1) / 2.0 ** e
    assert ((ratio > 224.0) & (ratio <= 448.0)).all()
    y = x / 2.0 ** e[:, None]
    a = np.maximum(np.abs(y), 2.0 ** -6)
    half_quantum = 2.0 ** (np.floor(np.log2(a)) - 4)
    assert (np.abs(q - y) <= half_quantum + 1e-300).all()


def test_fp8_attention_emulation_against_exact_softmax():
    """The fp8 emulation's scores are q k^T / sqrt(hd) (in base 2) up to the two E4M3 roundings: with
    queries and keys exactly representable after scaling (small integers times a power of two) the
    emulated attention equals the exact one up to the bf16 rounding of P and V."""
    rng = np.random.default_rng(33)
    hd = 64
    c = np.float32(math.log2(math.e) / math.sqrt(hd))
    # queries: integers / c so that q * c (fp32) lands on small integers -> exactly representable
    k = rng.integers(-7, 8, (40, hd)).astype(np.float64)
    v = rng.normal(0, 1, (40, hd))
    qi = rng.integers(-3, 4, (9, hd)).astype(np.float64)
    q = (qi.astype(np.float32) / c).astype(np.float64)
    exactq = (np.asarray(q, np.float32) * c).astype(np.float64)
    assert np.array_equal(exactq, qi) or np.abs(exactq - qi).max() < 1e-6
    got = vit.attention(q, k, v, vit.Prec("fp8"))
    s = (exactq @ k.T)
    p = np.exp2(s - s.max(axis=1, keepdims=True))
    want = (p @ v) / p.sum(axis=1, keepdims=True)
    assert np.abs(got - want).max() < 2e-2 * np.abs(want).max()
