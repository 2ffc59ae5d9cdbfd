"""Kernel-level parity: MFMA GEMM, segment flash attention and LayerNorm against the oracle
(or exact integer arithmetic), through the C ABI op entry points."""
import numpy as np
import pytest

from gpu_util import mf, round_bf16, torch_cuda
from oracle import vit

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
# (16400, 1024, 256): enough tiles for the 256 x 128 tile of the bf16 path, with a ragged last row block
@pytest.mark.parametrize("M,N,K", [(300, 256, 256), (1, 128, 640), (517, 384, 1536), (16400, 1024, 256)])
def test_gemm_small_integers_bit_exact(prec, M, N, K):
    torch = torch_cuda()
    m = mf()
    rng = np.random.default_rng(M + N + K)
    A = rng.integers(-3, 4, size=(M, K)).astype(np.float32)
    B = rng.integers(-3, 4, size=(N, K)).astype(np.float32)
    bias = rng.integers(-5, 6, size=N).astype(np.float32)
    # integer-valued float64 products and sums (|sum| <= 9 K + 5 < 2^53): exact
    ref = A.astype(np.float64) @ B.astype(np.float64).T + bias.astype(np.float64)
    tdt = torch.bfloat16 if prec == "bf16" else torch.float32
    dA = torch.from_numpy(A).to("cuda", tdt).contiguous()
    dB = torch.from_numpy(B).to("cuda", tdt).contiguous()
    db = torch.from_numpy(bias).cuda()
    dC = torch.full((M, N), 7.0, device="cuda")
    m.op_gemm(prec, dA, dB, db, dC)
    got = dC.cpu().numpy().astype(np.float64)
    assert np.array_equal(got, ref)


def _attn_case(torch, prec, hd, heads, frames, n, seed):
    """Random Q, K, V in the library layouts plus the per-segment oracle."""
    rng = np.random.default_rng(seed)
    npad = (n + 7) // 8 * 8
    D = hd * heads
    rows = frames * npad
    mpad = rows + 256 + 64
    q = rng.normal(size=(heads, mpad, hd)).astype(np.float32)
    k = rng.normal(size=(heads, mpad, hd)).astype(np.float32)
    v = rng.normal(size=(heads, mpad, hd)).astype(np.float32)
    if prec == "bf16":
        q, k, v = round_bf16(q), round_bf16(k), round_bf16(v)
    tdt = torch.bfloat16 if prec == "bf16" else torch.float32
    dq = torch.from_numpy(q).to("cuda", tdt).contiguous()
    dk = torch.from_numpy(k).to("cuda", tdt).contiguous()
    dvt = torch.from_numpy(np.ascontiguousarray(v.transpose(0, 2, 1))).to("cuda", tdt).contiguous()
    do = torch.zeros((mpad, D), device="cuda", dtype=tdt)
    return q.astype(np.float64), k.astype(np.float64), v.astype(np.float64), dq, dk, dvt, do, npad, mpad


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-5), ("bf16", 1.5e-2)])
@pytest.mark.parametrize("hd,heads", [(64, 2), (32, 3)])
@pytest.mark.parametrize("n", [65, 145, 200])
def test_attention_framewise_and_global(prec, tol, hd, heads, n):
    torch = torch_cuda()
    m = mf()
    frames = 3
    q, k, v, dq, dk, dvt, do, npad, mpad = _attn_case(torch, prec, hd, heads, frames, n, n + hd)
    D = hd * heads
    # frame-wise: one segment per frame
    segs = [[f * npad, 1, n, npad] for f in range(frames)]
    m.op_attention(prec, hd, heads, D, dq, dk, dvt, do, mpad, segs)
    got = do.float().cpu().numpy()
    for f in range(frames):
        r = slice(f * npad, f * npad + n)
        for h in range(heads):
            ref = vit.attention(q[h, r], k[h, r], v[h, r])
            np.testing.assert_allclose(got[r, h * hd:(h + 1) * hd], ref, atol=tol, rtol=tol)
    # global: one segment over all frames, padding rows masked
    do.zero_()
    m.op_attention(prec, hd, heads, D, dq, dk, dvt, do, mpad, [[0, frames, n, npad]])
    got = do.float().cpu().numpy()
    valid = np.concatenate([np.arange(f * npad, f * npad + n) for f in range(frames)])
    for h in range(heads):
        ref = vit.attention(q[h, valid], k[h, valid], v[h, valid])
        np.testing.assert_allclose(got[valid, h * hd:(h + 1) * hd], ref, atol=tol, rtol=tol)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 1e-2)])
def test_attention_rows_sum_to_one(prec, tol):
    """V = 1: every output is 1 (the softmax rows sum to one), with large score ranges.

    fp32: the normaliser and the PV product sum the same ~600 fp32 probabilities in different
    orders, each exp2 within a few ulp: |O - 1| <= ~600 * 2^-24 * few < 1e-5.  bf16: P is rounded
    to bf16 (2^-9 relative) before the PV product while the normaliser is not."""
    torch = torch_cuda()
    m = mf()
    hd, heads, frames, n = 64, 2, 2, 300
    q, k, v, dq, dk, dvt, do, npad, mpad = _attn_case(torch, prec, hd, heads, frames, n, 3)
    dq.mul_(4.0)
    dvt.fill_(1.0)
    m.op_attention(prec, hd, heads, hd * heads, dq, dk, dvt, do, mpad, [[0, frames, n, npad]])
    got = do.float().cpu().numpy()
    valid = np.concatenate([np.arange(f * npad, f * npad + n) for f in range(frames)])
    np.testing.assert_allclose(got[valid], 1.0, atol=tol)


def _scored_case(torch, prec, kind, hd=64, heads=2, frames=3, n=300, seed=21):
    """Q, K whose scores follow a chosen pattern along the keys of a 3-frame segment, V random.

    growing:  scores rise ~0.23 log2 units per key (200+ over the segment), so the reference
              maximum must be raised many times after the first step;
    falling:  the same, decreasing (the first step holds the maximum, later probabilities vanish);
    negative: every score near -200 log2 units (the reference must come from the first step's
              maximum, not from 0, or every probability underflows);
    spike:    random scores plus one key per frame 40 log2 units above the rest, late in the frame."""
    rng = np.random.default_rng(seed)
    npad = (n + 7) // 8 * 8
    mpad = frames * npad + 256 + 64
    q = np.zeros((heads, mpad, hd), np.float32)
    k = np.zeros((heads, mpad, hd), np.float32)
    v = rng.normal(size=(heads, mpad, hd)).astype(np.float32)
    rows = np.concatenate([np.arange(f * npad, f * npad + n) for f in range(frames)])
    j = np.arange(len(rows), dtype=np.float32)
    if kind in ("growing", "falling"):
        a = 0.02 * (j if kind == "growing" else j[::-1])
        q[:, rows] = 1.0 + 0.1 * rng.normal(size=(heads, len(rows), hd))
        k[:, rows] = a[None, :, None] + 0.1 * rng.normal(size=(heads, len(rows), hd))
    elif kind == "negative":
        q[:, rows] = 4.16 + 0.05 * rng.normal(size=(heads, len(rows), hd))
        k[:, rows] = -4.16 + 0.3 * rng.normal(size=(heads, len(rows), hd))
    else:
        q[:, rows] = rng.normal(size=(heads, len(rows), hd))
        k[:, rows] = rng.normal(size=(heads, len(rows), hd))
        for f in range(frames):
            r = f * npad + n - 5
            k[:, r] = q[:, f * npad] * 0.0 + 3.0 * np.sign(q[:, f * npad + 1])
    if prec == "bf16":
        q, k, v = round_bf16(q), round_bf16(k), round_bf16(v)
    tdt = torch.bfloat16 if prec == "bf16" else torch.float32
    dq = torch.from_numpy(q).to("cuda", tdt).contiguous()
    dk = torch.from_numpy(k).to("cuda", tdt).contiguous()
    dvt = torch.from_numpy(np.ascontiguousarray(v.transpose(0, 2, 1))).to("cuda", tdt).contiguous()
    do = torch.zeros((mpad, hd * heads), device="cuda", dtype=tdt)
    return (q.astype(np.float64), k.astype(np.float64), v.astype(np.float64), dq, dk, dvt, do, npad, mpad, rows)


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-5), ("bf16", 2e-2)])
@pytest.mark.parametrize("kind", ["growing", "falling", "negative", "spike"])
def test_attention_score_ranges(prec, tol, kind):
    """The reference-maximum logic of the softmax (set on a query's first key step, raised when a
    step's probabilities grow large) against the FP64 oracle, on score patterns that exercise it;
    frame-wise and global segments.  Errors are relative to max |V|."""
    torch = torch_cuda()
    m = mf()
    hd, heads, frames, n = 64, 2, 3, 300
    q, k, v, dq, dk, dvt, do, npad, mpad, rows = _scored_case(torch, prec, kind, hd, heads, frames, n)
    s_max = max(np.abs(q[h, rows] @ k[h, rows].T).max() for h in range(heads)) / np.sqrt(hd) * np.log2(np.e)
    print(f"{kind}: max |score| {s_max:.0f} log2 units")
    vmax = np.abs(v).max()
    m.op_attention(prec, hd, heads, hd * heads, dq, dk, dvt, do, mpad, [[0, frames, n, npad]])
    got = do.float().cpu().numpy()
    assert np.isfinite(got[rows]).all()
    for h in range(heads):
        ref = vit.attention(q[h, rows], k[h, rows], v[h, rows])
        err = np.abs(got[rows, h * hd:(h + 1) * hd] - ref).max() / vmax
        assert err < tol, (kind, h, err)
    do.zero_()
    segs = [[f * npad, 1, n, npad] for f in range(frames)]
    m.op_attention(prec, hd, heads, hd * heads, dq, dk, dvt, do, mpad, segs)
    got = do.float().cpu().numpy()
    for f in range(frames):
        r = slice(f * npad, f * npad + n)
        for h in range(heads):
            ref = vit.attention(q[h, r], k[h, r], v[h, r])
            err = np.abs(got[r, h * hd:(h + 1) * hd] - ref).max() / vmax
            assert err < tol, (kind, "frame", f, h, err)


@pytest.mark.parametrize("prec,tol", [("fp32", 3e-6), ("bf16", 1e-2)])
@pytest.mark.parametrize("dim", [128, 384, 1024])
def test_layernorm(prec, tol, dim):
    torch = torch_cuda()
    m = mf()
    rng = np.random.default_rng(dim)
    x = (rng.normal(size=(333, dim)) * 3 + 1).astype(np.float32)
    g = (1 + 0.1 * rng.normal(size=dim)).astype(np.float32)
    b = (0.1 * rng.normal(size=dim)).astype(np.float32)
    dx, dg, db = (torch.from_numpy(a).cuda() for a in (x, g, b))
    dy = torch.zeros((333, dim), device="cuda", dtype=torch.bfloat16 if prec == "bf16" else torch.float32)
    m.op_layernorm(prec, dx, dy, dg, db)
    ref = vit.layer_norm(x.astype(np.float64), g, b)
    np.testing.assert_allclose(dy.float().cpu().numpy(), ref, atol=tol, rtol=tol)
