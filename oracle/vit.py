"""Multi-view ViT pose regressor, FP64 (oracle; test infrastructure only).

The paper takes per-window camera poses from a multi-view foundation model
(Sec. 2.2, Table 2) without describing it.  The network computed here is the
one this project fixes for that stage: patch embedding of ImageNet-normalised
frames with a 2-D sin-cos position code, one camera token per frame (a
reference token for the window's first frame, a shared one for the others),
pre-LN transformer blocks alternating frame-wise attention (even layers) and
global attention over every token of the window (odd layers), an erf-GELU MLP,
and a camera-token head regressing 9 numbers (translation 3, quaternion 4
scalar-last, field of view 2) per frame.

The window forward of Sec. 2.2 predicts depth maps {D_t} beside the poses; the
paper does not describe that head either.  The optional one computed here
(depth_head) is the simplest dense head on the same tokens: a LayerNorm with its
own affine on every patch token of the last block, a linear map to the 14 x 14
pixels of that patch (row-major within the patch), and exp of the result, so a
depth map is positive and in the window's own (local) units.

Options
  precision="fp64"  plain float64 everywhere (the parity reference)
  precision="bf16"  every matmul operand (and the softmax probabilities before
                    the PV product) rounded to bfloat16 RNE, accumulation in
                    float64: an emulation that calibrates how much a bf16 path
                    is expected to deviate; it is not a parity reference.
  precision="fp8"   as "bf16", except that the QKV, fc1 and fc2 products take
                    OCP E4M3 operands: the bf16-rounded activations of the whole
                    window and each weight matrix are divided by their own
                    per-tensor scale amax/448, rounded to E4M3 (nearest even,
                    saturating), and the product is multiplied back by both
                    scales; and the attention scores q k^T take E4M3 operands
                    too: every query row (multiplied by log2(e)/sqrt(hd) in
                    fp32) and every key row of a head is divided by its own
                    power-of-two scale 2^e, e the smallest integer with
                    448 * 2^e >= the row's amax, and rounded to E4M3, so the
                    scores come out in base-2 exponent units; the probabilities
                    and V stay bf16.  Also a calibration, not a parity reference.
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
from scipy.special import erf

IMAGENET_MEAN = np.array([0.485, 0.456, 0.406], dtype=np.float64)
IMAGENET_STD = np.array([0.229, 0.224, 0.225], dtype=np.float64)
LN_EPS = 1e-6


# ----------------------------------------------------------------------------- precision helpers
def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


E4M3_MAX = 448.0          # largest finite OCP E4M3 value, 1.75 * 2^8
E4M3_MIN_NORMAL = 2.0 ** -6
E4M3_MANT_BITS = 3


def round_e4m3(x: np.ndarray) -> np.ndarray:
    """Round to the nearest OCP E4M3 value (ties to even), saturating at +-448; float64 out.

    Normal binade [2^e, 2^(e+1)), e >= -6, has spacing 2^(e-3); below 2^-6 the subnormals have
    the fixed spacing 2^-9."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), E4M3_MAX)
    e = np.floor(np.log2(np.maximum(a, E4M3_MIN_NORMAL)))
    quantum = 2.0 ** (e - E4M3_MANT_BITS)
    r = np.round(a / quantum) * quantum        # numpy rounds halves to even
    return np.copysign(np.minimum(r, E4M3_MAX), x)


def quantise_e4m3(x: np.ndarray) -> tuple[np.ndarray, float]:
    """Per-tensor scaling: s = amax / 448 (1 for an all-zero tensor), q = E4M3(x / s); returns (q, s)."""
    amax = float(np.max(np.abs(x))) if np.size(x) else 0.0
    s = amax / E4M3_MAX if amax > 0.0 else 1.0
    return round_e4m3(np.asarray(x, dtype=np.float64) / s), s


def pow2_row_scale(amax: np.ndarray) -> np.ndarray:
    """Per row: the smallest integer e with 448 * 2^e >= amax (amax > 0), as float64; 0 for a zero row."""
    a = np.asarray(amax, dtype=np.float64)
    e = np.ceil(np.log2(np.where(a > 0, a, E4M3_MAX) / E4M3_MAX))
    # guard the logarithm's last bit: move e to the exact boundary
    e = np.where(E4M3_MAX * 2.0 ** (e - 1) >= a, e - 1, e)
    e = np.where(E4M3_MAX * 2.0 ** e < a, e + 1, e)
    return np.where(a > 0, e, 0.0)


def quantise_rows_e4m3(x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Per-row power-of-two scaling: q = E4M3(x / 2^e) with e = pow2_row_scale(row amax); returns
    (q, e) so that x ~ q * 2^e row by row."""
    x = np.asarray(x, dtype=np.float64)
    e = pow2_row_scale(np.max(np.abs(x), axis=-1))
    return round_e4m3(x / 2.0 ** e[..., None]), e


class Prec:
    def __init__(self, precision: str = "fp64"):
        if precision not in ("fp64", "bf16", "fp8"):
            raise ValueError(precision)
        self.name = precision

    def op(self, x):
        return x if self.name == "fp64" else round_bf16(x)

    def matmul(self, a, b):
        return self.op(a) @ self.op(b)

    def matmul_q(self, a, b):
        """Products that the fp8 mode runs on E4M3 operands (QKV, fc1, fc2)."""
        if self.name != "fp8":
            return self.matmul(a, b)
        qa, sa = quantise_e4m3(round_bf16(a))
        qb, sb = quantise_e4m3(b)
        return (qa @ qb) * (sa * sb)


# ----------------------------------------------------------------------------- weights
def unpack_weights(blob: np.ndarray, depth: int, dim: int, mlp: int, patch: int = 14,
                   depth_head: bool = False) -> dict:
    """Split the flat fp32 blob into named float64 tensors (order of the blob format; with
    depth_head the depth head's lnd_g, lnd_b, W_d [D, patch^2], b_d follow the pose head)."""
    blob = np.asarray(blob, dtype=np.float32).astype(np.float64)
    pos = 0

    def take(*shape):
        nonlocal pos
        n = int(np.prod(shape))
        if pos + n > blob.size:
            raise ValueError("weight blob too short")
        t = blob[pos:pos + n].reshape(shape)
        pos += n
        return t

    D, F = dim, mlp
    w = {"W_p": take(3 * patch * patch, D), "b_p": take(D), "c_ref": take(D), "c_other": take(D),
         "layers": []}
    for _ in range(depth):
        w["layers"].append({
            "ln1_g": take(D), "ln1_b": take(D), "W_qkv": take(D, 3 * D), "b_qkv": take(3 * D),
            "W_o": take(D, D), "b_o": take(D), "ln2_g": take(D), "ln2_b": take(D),
            "W_1": take(D, F), "b_1": take(F), "W_2": take(F, D), "b_2": take(D)})
    w["lnf_g"] = take(D)
    w["lnf_b"] = take(D)
    w["H_1"] = take(D, D)
    w["h_1"] = take(D)
    w["H_2"] = take(D, 9)
    w["h_2"] = take(9)
    if depth_head:
        w["lnd_g"] = take(D)
        w["lnd_b"] = take(D)
        w["W_d"] = take(D, patch * patch)
        w["b_d"] = take(patch * patch)
    if pos != blob.size:
        raise ValueError(f"weight blob has {blob.size - pos} trailing values")
    return w


# ----------------------------------------------------------------------------- building blocks
def normalise(frames: np.ndarray) -> np.ndarray:
    """ImageNet mean/std normalisation of [S,3,H,W] pixels in [0,1)."""
    x = np.asarray(frames, dtype=np.float64)
    return (x - IMAGENET_MEAN[None, :, None, None]) / IMAGENET_STD[None, :, None, None]


def patchify(x: np.ndarray, patch: int = 14) -> np.ndarray:
    """[S,3,H,W] -> [S, (H/p)(W/p), 3 p p]; patches row-major over the grid, each flattened (c, ky, kx)."""
    S, C, H, W = x.shape
    gh, gw = H // patch, W // patch
    if gh * patch != H or gw * patch != W:
        raise ValueError("frame size must be a multiple of the patch size")
    t = x.reshape(S, C, gh, patch, gw, patch).transpose(0, 2, 4, 1, 3, 5)
    return t.reshape(S, gh * gw, C * patch * patch)


def sincos_pe(gh: int, gw: int, dim: int) -> np.ndarray:
    """2-D sin-cos position code [gh*gw, dim]: [sin(y w), cos(y w), sin(x w), cos(x w)],
    w_i = 10000^(-i/(dim/4)), i < dim/4, y = patch row, x = patch column."""
    q = dim // 4
    omega = 10000.0 ** (-np.arange(q, dtype=np.float64) / q)
    ys, xs = np.meshgrid(np.arange(gh, dtype=np.float64), np.arange(gw, dtype=np.float64),
                         indexing="ij")
    y = ys.reshape(-1, 1) * omega[None, :]
    x = xs.reshape(-1, 1) * omega[None, :]
    return np.concatenate([np.sin(y), np.cos(y), np.sin(x), np.cos(x)], axis=1)


def layer_norm(x: np.ndarray, g: np.ndarray, b: np.ndarray, eps: float = LN_EPS) -> np.ndarray:
    mu = x.mean(axis=-1, keepdims=True)
    var = ((x - mu) ** 2).mean(axis=-1, keepdims=True)
    return (x - mu) / np.sqrt(var + eps) * g + b


def gelu(z: np.ndarray) -> np.ndarray:
    """Exact (erf) GELU: z * Phi(z)."""
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def attention(q: np.ndarray, k: np.ndarray, v: np.ndarray, prec: Prec | None = None,
              chunk: int = 1024) -> np.ndarray:
    """softmax(q k^T / sqrt(hd)) v for one head, no mask.  q [Tq,hd], k,v [Tk,hd].

    Queries are processed in chunks so the [Tq, Tk] score matrix is never held whole;
    each query row is still the exact softmax over all keys.
    """
    prec = prec or Prec()
    hd = q.shape[-1]
    scale = 1.0 / math.sqrt(hd)
    vv = prec.op(v)
    out = np.empty((q.shape[0], v.shape[1]), dtype=np.float64)
    if prec.name == "fp8":
        # scores on E4M3 operands with per-row power-of-two scales, in base-2 exponent units
        c = np.float32(math.log2(math.e) / math.sqrt(hd))
        qs = (np.asarray(q, dtype=np.float32) * c).astype(np.float64)
        q8, eq = quantise_rows_e4m3(qs)
        k8, ek = quantise_rows_e4m3(np.asarray(k, dtype=np.float32).astype(np.float64))
        for s in range(0, q.shape[0], chunk):
            sc = (q8[s:s + chunk] @ k8.T) * 2.0 ** (eq[s:s + chunk, None] + ek[None, :])
            sc -= sc.max(axis=1, keepdims=True)
            p = np.exp2(sc)
            l = p.sum(axis=1, keepdims=True)
            out[s:s + chunk] = (prec.op(p) @ vv) / l
        return out
    kk = prec.op(k)
    for s in range(0, q.shape[0], chunk):
        sc = (prec.op(q[s:s + chunk]) @ kk.T) * scale
        sc -= sc.max(axis=1, keepdims=True)
        p = np.exp(sc)
        l = p.sum(axis=1, keepdims=True)
        out[s:s + chunk] = (prec.op(p) @ vv) / l
    return out


def multihead(xn: np.ndarray, lw: dict, heads: int, groups: list, prec: Prec,
              workers: int = 1) -> np.ndarray:
    """Self-attention of the LayerNormed tokens xn [T, D] within each token group.

    groups: list of (start, length) token ranges; tokens attend only inside their group.
    Returns the output projection O W_o + b_o [T, D].
    workers > 1 computes the heads on that many threads (the heads are independent and each
    writes its own columns of O, so the values are the same as with one worker; NumPy releases
    the interpreter lock inside its array loops, which is what makes the threads run at once).
    """
    T, D = xn.shape
    hd = D // heads
    qkv = prec.matmul_q(xn, lw["W_qkv"]) + lw["b_qkv"]
    q, k, v = qkv[:, :D], qkv[:, D:2 * D], qkv[:, 2 * D:]
    o = np.empty((T, D), dtype=np.float64)

    def one_head(h):
        c = slice(h * hd, (h + 1) * hd)
        for (s, n) in groups:
            o[s:s + n, c] = attention(q[s:s + n, c], k[s:s + n, c], v[s:s + n, c], prec)

    if workers > 1:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(one_head, range(heads)))
    else:
        for h in range(heads):
            one_head(h)
    return prec.matmul(o, lw["W_o"]) + lw["b_o"]


def block(x: np.ndarray, lw: dict, heads: int, groups: list, prec: Prec, workers: int = 1) -> np.ndarray:
    """One pre-LN transformer block: X += Attn(LN1 X); X += W2 GELU(W1 LN2 X)."""
    x = x + multihead(layer_norm(x, lw["ln1_g"], lw["ln1_b"]), lw, heads, groups, prec, workers)
    h = gelu(prec.matmul_q(layer_norm(x, lw["ln2_g"], lw["ln2_b"]), lw["W_1"]) + lw["b_1"])
    return x + prec.matmul_q(h, lw["W_2"]) + lw["b_2"]


def embed(frames: np.ndarray, w: dict, patch: int = 14, prec: Prec | None = None) -> np.ndarray:
    """Window tokens [S*n, D]: per frame a camera token followed by its patch tokens."""
    prec = prec or Prec()
    S, _, H, W = frames.shape
    gh, gw = H // patch, W // patch
    D = w["W_p"].shape[1]
    pt = prec.matmul(patchify(normalise(frames), patch), w["W_p"]) + w["b_p"]  # [S, P, D]
    pt = pt + sincos_pe(gh, gw, D)[None]
    cam = np.stack([w["c_ref"] if f == 0 else w["c_other"] for f in range(S)])[:, None, :]
    return np.concatenate([cam, pt], axis=1).reshape(S * (gh * gw + 1), D)


def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrix of a scalar-last quaternion (x, y, z, w) after normalisation
    (Hamilton convention); the identity when |q| < 1e-12."""
    n = float(np.linalg.norm(q))
    if n < 1e-12:
        return np.eye(3)
    x, y, z, w_ = (np.asarray(q, dtype=np.float64) / n)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w_), 2 * (x * z + y * w_)],
        [2 * (x * y + z * w_), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w_)],
        [2 * (x * z - y * w_), 2 * (y * z + x * w_), 1 - 2 * (x * x + y * y)]])


def pose_head(cam_tokens: np.ndarray, w: dict) -> np.ndarray:
    """Final LN of the camera tokens, Linear-GELU-Linear -> [S, 9] = (t3, quat4 xyzw, fov2).

    The head stays in float64 in both oracle precisions (the path keeps it fp32)."""
    z = layer_norm(cam_tokens, w["lnf_g"], w["lnf_b"])
    return gelu(z @ w["H_1"] + w["h_1"]) @ w["H_2"] + w["h_2"]


def depth_head(tokens: np.ndarray, w: dict, S: int, height: int, width: int, patch: int = 14,
               prec: Prec | None = None) -> np.ndarray:
    """Depth maps [S, H, W] of a window from its last-block tokens [S*n, D]: every patch token
    (not the camera token) goes through LN(lnd) and W_d, b_d to patch*patch values, exp'd, that
    fill the patch's pixels row by row: pixel (py*patch + ky, px*patch + kx) of frame f takes
    output ky*patch + kx of patch (py, px)."""
    prec = prec or Prec()
    gh, gw = height // patch, width // patch
    n = gh * gw + 1
    D = tokens.shape[1]
    x = tokens.reshape(S, n, D)[:, 1:, :]
    z = prec.matmul(layer_norm(x, w["lnd_g"], w["lnd_b"]), w["W_d"]) + w["b_d"]   # [S, P, patch^2]
    d = np.exp(z).reshape(S, gh, gw, patch, patch)
    return d.transpose(0, 1, 3, 2, 4).reshape(S, gh * patch, gw * patch)


def pose9_to_T(p9: np.ndarray) -> np.ndarray:
    """World-to-camera 4x4 [R(q) | t] from one 9-vector."""
    T = np.eye(4)
    T[:3, :3] = quat_to_rot(p9[3:7])
    T[:3, 3] = p9[0:3]
    return T


def forward_window(frames: np.ndarray, w: dict, heads: int, patch: int = 14,
                   precision: str = "fp64", return_tokens: bool = False, workers: int = 1,
                   depth: bool = False):
    """Pose regression for one window of S frames [S,3,H,W] -> pose9 [S, 9].

    Even layers attend within each frame (n = P+1 tokens), odd layers over all S*n tokens.
    workers: threads over the attention heads (same values for any count).
    depth: also return the window's depth maps [S, H, W] (depth_head): (p9, depth[, tokens]).
    """
    prec = Prec(precision)
    S, _, H, W = frames.shape
    n = (H // patch) * (W // patch) + 1
    x = embed(frames, w, patch, prec)
    frame_groups = [(f * n, n) for f in range(S)]
    window_group = [(0, S * n)]
    for l, lw in enumerate(w["layers"]):
        x = block(x, lw, heads, frame_groups if l % 2 == 0 else window_group, prec, workers)
    p9 = pose_head(x[0::n], w)
    out = (p9,)
    if depth:
        out += (depth_head(x, w, S, H, W, patch, prec),)
    if return_tokens:
        out += (x,)
    return out if len(out) > 1 else p9
