"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *generates inputs*: model configurations (sizes), the fp32
weight blob, uniform pixels and synthetic camera trajectories.  It holds none
of the method's arithmetic (no forward pass, no chaining, no focus projection),
so the CPU oracle and the HIP path can both consume it without sharing code.

Weight blob order (a flat fp32 array, every linear layer stored [in, out] so
that y = x W + b):
    W_p[588, D], b_p[D], c_ref[D], c_other[D]
    per layer l:  ln1.g[D], ln1.b[D], W_qkv[D, 3D], b_qkv[3D], W_o[D, D], b_o[D],
                  ln2.g[D], ln2.b[D], W_1[D, F], b_1[F], W_2[F, D], b_2[D]
    lnf.g[D], lnf.b[D], H_1[D, D], h_1[D], H_2[D, 9], h_2[9]
    with a depth head (ModelConfig.depth_head), appended:
    lnd.g[D], lnd.b[D], W_d[D, 196], b_d[196]
Every entry is N(0, 0.02) drawn in float64 and rounded to fp32; LayerNorm
gains are 1 + N(0, 0.02).  W_qkv columns are q | k | v, each split into heads
of hd contiguous columns.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

PATCH = 14
POSE_DIM = 9


@dataclasses.dataclass(frozen=True)
class ModelConfig:
    depth: int
    dim: int
    heads: int
    mlp: int
    patch: int = PATCH
    depth_head: bool = False      # the blob also carries the per-patch depth head

    @property
    def head_dim(self) -> int:
        return self.dim // self.heads


@dataclasses.dataclass(frozen=True)
class Workload:
    """A synthetic workload: model sizes, frame geometry, window, intrinsics, seeds."""
    name: str
    model: ModelConfig
    frames: int
    height: int
    width: int
    window: int
    overlap: int
    fx: float
    fy: float
    cx: float
    cy: float
    seed_weights: int
    seed_pixels: int
    precision: str

    @property
    def tokens_per_frame(self) -> int:
        return (self.height // PATCH) * (self.width // PATCH) + 1


TINY = Workload("tiny-8x112x112-4L-d128", ModelConfig(4, 128, 4, 512), 8, 112, 112, 8, 4,
                100.0, 100.0, 56.0, 56.0, 0, 1, "fp32")
SMALL = Workload("small-64x280x504-12L-d384-w16s8", ModelConfig(12, 384, 6, 1536), 64, 280, 504,
                 16, 8, 400.0, 400.0, 252.0, 140.0, 0, 2, "bf16")
LARGE = Workload("large-256x378x504-24L-d1024-w32s16", ModelConfig(24, 1024, 16, 4096), 256, 378,
                 504, 32, 16, 500.0, 500.0, 252.0, 189.0, 0, 3, "bf16")
FP8 = Workload("fp8-128x504x896-24L-d1024-w48s24", ModelConfig(24, 1024, 16, 4096), 128, 504, 896,
               48, 24, 600.0, 600.0, 448.0, 252.0, 0, 4, "fp8")
SERVE_MODEL = ModelConfig(24, 1024, 16, 4096)
SERVE_RESOLUTIONS = ((280, 504), (378, 504), (504, 504))

WORKLOADS = {w.name: w for w in (TINY, SMALL, LARGE, FP8)}


def weight_spec(cfg: ModelConfig):
    """Ordered (name, shape) list of the flat weight blob."""
    D, F = cfg.dim, cfg.mlp
    K = 3 * cfg.patch * cfg.patch
    spec = [("W_p", (K, D)), ("b_p", (D,)), ("c_ref", (D,)), ("c_other", (D,))]
    for l in range(cfg.depth):
        p = f"l{l}."
        spec += [(p + "ln1.g", (D,)), (p + "ln1.b", (D,)), (p + "W_qkv", (D, 3 * D)),
                 (p + "b_qkv", (3 * D,)), (p + "W_o", (D, D)), (p + "b_o", (D,)),
                 (p + "ln2.g", (D,)), (p + "ln2.b", (D,)), (p + "W_1", (D, F)), (p + "b_1", (F,)),
                 (p + "W_2", (F, D)), (p + "b_2", (D,))]
    spec += [("lnf.g", (D,)), ("lnf.b", (D,)), ("H_1", (D, D)), ("h_1", (D,)),
             ("H_2", (D, POSE_DIM)), ("h_2", (POSE_DIM,))]
    if cfg.depth_head:
        P2 = cfg.patch * cfg.patch
        spec += [("lnd.g", (D,)), ("lnd.b", (D,)), ("W_d", (D, P2)), ("b_d", (P2,))]
    return spec


def weight_count(cfg: ModelConfig) -> int:
    return sum(int(np.prod(s)) for _, s in weight_spec(cfg))


def make_weights(cfg: ModelConfig, seed: int = 0, std: float = 0.02) -> np.ndarray:
    """Flat fp32 blob: N(0, std) in float64 rounded to fp32; LayerNorm gains 1 + N(0, std)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in weight_spec(cfg):
        w = rng.normal(0.0, std, size=shape)
        if name.endswith(".g"):
            w = 1.0 + w
        parts.append(w.astype(np.float32).ravel())
    return np.concatenate(parts)


def make_frames(n: int, height: int, width: int, seed: int) -> np.ndarray:
    """[n, 3, H, W] fp32 pixels uniform in [0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.random((n, 3, height, width)).astype(np.float32)


def workload_frames(w: Workload, n: int | None = None) -> np.ndarray:
    return make_frames(w.frames if n is None else n, w.height, w.width, w.seed_pixels)


# ----------------------------------------------------------------------------------------------
# Synthetic camera trajectories (world-to-camera 4x4 poses, OpenCV axes: x right, y down,
# z forward; world = the first camera's upright frame, gravity along +y).
# ----------------------------------------------------------------------------------------------

def rot_x(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], dtype=np.float64)


def rot_y(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]], dtype=np.float64)


def rot_z(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], dtype=np.float64)


def pose_from_center(center, R_c2w) -> np.ndarray:
    """World-to-camera pose of a camera at `center` whose camera-to-world rotation is R_c2w."""
    R = np.asarray(R_c2w, dtype=np.float64).T
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = -R @ np.asarray(center, dtype=np.float64)
    return T


@dataclasses.dataclass(frozen=True)
class CameraPath:
    """c(t) = c0 + v t + a t^2 / 2, orientation R_c2w = R_y(yaw0 + yaw(t)) R_x(pitch(t)) R_z(roll0).

    yaw(t) = sway * sin(2 pi f t), pitch(t) = sway * sin(2 pi f t + phase).
    """
    fps: float = 30.0
    velocity: tuple = (0.0, 0.0, 1.5)
    accel: tuple = (0.0, 0.0, 0.0)
    c0: tuple = (0.0, 0.0, 0.0)
    sway_deg: float = 5.0
    sway_hz: float = 2.0
    pitch_phase: float = math.pi / 3
    pitch_sway: bool = True
    yaw0_deg: float = 0.0
    roll0_deg: float = 0.0

    def center(self, i: int) -> np.ndarray:
        t = i / self.fps
        return (np.asarray(self.c0) + np.asarray(self.velocity) * t
                + 0.5 * np.asarray(self.accel) * t * t)

    def angles(self, i: int):
        t = i / self.fps
        w = 2 * math.pi * self.sway_hz * t
        amp = math.radians(self.sway_deg)
        yaw = math.radians(self.yaw0_deg) + amp * math.sin(w)
        pitch = amp * math.sin(w + self.pitch_phase) if self.pitch_sway else 0.0
        return yaw, pitch, math.radians(self.roll0_deg)

    def R_c2w(self, i: int) -> np.ndarray:
        yaw, pitch, roll = self.angles(i)
        return rot_y(yaw) @ rot_x(pitch) @ rot_z(roll)

    def poses(self, n: int) -> np.ndarray:
        """[n, 4, 4] world-to-camera poses."""
        return np.stack([pose_from_center(self.center(i), self.R_c2w(i)) for i in range(n)])


def random_rigid(rng: np.random.Generator, max_angle: float = math.pi, max_t: float = 1.0) -> np.ndarray:
    """A random 4x4 rigid transform (axis-angle rotation, uniform translation)."""
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    ang = rng.uniform(-max_angle, max_angle)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    R = np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * (K @ K)
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = rng.uniform(-max_t, max_t, size=3)
    return T


def serve_streams(n_streams: int, seed: int = 5, min_len: int = 60, max_len: int = 1800,
                  rate: float = 0.4):
    """Stream descriptors for the serving workload: (arrival_s, length, H, W, pixel_seed)."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_streams))
    arrivals -= arrivals[0]
    out = []
    for i in range(n_streams):
        length = int(rng.integers(min_len, max_len + 1))
        H, W = SERVE_RESOLUTIONS[int(rng.integers(0, len(SERVE_RESOLUTIONS)))]
        out.append((float(arrivals[i]), length, H, W, 1000 + i))
    return out
