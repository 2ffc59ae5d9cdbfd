"""Helpers of the GPU parity tests: device access, the library handle, error measures."""
import math
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def mf():
    """The library binding; fails loudly when the library is missing (no fallback)."""
    import paper_2601_07154_amd as m
    m._lib.lib()
    return m


def rot_err_deg(R1, R2):
    """Angle of R1^T R2 in degrees, 2 asin(|R1 - R2|_F / sqrt 8): well conditioned near 0."""
    d = np.linalg.norm(np.asarray(R1) - np.asarray(R2), axis=(-2, -1)) / math.sqrt(8.0)
    return np.degrees(2.0 * np.arcsin(np.minimum(1.0, d)))


def dir_err_deg(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    na, nb = np.linalg.norm(a, axis=-1), np.linalg.norm(b, axis=-1)
    c = np.sum(a * b, axis=-1) / np.maximum(na * nb, 1e-300)
    s = np.linalg.norm(np.cross(a, b), axis=-1) / np.maximum(na * nb, 1e-300)
    return np.degrees(np.arctan2(s, c))


def round_bf16(x):
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)
