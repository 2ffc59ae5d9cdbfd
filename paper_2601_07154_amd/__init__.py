"""MI355X-native motion-focus recognition (arXiv 2601.07154): Python binding of libmfocus.so.

Thin wrappers with the C ABI's names and semantics (include/mf.h, include/mf_ops.h): the
arithmetic of every stage runs in the library's HIP kernels.  Host arrays are numpy; device
arrays are torch tensors (their data_ptr is passed with MF_DEVICE_PTR).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (FOCUS_DTYPE, MF_ANCHOR_SE3, MF_ANCHOR_YAW, MF_ANCHOR_YAW_SCALE, MF_FOCUS_ACCEL,
                   MF_FOCUS_VELOCITY, MF_BF16, MF_DEVICE_PTR, MF_EAGAIN, MF_ECLOSED,
                   MF_EOS, MF_FP32, MF_MAP_MAX, MF_MAP_SUM, MF_OK, MF_POSES_LOCAL)

PRECISIONS = {"fp32": MF_FP32, "bf16": MF_BF16, "fp8": _lib.MF_FP8}


class MfError(RuntimeError):
    def __init__(self, status: int, where: str, lib=None):
        lib = lib or _lib.lib()
        msg = lib.mf_last_error().decode(errors="replace")
        super().__init__(f"{where}: {lib.mf_status_str(status).decode()} ({status}): {msg}")
        self.status = status


def _check(status: int, where: str, ok=(MF_OK,), lib=None):
    if status not in ok:
        raise MfError(status, where, lib)
    return status


def _ptr(x):
    """(pointer, is_device) of a numpy array or torch tensor."""
    if hasattr(x, "data_ptr") and hasattr(x, "is_cuda"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(x.data_ptr()), bool(x.is_cuda)
    if not x.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return C.c_void_p(x.ctypes.data), False


def rows_per_frame(height: int, width: int) -> int:
    return _lib.lib().mf_rows_per_frame(height, width)


class _TorchAllocator:
    """Device buffers for the engine from torch's caching allocator (uint8 tensors kept alive by
    address until the engine hands them back)."""

    def __init__(self, device: int):
        import threading

        import torch
        self.torch, self.device, self.live, self.lock = torch, device, {}, threading.Lock()
        self.c_alloc = _lib.DEV_ALLOC(self._alloc)
        self.c_free = _lib.DEV_FREE(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            t = self.torch.empty(max(int(nbytes), 1), dtype=self.torch.uint8, device=f"cuda:{self.device}")
        except RuntimeError:
            return None
        with self.lock:
            self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, ptr, ctx):
        with self.lock:
            self.live.pop(ptr, None)


class Engine:
    """mf_engine: weights on the device, batch workspace, optional scheduler thread."""

    def __init__(self, depth: int, dim: int, heads: int, mlp: int, weights: np.ndarray,
                 precision: str = "bf16", threaded: bool = False, max_tokens: int = 0,
                 hbm_budget: int = 0, device: int = 0, stream: int | None = None, graphs: bool = True,
                 allocator: str | None = None, depth_head: bool = False, lib=None):
        """allocator="torch": the engine's device memory comes from torch's caching allocator.
        depth_head: the weight blob also carries the depth head (streams may emit depth maps)."""
        self.lib = lib or _lib.lib()
        w = np.ascontiguousarray(weights, dtype=np.float32)
        m = _lib.ModelCfg(depth, dim, heads, mlp, 14, PRECISIONS[precision], 1 if depth_head else 0)
        rt = _lib.RuntimeCfg(device, 1 if threaded else 0, max_tokens, hbm_budget,
                             C.c_void_p(stream) if stream else None, 1 if graphs else 0, 0)
        self._alloc = None
        if allocator == "torch":
            self._alloc = _TorchAllocator(device)
            rt.dev_alloc, rt.dev_free = self._alloc.c_alloc, self._alloc.c_free
        elif allocator is not None:
            raise ValueError(f"unknown allocator {allocator!r}")
        h = C.c_void_p()
        _check(self.lib.mf_engine_create(C.byref(m), C.c_void_p(w.ctypes.data), w.size, C.byref(rt),
                                         C.byref(h)), "mf_engine_create", lib=self.lib)
        self.h = h
        self.dim = dim
        self.precision = precision
        self.threaded = threaded

    @classmethod
    def from_model(cls, model, weights, **kw):
        return cls(model.depth, model.dim, model.heads, model.mlp, weights,
                   depth_head=getattr(model, "depth_head", False), **kw)

    def close(self):
        if getattr(self, "h", None):
            self.lib.mf_engine_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---------------------------------------------------------------- streams
    def open_stream(self, height: int, width: int, window: int, overlap: int, K, n_points: int = 15,
                    sigma: float = 1.0, sigma_min: float = 0.0, sigma_max: float = 0.0,
                    anchor_mode: int = MF_ANCHOR_YAW, emit_maps: bool = True, ring_frames: int = 0,
                    result_frames: int = 0, allow_again: bool = False, focus_mode: int = 0,
                    diff_stride: int = 1, map_mode: int = MF_MAP_MAX, emit_depth: bool = False) -> int:
        fx, fy, cx, cy = K
        c = _lib.StreamCfg(height, width, window, overlap, fx, fy, cx, cy, n_points, anchor_mode, sigma,
                           sigma_min, sigma_max, 1 if emit_maps else 0, ring_frames, result_frames, focus_mode,
                           diff_stride, map_mode, 1 if emit_depth else 0)
        sid = C.c_int32()
        st = self.lib.mf_open_stream(self.h, C.byref(c), C.byref(sid))
        if allow_again and st == MF_EAGAIN:
            return -1
        _check(st, "mf_open_stream", lib=self.lib)
        return sid.value

    def push_frames(self, sid: int, frames, eos: bool = False, allow_again: bool = False) -> int:
        n = int(frames.shape[0]) if frames is not None else 0
        if frames is None:
            p, dev = None, False
        else:
            if str(getattr(frames, "dtype", "")) not in ("float32", "torch.float32"):
                raise ValueError("frames must be float32")
            p, dev = _ptr(frames)
        flags = (MF_EOS if eos else 0) | (MF_DEVICE_PTR if dev else 0)
        st = self.lib.mf_push_frames(self.h, sid, p, n, flags)
        return _check(st, "mf_push_frames", (MF_OK, MF_EAGAIN) if allow_again else (MF_OK,), lib=self.lib)

    def push_poses(self, sid: int, T, first_frame: int, local: bool = False, eos: bool = False) -> int:
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(-1, 16)
        flags = (MF_EOS if eos else 0) | (MF_POSES_LOCAL if local else 0)
        return _check(self.lib.mf_push_poses(self.h, sid, C.c_void_p(T.ctypes.data), T.shape[0], first_frame,
                                             flags), "mf_push_poses", lib=self.lib)

    def close_stream(self, sid: int):
        _check(self.lib.mf_close_stream(self.h, sid), "mf_close_stream", lib=self.lib)

    def poll(self, sid: int, cap: int = 4096, maps=None, depth=None):
        """Returns (records [n] FOCUS_DTYPE, status) with status MF_OK, MF_EAGAIN or MF_ECLOSED.
        maps / depth (optional): [cap][H][W] float32, both host or both device."""
        out = np.zeros(cap, dtype=FOCUS_DTYPE)
        n = C.c_int32()
        mp, mdev = (None, False) if maps is None else _ptr(maps)
        if depth is None:
            st = self.lib.mf_poll_focus(self.h, sid, C.c_void_p(out.ctypes.data), cap, C.byref(n), mp,
                                        MF_DEVICE_PTR if mdev else 0)
            _check(st, "mf_poll_focus", (MF_OK, MF_EAGAIN, MF_ECLOSED), lib=self.lib)
        else:
            dp, ddev = _ptr(depth)
            if maps is not None and mdev != ddev:
                raise ValueError("maps and depth must both be host or both device memory")
            st = self.lib.mf_poll_focus_depth(self.h, sid, C.c_void_p(out.ctypes.data), cap, C.byref(n), mp, dp,
                                              MF_DEVICE_PTR if ddev else 0)
            _check(st, "mf_poll_focus_depth", (MF_OK, MF_EAGAIN, MF_ECLOSED), lib=self.lib)
        return out[:n.value].copy(), st

    def step(self) -> int:
        n = C.c_int32()
        _check(self.lib.mf_engine_step(self.h, C.byref(n)), "mf_engine_step", lib=self.lib)
        return n.value

    def sync(self):
        _check(self.lib.mf_engine_sync(self.h), "mf_engine_sync", lib=self.lib)

    def stats(self) -> dict:
        s = _lib.Stats()
        _check(self.lib.mf_engine_stats(self.h, C.byref(s)), "mf_engine_stats", lib=self.lib)
        return {f: getattr(s, f) for f, _ in _lib.Stats._fields_}

    # ---------------------------------------------------------------- op level
    def forward_window(self, frames_dev, max_layers: int = -1, want_tokens: bool = False):
        """frames_dev: torch float32 cuda tensor [S,3,H,W].  Returns (pose9, T, tokens|None)."""
        S, _, H, W = frames_dev.shape
        p, dev = _ptr(frames_dev)
        if not dev:
            raise ValueError("frames must be in device memory")
        pose9 = np.zeros((S, 9), np.float32)
        T = np.zeros((S, 4, 4), np.float64)
        tok = np.zeros((S * rows_per_frame(H, W), self.dim), np.float32) if want_tokens else None
        _check(self.lib.mf_forward_window(self.h, p, S, H, W, max_layers, C.c_void_p(pose9.ctypes.data),
                                          C.c_void_p(T.ctypes.data),
                                          C.c_void_p(tok.ctypes.data) if tok is not None else None),
               "mf_forward_window", lib=self.lib)
        return pose9, T, tok

    def debug_copy(self, which: int, shape, dtype) -> np.ndarray:
        out = np.zeros(shape, dtype=dtype)
        _check(self.lib.mf_debug_copy(self.h, which, C.c_void_p(out.ctypes.data), out.nbytes), "mf_debug_copy", lib=self.lib)
        return out

    def profile(self, enable: int = -1) -> dict:
        ag, af, gm = C.c_double(), C.c_double(), C.c_double()
        calls = C.c_int64()
        _check(self.lib.mf_profile(self.h, enable, C.byref(ag), C.byref(calls), C.byref(af), C.byref(gm)),
               "mf_profile", lib=self.lib)
        return dict(attn_global_ms=ag.value, attn_global_calls=calls.value, attn_frame_ms=af.value,
                    gemm_ms=gm.value)

    def profile_stages(self) -> dict:
        """Per-stage sums of the current timing: {stage: (ms, launches)} (stage names in _lib.STAGES)."""
        n = len(_lib.STAGES)
        ms = np.zeros(n, np.float64)
        calls = np.zeros(n, np.int64)
        _check(self.lib.mf_profile_stages(self.h, C.c_void_p(ms.ctypes.data), C.c_void_p(calls.ctypes.data), n),
               "mf_profile_stages", lib=self.lib)
        return {name: (float(ms[k]), int(calls[k])) for k, name in enumerate(_lib.STAGES)}


def op_attention(precision: str, head_dim: int, heads: int, dim: int, q, k, vt, o, mpad: int, segs,
                 stream: int = 0):
    s = np.ascontiguousarray(segs, dtype=np.int32).reshape(-1, 4)
    lib = _lib.lib()
    _check(lib.mf_op_attention(PRECISIONS[precision], head_dim, heads, dim, _ptr(q)[0], _ptr(k)[0], _ptr(vt)[0],
                               _ptr(o)[0], mpad, C.c_void_p(s.ctypes.data), s.shape[0], C.c_void_p(stream)),
           "mf_op_attention")


def op_gemm(precision: str, A, Bt, bias, Cout, stream: int = 0):
    M, K = A.shape
    N = Bt.shape[0]
    lib = _lib.lib()
    _check(lib.mf_op_gemm(PRECISIONS[precision], _ptr(A)[0], _ptr(Bt)[0],
                          _ptr(bias)[0] if bias is not None else None, _ptr(Cout)[0], M, N, K,
                          C.c_void_p(stream)), "mf_op_gemm")


def op_layernorm(precision: str, x, y, g, b, stream: int = 0):
    rows, dim = x.shape
    lib = _lib.lib()
    _check(lib.mf_op_layernorm(PRECISIONS[precision], _ptr(x)[0], _ptr(y)[0], _ptr(g)[0], _ptr(b)[0], rows, dim,
                               C.c_void_p(stream)), "mf_op_layernorm")


def op_gemm_fp8(A8, Bt8, ascale, bscale, bias, Cout, stream: int = 0):
    """A8 [M][K], Bt8 [N][K]: uint8 tensors of E4M3 bytes; ascale [M], bscale [1] float32 (device)."""
    M, K = A8.shape
    N = Bt8.shape[0]
    lib = _lib.lib()
    _check(lib.mf_op_gemm_fp8(_ptr(A8)[0], _ptr(Bt8)[0], _ptr(ascale)[0], _ptr(bscale)[0],
                              _ptr(bias)[0] if bias is not None else None, _ptr(Cout)[0], M, N, K,
                              C.c_void_p(stream)), "mf_op_gemm_fp8")


def op_quantize_fp8(x, scale: float, q, stream: int = 0):
    lib = _lib.lib()
    _check(lib.mf_op_quantize_fp8(_ptr(x)[0], x.numel(), scale, _ptr(q)[0], C.c_void_p(stream)),
           "mf_op_quantize_fp8")


def op_quantize_fp8_windows(y, segs, q, srow, stream: int = 0):
    """y [rows][C] bfloat16 (device); segs [nwin][4] {base, nf, n, npad}; q uint8 [rows][C], srow float32 [rows]."""
    s = np.ascontiguousarray(segs, dtype=np.int32).reshape(-1, 4)
    lib = _lib.lib()
    _check(lib.mf_op_quantize_fp8_windows(_ptr(y)[0], y.shape[1], C.c_void_p(s.ctypes.data), s.shape[0], _ptr(q)[0],
                                          _ptr(srow)[0], C.c_void_p(stream)), "mf_op_quantize_fp8_windows")


def op_quantize_fp8_windows_noalloc(y, segs, q, srow, stream: int = 0):
    """As op_quantize_fp8_windows, through the entry point that allocates no device memory (its
    window table and amax counters sit in the library's static per-GPU array)."""
    s = np.ascontiguousarray(segs, dtype=np.int32).reshape(-1, 4)
    lib = _lib.lib()
    _check(lib.mf_op_quantize_fp8_windows_noalloc(_ptr(y)[0], y.shape[1], C.c_void_p(s.ctypes.data), s.shape[0],
                                                  _ptr(q)[0], _ptr(srow)[0], C.c_void_p(stream)),
           "mf_op_quantize_fp8_windows_noalloc")


def op_attention_fp8(heads: int, dim: int, q8, qe, k8, ke, vt, o, mpad: int, segs, stream: int = 0):
    """Attention with E4M3 scores: q8/k8 uint8 [heads][mpad][64], qe/ke uint8 [heads][mpad] (E8M0 exponents),
    vt bfloat16 [heads][64][mpad], o bfloat16 [rows][dim] (device tensors); segs [nseg][4]."""
    s = np.ascontiguousarray(segs, dtype=np.int32).reshape(-1, 4)
    lib = _lib.lib()
    _check(lib.mf_op_attention_fp8(heads, dim, _ptr(q8)[0], _ptr(qe)[0], _ptr(k8)[0], _ptr(ke)[0], _ptr(vt)[0],
                                   _ptr(o)[0], mpad, C.c_void_p(s.ctypes.data), s.shape[0], C.c_void_p(stream)),
           "mf_op_attention_fp8")
