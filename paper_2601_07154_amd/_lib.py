"""ctypes binding of libmfocus.so (argument marshalling only; every step runs in the library).

The library is loaded from this package's directory; a missing library is an error, never a
silent fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfocus.so")

MF_OK, MF_EINVAL, MF_ENOMEM, MF_EAGAIN, MF_ECLOSED, MF_EDEVICE, MF_ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
MF_FP32, MF_BF16, MF_FP8 = 0, 1, 2
MF_ANCHOR_YAW, MF_ANCHOR_SE3, MF_ANCHOR_YAW_SCALE = 0, 1, 2
MF_FOCUS_ACCEL, MF_FOCUS_VELOCITY = 0, 1
MF_EOS, MF_DEVICE_PTR, MF_POSES_LOCAL = 1, 2, 4
MF_MAP_MAX, MF_MAP_SUM = 0, 1
STAGES = ("attn_global", "attn_frame", "qkv", "out_proj", "fc1", "fc2", "patch", "layernorm", "quant_fp8", "head")


class ModelCfg(C.Structure):
    _fields_ = [("depth", C.c_int32), ("dim", C.c_int32), ("heads", C.c_int32), ("mlp", C.c_int32),
                ("patch", C.c_int32), ("precision", C.c_int32), ("depth_head", C.c_int32)]


DEV_ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEV_FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class RuntimeCfg(C.Structure):
    _fields_ = [("device", C.c_int32), ("threaded", C.c_int32), ("max_tokens_per_batch", C.c_int64),
                ("hbm_budget_bytes", C.c_uint64), ("stream", C.c_void_p), ("use_graphs", C.c_int32),
                ("reserved", C.c_int32), ("dev_alloc", DEV_ALLOC), ("dev_free", DEV_FREE),
                ("alloc_ctx", C.c_void_p)]


class StreamCfg(C.Structure):
    _fields_ = [("height", C.c_int32), ("width", C.c_int32), ("window", C.c_int32), ("overlap", C.c_int32),
                ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("n_points", C.c_int32), ("anchor_mode", C.c_int32),
                ("sigma", C.c_double), ("sigma_min", C.c_double), ("sigma_max", C.c_double),
                ("emit_maps", C.c_int32), ("ring_frames", C.c_int32), ("result_frames", C.c_int32),
                ("focus_mode", C.c_int32), ("diff_stride", C.c_int32), ("map_mode", C.c_int32),
                ("emit_depth", C.c_int32)]


class Focus(C.Structure):
    _fields_ = [("frame", C.c_int64), ("window", C.c_int32), ("valid", C.c_int32),
                ("T_w2c", C.c_double * 16), ("pose9", C.c_float * 9), ("peak_x", C.c_int32),
                ("peak_y", C.c_int32), ("sigma_px", C.c_float), ("a_world", C.c_double * 3),
                ("a_cam", C.c_double * 3), ("u", C.c_double), ("v", C.c_double), ("s", C.c_double),
                ("t_push", C.c_double), ("t_ready", C.c_double), ("t_window", C.c_double),
                ("t_batch", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("frames_pushed", C.c_int64), ("frames_emitted", C.c_int64), ("windows_run", C.c_int64),
                ("batches_run", C.c_int64), ("tokens_run", C.c_int64), ("streams_open", C.c_int32),
                ("streams_pending", C.c_int32), ("hbm_used_bytes", C.c_uint64),
                ("hbm_budget_bytes", C.c_uint64), ("gpu_ms", C.c_double), ("frames_embed_shared", C.c_int64)]


FOCUS_DTYPE = np.dtype({
    "names": ["frame", "window", "valid", "T_w2c", "pose9", "peak_x", "peak_y", "sigma_px", "a_world", "a_cam",
              "u", "v", "s", "t_push", "t_ready", "t_window", "t_batch"],
    "formats": ["<i8", "<i4", "<i4", ("<f8", (16,)), ("<f4", (9,)), "<i4", "<i4", "<f4", ("<f8", (3,)),
                ("<f8", (3,)), "<f8", "<f8", "<f8", "<f8", "<f8", "<f8", "<f8"],
    "offsets": [Focus.frame.offset, Focus.window.offset, Focus.valid.offset, Focus.T_w2c.offset,
                Focus.pose9.offset, Focus.peak_x.offset, Focus.peak_y.offset, Focus.sigma_px.offset,
                Focus.a_world.offset,
                Focus.a_cam.offset, Focus.u.offset, Focus.v.offset, Focus.s.offset, Focus.t_push.offset,
                Focus.t_ready.offset, Focus.t_window.offset, Focus.t_batch.offset],
    "itemsize": C.sizeof(Focus),
})

EXPORTS = {
    # name: (restype, argtypes)
    "mf_engine_create": (C.c_int32, [C.POINTER(ModelCfg), C.c_void_p, C.c_size_t, C.POINTER(RuntimeCfg),
                                     C.POINTER(C.c_void_p)]),
    "mf_engine_destroy": (None, [C.c_void_p]),
    "mf_open_stream": (C.c_int32, [C.c_void_p, C.POINTER(StreamCfg), C.POINTER(C.c_int32)]),
    "mf_push_frames": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32]),
    "mf_push_poses": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int64, C.c_int32]),
    "mf_poll_focus": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                  C.c_void_p, C.c_int32]),
    "mf_poll_focus_depth": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                        C.c_void_p, C.c_void_p, C.c_int32]),
    "mf_close_stream": (C.c_int32, [C.c_void_p, C.c_int32]),
    "mf_engine_step": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32)]),
    "mf_engine_sync": (C.c_int32, [C.c_void_p]),
    "mf_engine_stats": (C.c_int32, [C.c_void_p, C.POINTER(Stats)]),
    "mf_status_str": (C.c_char_p, [C.c_int32]),
    "mf_last_error": (C.c_char_p, []),
    # op-level entry points
    "mf_rows_per_frame": (C.c_int32, [C.c_int32, C.c_int32]),
    "mf_forward_window": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                      C.c_void_p, C.c_void_p, C.c_void_p]),
    "mf_debug_copy": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t]),
    "mf_profile": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                               C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "mf_profile_stages": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "mf_op_attention": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p]),
    "mf_op_attention_fp8": (C.c_int32, [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p]),
    "mf_op_gemm": (C.c_int32, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                               C.c_int32, C.c_int32, C.c_void_p]),
    "mf_op_gemm_fp8": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_int32, C.c_int32, C.c_int32, C.c_void_p]),
    "mf_op_quantize_fp8": (C.c_int32, [C.c_void_p, C.c_int64, C.c_float, C.c_void_p, C.c_void_p]),
    "mf_op_quantize_fp8_windows": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                               C.c_void_p, C.c_void_p]),
    "mf_op_quantize_fp8_windows_noalloc": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                                       C.c_void_p, C.c_void_p, C.c_void_p]),
    "mf_op_layernorm": (C.c_int32, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                    C.c_int32, C.c_void_p]),
}


def bind(path: str, strict: bool = True):
    """Load a library and declare the prototypes of EXPORTS (strict: every one must exist)."""
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        if not strict and not hasattr(lib, name):
            continue
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_2601_07154_amd.build)")
        _lib = bind(LIB_PATH)
    return _lib
