"""Argument checks of the C ABI that return before any device work (run without a GPU): each
entry point rejects what its header says it rejects, with MF_EINVAL and a message."""
import ctypes as C

import numpy as np
import pytest

import mf_synth

FAKE = C.c_void_p(0x1000)     # never dereferenced: every call below fails its checks first


@pytest.fixture(scope="module")
def lib():
    from paper_2601_07154_amd import _lib
    return _lib.lib()


def _segs(rows):
    a = np.ascontiguousarray(np.asarray(rows, np.int32).reshape(-1, 4))
    return a, C.c_void_p(a.ctypes.data), a.shape[0]


def test_status_strings(lib):
    from paper_2601_07154_amd import _lib
    for st in (_lib.MF_OK, _lib.MF_EINVAL, _lib.MF_ENOMEM, _lib.MF_EAGAIN, _lib.MF_ECLOSED, _lib.MF_EDEVICE,
               _lib.MF_ENOTFOUND):
        assert lib.mf_status_str(st).decode()
    assert lib.mf_status_str(12345).decode() == "unknown status"


@pytest.mark.parametrize("hd,heads,dim,segs,mpad", [
    (48, 2, 96, [[0, 1, 10, 16]], 1024),       # head dim other than 32 / 64
    (64, 2, 100, [[0, 1, 10, 16]], 1024),      # heads * hd != dim
    (64, 2, 128, [[0, 1, 10, 12]], 1024),      # npad not a multiple of 8
    (64, 2, 128, [[0, 1, 20, 16]], 1024),      # n > npad
    (64, 2, 128, [[4, 1, 10, 16]], 1024),      # base not a multiple of 8
    (64, 2, 128, [[0, 60, 10, 16]], 1024),     # segment + 256 guard rows beyond mpad
    (64, 2, 128, [], 1024),                     # no segment
])
def test_op_attention_rejects(lib, hd, heads, dim, segs, mpad):
    from paper_2601_07154_amd import _lib
    arr, p, n = _segs(segs) if segs else (None, C.c_void_p(0x2000), 0)
    st = lib.mf_op_attention(_lib.MF_BF16, hd, heads, dim, FAKE, FAKE, FAKE, FAKE, mpad, p, n, None)
    assert st == _lib.MF_EINVAL


@pytest.mark.parametrize("prec,M,N,K", [(1, 10, 100, 64), (1, 10, 128, 100), (0, 10, 128, 48), (1, -1, 128, 64),
                                        (1, 10, 128, 0)])
def test_op_gemm_rejects(lib, prec, M, N, K):
    from paper_2601_07154_amd import _lib
    assert lib.mf_op_gemm(prec, FAKE, FAKE, None, FAKE, M, N, K, None) == _lib.MF_EINVAL


@pytest.mark.parametrize("M,N,K,scales", [(10, 128, 96, True), (10, 96, 128, True), (10, 128, 128, False)])
def test_op_gemm_fp8_rejects(lib, M, N, K, scales):
    from paper_2601_07154_amd import _lib
    s = FAKE if scales else None
    assert lib.mf_op_gemm_fp8(FAKE, FAKE, s, s, None, FAKE, M, N, K, None) == _lib.MF_EINVAL


@pytest.mark.parametrize("n,scale", [(6, 1.0), (8, 0.0), (8, -1.0), (8, float("nan")), (-4, 1.0)])
def test_op_quantize_fp8_rejects(lib, n, scale):
    from paper_2601_07154_amd import _lib
    assert lib.mf_op_quantize_fp8(FAKE, n, scale, FAKE, None) == _lib.MF_EINVAL


@pytest.mark.parametrize("C_,segs", [(20, [[0, 1, 8, 8]]), (32, [[0, 1, 9, 8]]), (32, [[-8, 1, 8, 8]]),
                                     (32, [[0, 0, 8, 8]])])
def test_op_quantize_fp8_windows_rejects(lib, C_, segs):
    from paper_2601_07154_amd import _lib
    arr, p, n = _segs(segs)
    assert lib.mf_op_quantize_fp8_windows(FAKE, C_, p, n, FAKE, FAKE, None) == _lib.MF_EINVAL
    assert lib.mf_op_quantize_fp8_windows_noalloc(FAKE, C_, p, n, FAKE, FAKE, None) == _lib.MF_EINVAL


def test_op_quantize_fp8_windows_noalloc_rejects_more_windows_than_its_array(lib):
    """The allocation-free quantiser holds at most MF_NOALLOC_MAX_WINDOWS windows (4096)."""
    from paper_2601_07154_amd import _lib
    rows = [[8 * i, 1, 8, 8] for i in range(4097)]
    arr, p, n = _segs(rows)
    assert lib.mf_op_quantize_fp8_windows_noalloc(FAKE, 32, p, n, FAKE, FAKE, None) == _lib.MF_EINVAL
    assert lib.mf_op_quantize_fp8_windows_noalloc(FAKE, 32, p, 0, FAKE, FAKE, None) == _lib.MF_EINVAL


def test_op_layernorm_rejects_null(lib):
    from paper_2601_07154_amd import _lib
    assert lib.mf_op_layernorm(_lib.MF_BF16, None, FAKE, FAKE, FAKE, 4, 128, None) == _lib.MF_EINVAL


@pytest.mark.parametrize("change", ["patch", "precision", "heads", "dim", "head_dim", "mlp", "blob"])
def test_engine_create_rejects_bad_models(lib, change):
    """Model checks happen before the device is touched; the message names the problem."""
    from paper_2601_07154_amd import _lib
    model = mf_synth.ModelConfig(2, 128, 2, 256)
    blob = mf_synth.make_weights(model, 0)
    depth, dim, heads, mlp, patch, prec = 2, 128, 2, 256, 14, _lib.MF_BF16
    n = blob.size
    if change == "patch":
        patch = 16
    elif change == "precision":
        prec = 7
    elif change == "heads":
        heads = 3
    elif change == "dim":
        dim, heads = 192, 3
    elif change == "head_dim":
        heads = 8             # hd 16
    elif change == "mlp":
        mlp = 200
    else:
        n = blob.size - 1
    m = _lib.ModelCfg(depth, dim, heads, mlp, patch, prec)
    rt = _lib.RuntimeCfg(0, 0, 0, 0, None, 0, 0)
    h = C.c_void_p()
    st = lib.mf_engine_create(C.byref(m), C.c_void_p(blob.ctypes.data), n, C.byref(rt), C.byref(h))
    assert st == _lib.MF_EINVAL and not h.value
    assert lib.mf_last_error().decode()


@pytest.mark.parametrize("flag,extra", [(1, 0), (0, 1)])
def test_engine_create_checks_the_depth_head_blob(lib, flag, extra):
    """A model with the depth head needs its tensors at the end of the blob and one without refuses
    them (checked before the device is touched)."""
    from paper_2601_07154_amd import _lib
    head = mf_synth.ModelConfig(2, 128, 2, 256, depth_head=bool(extra))
    blob = mf_synth.make_weights(head, 0)
    m = _lib.ModelCfg(2, 128, 2, 256, 14, _lib.MF_BF16, flag)
    rt = _lib.RuntimeCfg(0, 0, 0, 0, None, 0, 0)
    h = C.c_void_p()
    st = lib.mf_engine_create(C.byref(m), C.c_void_p(blob.ctypes.data), blob.size, C.byref(rt), C.byref(h))
    assert st == _lib.MF_EINVAL and not h.value
    assert "floats" in lib.mf_last_error().decode()


@pytest.mark.parametrize("heads,dim,segs,mpad", [(2, 100, [[0, 1, 10, 16]], 1024),   # dim != 64 heads
                                                 (2, 128, [[0, 1, 10, 12]], 1024),   # npad not a multiple of 8
                                                 (2, 128, [[0, 60, 10, 16]], 1024),  # past mpad - 256
                                                 (2, 128, [[0, 1, 10, 16]], 1020)])  # mpad not a multiple of 8
def test_op_attention_fp8_rejects(lib, heads, dim, segs, mpad):
    from paper_2601_07154_amd import _lib
    arr, p, n = _segs(segs)
    st = lib.mf_op_attention_fp8(heads, dim, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, mpad, p, n, None)
    assert st == _lib.MF_EINVAL
