"""The allocation-free window quantiser (mf_op_quantize_fp8_windows_noalloc) against the allocating
entry point it mirrors (mf_op_quantize_fp8_windows): identical E4M3 codes and scales, byte for
byte, on two calls in a row, the second with fewer windows, fewer rows and smaller magnitudes (so
amax counters left over from the first call would change its scales)."""
import numpy as np
import pytest

from gpu_util import mf, torch_cuda

pytestmark = pytest.mark.gpu


def _case(rng, segs, cdim, mag):
    rows = max(int(b + nf * npad) for b, nf, n, npad in segs)
    y = (rng.standard_normal((rows, cdim)) * mag * np.exp(rng.uniform(-2, 2, (rows, 1)))).astype(np.float32)
    return y


def _run(torch, m, fn, yb, segs, fill):
    rows, cdim = yb.shape
    q = torch.full((rows, cdim), fill, dtype=torch.uint8, device="cuda")
    s = torch.full((rows,), float(fill), device="cuda")
    fn(yb, segs, q, s)
    torch.cuda.synchronize()
    return q.cpu().numpy(), s.cpu().numpy()


def test_noalloc_quantiser_matches_allocating_one_on_two_calls():
    torch = torch_cuda()
    m = mf()
    rng = np.random.default_rng(11)
    # first call: 6 windows (frames of 200 valid tokens in 208 rows, a ragged last window)
    segs1 = np.array([[0, 4, 200, 208], [832, 4, 200, 208], [1664, 2, 200, 208], [2080, 1, 37, 40],
                      [2120, 3, 17, 24], [2192, 1, 64, 64]], np.int32)
    y1 = _case(rng, segs1, 384, 8.0)
    # second call: 3 windows over fewer rows and columns, values 100x smaller
    segs2 = np.array([[0, 2, 100, 104], [208, 1, 9, 16], [232, 2, 50, 56]], np.int32)
    y2 = _case(rng, segs2, 256, 0.08)
    y2[208:224] = 0.0          # an all-zero window: scale 1
    for y, segs in ((y1, segs1), (y2, segs2)):
        yb = torch.from_numpy(y).to(torch.bfloat16).cuda()
        q_ref, s_ref = _run(torch, m, m.op_quantize_fp8_windows, yb, segs, 0)
        q_new, s_new = _run(torch, m, m.op_quantize_fp8_windows_noalloc, yb, segs, 0xA5)
        covered = np.zeros(y.shape[0], bool)
        for base, nf, n, npad in segs:
            covered[base:base + nf * npad] = True
        assert np.array_equal(q_new[covered], q_ref[covered])
        assert np.array_equal(s_new[covered].view(np.uint32), s_ref[covered].view(np.uint32))
        assert np.all(s_ref[covered] > 0)
        # rows outside every window are left as they were
        assert np.all(q_new[~covered] == 0xA5) and np.all(s_new[~covered] == float(0xA5))
