"""Serving: streams of uneven lengths and resolutions arrive over time on the threaded engine
(admission by HBM budget, continuous batching); every stream's results equal the same stream
served alone, bit for bit."""
import numpy as np
import pytest

import mf_synth
from gpu_util import mf, torch_cuda

pytestmark = pytest.mark.gpu


def test_served_streams_equal_streams_alone():
    torch = torch_cuda()
    m = mf()
    from paper_2601_07154_amd import serving
    model = mf_synth.ModelConfig(4, 384, 6, 1536)
    blob = mf_synth.make_weights(model, 11)
    rng = np.random.default_rng(3)
    res = [(112, 168), (140, 252), (112, 112)]
    # all streams arrive at once (throughput regime), so ready windows of several streams share batches
    specs = [serving.StreamSpec(0.0, int(rng.integers(9, 40)), *res[i % 3], seed=200 + i) for i in range(7)]
    pools = {}

    def pool(H, W):
        if (H, W) not in pools:
            pools[(H, W)] = torch.from_numpy(mf_synth.make_frames(40, H, W, H * 1000 + W)).cuda()
        return pools[(H, W)]

    K = lambda H, W: (150.0, 150.0, W / 2, H / 2)
    eng = m.Engine.from_model(model, blob, precision="bf16", threaded=True, max_tokens=32768)
    out = serving.serve(eng, specs, pool, 8, 4, K, paced=False, time_limit=120)
    st = eng.stats()
    eng.close()
    assert st["batches_run"] < st["windows_run"]          # windows of several streams shared batches
    lat = serving.latency_summary(out["records"])
    print(f"served {lat['frames']} frames in {st['batches_run']} batches, p50 {lat['p50_ms']:.1f} ms, "
          f"p99 {lat['p99_ms']:.1f} ms (mean buffering {lat['buffering']['mean_ms']:.1f}, queueing "
          f"{lat['queueing']['mean_ms']:.1f}, compute {lat['compute']['mean_ms']:.1f} ms)")
    for r in out["records"]:
        assert (r["t_push"] <= r["t_window"]).all() and (r["t_window"] <= r["t_batch"]).all()
        assert (r["t_batch"] <= r["t_ready"]).all()
    for i, spec in enumerate(specs):
        eng1 = m.Engine.from_model(model, blob, precision="bf16", threaded=False, max_tokens=32768)
        alone = serving.serve(eng1, [serving.StreamSpec(0.0, spec.length, spec.height, spec.width)], pool, 8, 4, K,
                              paced=False, time_limit=60)["records"][0]
        eng1.close()
        got = out["records"][i]
        assert list(got["frame"]) == list(range(spec.length))
        for f in ("T_w2c", "pose9", "a_world", "u", "v", "valid"):
            np.testing.assert_array_equal(got[f], alone[f], err_msg=f"stream {i} field {f}")
