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


def test_arrivals_while_busy_and_admission_under_a_tight_budget():
    """Streams arrive while batches of earlier streams run on the device, under an HBM budget that
    holds the engine and two streams: later streams are refused (MF_EAGAIN) until earlier ones drain
    and are then admitted; their windows join batches already in flight; every stream's results
    equal the same stream served alone, bit for bit."""
    torch = torch_cuda()
    m = mf()
    from paper_2601_07154_amd import serving
    model = mf_synth.ModelConfig(4, 384, 6, 1536)
    blob = mf_synth.make_weights(model, 12)
    H, W, L, O = 140, 252, 8, 4
    K = lambda h, w: (150.0, 150.0, w / 2, h / 2)
    frames = torch.from_numpy(mf_synth.make_frames(48, H, W, 77)).cuda()
    pool = lambda h, w: frames
    # what the engine and one stream take, measured on a probe engine with room to spare
    probe = m.Engine.from_model(model, blob, precision="bf16", threaded=True, max_tokens=32768)
    fixed = probe.stats()["hbm_used_bytes"]
    sid = probe.open_stream(H, W, L, O, K(H, W), sigma=1000.0, emit_maps=False, ring_frames=2 * L + 8)
    per_stream = probe.stats()["hbm_used_bytes"] - fixed
    probe.close_stream(sid)
    probe.close()
    budget = fixed + int(2.5 * per_stream)
    rng = np.random.default_rng(8)
    # four streams at once (two fit, two are turned away), two more while the first batches run
    specs = [serving.StreamSpec(0.0 if i < 4 else 0.01 * i, int(rng.integers(20, 48)), H, W) for i in range(6)]
    eng = m.Engine.from_model(model, blob, precision="bf16", threaded=True, max_tokens=32768, hbm_budget=budget)
    out = serving.serve(eng, specs, pool, L, O, K, paced=False, time_limit=120)
    st = eng.stats()
    eng.close()
    print(f"budget {budget} B (fixed {fixed} + 2.5 x {per_stream}); refusals per stream {out['refused']}; "
          f"admitted at {np.round(out['admitted_at'], 3).tolist()} s; {st['batches_run']} batches, "
          f"{st['windows_run']} windows")
    assert sum(out["refused"]) > 0                                   # the budget turned streams away
    late = [i for i, a in enumerate(out["admitted_at"]) if a > specs[i].arrival + 1e-3]
    assert late                                                      # ... and admitted them later
    assert st["batches_run"] < st["windows_run"]                     # windows shared batches
    for i, spec in enumerate(specs):
        eng1 = m.Engine.from_model(model, blob, precision="bf16", threaded=False, max_tokens=32768)
        alone = serving.serve(eng1, [serving.StreamSpec(0.0, spec.length, H, W)], pool, L, O, K,
                              paced=False, time_limit=60)["records"][0]
        eng1.close()
        got = out["records"][i]
        assert list(got["frame"]) == list(range(spec.length))
        for f in ("T_w2c", "pose9", "a_world", "u", "v", "valid"):
            np.testing.assert_array_equal(got[f], alone[f], err_msg=f"stream {i} field {f}")
