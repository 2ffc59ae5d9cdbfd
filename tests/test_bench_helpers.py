"""bench.py's own workload arithmetic (window count and flop counts) against the oracle's schedule."""
import importlib.util
import os

import pytest

import mf_synth
from oracle import motion

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


@pytest.mark.parametrize("n,L,O", [(64, 16, 8), (128, 48, 24), (7, 16, 8), (16, 16, 8), (17, 16, 8), (100, 8, 1),
                                   (1, 4, 2), (0, 4, 2)])
def test_window_sizes_match_schedule(n, L, O):
    b = _bench()
    assert b.window_sizes(n, L, O) == [w["size"] for w in motion.window_schedule(n, L, O)]


def test_flop_counts_small_workload():
    b = _bench()
    wl = mf_synth.SMALL
    T = wl.window * wl.tokens_per_frame
    assert b.global_attention_flops(wl) == 7 * 4.0 * T * T * wl.model.dim
    assert abs(b.global_attention_flops(wl) - 1.4309e12) / 1.4309e12 < 1e-4


def test_traffic_figure_only_for_its_workload_and_source(tmp_path, monkeypatch):
    """roofline.traffic comes from the committed counter summary only for the workload and the
    attention source it was measured on."""
    b = _bench()
    text = (f"source_sha256: {b.kernel_source_hash()}\ntraffic_bytes_per_launch: 123456\n"
            f"workload: {mf_synth.SMALL.name}\n")
    f = tmp_path / "traffic.md"
    f.write_text(text)
    monkeypatch.setattr(b, "TRAFFIC_FILES", {mf_synth.SMALL.name: str(f), mf_synth.LARGE.name: str(f)})
    assert b.measured_traffic(mf_synth.SMALL.name) == 123456.0
    assert b.measured_traffic(mf_synth.LARGE.name) is None      # the file names another workload
    assert b.measured_traffic(mf_synth.FP8.name) is None        # no file for this workload
    f.write_text(text.replace(b.kernel_source_hash(), "0" * 64))
    assert b.measured_traffic(mf_synth.SMALL.name) is None


def test_gemm_stage_flops_sum_to_the_layer_formula():
    """Per-GEMM algorithmic flops (QKV 6TD^2, out-projection 2TD^2, fc1 and fc2 2TDF each) add up to
    the per-layer 2TD(3D + D + 2F) of the step total."""
    b = _bench()
    for wl in (mf_synth.SMALL, mf_synth.LARGE, mf_synth.FP8):
        per = b.gemm_stage_flops(wl)
        assert set(per) == set(b.GEMM_STAGES)
        assert abs(wl.model.depth * sum(per.values()) - b.gemm_flops(wl)) <= 1e-9 * b.gemm_flops(wl)
        T = sum(b.window_sizes(wl.frames, wl.window, wl.overlap)) * wl.tokens_per_frame
        D, F = wl.model.dim, wl.model.mlp
        assert per["qkv"] == 6.0 * T * D * D and per["fc1"] == per["fc2"] == 2.0 * T * D * F


def test_attention_bytes_large_workload():
    """Q, K, V and O once each in bf16: 8 T D bytes per window, 15 windows of 32 x 973 tokens."""
    b = _bench()
    wl = mf_synth.LARGE
    assert b.global_attention_bytes(wl) == 15 * 8.0 * 32 * 973 * 1024
