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
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(f))
    assert b.measured_traffic(mf_synth.SMALL.name) == 123456.0
    assert b.measured_traffic(mf_synth.LARGE.name) is None
    f.write_text(text.replace(b.kernel_source_hash(), "0" * 64))
    assert b.measured_traffic(mf_synth.SMALL.name) is None
