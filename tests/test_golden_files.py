"""The stored oracle outputs (tests/golden) were written for the inputs the generators give today:
each file's key (workload, windows, precision, SHA-256 of the weight blob and of the frames read) is
recomputed, and the stored poses are rigid transforms with finite focus tracks.  CPU only."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
if HERE not in sys.path:
    sys.path.insert(0, HERE)
import make_golden  # noqa: E402

PRESENT = [n for n in make_golden.FIXTURES if os.path.exists(make_golden.path(n))]


@pytest.mark.parametrize("name", PRESENT)
def test_stored_output_matches_todays_inputs(name):
    g = make_golden.load(name)            # raises if the key differs from the recomputed one
    wl, nwin, precision = make_golden.FIXTURES[name]
    assert g["key"]["precision"] == precision and g["key"]["windows"] == nwin
    assert len(g["schedule"]) == nwin and len(g["pose9"]) == nwin
    T = g["T_w"]
    R = T[:, :3, :3]
    np.testing.assert_allclose(R @ R.transpose(0, 2, 1), np.tile(np.eye(3), (len(T), 1, 1)), atol=1e-9)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-9)
    tr = g["track"]
    v = tr["valid"]
    assert np.isfinite(tr["p"]).all() and np.isfinite(tr["uv"][v]).all()
    assert not v[:2].any()                # frames 0 and 1 carry no focus (second difference)


def test_the_benchmark_workloads_have_stored_fp64_outputs():
    for name in ("small_fp64_w01", "large_fp64_w01", "fp8_fp64_w0"):
        assert name in PRESENT, name
