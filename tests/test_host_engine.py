"""Host logic of the engine (scheduler, admission, ordering, errors) on the CPU: the real
engine.cpp and C ABI linked against a stub executor that computes nothing (tests/host_stub)."""
import os
import subprocess
import threading

import numpy as np
import pytest

import paper_2601_07154_amd as mfp
from paper_2601_07154_amd import _lib
from oracle import motion

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
W16 = np.zeros(16, np.float32)   # the stub ignores weights


@pytest.fixture(scope="session")
def hostlib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("host") / "libmfhost.so")
    src = [os.path.join(ROOT, "paper_2601_07154_amd", "csrc", "engine.cpp"),
           os.path.join(HERE, "host_stub", "exec_stub.cpp")]
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-Wall", "-Werror",
                    "-I" + os.path.join(ROOT, "include"), *src, "-o", out, "-lpthread"], check=True)
    return _lib.bind(out, strict=False)   # the op-level entry points are device-only


def engine(lib, **kw):
    return mfp.Engine(2, 128, 4, 512, W16, precision="bf16", lib=lib, **kw)


def drain(eng, sid, cap=1000, maps=None):
    recs = []
    while True:
        r, st = eng.poll(sid, cap, maps)
        if len(r):
            recs.append(r)
        if st != mfp.MF_OK or len(r) == 0:
            return (np.concatenate(recs) if recs else np.zeros(0, mfp.FOCUS_DTYPE)), st


FR = np.zeros((1, 3, 28, 28), np.float32)


def frames(n):
    return np.zeros((n, 3, 28, 28), np.float32)


@pytest.mark.parametrize("N,L,O,chunk", [(64, 16, 8, 5), (8, 8, 4, 8), (5, 8, 4, 2), (128, 48, 24, 7),
                                         (50, 12, 3, 50), (17, 16, 1, 1), (1, 4, 1, 1)])
def test_schedule_and_ordering(hostlib, N, L, O, chunk):
    eng = engine(hostlib)
    sid = eng.open_stream(28, 28, L, O, (50, 50, 14, 14), ring_frames=N + L, result_frames=max(4 * L, N))
    pushed = 0
    while pushed < N:
        n = min(chunk, N - pushed)
        eng.push_frames(sid, frames(n), eos=pushed + n == N)
        pushed += n
        eng.step()
    eng.sync()
    recs, st = drain(eng, sid)
    assert list(recs["frame"]) == list(range(N))                   # once each, in order
    sched = motion.window_schedule(N, L, O)
    for k, w in enumerate(sched):
        sel = recs[(recs["frame"] >= w["emit_begin"]) & (recs["frame"] < w["emit_end"])]
        assert (sel["window"] == k).all()
        assert (sel["pose9"][:, 0] == w["start"]).all() and (sel["pose9"][:, 1] == w["size"]).all()
    np.testing.assert_array_equal(recs["T_w2c"][:, 3], np.arange(N))
    # latency parts are ordered: pushed <= window complete <= batch start <= result ready
    assert (recs["t_push"] <= recs["t_window"]).all() and (recs["t_window"] <= recs["t_batch"]).all()
    assert (recs["t_batch"] <= recs["t_ready"]).all() and (recs["t_push"] > 0).all()
    # a regular window is complete when its last frame is pushed; the tail window needs the EOS push
    for k, w in enumerate(sched):
        sel = recs[(recs["frame"] >= w["emit_begin"]) & (recs["frame"] < w["emit_end"])]
        last = recs[recs["frame"] == w["start"] + w["size"] - 1]["t_push"][0]
        assert (sel["t_window"] >= last).all()
    # drained and closed: ECLOSED once, then the id is released
    assert st == mfp.MF_ECLOSED
    with pytest.raises(mfp.MfError) as e:
        eng.poll(sid, 10)
    assert e.value.status == mfp._lib.MF_ENOTFOUND
    eng.close()


def test_continuous_batching_across_streams(hostlib):
    eng = engine(hostlib)
    sids = [eng.open_stream(28, 28, 8, 4, (50, 50, 14, 14), ring_frames=40) for _ in range(3)]
    for s in sids:
        eng.push_frames(s, frames(20), eos=True)
    assert eng.step() == 3 * len(motion.window_schedule(20, 8, 4))   # every ready window, one batch
    recs = [drain(eng, s)[0] for s in sids]
    for r in recs:
        assert list(r["frame"]) == list(range(20))
        assert len(set(r["pose9"][:, 2])) == 1                       # same batch
    assert len({r["pose9"][0, 2] for r in recs}) == 1
    eng.close()


def test_token_budget_splits_batches(hostlib):
    rows = 8                                                        # 28x28: 4 patches + camera -> 8 rows
    eng = engine(hostlib, max_tokens=2 * 8 * rows)                  # two windows of 8 frames
    sid = eng.open_stream(28, 28, 8, 4, (50, 50, 14, 14), ring_frames=64, result_frames=64)
    eng.push_frames(sid, frames(40), eos=True)
    n = 0
    sizes = []
    while True:
        k = eng.step()
        if k == 0:
            break
        sizes.append(k)
        n += k
    assert max(sizes) == 2 and n == len(motion.window_schedule(40, 8, 4))
    recs, _ = drain(eng, sid)
    assert list(recs["frame"]) == list(range(40))
    eng.close()


def test_window_larger_than_token_budget_is_rejected(hostlib):
    eng = engine(hostlib, max_tokens=64)
    with pytest.raises(mfp.MfError) as e:
        eng.open_stream(28, 28, 16, 8, (50, 50, 14, 14))
    assert e.value.status == mfp._lib.MF_EINVAL
    eng.close()


def test_ring_backpressure(hostlib):
    eng = engine(hostlib)
    sid = eng.open_stream(28, 28, 8, 4, (50, 50, 14, 14), ring_frames=12)
    assert eng.push_frames(sid, frames(12)) == mfp.MF_OK
    assert eng.push_frames(sid, frames(4), allow_again=True) == mfp.MF_EAGAIN   # ring full
    eng.sync()                                                                    # window 0 runs
    assert eng.push_frames(sid, frames(1), allow_again=True) == mfp.MF_OK       # frame 0 freed
    eng.close()


def test_result_backpressure_with_maps(hostlib):
    eng = engine(hostlib)
    sid = eng.open_stream(28, 28, 8, 4, (50, 50, 14, 14), ring_frames=64, result_frames=8, emit_maps=True)
    eng.push_frames(sid, frames(24), eos=True)
    eng.sync()
    maps = np.zeros((100, 28, 28), np.float32)
    r, st = eng.poll(sid, 100, maps)
    assert list(r["frame"]) == list(range(8))            # window 1 waits until maps are polled
    np.testing.assert_array_equal(maps[:8, 0, 0], np.arange(8))
    got = []
    for _ in range(20):                                   # non-threaded: windows run in sync()
        eng.sync()
        r2, st = eng.poll(sid, 100, maps)
        got += list(r2["frame"])
        assert len(r2) <= 8
        if st == mfp.MF_ECLOSED:
            break
    assert got == list(range(8, 24))
    eng.close()


def test_admission_by_hbm_budget(hostlib):
    per = 3 * 28 * 28 * 4 * 24 + 512 * 168   # ring + history ring
    eng = engine(hostlib, hbm_budget=(1 << 20) + int(per * 1.5) + 4096)
    a = eng.open_stream(28, 28, 8, 4, (50, 50, 14, 14), ring_frames=24)
    assert eng.open_stream(28, 28, 8, 4, (50, 50, 14, 14), ring_frames=24, allow_again=True) == -1  # EAGAIN
    with pytest.raises(mfp.MfError) as e:                                                           # never fits
        eng.open_stream(28, 28, 8, 4, (50, 50, 14, 14), ring_frames=2400)
    assert e.value.status == mfp._lib.MF_ENOMEM
    eng.push_frames(a, frames(8), eos=True)
    eng.sync()
    drain(eng, a)                                                  # drained and closed: released
    b = eng.open_stream(28, 28, 8, 4, (50, 50, 14, 14), ring_frames=24)
    assert b != a
    st = eng.stats()
    assert st["streams_pending"] >= 1 and st["hbm_used_bytes"] <= st["hbm_budget_bytes"]
    eng.close()


@pytest.mark.parametrize("kw", [dict(height=30), dict(width=0), dict(overlap=0), dict(overlap=8), dict(n_points=0),
                                dict(n_points=33), dict(anchor_mode=7), dict(fx=0.0), dict(focus_mode=2),
                                dict(diff_stride=-1), dict(diff_stride=65)])
def test_invalid_stream_configs(hostlib, kw):
    eng = engine(hostlib)
    args = dict(height=28, width=28, window=8, overlap=4, fx=50.0, n_points=15, anchor_mode=0, focus_mode=0,
                diff_stride=1)
    args.update(kw)
    with pytest.raises(mfp.MfError) as e:
        eng.open_stream(args["height"], args["width"], args["window"], args["overlap"], (args["fx"], 50, 14, 14),
                        n_points=args["n_points"], anchor_mode=args["anchor_mode"], focus_mode=args["focus_mode"],
                        diff_stride=args["diff_stride"])
    assert e.value.status == mfp._lib.MF_EINVAL
    eng.close()


def test_call_order_errors(hostlib):
    eng = engine(hostlib)
    sid = eng.open_stream(28, 28, 8, 4, (50, 50, 14, 14))
    eng.push_frames(sid, frames(3))
    with pytest.raises(mfp.MfError) as e:
        eng.push_poses(sid, np.tile(np.eye(4), (2, 1, 1)), 3)      # a frame stream takes no poses
    assert e.value.status == mfp._lib.MF_EINVAL
    eng.close_stream(sid)
    with pytest.raises(mfp.MfError) as e:
        eng.push_frames(sid, frames(1))
    assert e.value.status == mfp._lib.MF_ECLOSED
    with pytest.raises(mfp.MfError) as e:
        eng.push_frames(12345, frames(1))
    assert e.value.status == mfp._lib.MF_ENOTFOUND
    eng.sync()
    recs, st = drain(eng, sid)
    assert list(recs["frame"]) == [0, 1, 2]                         # short stream: one window
    eng.close()


def test_pose_streams(hostlib):
    eng = engine(hostlib)
    sid = eng.open_stream(28, 28, 8, 4, (50, 50, 14, 14), result_frames=64)
    T = np.tile(np.eye(4), (10, 1, 1))
    T[:, 0, 3] = np.arange(10)                                     # the stub echoes T[0,3]
    eng.push_poses(sid, T, 0)
    with pytest.raises(mfp.MfError):
        eng.push_poses(sid, T, 5)                                   # must continue at frame 10
    eng.push_poses(sid, T[:3], 10, eos=True)
    eng.sync()
    recs, st = drain(eng, sid)
    assert list(recs["frame"]) == list(range(13))
    np.testing.assert_array_equal(recs["T_w2c"][:10, 7], np.arange(10))
    # local windows: the next window must contain the anchor (last emitted frame)
    s2 = eng.open_stream(28, 28, 8, 4, (50, 50, 14, 14))
    with pytest.raises(mfp.MfError):
        eng.push_poses(s2, T[:8], 2, local=True)                    # first window starts at 0
    eng.push_poses(s2, T[:8], 0, local=True)
    with pytest.raises(mfp.MfError):
        eng.push_poses(s2, T[:8], 8, local=True)                    # misses the anchor frame 7
    eng.push_poses(s2, T[:8], 4, local=True, eos=True)
    eng.sync()
    r2, _ = drain(eng, s2)
    assert list(r2["frame"]) == list(range(12)) and list(r2["window"][7:9]) == [0, 1]
    eng.close()


def test_threaded_scheduler_concurrent_streams(hostlib):
    eng = engine(hostlib, threaded=True)
    with pytest.raises(mfp.MfError):
        eng.step()
    sids = [eng.open_stream(28, 28, 8, 4, (50, 50, 14, 14), ring_frames=16) for _ in range(4)]
    results = {}

    def feed(sid, n):
        got, pushed = [], 0
        while pushed < n or True:
            if pushed < n:
                if eng.push_frames(sid, frames(1), eos=pushed + 1 == n, allow_again=True) == mfp.MF_OK:
                    pushed += 1
            r, st = eng.poll(sid, 64)
            if len(r):
                got.append(r)
            if st == mfp.MF_ECLOSED:
                break
        results[sid] = np.concatenate(got)

    ths = [threading.Thread(target=feed, args=(s, 37 + 11 * i)) for i, s in enumerate(sids)]
    for t in ths:
        t.start()
    for t in ths:
        t.join(timeout=60)
    for i, s in enumerate(sids):
        assert list(results[s]["frame"]) == list(range(37 + 11 * i))
    eng.close()


def test_threaded_engine_under_thread_sanitizer(tmp_path):
    """The scheduler thread, pushes and polls of 6 streams from 6 threads: no data race reported."""
    exe = str(tmp_path / "race_drive")
    src = [os.path.join(ROOT, "paper_2601_07154_amd", "csrc", "engine.cpp"),
           os.path.join(HERE, "host_stub", "exec_stub.cpp"), os.path.join(HERE, "host_stub", "race_drive.cpp")]
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-I" + os.path.join(ROOT, "include"),
                    *src, "-o", exe, "-lpthread"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]
    assert "bad=0" in r.stdout


def test_serving_loop_on_host_stub(hostlib):
    """The request loop admits streams as the budget frees up and returns every frame in order."""
    from paper_2601_07154_amd import serving
    per = 3 * 28 * 28 * 4 * (2 * 8 + 8) + 512 * 168
    eng = engine(hostlib, threaded=True, hbm_budget=(1 << 20) + 3 * per + 1000)   # 3 streams at a time
    rng = np.random.default_rng(0)
    specs = [serving.StreamSpec(0.0, int(rng.integers(5, 60)), 28, 28) for i in range(10)]   # all at once
    out = serving.serve(eng, specs, lambda H, W: np.zeros((16, 3, H, W), np.float32), 8, 4,
                        lambda H, W: (50.0, 50.0, W / 2, H / 2), paced=False, time_limit=60)
    for s, r in zip(specs, out["records"]):
        assert list(r["frame"]) == list(range(s.length))
    lat = serving.latency_summary(out["records"])
    assert lat["frames"] == sum(s.length for s in specs)
    parts = lat["buffering"]["mean_ms"] + lat["queueing"]["mean_ms"] + lat["compute"]["mean_ms"]
    assert abs(parts - lat["mean_ms"]) < 1e-6 * max(1.0, lat["mean_ms"])   # the split adds up
    assert out["stats"]["streams_pending"] > 0          # admission had to wait
    eng.close()
