"""Request loop for serving many video streams on one engine (continuous batching).

Streams arrive over time (arrival second, length, H, W); each is admitted when the engine's HBM
budget allows (mf_open_stream returns MF_EAGAIN until memory frees up), its frames are pushed at
their capture rate (or all at once in the throughput regime), and results are polled as the
engine's scheduler thread completes windows.  Every window that is ready when a batch starts
joins that batch, whatever stream it belongs to.

Reported per frame, in the paced regime: latency from the frame's capture time (the stream's
arrival + i / fps) to its result, split into admission (capture to push: waiting for the stream to
be admitted under the HBM budget, or for room in its frame ring), buffering (t_window - t_push:
waiting for the window's last frame, or the end of the stream for a tail window), queueing (t_batch -
t_window: waiting for a batch to start) and compute (t_ready - t_batch: the batch itself).  In the
throughput regime every frame is available at its stream's arrival and the run measures frames/s;
its latency is counted from the push (t_ready - t_push).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import MF_EAGAIN, MF_ECLOSED, MF_OK


@dataclass
class StreamSpec:
    arrival: float      # seconds after the start
    length: int         # frames
    height: int
    width: int
    seed: int = 0


@dataclass
class StreamState:
    spec: StreamSpec
    sid: int = -1
    pushed: int = 0
    done: bool = False
    admitted_at: float = -1.0
    records: list = field(default_factory=list)
    wait: list = field(default_factory=list)   # per pushed frame: push time - capture time (s)


def serve(engine, specs, frame_pool, window: int, overlap: int, K_of, fps: float = 30.0,
          paced: bool = True, poll_cap: int = 256, time_limit: float = 600.0, sigma: float = 1000.0,
          emit_maps: bool = False, push_chunk: int = 1, progress=None, progress_every: float = 30.0):
    """Run the streams to completion on a threaded engine.

    frame_pool(height, width) -> array/tensor [P, 3, H, W] of frames pushed cyclically.
    K_of(height, width) -> intrinsics.  progress(dict) is called every progress_every seconds with
    the run's counts.  Returns dict(records per stream, wall seconds, stats, states; per stream:
    admitted_at and the number of MF_EAGAIN refusals of its admission).
    """
    states = [StreamState(s) for s in specs]
    pending = list(range(len(states)))          # not yet admitted, in arrival order
    active = []
    t0 = time.perf_counter()
    pools = {}
    refused = [0] * len(states)
    max_active = 0
    next_report = progress_every
    while True:
        now = time.perf_counter() - t0
        if now > time_limit:
            raise TimeoutError("serving run exceeded its time limit")
        if progress is not None and now >= next_report:
            next_report += progress_every
            progress({"t": now, "admitted": len(states) - len(pending), "active": len(active),
                      "done": sum(st.done for st in states),
                      "frames": sum(sum(len(r) for r in st.records) for st in states)})
        # admission in arrival order
        while pending and states[pending[0]].spec.arrival <= now:
            st = states[pending[0]]
            s = st.spec
            sid = engine.open_stream(s.height, s.width, window, overlap, K_of(s.height, s.width), sigma=sigma,
                                     emit_maps=emit_maps, ring_frames=2 * window + 8 * push_chunk,
                                     allow_again=True)
            if sid < 0:
                refused[pending[0]] += 1
                break                            # budget held by other streams: retry later
            st.sid = sid
            st.admitted_at = now
            active.append(st)
            pending.pop(0)
            max_active = max(max_active, len(active))
        # pushes: frames whose capture time (arrival + i / fps) has come (paced), or everything
        # (throughput regime)
        for st in active:
            s = st.spec
            if st.pushed >= s.length:
                continue
            due = s.length if not paced else min(s.length, int((now - s.arrival) * fps) + 1)
            key = (s.height, s.width)
            if key not in pools:
                pools[key] = frame_pool(s.height, s.width)
            pool = pools[key]
            while st.pushed < due:
                n = min(push_chunk, due - st.pushed, pool.shape[0] - st.pushed % pool.shape[0])
                off = st.pushed % pool.shape[0]
                rc = engine.push_frames(st.sid, pool[off:off + n], eos=st.pushed + n == s.length, allow_again=True)
                if rc == MF_EAGAIN:
                    break
                t_pushed = time.perf_counter() - t0
                for i in range(st.pushed, st.pushed + n):
                    st.wait.append(max(0.0, t_pushed - (s.arrival + i / fps)) if paced else 0.0)
                st.pushed += n
        if not getattr(engine, "threaded", True):
            engine.step()
        # polls
        for st in list(active):
            r, rc = engine.poll(st.sid, poll_cap)
            if len(r):
                st.records.append(r)
            if rc == MF_ECLOSED:
                st.done = True
                active.remove(st)
        if not pending and not active:
            break
        if not paced:
            time.sleep(0.0005)
        else:
            time.sleep(0.001)
    wall = time.perf_counter() - t0
    recs = [np.concatenate(st.records) if st.records else np.zeros(0) for st in states]
    waits = [np.asarray(st.wait, dtype=np.float64) for st in states]
    return dict(records=recs, waits=waits, wall=wall, stats=engine.stats(), states=states, refused=refused,
                admitted_at=[st.admitted_at for st in states], max_active=max_active)


def latency_summary(recs_list, waits=None):
    """p50 / p99 / mean per-frame latency in ms, and the same for its parts: admission (capture to
    push, when waits [per stream, per frame, seconds] is given), buffering, queueing and compute.
    With waits the latency counts from each frame's capture time, else from its push."""
    pairs = [(r, None if waits is None else waits[i]) for i, r in enumerate(recs_list) if len(r)]
    recs = [r for r, _ in pairs]
    cat = lambda f: np.concatenate([f(r) for r in recs]) * 1e3
    adm = (np.concatenate([w[r["frame"]] for r, w in pairs]) * 1e3 if waits is not None
           else np.zeros(sum(len(r) for r in recs)))
    lat = cat(lambda r: r["t_ready"] - r["t_push"]) + adm
    out = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_ms": float(lat.mean()), "frames": int(lat.size),
           "from": "capture" if waits is not None else "push"}
    parts = [("buffering", lambda r: r["t_window"] - r["t_push"]),
             ("queueing", lambda r: r["t_batch"] - r["t_window"]),
             ("compute", lambda r: r["t_ready"] - r["t_batch"])]
    if waits is not None:
        out["admission"] = {"p50_ms": float(np.percentile(adm, 50)), "p99_ms": float(np.percentile(adm, 99)),
                            "mean_ms": float(adm.mean())}
    for name, f in parts:
        part = cat(f)
        out[name] = {"p50_ms": float(np.percentile(part, 50)), "p99_ms": float(np.percentile(part, 99)),
                     "mean_ms": float(part.mean())}
    return out
