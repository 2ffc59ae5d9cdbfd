"""Host logic of the serving loop (no GPU): admission by budget, pacing from capture times, and the
latency definition, on a fake engine with the binding's interface that emits every pushed frame at
once."""
import time

import numpy as np

from paper_2601_07154_amd import FOCUS_DTYPE, MF_EAGAIN, MF_ECLOSED, MF_OK, serving


class FakeEngine:
    """Admits one stream at a time (the budget); a pushed frame's record is ready immediately."""
    threaded = True

    def __init__(self):
        self.t0 = time.perf_counter()
        self.open = None
        self.ready, self.closed, self.count = {}, set(), {}
        self.next = 1

    def now(self):
        return time.perf_counter() - self.t0

    def open_stream(self, H, W, L, O, K, allow_again=False, **kw):
        if self.open is not None:
            return -1 if allow_again else MF_EAGAIN
        sid = self.next
        self.next += 1
        self.open = sid
        self.ready[sid] = []
        self.count[sid] = 0
        return sid

    def push_frames(self, sid, frames, eos=False, allow_again=False):
        t = self.now()
        for _ in range(frames.shape[0]):
            r = np.zeros(1, FOCUS_DTYPE)
            r["frame"] = self.count[sid]
            r["t_push"] = r["t_window"] = r["t_batch"] = t
            r["t_ready"] = t + 0.002
            self.count[sid] += 1
            self.ready[sid].append(r)
        if eos:
            self.closed.add(sid)
        return MF_OK

    def poll(self, sid, cap):
        out = self.ready[sid][:cap]
        self.ready[sid] = self.ready[sid][cap:]
        recs = np.concatenate(out) if out else np.zeros(0, FOCUS_DTYPE)
        if not self.ready[sid] and sid in self.closed:
            if self.open == sid:
                self.open = None
            return recs, MF_ECLOSED
        return recs, MF_OK

    def stats(self):
        return {}


def test_paced_latency_counts_from_capture_including_admission():
    eng = FakeEngine()
    fps = 200.0
    specs = [serving.StreamSpec(0.0, 20, 28, 28), serving.StreamSpec(0.005, 10, 28, 28)]
    pool = lambda H, W: np.zeros((4, 3, H, W), np.float32)
    out = serving.serve(eng, specs, pool, 8, 4, lambda H, W: (1.0, 1.0, 1.0, 1.0), fps=fps, paced=True,
                        time_limit=20)
    recs, waits = out["records"], out["waits"]
    assert [len(r) for r in recs] == [20, 10] and [len(w) for w in waits] == [20, 10]
    # the second stream arrives while the first holds the budget: its early frames wait to be admitted,
    # at least until the first stream's last capture (19 / fps after its arrival)
    assert waits[1][0] >= 19 / fps - 0.005 - 1e-3
    lat_cap = serving.latency_summary(recs, waits)
    lat_push = serving.latency_summary(recs)
    assert lat_cap["from"] == "capture" and lat_push["from"] == "push"
    assert lat_cap["admission"]["p99_ms"] >= 1e3 * (19 / fps - 0.005) - 1.0
    assert lat_cap["p99_ms"] > lat_push["p99_ms"]
    # every frame's latency from capture = its wait + its engine latency
    assert abs(lat_cap["mean_ms"] - (lat_push["mean_ms"] + lat_cap["admission"]["mean_ms"])) < 1e-6


def test_throughput_regime_counts_from_push():
    eng = FakeEngine()
    specs = [serving.StreamSpec(0.0, 12, 28, 28), serving.StreamSpec(0.0, 5, 28, 28)]
    pool = lambda H, W: np.zeros((4, 3, H, W), np.float32)
    out = serving.serve(eng, specs, pool, 8, 4, lambda H, W: (1.0, 1.0, 1.0, 1.0), paced=False, time_limit=20)
    assert all((w == 0).all() for w in out["waits"])
    lat = serving.latency_summary(out["records"])
    assert lat["frames"] == 17 and abs(lat["compute"]["mean_ms"] - 2.0) < 0.5
