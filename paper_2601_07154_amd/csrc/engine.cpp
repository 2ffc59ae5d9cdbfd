// Motion-focus engine: stream admission, the sliding-window schedule, continuous batching of
// ready windows across streams, result ordering, and the C ABI.  Plain C++; the device work
// is behind mf::Executor.
//
// Windows (Sec. 2.2): window k of a stream covers frames [s_k, s_k + L), s_k = k (L - O),
// while it fits; at end of stream a tail window [N - L, N) covers what is left, and a stream
// of N <= L frames is one window of N frames.  Window k emits the frames after those emitted
// by window k-1; its poses are anchored at the last of those (a frame both windows contain).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "engine.h"

namespace mf {

enum { CHAIN_ANCHOR_ = 0, CHAIN_FIRST_ = 1, CHAIN_WORLD_ = 2 };

static thread_local char g_err[512] = "";
static void set_err(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

struct PoseJob {
  int64_t start;
  int32_t size;
  int64_t emit_begin, emit_end;
  int32_t mode;
  int32_t window_id;
  std::vector<double> T;
};

struct Stream {
  int32_t id = 0;
  mf_stream_cfg cfg{};
  StreamRes res;
  int kind = 0;                 // 0 undecided, 1 frames, 2 poses
  int64_t pushed = 0;           // frames (or poses) received
  int64_t ring_lo = 0;          // oldest frame a future window may still read
  bool eos = false;
  double eos_time = 0.0;        // when eos was set
  int64_t next_start = 0;       // start of the next regular window
  int32_t next_k = 0;           // windows scheduled so far
  int64_t emitted_end = 0;      // frames scheduled for emission so far
  int64_t last_start = -1;
  bool windows_done = false;
  int inflight = 0;
  std::deque<PoseJob> pose_jobs;
  std::deque<mf_focus> ready;
  int64_t polled = 0;           // next frame to be handed out
  std::deque<double> push_time; // t_push of frames push_time_base ..
  int64_t push_time_base = 0;
  bool released = false;
  std::mutex io;                // serialises pushes and polls of this stream
};

struct Engine {
  std::unique_ptr<Executor> ex;
  mf_model_cfg model{};
  mf_runtime_cfg rt{};
  std::mutex run_mu;            // one batch at a time (mf_engine_step / mf_engine_sync may race)
  std::mutex mu;
  std::condition_variable cv;
  std::map<int32_t, std::shared_ptr<Stream>> streams;
  int32_t next_id = 1;
  int32_t rr = 0;               // round-robin cursor (stream id)
  uint64_t budget = 0, used = 0;
  bool broken = false;
  bool stop = false, dirty = false, running = false;
  std::thread worker;
  std::chrono::steady_clock::time_point t0;
  mf_stats st{};

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

// Frames of history the device looks back on beyond those a batch emits: the N map points, the
// anchor inside the window, and the 2 s frames of the centre differences.
static int hist_lookback(const mf_stream_cfg& c) { return c.n_points + c.window + 8 + 2 * c.diff_stride; }
// streams that keep per-frame maps (focus maps, depth maps) in result slots until they are polled
static bool keeps_results(const mf_stream_cfg& c) { return c.emit_maps || c.emit_depth; }

// ------------------------------------------------------------------ schedule
// The next window of a frame stream if all its frames are here (not committed).
static bool peek_window(const Stream& s, BatchWindow& w) {
  if (s.windows_done || s.kind != 1) return false;
  const int L = s.cfg.window;
  const int64_t N = s.pushed;
  int64_t start;
  int32_t size;
  if (s.next_start + L <= N) {
    start = s.next_start;
    size = L;
  } else if (!s.eos) {
    return false;
  } else if (s.next_k == 0) {
    if (N == 0) return false;
    start = 0;
    size = (int32_t)N;
  } else if (s.emitted_end < N) {
    start = N - L;
    size = L;
  } else {
    return false;
  }
  w.stream_id = s.id;
  w.window_id = s.next_k;
  w.chain_mode = s.next_k == 0 ? CHAIN_FIRST_ : CHAIN_ANCHOR_;
  w.start = start;
  w.size = size;
  w.emit_begin = s.emitted_end;
  w.emit_end = start + size;
  w.poses = nullptr;
  return true;
}

static void commit_window(Stream& s, const BatchWindow& w) {
  const int stride = s.cfg.window - s.cfg.overlap;
  s.next_k++;
  s.emitted_end = w.emit_end;
  s.last_start = w.start;
  if (w.start == s.next_start && w.size == s.cfg.window) s.next_start = w.start + stride;
  else s.windows_done = true;   // short stream or tail window
  if (s.eos && s.emitted_end == s.pushed) s.windows_done = true;
  s.inflight++;
}

static bool maps_fit(const Stream& s, int64_t emit_end) {
  return !keeps_results(s.cfg) || emit_end - s.polled <= s.res.map_cap;
}

static bool work_ready_locked(Engine& e) {
  for (auto& kv : e.streams) {
    Stream& s = *kv.second;
    if (s.released) continue;
    BatchWindow w;
    if (peek_window(s, w) && maps_fit(s, w.emit_end)) return true;
    if (!s.pose_jobs.empty() && maps_fit(s, s.pose_jobs.front().emit_end)) return true;
  }
  return false;
}

// Gather ready windows of every stream (round robin from the cursor) up to the token budget,
// run them as one batch and hand the results to the streams.  Returns windows run, or < 0.
static int step(Engine& e) {
  std::lock_guard<std::mutex> run(e.run_mu);
  Batch b;
  std::vector<std::vector<double>> pose_store;
  std::vector<int> pose_idx;   // per batch window: index into pose_store or -1
  {
    std::lock_guard<std::mutex> lk(e.mu);
    if (e.broken) {
      set_err("engine is in a failed state after a device error");
      return MF_EDEVICE;
    }
    std::vector<std::shared_ptr<Stream>> order;
    for (auto it = e.streams.lower_bound(e.rr); it != e.streams.end(); ++it) order.push_back(it->second);
    for (auto it = e.streams.begin(); it != e.streams.end() && it->first < e.rr; ++it)
      order.push_back(it->second);
    const int64_t cap = e.ex->max_tokens();
    const int64_t fcap = e.ex->max_frames();
    int64_t frames_in = 0;   // T_loc rows (window frames) of the batch; emitted records <= this
    bool full = false;
    for (auto& sp : order) {
      Stream& s = *sp;
      if (s.released) continue;
      // frames one stream may emit in a batch: its device history must still hold the
      // accelerations the maps of the oldest of them read
      const int64_t span = s.res.hist_n - hist_lookback(s.cfg);
      int64_t emitted_here = 0;
      if (s.kind == 1) {
        const int64_t rows = e.ex->rows_per_frame(s.cfg.height, s.cfg.width);
        BatchWindow w;
        while (peek_window(s, w)) {
          if (!maps_fit(s, w.emit_end)) break;
          if (b.tokens + rows * w.size > cap || frames_in + w.size > fcap ||
              (emitted_here > 0 && emitted_here + (w.emit_end - w.emit_begin) > span)) {
            full = true;
            break;
          }
          frames_in += w.size;
          emitted_here += w.emit_end - w.emit_begin;
          w.cfg = &s.cfg;
          w.res = &s.res;
          commit_window(s, w);
          b.wins.push_back(w);
          pose_idx.push_back(-1);
          b.tokens += rows * w.size;
        }
      } else if (s.kind == 2) {
        while (!s.pose_jobs.empty() && maps_fit(s, s.pose_jobs.front().emit_end)) {
          PoseJob& j = s.pose_jobs.front();
          if (frames_in + j.size > fcap || (emitted_here > 0 && emitted_here + (j.emit_end - j.emit_begin) > span)) {
            full = true;
            break;
          }
          frames_in += j.size;
          emitted_here += j.emit_end - j.emit_begin;
          BatchWindow w;
          w.stream_id = s.id;
          w.cfg = &s.cfg;
          w.res = &s.res;
          w.window_id = j.window_id;
          w.chain_mode = j.mode;
          w.start = j.start;
          w.size = j.size;
          w.emit_begin = j.emit_begin;
          w.emit_end = j.emit_end;
          w.poses = nullptr;
          pose_idx.push_back((int)pose_store.size());
          pose_store.push_back(std::move(j.T));
          b.wins.push_back(w);
          s.inflight++;
          s.pose_jobs.pop_front();
        }
      }
      if (full) {
        e.rr = s.id;   // this stream goes first next time
        break;
      }
    }
    if (!full && !order.empty()) e.rr = order.front()->id + 1;
    if (b.wins.empty()) return 0;
    e.running = true;
  }
  for (size_t i = 0; i < b.wins.size(); ++i)
    if (pose_idx[i] >= 0) b.wins[i].poses = pose_store[pose_idx[i]].data();

  std::vector<mf_focus> out;
  std::string err;
  double ms = 0.0;
  const double t_batch = e.now();
  const mf_status rc = e.ex->run_batch(b, out, &ms, err);
  const double t_ready = e.now();

  std::lock_guard<std::mutex> lk(e.mu);
  e.running = false;
  if (rc != MF_OK) {
    e.broken = true;
    set_err("%s", err.c_str());
    e.cv.notify_all();
    return rc;
  }
  size_t k = 0;
  for (auto& w : b.wins) {
    Stream& s = *e.streams.at(w.stream_id);
    // the window was complete when its last frame arrived; a window cut short by the end of the
    // stream (tail or only window) also needed the end of stream
    const int64_t tl = w.emit_end - 1 - s.push_time_base;
    double t_window = (tl >= 0 && tl < (int64_t)s.push_time.size()) ? s.push_time[tl] : 0.0;
    const int stride = s.cfg.window - s.cfg.overlap;
    const bool regular = s.kind == 1 && w.size == s.cfg.window && stride > 0 && w.start % stride == 0;
    if (!regular && s.eos) t_window = std::max(t_window, s.eos_time);
    for (int64_t t = w.emit_begin; t < w.emit_end; ++t, ++k) {
      mf_focus r = out[k];
      const int64_t ti = t - s.push_time_base;
      r.t_push = (ti >= 0 && ti < (int64_t)s.push_time.size()) ? s.push_time[ti] : 0.0;
      r.t_window = std::max(t_window, r.t_push);
      r.t_batch = std::max(t_batch, r.t_window);
      r.t_ready = t_ready;
      s.ready.push_back(r);
    }
    s.inflight--;
    if (s.kind == 1) s.ring_lo = s.windows_done ? s.pushed : std::max(s.ring_lo, s.last_start + 1);
    while (!s.push_time.empty() && s.push_time_base < w.emit_end) {
      s.push_time.pop_front();
      s.push_time_base++;
    }
    e.st.frames_emitted += w.emit_end - w.emit_begin;
    e.st.windows_run++;
  }
  e.st.batches_run++;
  e.st.tokens_run += b.tokens;
  e.st.gpu_ms += ms;
  e.st.frames_embed_shared += e.ex->last_batch_shared();
  e.cv.notify_all();
  return (int)b.wins.size();
}

static void worker_loop(Engine* e) {
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(e->mu);
      e->cv.wait(lk, [&] { return e->stop || e->dirty; });
      if (e->stop) return;
      e->dirty = false;
      e->running = true;
    }
    for (;;) {
      const int n = step(*e);
      if (n <= 0) break;
    }
    std::lock_guard<std::mutex> lk(e->mu);
    e->running = false;
    e->cv.notify_all();
  }
}

static void poke(Engine& e) {   // caller holds e.mu
  e.dirty = true;
  e.cv.notify_all();
}

static std::shared_ptr<Stream> find_locked(Engine& e, int32_t id) {
  auto it = e.streams.find(id);
  if (it == e.streams.end() || it->second->released) return nullptr;
  return it->second;
}

}  // namespace mf

using namespace mf;

struct mf_engine : public Engine {};

#define GUARD_BEGIN try {
#define GUARD_END                             \
  }                                           \
  catch (const std::exception& ex) {          \
    set_err("internal error: %s", ex.what()); \
    return MF_EINVAL;                         \
  }                                           \
  catch (...) {                               \
    set_err("internal error");                \
    return MF_EINVAL;                         \
  }

extern "C" {

const char* mf_status_str(mf_status s) {
  switch (s) {
    case MF_OK: return "ok";
    case MF_EINVAL: return "invalid argument";
    case MF_ENOMEM: return "does not fit the HBM budget";
    case MF_EAGAIN: return "try again";
    case MF_ECLOSED: return "stream closed";
    case MF_EDEVICE: return "device error";
    case MF_ENOTFOUND: return "unknown stream";
  }
  return "unknown status";
}

const char* mf_last_error(void) { return g_err; }

mf_status mf_engine_create(const mf_model_cfg* model, const float* weights, size_t n_floats,
                           const mf_runtime_cfg* rt, mf_engine** out) {
  GUARD_BEGIN
  if (!model || !weights || !out) {
    set_err("null argument");
    return MF_EINVAL;
  }
  *out = nullptr;
  mf_runtime_cfg r{};
  if (rt) r = *rt;
  std::unique_ptr<mf_engine> e(new mf_engine());
  e->model = *model;
  e->rt = r;
  e->t0 = std::chrono::steady_clock::now();
  e->ex.reset(make_executor());
  std::string err;
  const mf_status rc = e->ex->init(*model, weights, n_floats, r, err);
  if (rc != MF_OK) {
    set_err("%s", err.c_str());
    return rc;
  }
  e->budget = e->ex->budget_bytes();
  e->used = e->ex->fixed_bytes();
  if (r.threaded) e->worker = std::thread(worker_loop, e.get());
  *out = e.release();
  return MF_OK;
  GUARD_END
}

void mf_engine_destroy(mf_engine* e) {
  if (!e) return;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    e->stop = true;
    e->cv.notify_all();
  }
  if (e->worker.joinable()) e->worker.join();
  for (auto& kv : e->streams)
    if (!kv.second->released) e->ex->close_stream(&kv.second->res);
  e->streams.clear();
  delete e;
}

mf_status mf_open_stream(mf_engine* e, const mf_stream_cfg* cfg, int32_t* stream_id) {
  GUARD_BEGIN
  if (!e || !cfg || !stream_id) {
    set_err("null argument");
    return MF_EINVAL;
  }
  mf_stream_cfg c = *cfg;
  if (c.height <= 0 || c.width <= 0 || c.height % 14 || c.width % 14) {
    set_err("frame size %dx%d must be positive multiples of 14", c.height, c.width);
    return MF_EINVAL;
  }
  if (c.window < 1 || c.overlap < 1 || c.overlap >= c.window) {
    set_err("need 1 <= overlap < window (got window %d overlap %d)", c.window, c.overlap);
    return MF_EINVAL;
  }
  if (c.n_points < 1 || c.n_points > 32) {
    set_err("n_points must be in 1..32");
    return MF_EINVAL;
  }
  if (c.anchor_mode != MF_ANCHOR_YAW && c.anchor_mode != MF_ANCHOR_SE3 && c.anchor_mode != MF_ANCHOR_YAW_SCALE) {
    set_err("unknown anchor mode %d", c.anchor_mode);
    return MF_EINVAL;
  }
  if (c.focus_mode != MF_FOCUS_ACCEL && c.focus_mode != MF_FOCUS_VELOCITY) {
    set_err("unknown focus mode %d", c.focus_mode);
    return MF_EINVAL;
  }
  if (c.map_mode != MF_MAP_MAX && c.map_mode != MF_MAP_SUM) {
    set_err("unknown map mode %d", c.map_mode);
    return MF_EINVAL;
  }
  if (c.emit_depth && !e->model.depth_head) {
    set_err("emit_depth needs a model with a depth head");
    return MF_EINVAL;
  }
  if (c.diff_stride == 0) c.diff_stride = 1;
  if (c.diff_stride < 1 || c.diff_stride > 64) {
    set_err("diff_stride must be in 1..64");
    return MF_EINVAL;
  }
  if (!(c.fx != 0.0) || !(c.fy != 0.0)) {
    set_err("focal lengths must be non-zero");
    return MF_EINVAL;
  }
  if (c.sigma_min <= 0.0) c.sigma_min = 0.5;
  if (c.sigma_max <= 0.0) c.sigma_max = 4.0 * std::max(c.height, c.width);
  if (c.sigma_max < c.sigma_min) {
    set_err("sigma_max < sigma_min");
    return MF_EINVAL;
  }
  if (c.ring_frames <= 0) c.ring_frames = 2 * c.window + 8;
  if (c.ring_frames < c.window) {
    set_err("ring_frames must be >= window");
    return MF_EINVAL;
  }
  if (c.result_frames <= 0) c.result_frames = 4 * c.window;
  if (c.result_frames < c.window) {
    set_err("result_frames must be >= window");
    return MF_EINVAL;
  }
  const int64_t rows = (int64_t)c.window * e->ex->rows_per_frame(c.height, c.width);
  if (rows > e->ex->max_tokens()) {
    set_err("a window of %d frames (%lld token rows) exceeds the batch token budget %lld", c.window,
            (long long)rows, (long long)e->ex->max_tokens());
    return MF_EINVAL;
  }
  // history ring: the frames one batch may emit for this stream (at least 8 windows' worth),
  // plus what the maps, the anchor and the differences look back on
  int hist_n = 64;
  while (hist_n < std::max(8 * c.window, 256) + hist_lookback(c)) hist_n *= 2;
  const uint64_t need = e->ex->stream_bytes(c, c.ring_frames, keeps_results(c) ? c.result_frames : 0, hist_n);
  auto s = std::make_shared<Stream>();
  {
    std::lock_guard<std::mutex> lk(e->mu);
    if (e->broken) {
      set_err("engine is in a failed state after a device error");
      return MF_EDEVICE;
    }
    const uint64_t fixed = e->ex->fixed_bytes();
    if (fixed + need > e->budget) {
      set_err("stream needs %llu bytes; budget %llu minus fixed %llu can never hold it",
              (unsigned long long)need, (unsigned long long)e->budget, (unsigned long long)fixed);
      return MF_ENOMEM;
    }
    if (e->used + need > e->budget) {
      set_err("HBM budget in use by other streams (%llu of %llu bytes)", (unsigned long long)e->used,
              (unsigned long long)e->budget);
      e->st.streams_pending++;
      return MF_EAGAIN;
    }
    e->used += need;   // reserve before allocating outside the lock
  }
  s->cfg = c;
  s->res.ring_cap = c.ring_frames;
  s->res.map_cap = keeps_results(c) ? c.result_frames : 0;
  s->res.hist_n = hist_n;
  std::string err;
  const mf_status rc = e->ex->open_stream(c, &s->res, err);
  std::lock_guard<std::mutex> lk(e->mu);
  if (rc != MF_OK) {
    e->used -= need;
    set_err("%s", err.c_str());
    return rc;
  }
  s->res.bytes = need;
  s->id = e->next_id++;
  e->streams[s->id] = s;
  e->st.streams_open++;
  *stream_id = s->id;
  return MF_OK;
  GUARD_END
}

mf_status mf_push_frames(mf_engine* e, int32_t stream_id, const float* rgb, int32_t n, int32_t flags) {
  GUARD_BEGIN
  if (!e || (n > 0 && !rgb) || n < 0) {
    set_err("bad arguments");
    return MF_EINVAL;
  }
  std::shared_ptr<Stream> s;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    s = find_locked(*e, stream_id);
  }
  if (!s) {
    set_err("unknown stream %d", stream_id);
    return MF_ENOTFOUND;
  }
  std::lock_guard<std::mutex> io(s->io);
  int64_t first;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    if (e->broken) {
      set_err("engine is in a failed state after a device error");
      return MF_EDEVICE;
    }
    if (s->eos) {
      set_err("stream %d is closed", stream_id);
      return MF_ECLOSED;
    }
    if (s->kind == 2) {
      set_err("stream %d takes poses, not frames", stream_id);
      return MF_EINVAL;
    }
    if (s->pushed + n - s->ring_lo > s->res.ring_cap) {
      set_err("frame ring full (%d frames): poll results and retry", s->res.ring_cap);
      return MF_EAGAIN;
    }
    first = s->pushed;
    s->kind = 1;
  }
  if (n > 0) {
    std::string err;
    const mf_status rc = e->ex->upload_frames(s->cfg, &s->res, first, rgb, n, (flags & MF_DEVICE_PTR) != 0, err);
    if (rc != MF_OK) {
      set_err("%s", err.c_str());
      return rc;
    }
  }
  std::lock_guard<std::mutex> lk(e->mu);
  const double t = e->now();
  for (int i = 0; i < n; ++i) s->push_time.push_back(t);
  s->pushed += n;
  e->st.frames_pushed += n;
  if ((flags & MF_EOS) && !s->eos) {
    s->eos = true;
    s->eos_time = t;
  }
  poke(*e);
  return MF_OK;
  GUARD_END
}

mf_status mf_push_poses(mf_engine* e, int32_t stream_id, const double* T, int32_t n, int64_t first_frame,
                        int32_t flags) {
  GUARD_BEGIN
  if (!e || n < 0 || (n > 0 && !T)) {
    set_err("bad arguments");
    return MF_EINVAL;
  }
  std::lock_guard<std::mutex> lk(e->mu);
  auto s = find_locked(*e, stream_id);
  if (!s) {
    set_err("unknown stream %d", stream_id);
    return MF_ENOTFOUND;
  }
  if (s->eos) {
    set_err("stream %d is closed", stream_id);
    return MF_ECLOSED;
  }
  if (s->kind == 1) {
    set_err("stream %d takes frames, not poses", stream_id);
    return MF_EINVAL;
  }
  if (s->cfg.emit_depth) {
    set_err("stream %d emits depth maps: depth comes from frames, not poses", stream_id);
    return MF_EINVAL;
  }
  if (n > e->ex->max_frames()) {
    set_err("at most %lld poses per call", (long long)e->ex->max_frames());
    return MF_EINVAL;
  }
  if (n > 0) {
    PoseJob j;
    j.start = first_frame;
    j.size = n;
    j.window_id = s->next_k;
    if (flags & MF_POSES_LOCAL) {
      if (n > s->cfg.window) {
        set_err("a window of local poses has at most %d frames", s->cfg.window);
        return MF_EINVAL;
      }
      if (s->emitted_end == 0) {
        if (first_frame != 0) {
          set_err("the first window of local poses must start at frame 0");
          return MF_EINVAL;
        }
        j.mode = CHAIN_FIRST_;
      } else {
        if (first_frame > s->emitted_end - 1 || first_frame < 0 || first_frame + n <= s->emitted_end) {
          set_err("window [%lld, %lld) must contain frame %lld (the anchor) and extend past it",
                  (long long)first_frame, (long long)(first_frame + n), (long long)(s->emitted_end - 1));
          return MF_EINVAL;
        }
        j.mode = CHAIN_ANCHOR_;
      }
      j.emit_begin = s->emitted_end;
      j.emit_end = first_frame + n;
    } else {
      if (first_frame != s->emitted_end) {
        set_err("world poses must continue the stream at frame %lld", (long long)s->emitted_end);
        return MF_EINVAL;
      }
      const int span = s->res.hist_n - hist_lookback(s->cfg);
      if (n > span) {
        set_err("push at most %d world poses per call", span);
        return MF_EINVAL;
      }
      j.mode = CHAIN_WORLD_;
      j.emit_begin = first_frame;
      j.emit_end = first_frame + n;
    }
    if (keeps_results(s->cfg) && j.emit_end - j.emit_begin > s->res.map_cap) {
      set_err("%lld frames at once exceed result_frames %d", (long long)(j.emit_end - j.emit_begin),
              s->res.map_cap);
      return MF_EINVAL;
    }
    j.T.assign(T, T + (size_t)n * 16);
    const double t = e->now();
    for (int64_t f = s->emitted_end; f < j.emit_end; ++f) s->push_time.push_back(t);
    s->kind = 2;
    s->next_k++;
    s->emitted_end = j.emit_end;
    s->pushed = j.emit_end;
    e->st.frames_pushed += j.emit_end - j.emit_begin;
    s->pose_jobs.push_back(std::move(j));
  }
  if (flags & MF_EOS) {
    if (!s->eos) s->eos_time = e->now();
    s->eos = true;
    s->windows_done = true;
  }
  poke(*e);
  return MF_OK;
  GUARD_END
}

mf_status mf_poll_focus(mf_engine* e, int32_t stream_id, mf_focus* out, int32_t cap, int32_t* n_out,
                        float* maps, int32_t maps_flags) {
  return mf_poll_focus_depth(e, stream_id, out, cap, n_out, maps, nullptr, maps_flags);
}

mf_status mf_poll_focus_depth(mf_engine* e, int32_t stream_id, mf_focus* out, int32_t cap, int32_t* n_out,
                              float* maps, float* depth, int32_t maps_flags) {
  GUARD_BEGIN
  if (!e || !n_out || cap < 0 || (cap > 0 && !out)) {
    set_err("bad arguments");
    return MF_EINVAL;
  }
  *n_out = 0;
  std::shared_ptr<Stream> s;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    s = find_locked(*e, stream_id);
  }
  if (!s) {
    set_err("unknown stream %d", stream_id);
    return MF_ENOTFOUND;
  }
  if (depth && !s->cfg.emit_depth) {
    set_err("stream %d was opened without emit_depth", stream_id);
    return MF_EINVAL;
  }
  std::lock_guard<std::mutex> io(s->io);
  int32_t k = 0;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    if (e->broken) {
      set_err("engine is in a failed state after a device error");
      return MF_EDEVICE;
    }
    k = (int32_t)std::min<size_t>((size_t)cap, s->ready.size());
    for (int32_t i = 0; i < k; ++i) out[i] = s->ready[i];
    if (k == 0) {
      const bool drained = s->eos && s->inflight == 0 && s->pose_jobs.empty() &&
                           (s->kind != 1 || s->windows_done || s->pushed == 0);
      BatchWindow w;
      const bool more = s->kind == 1 && peek_window(*s, w);
      if (drained && !more) {
        e->ex->close_stream(&s->res);
        e->used -= s->res.bytes;
        s->released = true;
        e->streams.erase(stream_id);
        e->st.streams_open--;
        poke(*e);
        set_err("stream %d closed and drained", stream_id);
        return MF_ECLOSED;
      }
      set_err("no result ready");
      return MF_EAGAIN;
    }
  }
  // copy the maps before releasing their ring slots (the scheduler may reuse them afterwards)
  for (int kind = 0; kind < 2; ++kind) {
    float* dst = kind == 0 ? (s->cfg.emit_maps ? maps : nullptr) : (s->cfg.emit_depth ? depth : nullptr);
    if (!dst) continue;
    const int64_t hw = (int64_t)s->cfg.height * s->cfg.width;
    int32_t i = 0;
    while (i < k) {
      const int64_t f0 = out[i].frame;
      int32_t run = 1;
      while (i + run < k && out[i + run].frame == f0 + run && (f0 + run) % s->res.map_cap != 0) ++run;
      std::string err;
      const bool dev = (maps_flags & MF_DEVICE_PTR) != 0;
      const mf_status rc = kind == 0 ? e->ex->copy_maps(s->cfg, &s->res, f0, run, dst + (int64_t)i * hw, dev, err)
                                     : e->ex->copy_depth(s->cfg, &s->res, f0, run, dst + (int64_t)i * hw, dev, err);
      if (rc != MF_OK) {
        set_err("%s", err.c_str());
        return rc;
      }
      i += run;
    }
  }
  std::lock_guard<std::mutex> lk(e->mu);
  for (int32_t i = 0; i < k; ++i) s->ready.pop_front();
  s->polled += k;
  *n_out = k;
  poke(*e);
  return MF_OK;
  GUARD_END
}

mf_status mf_close_stream(mf_engine* e, int32_t stream_id) {
  GUARD_BEGIN
  if (!e) return MF_EINVAL;
  std::lock_guard<std::mutex> lk(e->mu);
  auto s = find_locked(*e, stream_id);
  if (!s) {
    set_err("unknown stream %d", stream_id);
    return MF_ENOTFOUND;
  }
  if (!s->eos) s->eos_time = e->now();
  s->eos = true;
  if (s->kind != 1) s->windows_done = true;
  poke(*e);
  return MF_OK;
  GUARD_END
}

mf_status mf_engine_step(mf_engine* e, int32_t* n_windows) {
  GUARD_BEGIN
  if (!e) return MF_EINVAL;
  if (e->rt.threaded) {
    set_err("mf_engine_step is for engines without a scheduler thread");
    return MF_EINVAL;
  }
  const int n = step(*e);
  if (n_windows) *n_windows = n < 0 ? 0 : n;
  return n < 0 ? n : MF_OK;
  GUARD_END
}

mf_status mf_engine_sync(mf_engine* e) {
  GUARD_BEGIN
  if (!e) return MF_EINVAL;
  if (!e->rt.threaded) {
    for (;;) {
      const int n = step(*e);
      if (n < 0) return n;
      if (n == 0) return MF_OK;
    }
  }
  std::unique_lock<std::mutex> lk(e->mu);
  e->cv.wait(lk, [&] { return e->broken || (!e->dirty && !e->running && !work_ready_locked(*e)); });
  if (e->broken) {
    set_err("engine is in a failed state after a device error");
    return MF_EDEVICE;
  }
  return MF_OK;
  GUARD_END
}

mf_status mf_engine_stats(mf_engine* e, mf_stats* out) {
  if (!e || !out) return MF_EINVAL;
  std::lock_guard<std::mutex> lk(e->mu);
  *out = e->st;
  out->hbm_used_bytes = e->used;
  out->hbm_budget_bytes = e->budget;
  return MF_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ op-level entry points
#include "../../include/mf_ops.h"

extern "C" {

mf_status mf_forward_window(mf_engine* e, const float* frames_dev, int32_t S, int32_t height, int32_t width,
                            int32_t max_layers, float* pose9, double* T, float* tokens) {
  GUARD_BEGIN
  if (!e || !frames_dev || S < 1) {
    set_err("bad arguments");
    return MF_EINVAL;
  }
  std::lock_guard<std::mutex> lk(e->mu);
  if (e->running) {
    set_err("engine busy");
    return MF_EAGAIN;
  }
  const int64_t rows = (int64_t)S * e->ex->rows_per_frame(height, width);
  if (rows > e->ex->max_tokens()) {
    set_err("window of %lld rows exceeds the token budget", (long long)rows);
    return MF_EINVAL;
  }
  std::string err;
  const mf_status rc = e->ex->forward_frames(frames_dev, S, height, width, pose9, T, max_layers, tokens, err);
  if (rc != MF_OK) set_err("%s", err.c_str());
  return rc;
  GUARD_END
}

mf_status mf_debug_copy(mf_engine* e, int32_t which, void* host, size_t bytes) {
  GUARD_BEGIN
  if (!e || !host) return MF_EINVAL;
  std::lock_guard<std::mutex> lk(e->mu);
  if (e->running) {
    set_err("engine busy");
    return MF_EAGAIN;
  }
  std::string err;
  const mf_status rc = e->ex->debug_copy(which, host, bytes, err);
  if (rc != MF_OK) set_err("%s", err.c_str());
  return rc;
  GUARD_END
}

mf_status mf_profile(mf_engine* e, int32_t enable, double* ag, int64_t* calls, double* af, double* gm) {
  if (!e) return MF_EINVAL;
  std::lock_guard<std::mutex> lk(e->mu);
  e->ex->profile(ag, calls, af, gm, enable);
  return MF_OK;
}

mf_status mf_profile_stages(mf_engine* e, double* ms, int64_t* calls, int32_t n) {
  if (!e || n < 0) return MF_EINVAL;
  std::lock_guard<std::mutex> lk(e->mu);
  e->ex->profile_stages(ms, calls, n < MF_STAGE_COUNT ? n : MF_STAGE_COUNT);
  return MF_OK;
}

}  // extern "C"
