// Race check of the threaded engine (built with -fsanitize=thread against the stub executor):
// several streams pushed and polled from their own threads while the scheduler thread runs
// batches; every stream must come back complete and in order.
#include <stdio.h>
#include <string.h>

#include <thread>
#include <vector>

#include "mf.h"
#include "mf_ops.h"

#include <mutex>

static int run_stream(mf_engine* e, int n, int res, int* bad) {
  mf_stream_cfg c;
  memset(&c, 0, sizeof c);
  c.height = 28 + 14 * res; c.width = 28; c.window = 8; c.overlap = 4;
  c.fx = c.fy = 50; c.cx = c.cy = 14; c.n_points = 15; c.sigma = 1.0; c.ring_frames = 16;
  int32_t sid;
  while (mf_open_stream(e, &c, &sid) == MF_EAGAIN) std::this_thread::yield();
  std::vector<float> fr(3 * c.height * c.width, 0.0f);
  int pushed = 0;
  int64_t next = 0;
  mf_focus out[32];
  for (;;) {
    if (pushed < n) {
      const mf_status st = mf_push_frames(e, sid, fr.data(), 1, pushed + 1 == n ? MF_EOS : 0);
      if (st == MF_OK) ++pushed;
      else if (st != MF_EAGAIN) { ++*bad; return 1; }
    }
    int32_t k = 0;
    const mf_status st = mf_poll_focus(e, sid, out, 32, &k, nullptr, 0);
    for (int i = 0; i < k; ++i)
      if (out[i].frame != next++) ++*bad;
    if (st == MF_ECLOSED) break;
    if (st != MF_OK && st != MF_EAGAIN) { ++*bad; return 1; }
  }
  if (next != n) ++*bad;
  return 0;
}

int main() {
  mf_model_cfg m = {2, 128, 4, 512, 14, MF_BF16};
  mf_runtime_cfg rt;
  memset(&rt, 0, sizeof rt);
  rt.threaded = 1;
  rt.hbm_budget_bytes = 4u << 20;   // admits a few streams at a time
  float w = 0.0f;
  mf_engine* e = nullptr;
  if (mf_engine_create(&m, &w, 1, &rt, &e) != MF_OK) { printf("create failed: %s\n", mf_last_error()); return 2; }
  int bad[6] = {0};
  std::vector<std::thread> th;
  // streams of three resolutions opened from their own threads (the executor's per-resolution table
  // grows concurrently), while another thread switches per-kernel profiling on and off
  for (int i = 0; i < 6; ++i) th.emplace_back([&, i] { run_stream(e, 30 + 7 * i, i % 3, &bad[i]); });
  bool stop = false;
  std::mutex stop_mu;
  std::thread prof([&] {
    for (int k = 0;; ++k) {
      {
        std::lock_guard<std::mutex> lk(stop_mu);
        if (stop) break;
      }
      double ms = 0.0;
      int64_t calls = 0;
      mf_profile(e, k & 1, &ms, &calls, nullptr, nullptr);
      std::this_thread::yield();
    }
  });
  for (auto& t : th) t.join();
  {
    std::lock_guard<std::mutex> lk(stop_mu);
    stop = true;
  }
  prof.join();
  mf_stats st;
  mf_engine_stats(e, &st);
  mf_engine_destroy(e);
  int tot = 0;
  for (int b : bad) tot += b;
  printf("streams done: bad=%d batches=%lld emitted=%lld\n", tot, (long long)st.batches_run, (long long)st.frames_emitted);
  return tot ? 1 : 0;
}
