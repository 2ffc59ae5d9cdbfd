// CPU stand-in for the device executor, used only by the host-logic tests: it links the real
// scheduler and C ABI (engine.cpp) against an executor that computes nothing.  Each emitted
// record describes where it came from so the tests can check the schedule:
//   T_w2c[3] = frame index, pose9[0] = window start, pose9[1] = window size,
//   pose9[2] = batch ordinal, pose9[3] = frames of the same stream in that batch.
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../paper_2601_07154_amd/csrc/engine.h"

namespace mf {

class StubExecutor : public Executor {
 public:
  mf_status init(const mf_model_cfg& m, const float*, size_t n, const mf_runtime_cfg& rt, std::string& err) override {
    if (m.dim <= 0 || m.depth <= 0) { err = "bad model"; return MF_EINVAL; }
    (void)n;
    budget_ = rt.hbm_budget_bytes ? rt.hbm_budget_bytes : (1ull << 30);
    mcap_ = rt.max_tokens_per_batch > 0 ? rt.max_tokens_per_batch : 262144;
    fixed_ = 1 << 20;
    if (fixed_ > budget_) { err = "budget below the fixed workspace"; return MF_ENOMEM; }
    return MF_OK;
  }
  uint64_t fixed_bytes() const override { return fixed_; }
  uint64_t budget_bytes() const override { return budget_; }
  int64_t max_tokens() const override { return mcap_; }
  int64_t max_frames() const override { return mcap_ / 8 + 64; }
  int rows_per_frame(int H, int W) const override { return ((H / 14) * (W / 14) + 1 + 7) / 8 * 8; }
  uint64_t stream_bytes(const mf_stream_cfg& c, int ring_cap, int map_cap, int hist_n) const override {
    const uint64_t hw = (uint64_t)c.height * c.width;
    const uint64_t rings = (c.emit_maps ? 1 : 0) + (c.emit_depth ? 1 : 0);
    return (uint64_t)ring_cap * 3 * hw * 4 + rings * map_cap * hw * 4 + (uint64_t)hist_n * 168;
  }
  // Shared state as the device executor has it: a per-resolution table that stream opens extend
  // (opens run on API threads, outside the engine lock) and a profiling switch that API threads
  // flip while the scheduler thread runs batches.  The locks mirror the device executor's, so the
  // race test exercises the same discipline.
  mf_status open_stream(const mf_stream_cfg& c, StreamRes* r, std::string&) override {
    r->ring = (void*)0x1;
    std::lock_guard<std::mutex> lk(pe_mu_);
    auto key = std::make_pair(c.height / 14, c.width / 14);
    auto it = pe_index_.find(key);
    if (it == pe_index_.end()) {
      pe_index_[key] = pe_rows_;
      r->pe_base = pe_rows_;
      pe_rows_ += key.first * key.second;
    } else {
      r->pe_base = it->second;
    }
    return MF_OK;
  }
  void close_stream(StreamRes* r) override { r->ring = nullptr; }
  mf_status upload_frames(const mf_stream_cfg&, StreamRes*, int64_t, const float*, int, bool, std::string&) override {
    return MF_OK;
  }
  mf_status run_batch(const Batch& b, std::vector<mf_focus>& out, double* ms, std::string&) override {
    bool prof;
    {
      std::lock_guard<std::mutex> lk(prof_mu_);
      prof = profiling_;
    }
    ++batches_;
    for (const BatchWindow& w : b.wins) {
      int same = 0;
      for (const BatchWindow& x : b.wins)
        if (x.stream_id == w.stream_id) same += (int)(x.emit_end - x.emit_begin);
      for (int64_t t = w.emit_begin; t < w.emit_end; ++t) {
        mf_focus r;
        memset(&r, 0, sizeof r);
        r.frame = t;
        r.window = w.window_id;
        for (int i = 0; i < 16; ++i) r.T_w2c[i] = (i % 5 == 0) ? 1.0 : 0.0;
        r.T_w2c[3] = (double)t;
        r.pose9[0] = (float)w.start;
        r.pose9[1] = (float)w.size;
        r.pose9[2] = (float)batches_;
        r.pose9[3] = (float)same;
        if (w.poses) r.T_w2c[7] = w.poses[(t - w.start) * 16 + 3];   // echo the pushed pose
        out.push_back(r);
      }
    }
    if (ms) *ms = 0.0;
    if (prof) {
      std::lock_guard<std::mutex> lk(prof_mu_);
      prof_batches_ += 1.0;
    }
    return MF_OK;
  }
  mf_status copy_maps(const mf_stream_cfg& c, StreamRes*, int64_t frame, int n, float* dst, bool, std::string&) override {
    const size_t hw = (size_t)c.height * c.width;
    for (int i = 0; i < n; ++i)
      for (size_t p = 0; p < hw; ++p) dst[i * hw + p] = (float)(frame + i);
    return MF_OK;
  }
  mf_status forward_frames(const float*, int, int, int, float*, double*, int, float*, std::string& err) override {
    err = "no device";
    return MF_EDEVICE;
  }
  mf_status debug_copy(int, void*, size_t, std::string& err) override {
    err = "no device";
    return MF_EDEVICE;
  }
  void profile(double* ag, int64_t* calls, double*, double*, int enable) override {
    std::lock_guard<std::mutex> lk(prof_mu_);
    if (ag) *ag = prof_batches_;
    if (calls) *calls = 0;
    if (enable >= 0) {
      profiling_ = enable != 0;
      prof_batches_ = 0.0;
    }
  }

 private:
  uint64_t budget_ = 0, fixed_ = 0;
  int64_t mcap_ = 0;
  int batches_ = 0;
  std::mutex pe_mu_, prof_mu_;
  std::map<std::pair<int, int>, int> pe_index_;
  int pe_rows_ = 0;
  bool profiling_ = false;
  double prof_batches_ = 0.0;
};

Executor* make_executor() { return new StubExecutor(); }

}  // namespace mf
