// Scheduler-side types of the motion-focus engine (plain C++, no HIP): streams, windows,
// batches, and the executor interface that runs a batch on a device.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mf.h"

namespace mf {

// Device resources of one stream, owned by the executor.
struct StreamRes {
  void* ring = nullptr;      // frame ring [ring_cap][3][H][W] fp32
  void* maps = nullptr;      // map ring [map_cap][H][W] fp32 (emit_maps)
  void* depth = nullptr;     // depth-map ring [map_cap][H][W] fp32 (emit_depth)
  void* hist = nullptr;      // FP64 pose/acceleration history [hist_n]
  int ring_cap = 0, map_cap = 0, hist_n = 0;
  int pe_base = 0;           // first row of this resolution in the position-code table
  uint64_t bytes = 0;
};

// One unit of work for a batch: a window of frames through the network, or poses pushed by
// the caller (world poses, or one window of local poses).
struct BatchWindow {
  int32_t stream_id;
  const mf_stream_cfg* cfg;
  StreamRes* res;
  int32_t window_id;
  int32_t chain_mode;        // CHAIN_ANCHOR / CHAIN_FIRST / CHAIN_WORLD
  int64_t start;             // first frame of the window
  int32_t size;              // frames in the window
  int64_t emit_begin, emit_end;
  const double* poses;       // host [size][16] for pushed poses, null for frames
};

// Streams appear in a batch in first-come order; a stream's windows are consecutive and in
// frame order.
struct Batch {
  std::vector<BatchWindow> wins;
  int64_t tokens = 0;
};

class Executor {
 public:
  virtual ~Executor() {}
  virtual mf_status init(const mf_model_cfg& m, const float* w, size_t n, const mf_runtime_cfg& rt,
                         std::string& err) = 0;
  virtual uint64_t fixed_bytes() const = 0;   // weights + batch workspace
  virtual uint64_t budget_bytes() const = 0;  // HBM the engine may use
  virtual int64_t max_tokens() const = 0;
  virtual int64_t max_frames() const = 0;     // frames (pose rows and emitted records) per batch
  virtual int rows_per_frame(int H, int W) const = 0;   // token rows a frame occupies
  // device bytes of a stream: frame ring, map_cap result slots of each kept map kind (focus maps if
  // c.emit_maps, depth maps if c.emit_depth) and the history
  virtual uint64_t stream_bytes(const mf_stream_cfg& c, int ring_cap, int map_cap, int hist_n) const = 0;
  virtual mf_status open_stream(const mf_stream_cfg& c, StreamRes* r, std::string& err) = 0;
  virtual void close_stream(StreamRes* r) = 0;
  // Copy n frames [n][3][H][W] into ring slots of frames first.., synchronously.
  virtual mf_status upload_frames(const mf_stream_cfg& c, StreamRes* r, int64_t first, const float* src,
                                  int n, bool device_src, std::string& err) = 0;
  // Run a batch; out receives the records of every emitted frame, window by window.
  virtual mf_status run_batch(const Batch& b, std::vector<mf_focus>& out, double* gpu_ms,
                              std::string& err) = 0;
  virtual mf_status copy_maps(const mf_stream_cfg& c, StreamRes* r, int64_t frame, int n, float* dst,
                              bool device_dst, std::string& err) = 0;
  // depth maps of n consecutive result slots (streams with emit_depth); executors without a depth
  // head refuse
  virtual mf_status copy_depth(const mf_stream_cfg&, StreamRes*, int64_t, int, float*, bool, std::string& err) {
    err = "depth maps are not supported by this executor";
    return MF_EINVAL;
  }
  // op-level access used by the test/benchmark entry points
  virtual mf_status forward_frames(const float* frames_dev, int S, int H, int W, float* pose9_host,
                                   double* T_host, int max_layers, float* tokens_host,
                                   std::string& err) = 0;
  // diagnostics: copy an internal buffer (0 X, 1 LN out, 2 Q, 3 K, 4 Vt, 5 O, 6 MLP hidden) to host
  virtual mf_status debug_copy(int which, void* host, size_t bytes, std::string& err) = 0;
  virtual void profile(double* attn_global_ms, int64_t* attn_global_calls, double* attn_frame_ms,
                       double* gemm_ms, int enable) = 0;
  // per-stage sums (MF_STAGE_* order) of the same timing; executors without it report zeros
  virtual int64_t last_batch_shared() const { return 0; }   // frames of the last batch that reused an embedding
  virtual void profile_stages(double* ms, int64_t* calls, int n) {
    for (int k = 0; k < n; ++k) {
      if (ms) ms[k] = 0.0;
      if (calls) calls[k] = 0;
    }
  }
};

Executor* make_executor();   // provided by the linked executor (HIP, or the CPU test stub)

}  // namespace mf
