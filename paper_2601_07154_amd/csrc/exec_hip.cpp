// HIP executor: device weights and workspace, the per-batch launch sequence of the ViT
// forward (patch embedding, alternating frame-wise / global blocks, pose head), then FP64
// anchoring + focus and the focus maps.  Every arithmetic step runs in the kernels of this
// library; the host only builds the batch tables.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"
#include "kernels.h"
#include "../../include/mf_ops.h"

namespace mf {

#define HIPCHECK(x)                                                              \
  do {                                                                           \
    hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess) {                                                      \
      err = std::string(#x) + " failed: " + hipGetErrorString(e_);               \
      return MF_EDEVICE;                                                         \
    }                                                                            \
  } while (0)

static constexpr int KP = 640;     // patch length 3*14*14 = 588 padded to the GEMM k-tile
static constexpr int DEPTH_OUT = 196;   // depth head outputs per patch token (its 14 x 14 pixels)
static constexpr int DEPTH_N = 256;     // ... padded to a GEMM tile width

static int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

struct LayerW {
  const float *ln1_g, *ln1_b, *b_qkv, *b_o, *ln2_g, *ln2_b, *b_1, *b_2;
  void *Wqkv, *Wo, *W1, *W2;       // transposed [out][in], compute type (E4M3 bytes for Wqkv/W1/W2 in fp8 mode)
};

struct Plan {                      // host-side tables of one batch
  std::vector<FrameDesc> frames;
  std::vector<AttnSeg> fsegs, gsegs;
  std::vector<AttnWork> fwork, gwork;
  std::vector<int32_t> cam_rows;
  std::vector<int32_t> dups;       // frames whose patch embedding is copied from an earlier window
  std::map<std::pair<int32_t, int64_t>, int32_t> seen;   // (stream, frame) -> first token row
  int64_t mtot = 0;
  int64_t patch_rows = 0;          // rows of the patch matrix (frames embedded by the GEMM)
  int max_npad = 0;
  int max_rows = 0;                // token rows of the largest window
};

class HipExecutor : public Executor {
 public:
  ~HipExecutor() override { release(); }

  mf_status init(const mf_model_cfg& m, const float* w, size_t n, const mf_runtime_cfg& rt,
                 std::string& err) override {
    m_ = m;
    if (m.patch != 14) { err = "patch must be 14"; return MF_EINVAL; }
    if (m.precision != MF_FP32 && m.precision != MF_BF16 && m.precision != MF_FP8) {
      err = "precision must be MF_FP32, MF_BF16 or MF_FP8";
      return MF_EINVAL;
    }
    if (m.depth < 1 || m.heads < 1 || m.dim % m.heads) { err = "bad depth/heads/dim"; return MF_EINVAL; }
    D_ = m.dim; H_ = m.heads; hd_ = D_ / H_; F_ = m.mlp; depth_ = m.depth;
    if (!(D_ == 128 || D_ == 256 || D_ == 384 || D_ == 512 || D_ == 768 || D_ == 1024)) { err = "dim must be one of 128, 256, 384, 512, 768, 1024"; return MF_EINVAL; }
    if (hd_ != 32 && hd_ != 64) { err = "head dim must be 32 or 64"; return MF_EINVAL; }
    if (F_ <= 0 || F_ % 128) { err = "mlp must be a positive multiple of 128"; return MF_EINVAL; }
    // MF_FP8: the QKV and MLP GEMMs take E4M3 operands; everything else runs as in MF_BF16
    fp8_ = m.precision == MF_FP8;
    depth_head_ = m.depth_head != 0;
    dt_ = m.precision == MF_FP32 ? DT_F32 : DT_BF16;
    es_ = dt_ == DT_BF16 ? 2 : 4;
    qt_ = attention_q_tile(dt_, hd_);
    fp8_attn_ = fp8_ && hd_ == 64;   // MF_FP8 scores on E4M3 operands (head dim 64)
    const size_t want = expected_floats();
    if (n != want) { err = "weight blob has " + std::to_string(n) + " floats, the model needs " + std::to_string(want); return MF_EINVAL; }
    if (!rt.dev_alloc != !rt.dev_free) { err = "dev_alloc and dev_free go together"; return MF_EINVAL; }
    ualloc_ = rt.dev_alloc;
    ufree_ = rt.dev_free;
    uctx_ = rt.alloc_ctx;
    HIPCHECK(hipSetDevice(rt.device));
    device_ = rt.device;
    use_graphs_ = rt.use_graphs != 0;
    if (rt.stream) { st_ = (hipStream_t)rt.stream; own_stream_ = false; }
    else { HIPCHECK(hipStreamCreateWithFlags(&st_, hipStreamNonBlocking)); own_stream_ = true; }
    HIPCHECK(hipStreamCreateWithFlags(&copy_, hipStreamNonBlocking));
    size_t free_b = 0, total_b = 0;
    HIPCHECK(hipMemGetInfo(&free_b, &total_b));
    budget_ = rt.hbm_budget_bytes ? rt.hbm_budget_bytes : (uint64_t)(free_b * 0.8);
    mcap_ = rt.max_tokens_per_batch > 0 ? rt.max_tokens_per_batch : 262144;
    mcap_ = align_up(mcap_, 8);
    mpad_ = mcap_ + 256;
    fcap_ = mcap_ / 8 + 64;
    if (workspace_bytes() + weight_bytes() > budget_) {
      err = "weights + workspace (" + std::to_string(workspace_bytes() + weight_bytes()) + " bytes) exceed the HBM budget";
      return MF_ENOMEM;
    }
    mf_status rc = load_weights(w, n, err);
    if (rc != MF_OK) return rc;
    rc = alloc_workspace(err);
    if (rc != MF_OK) return rc;
    HIPCHECK(hipEventCreate(&ev0_));
    HIPCHECK(hipEventCreate(&ev1_));
    return MF_OK;
  }

  uint64_t fixed_bytes() const override { return weight_bytes() + workspace_bytes(); }
  uint64_t budget_bytes() const override { return budget_; }
  int64_t max_tokens() const override { return mcap_; }
  int64_t max_frames() const override { return fcap_; }
  int rows_per_frame(int H, int W) const override { return (int)align_up((H / 14) * (W / 14) + 1, 8); }

  uint64_t stream_bytes(const mf_stream_cfg& c, int ring_cap, int map_cap, int hist_n) const override {
    const uint64_t hw = (uint64_t)c.height * c.width;
    const uint64_t rings = (c.emit_maps ? 1 : 0) + (c.emit_depth ? 1 : 0);
    return (uint64_t)ring_cap * 3 * hw * 4 + rings * map_cap * hw * 4 + (uint64_t)hist_n * sizeof(FrameHist);
  }

  mf_status open_stream(const mf_stream_cfg& c, StreamRes* r, std::string& err) override {
    HIPCHECK(hipSetDevice(device_));
    const uint64_t hw = (uint64_t)c.height * c.width;
    HIPCHECK(dmalloc(&r->ring, (size_t)r->ring_cap * 3 * hw * 4));
    if (r->map_cap > 0 && c.emit_maps) HIPCHECK(dmalloc(&r->maps, (size_t)r->map_cap * hw * 4));
    if (r->map_cap > 0 && c.emit_depth) {
      if (!depth_head_) { err = "emit_depth needs a model with a depth head"; return MF_EINVAL; }
      HIPCHECK(dmalloc(&r->depth, (size_t)r->map_cap * hw * 4));
    }
    HIPCHECK(dmalloc(&r->hist, (size_t)r->hist_n * sizeof(FrameHist)));
    HIPCHECK(hipMemsetAsync(r->hist, 0, (size_t)r->hist_n * sizeof(FrameHist), copy_));
    HIPCHECK(hipMemsetAsync(r->ring, 0, (size_t)r->ring_cap * 3 * hw * 4, copy_));
    HIPCHECK(hipStreamSynchronize(copy_));
    return pe_rows_for(c.height / 14, c.width / 14, &r->pe_base, err);
  }

  void close_stream(StreamRes* r) override {
    hipSetDevice(device_);
    dfree(r->ring);
    dfree(r->maps);
    dfree(r->depth);
    dfree(r->hist);
    r->ring = r->maps = r->depth = r->hist = nullptr;
  }

  mf_status upload_frames(const mf_stream_cfg& c, StreamRes* r, int64_t first, const float* src, int n,
                          bool device_src, std::string& err) override {
    HIPCHECK(hipSetDevice(device_));
    const size_t fb = (size_t)3 * c.height * c.width * 4;
    int done = 0;
    while (done < n) {
      const int64_t f = first + done;
      const int slot = (int)(f % r->ring_cap);
      const int run = std::min(n - done, r->ring_cap - slot);
      HIPCHECK(hipMemcpyAsync((char*)r->ring + (size_t)slot * fb, (const char*)src + (size_t)done * fb,
                              (size_t)run * fb, device_src ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                              copy_));
      done += run;
    }
    HIPCHECK(hipStreamSynchronize(copy_));
    return MF_OK;
  }

  mf_status copy_maps(const mf_stream_cfg& c, StreamRes* r, int64_t frame, int n, float* dst, bool device_dst,
                      std::string& err) override {
    HIPCHECK(hipSetDevice(device_));
    const size_t mb = (size_t)c.height * c.width * 4;
    const int slot = (int)(frame % r->map_cap);
    HIPCHECK(hipMemcpyAsync(dst, (char*)r->maps + (size_t)slot * mb, (size_t)n * mb,
                            device_dst ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, copy_));
    HIPCHECK(hipStreamSynchronize(copy_));
    return MF_OK;
  }

  mf_status copy_depth(const mf_stream_cfg& c, StreamRes* r, int64_t frame, int n, float* dst, bool device_dst,
                       std::string& err) override {
    HIPCHECK(hipSetDevice(device_));
    if (!r->depth) { err = "the stream keeps no depth maps"; return MF_EINVAL; }
    const size_t mb = (size_t)c.height * c.width * 4;
    const int slot = (int)(frame % r->map_cap);
    HIPCHECK(hipMemcpyAsync(dst, (char*)r->depth + (size_t)slot * mb, (size_t)n * mb,
                            device_dst ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, copy_));
    HIPCHECK(hipStreamSynchronize(copy_));
    return MF_OK;
  }

  mf_status run_batch(const Batch& b, std::vector<mf_focus>& out, double* gpu_ms, std::string& err) override {
    HIPCHECK(hipSetDevice(device_));
    latch_profiling();
    // ---- plan the forward part
    Plan p;
    std::vector<int32_t> loc_off(b.wins.size(), -1);
    int32_t fwd_frames = 0;
    for (size_t i = 0; i < b.wins.size(); ++i) {
      const BatchWindow& w = b.wins[i];
      if (w.poses) continue;
      loc_off[i] = fwd_frames;
      add_window(p, w, true);
      fwd_frames += w.size;
    }
    int32_t pose_rows = 0;
    for (size_t i = 0; i < b.wins.size(); ++i)
      if (b.wins[i].poses) { loc_off[i] = fwd_frames + pose_rows; pose_rows += b.wins[i].size; }
    // depth targets of the forward frames, in the order add_window listed them
    std::vector<DepthFrame> dframes;
    bool has_depth = false;
    for (size_t i = 0; i < b.wins.size(); ++i) {
      const BatchWindow& w = b.wins[i];
      if (w.poses) continue;
      const size_t hw = (size_t)w.cfg->height * w.cfg->width;
      for (int j = 0; j < w.size; ++j) {
        const int64_t t = w.start + j;
        DepthFrame df{};
        if (w.cfg->emit_depth && w.res->depth && t >= w.emit_begin && t < w.emit_end) {
          df.dst = (float*)w.res->depth + (size_t)(t % w.res->map_cap) * hw;
          has_depth = true;
        }
        df.W = w.cfg->width;
        df.gw = w.cfg->width / 14;
        df.pe_base = w.res->pe_base;
        df.win = (int32_t)i;
        dframes.push_back(df);
      }
    }
    if (p.mtot > mcap_ || fwd_frames + pose_rows > fcap_) { err = "batch exceeds the workspace"; return MF_EINVAL; }

    // ---- chain / focus / map tables
    std::vector<StreamDev> sdev;
    std::vector<ChainGroup> groups;
    std::vector<ChainWin> cwins;
    std::vector<MapJob> jobs;
    int32_t out_n = 0, max_h = 0, max_w = 0;
    int32_t prev_stream = -1;
    for (size_t i = 0; i < b.wins.size(); ++i) {
      const BatchWindow& w = b.wins[i];
      if (w.stream_id != prev_stream) {
        StreamDev sd{};
        sd.hist = (FrameHist*)w.res->hist;
        sd.hist_mask = w.res->hist_n - 1;
        sd.n_points = w.cfg->n_points;
        sd.fx = w.cfg->fx; sd.fy = w.cfg->fy; sd.cx = w.cfg->cx; sd.cy = w.cfg->cy;
        sd.sigma = w.cfg->sigma; sd.sigma_min = w.cfg->sigma_min; sd.sigma_max = w.cfg->sigma_max;
        sd.anchor_mode = w.cfg->anchor_mode;
        sd.focus_mode = w.cfg->focus_mode;
        sd.stride = w.cfg->diff_stride > 0 ? w.cfg->diff_stride : 1;
        sd.map_mode = w.cfg->map_mode;
        sd.H = w.cfg->height; sd.W = w.cfg->width;
        sd.map_cap = w.res->map_cap;
        sd.maps = (float*)w.res->maps;
        sdev.push_back(sd);
        groups.push_back({(int32_t)cwins.size(), 0});
        prev_stream = w.stream_id;
      }
      ChainWin cw{};
      cw.stream = (int32_t)sdev.size() - 1;
      cw.mode = w.chain_mode;
      cw.loc_off = loc_off[i];
      cw.window_id = w.window_id;
      cw.start = w.start;
      cw.emit_begin = w.emit_begin;
      cw.emit_end = w.emit_end;
      cw.out_off = out_n;
      cw.has_pose9 = w.poses ? 0 : 1;
      cwins.push_back(cw);
      groups.back().n_win++;
      if (w.cfg->emit_maps) {
        for (int64_t t = w.emit_begin; t < w.emit_end; ++t)
          jobs.push_back({cw.stream, out_n + (int32_t)(t - w.emit_begin), t});
        max_h = std::max(max_h, w.cfg->height);
        max_w = std::max(max_w, w.cfg->width);
      }
      out_n += (int32_t)(w.emit_end - w.emit_begin);
    }
    if (out_n > fcap_ || (int64_t)jobs.size() > fcap_) { err = "batch emits more frames than the workspace holds"; return MF_EINVAL; }
    if (!jobs.empty()) {
      const mf_status rp = ensure_psum((size_t)jobs.size() * map_row_blocks(max_h), err);
      if (rp != MF_OK) return rp;
    }

    // ---- pack every table into one pinned buffer, one upload
    size_t off = 0;
    auto reserve = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes, 256); return o; };
    const size_t o_frames = reserve(p.frames.size() * sizeof(FrameDesc));
    const size_t o_fsegs = reserve(p.fsegs.size() * sizeof(AttnSeg));
    const size_t o_fwork = reserve(p.fwork.size() * sizeof(AttnWork));
    const size_t o_gsegs = reserve(p.gsegs.size() * sizeof(AttnSeg));
    const size_t o_gwork = reserve(p.gwork.size() * sizeof(AttnWork));
    const size_t o_cam = reserve(p.cam_rows.size() * sizeof(int32_t));
    const size_t o_sdev = reserve(sdev.size() * sizeof(StreamDev));
    const size_t o_groups = reserve(groups.size() * sizeof(ChainGroup));
    const size_t o_cwins = reserve(cwins.size() * sizeof(ChainWin));
    const size_t o_jobs = reserve(jobs.size() * sizeof(MapJob));
    const size_t o_poses = reserve((size_t)pose_rows * 16 * sizeof(double));
    const size_t o_dframes = reserve(dframes.size() * sizeof(DepthFrame));
    const size_t o_dups = reserve(p.dups.size() * sizeof(int32_t));
    mf_status rc = ensure_tables(off, err);
    if (rc != MF_OK) return rc;
    auto put = [&](size_t o, const void* src, size_t bytes) { if (bytes) memcpy(tab_host_ + o, src, bytes); };
    put(o_frames, p.frames.data(), p.frames.size() * sizeof(FrameDesc));
    put(o_fsegs, p.fsegs.data(), p.fsegs.size() * sizeof(AttnSeg));
    put(o_fwork, p.fwork.data(), p.fwork.size() * sizeof(AttnWork));
    put(o_gsegs, p.gsegs.data(), p.gsegs.size() * sizeof(AttnSeg));
    put(o_gwork, p.gwork.data(), p.gwork.size() * sizeof(AttnWork));
    put(o_cam, p.cam_rows.data(), p.cam_rows.size() * sizeof(int32_t));
    put(o_sdev, sdev.data(), sdev.size() * sizeof(StreamDev));
    put(o_groups, groups.data(), groups.size() * sizeof(ChainGroup));
    put(o_cwins, cwins.data(), cwins.size() * sizeof(ChainWin));
    put(o_jobs, jobs.data(), jobs.size() * sizeof(MapJob));
    put(o_dframes, dframes.data(), dframes.size() * sizeof(DepthFrame));
    put(o_dups, p.dups.data(), p.dups.size() * sizeof(int32_t));
    {
      size_t po = o_poses;
      for (const BatchWindow& w : b.wins)
        if (w.poses) { put(po, w.poses, (size_t)w.size * 16 * sizeof(double)); po += (size_t)w.size * 16 * sizeof(double); }
    }
    auto T = [&](size_t o) { return (void*)(tab_dev_ + o); };
    // Everything the batch runs on the device, in stream order.  The tables are read from the
    // pinned buffer when the copy executes, so a captured graph replays with new contents.
    auto enqueue = [&]() -> mf_status {
      HIPCHECK(hipMemcpyAsync(tab_dev_, tab_host_, off, hipMemcpyHostToDevice, st_));
      if (!p.frames.empty()) {
        const mf_status r = forward(p, (const FrameDesc*)T(o_frames), (const AttnSeg*)T(o_fsegs),
                                    (const AttnWork*)T(o_fwork), (const AttnSeg*)T(o_gsegs),
                                    (const AttnWork*)T(o_gwork), (const int32_t*)T(o_cam),
                                    (const int32_t*)T(o_dups), depth_, err);
        if (r != MF_OK) return r;
      }
      if (pose_rows)
        HIPCHECK(hipMemcpyAsync(tloc_ + (size_t)fwd_frames * 16, T(o_poses), (size_t)pose_rows * 16 * sizeof(double),
                                hipMemcpyDeviceToDevice, st_));
      HIPCHECK(chain_focus((const ChainGroup*)T(o_groups), (int)groups.size(), (const ChainWin*)T(o_cwins),
                           (const StreamDev*)T(o_sdev), tloc_, pose9_, res_, win_scale_, st_));
      if (has_depth) {
        // depth maps of the emitted frames from the last block's tokens, times their window's scale
        prof_begin();
        HIPCHECK(layernorm(dt_, X_, Y_, lnd_g_, lnd_b_, p.mtot, D_, nullptr, st_));
        GemmArgs d{};
        d.A = Y_; d.lda = D_; d.Bt = Wd_; d.ldb = D_; d.M = (int)p.mtot; d.N = DEPTH_N; d.K = D_; d.bias = bd_;
        d.rowinfo = rowinfo_; d.rowframe = rowframe_; d.dframes = (const DepthFrame*)T(o_dframes);
        d.win_scale = win_scale_;
        HIPCHECK(gemm(dt_, EPI_DEPTH, d, st_));
        prof_end(MF_STAGE_HEAD);
      }
      HIPCHECK(focus_maps((const MapJob*)T(o_jobs), (int)jobs.size(), max_h, max_w, (const StreamDev*)T(o_sdev),
                          res_, keys_, psum_, st_));
      HIPCHECK(hipMemcpyAsync(res_host_, res_, (size_t)out_n * sizeof(mf_focus), hipMemcpyDeviceToHost, st_));
      return MF_OK;
    };
    HIPCHECK(hipEventRecord(ev0_, st_));
    // per-kernel timing brackets launches with events on the stream: profiled batches run eagerly
    if (use_graphs_ && !prof_batch_) {
      // Every kernel argument and copy size follows from these counts (table offsets included):
      // the token rows, the frames and work lists, the windows and the largest of them (the fp8
      // window quantiser's grid), the chain and map tables, the poses and the records, the patch
      // rows and the frames that take an earlier window's embedding.
      char sig[256];
      snprintf(sig, sizeof sig, "%lld/%d/%zu/%zu/%zu/%zu/%d/%zu/%zu/%zu/%d/%d/%d/%d/%d/%zu/%d/%lld/%zu",
               (long long)p.mtot, p.max_npad, p.frames.size(), p.fwork.size(), p.gwork.size(), p.gsegs.size(),
               p.max_rows, groups.size(), cwins.size(), jobs.size(), max_h, max_w, pose_rows, fwd_frames, out_n, off,
               has_depth ? 1 : 0, (long long)p.patch_rows, p.dups.size());
      auto it = graphs_.find(sig);
      if (it == graphs_.end()) {
        if (graphs_.size() >= 64) clear_graphs();
        GraphEntry ge;
        // the per-kernel timing events of a profiled batch are recorded by the graph itself
        prof_target_ = &ge.prof;
        HIPCHECK(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
        const mf_status r = enqueue();
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(st_, &g);
        prof_target_ = nullptr;
        if (r != MF_OK) {
          if (g) hipGraphDestroy(g);
          return r;
        }
        if (ec != hipSuccess) {
          err = std::string("hipStreamEndCapture failed: ") + hipGetErrorString(ec);
          return MF_EDEVICE;
        }
        const hipError_t ei = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (ei != hipSuccess) {
          err = std::string("hipGraphInstantiate failed: ") + hipGetErrorString(ei);
          return MF_EDEVICE;
        }
        it = graphs_.emplace(sig, std::move(ge)).first;
      }
      HIPCHECK(hipGraphLaunch(it->second.exec, st_));
      replayed_prof_ = &it->second.prof;
    } else {
      rc = enqueue();
      if (rc != MF_OK) return rc;
    }
    HIPCHECK(hipEventRecord(ev1_, st_));
    HIPCHECK(hipStreamSynchronize(st_));
    float ms = 0.0f;
    HIPCHECK(hipEventElapsedTime(&ms, ev0_, ev1_));
    if (gpu_ms) *gpu_ms = ms;
    reused_ = (int64_t)p.dups.size();
    collect_profile(err);
    out.assign(res_host_, res_host_ + out_n);
    return MF_OK;
  }

  mf_status forward_frames(const float* frames_dev, int S, int H, int W, float* pose9_host, double* T_host,
                           int max_layers, float* tokens_host, std::string& err) override {
    HIPCHECK(hipSetDevice(device_));
    latch_profiling();
    if (S < 1 || H % 14 || W % 14 || H <= 0 || W <= 0) { err = "bad frame geometry"; return MF_EINVAL; }
    StreamRes r;
    r.ring = (void*)frames_dev;
    r.ring_cap = S;
    mf_status rc = pe_rows_for(H / 14, W / 14, &r.pe_base, err);
    if (rc != MF_OK) return rc;
    mf_stream_cfg c{};
    c.height = H;
    c.width = W;
    c.window = S;
    BatchWindow w{};
    w.cfg = &c;
    w.res = &r;
    w.start = 0;
    w.size = S;
    Plan p;
    add_window(p, w, false);
    if (p.mtot > mcap_) { err = "window exceeds the token workspace"; return MF_EINVAL; }
    size_t off = 0;
    auto reserve = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes, 256); return o; };
    const size_t o_frames = reserve(p.frames.size() * sizeof(FrameDesc));
    const size_t o_fsegs = reserve(p.fsegs.size() * sizeof(AttnSeg));
    const size_t o_fwork = reserve(p.fwork.size() * sizeof(AttnWork));
    const size_t o_gsegs = reserve(p.gsegs.size() * sizeof(AttnSeg));
    const size_t o_gwork = reserve(p.gwork.size() * sizeof(AttnWork));
    const size_t o_cam = reserve(p.cam_rows.size() * sizeof(int32_t));
    rc = ensure_tables(off, err);
    if (rc != MF_OK) return rc;
    memcpy(tab_host_ + o_frames, p.frames.data(), p.frames.size() * sizeof(FrameDesc));
    memcpy(tab_host_ + o_fsegs, p.fsegs.data(), p.fsegs.size() * sizeof(AttnSeg));
    memcpy(tab_host_ + o_fwork, p.fwork.data(), p.fwork.size() * sizeof(AttnWork));
    memcpy(tab_host_ + o_gsegs, p.gsegs.data(), p.gsegs.size() * sizeof(AttnSeg));
    memcpy(tab_host_ + o_gwork, p.gwork.data(), p.gwork.size() * sizeof(AttnWork));
    memcpy(tab_host_ + o_cam, p.cam_rows.data(), p.cam_rows.size() * sizeof(int32_t));
    HIPCHECK(hipMemcpyAsync(tab_dev_, tab_host_, off, hipMemcpyHostToDevice, st_));
    auto T = [&](size_t o) { return (void*)(tab_dev_ + o); };
    const int layers = max_layers < 0 ? depth_ : std::min(max_layers, depth_);
    rc = forward(p, (const FrameDesc*)T(o_frames), (const AttnSeg*)T(o_fsegs), (const AttnWork*)T(o_fwork),
                 (const AttnSeg*)T(o_gsegs), (const AttnWork*)T(o_gwork), (const int32_t*)T(o_cam), nullptr, layers,
                 err);
    if (rc != MF_OK) return rc;
    if (pose9_host) HIPCHECK(hipMemcpyAsync(pose9_host, pose9_, (size_t)S * 9 * 4, hipMemcpyDeviceToHost, st_));
    if (T_host) HIPCHECK(hipMemcpyAsync(T_host, tloc_, (size_t)S * 16 * 8, hipMemcpyDeviceToHost, st_));
    if (tokens_host) HIPCHECK(hipMemcpyAsync(tokens_host, X_, (size_t)p.mtot * D_ * 4, hipMemcpyDeviceToHost, st_));
    HIPCHECK(hipStreamSynchronize(st_));
    collect_profile(err);
    return MF_OK;
  }

  int64_t last_batch_shared() const override { return reused_; }

  mf_status debug_copy(int which, void* host, size_t bytes, std::string& err) override {
    HIPCHECK(hipSetDevice(device_));
    const void* src[11] = {X_, Y_, Q_, K_, Vt_, O_, Hb_, Q8_, K8_, QE_, KE_};
    const size_t D = D_, wide = std::max<int64_t>(F_, KP);
    const size_t q8b = fp8_attn_ ? (size_t)mpad_ * D : 0, qeb = fp8_attn_ ? (size_t)mpad_ * H_ : 0;
    const size_t cap[11] = {(size_t)mcap_ * D * 4, (size_t)mcap_ * D * es_, (size_t)mpad_ * D * es_,
                           (size_t)mpad_ * D * es_, (size_t)mpad_ * D * es_, (size_t)mcap_ * D * es_,
                           (size_t)mcap_ * wide * es_, q8b, q8b, qeb, qeb};
    if (which < 0 || which > 10 || bytes > cap[which] || !src[which]) { err = "bad buffer or size"; return MF_EINVAL; }
    HIPCHECK(hipStreamSynchronize(st_));
    HIPCHECK(hipMemcpy(host, src[which], bytes, hipMemcpyDeviceToHost));
    return MF_OK;
  }

  void profile(double* ag_ms, int64_t* ag_calls, double* af_ms, double* g_ms, int enable) override {
    // may run on an API thread while the scheduler thread runs a batch: the switch and the sums are
    // shared under prof_mu_, and a batch reads the switch once, when it starts (latch_profiling)
    std::lock_guard<std::mutex> lk(prof_mu_);
    if (ag_ms) *ag_ms = prof_ms_[MF_STAGE_ATTN_GLOBAL];
    if (ag_calls) *ag_calls = prof_calls_[MF_STAGE_ATTN_GLOBAL];
    if (af_ms) *af_ms = prof_ms_[MF_STAGE_ATTN_FRAME];
    if (g_ms) {
      *g_ms = 0.0;
      for (int k : {MF_STAGE_QKV, MF_STAGE_OUT_PROJ, MF_STAGE_FC1, MF_STAGE_FC2, MF_STAGE_PATCH}) *g_ms += prof_ms_[k];
    }
    if (enable >= 0) {
      profiling_ = enable != 0;
      for (int k = 0; k < MF_STAGE_COUNT; ++k) { prof_ms_[k] = 0.0; prof_calls_[k] = 0; }
    }
  }

  void profile_stages(double* ms, int64_t* calls, int n) override {
    std::lock_guard<std::mutex> lk(prof_mu_);
    for (int k = 0; k < n && k < MF_STAGE_COUNT; ++k) {
      if (ms) ms[k] = prof_ms_[k];
      if (calls) calls[k] = prof_calls_[k];
    }
  }

 private:
  // ------------------------------------------------------------------ sizes
  size_t expected_floats() const {
    const size_t D = D_, F = F_;
    return 588 * D + 3 * D + depth_ * (2 * D + D * 3 * D + 3 * D + D * D + D + 2 * D + D * F + F + F * D + D) +
           2 * D + D * D + D + D * 9 + 9 + (depth_head_ ? 2 * D + D * DEPTH_OUT + DEPTH_OUT : 0);
  }
  uint64_t weight_bytes() const {
    const uint64_t D = D_, F = F_;
    return expected_floats() * 4 + (D * KP + depth_ * (3 * D * D + D * D + 2 * D * F)) * es_ + D * D * 4 +
           (depth_head_ ? (uint64_t)DEPTH_N * D * es_ + DEPTH_N * 4 : 0);
  }
  uint64_t workspace_bytes() const {
    const uint64_t D = D_, wide = std::max<int64_t>(F_, KP);
    // fp8: Y8, H8, the two row-scale arrays and the LayerNorm row maxima; E4M3 q / k and exponents
    const uint64_t f8 = (fp8_ ? (uint64_t)mcap_ * (D + F_ + 12) : 0) +
                        (fp8_attn_ ? (uint64_t)mpad_ * 2 * (D + (uint64_t)H_) : 0);
    // per token row: X, Y, O, the hidden, and four int32 maps (rowinfo, rowframe, patch row info
    // and destination)
    return f8 + (uint64_t)mcap_ * (D * 4 + D * es_ + D * es_ + wide * es_ + 4 * 4) + (uint64_t)mpad_ * 3 * D * es_ +
           (uint64_t)fcap_ * (2 * D * 4 + 9 * 4 + 16 * 8 + sizeof(mf_focus) * 2 + 8 + 8) + (64u << 20);
  }

  // ------------------------------------------------------------------ weights
  mf_status load_weights(const float* w, size_t n, std::string& err) {
    HIPCHECK(dmalloc(&wdev_, n * 4));
    HIPCHECK(hipMemcpy(wdev_, w, n * 4, hipMemcpyHostToDevice));
    const float* p = wdev_;
    auto take = [&](size_t cnt) { const float* q = p; p += cnt; return q; };
    const size_t D = D_, F = F_;
    const float* Wp = take(588 * D);
    b_p_ = take(D); c_ref_ = take(D); c_other_ = take(D);
    HIPCHECK(dmalloc(&Wp_, D * KP * es_));
    HIPCHECK(hipMemsetAsync(Wp_, 0, D * KP * es_, st_));
    HIPCHECK(convert_transpose(dt_, Wp, 588, (int)D, Wp_, KP, st_));
    layers_.resize(depth_);
    if (fp8_) {
      HIPCHECK(dmalloc(&wscale_, (size_t)depth_ * 3 * sizeof(float)));
      HIPCHECK(dmalloc(&wamax_, 64));
    }
    for (int l = 0; l < depth_; ++l) {
      LayerW& L = layers_[l];
      L.ln1_g = take(D); L.ln1_b = take(D);
      const float* Wqkv = take(D * 3 * D);
      L.b_qkv = take(3 * D);
      const float* Wo = take(D * D);
      L.b_o = take(D);
      L.ln2_g = take(D); L.ln2_b = take(D);
      const float* W1 = take(D * F);
      L.b_1 = take(F);
      const float* W2 = take(F * D);
      L.b_2 = take(D);
      const size_t ws = fp8_ ? 1 : es_;
      HIPCHECK(dmalloc(&L.Wqkv, 3 * D * D * ws));
      HIPCHECK(dmalloc(&L.Wo, D * D * es_));
      HIPCHECK(dmalloc(&L.W1, D * F * ws));
      HIPCHECK(dmalloc(&L.W2, F * D * ws));
      if (fp8_) {
        float* sc = wscale_ + 3 * l;
        HIPCHECK(quantize_weight_fp8(Wqkv, (int)D, (int)(3 * D), (unsigned char*)L.Wqkv, (int)D, wamax_, sc, st_));
        HIPCHECK(quantize_weight_fp8(W1, (int)D, (int)F, (unsigned char*)L.W1, (int)D, wamax_, sc + 1, st_));
        HIPCHECK(quantize_weight_fp8(W2, (int)F, (int)D, (unsigned char*)L.W2, (int)F, wamax_, sc + 2, st_));
        HIPCHECK(convert_transpose(dt_, Wo, (int)D, (int)D, L.Wo, (int)D, st_));
        continue;
      }
      HIPCHECK(convert_transpose(dt_, Wqkv, (int)D, (int)(3 * D), L.Wqkv, (int)D, st_));
      HIPCHECK(convert_transpose(dt_, Wo, (int)D, (int)D, L.Wo, (int)D, st_));
      HIPCHECK(convert_transpose(dt_, W1, (int)D, (int)F, L.W1, (int)D, st_));
      HIPCHECK(convert_transpose(dt_, W2, (int)F, (int)D, L.W2, (int)F, st_));
    }
    lnf_g_ = take(D); lnf_b_ = take(D);
    const float* H1 = take(D * D);
    h_1_ = take(D);
    H_2_ = take(D * 9);
    h_2_ = take(9);
    HIPCHECK(dmalloc(&H1t_, D * D * 4));
    HIPCHECK(convert_transpose(DT_F32, H1, (int)D, (int)D, H1t_, (int)D, st_));
    if (depth_head_) {
      // depth head: W_d [D][196] transposed to [256][D] (rows 196.. zero), bias padded to 256
      lnd_g_ = take(D); lnd_b_ = take(D);
      const float* Wd = take(D * DEPTH_OUT);
      const float* bd = take(DEPTH_OUT);
      HIPCHECK(dmalloc(&Wd_, (size_t)DEPTH_N * D * es_));
      HIPCHECK(hipMemsetAsync(Wd_, 0, (size_t)DEPTH_N * D * es_, st_));
      HIPCHECK(convert_transpose(dt_, Wd, (int)D, DEPTH_OUT, Wd_, (int)D, st_));
      HIPCHECK(dmalloc(&bd_, DEPTH_N * 4));
      HIPCHECK(hipMemsetAsync(bd_, 0, DEPTH_N * 4, st_));
      HIPCHECK(hipMemcpyAsync(bd_, bd, DEPTH_OUT * 4, hipMemcpyDeviceToDevice, st_));
    }
    HIPCHECK(hipStreamSynchronize(st_));
    return MF_OK;
  }

  mf_status alloc_workspace(std::string& err) {
    const size_t D = D_, wide = std::max<int64_t>(F_, KP);
    HIPCHECK(dmalloc(&X_, (size_t)mcap_ * D * 4));
    HIPCHECK(dmalloc(&Y_, (size_t)mcap_ * D * es_));
    HIPCHECK(dmalloc(&O_, (size_t)mcap_ * D * es_));
    HIPCHECK(dmalloc(&Hb_, (size_t)mcap_ * wide * es_));
    HIPCHECK(dmalloc(&rowinfo_, (size_t)mcap_ * 4));
    HIPCHECK(dmalloc(&rowframe_, (size_t)mcap_ * 4));
    HIPCHECK(dmalloc(&prow_, (size_t)mcap_ * 4));
    HIPCHECK(dmalloc(&pdst_, (size_t)mcap_ * 4));
    HIPCHECK(dmalloc(&win_scale_, (size_t)fcap_ * 8));
    HIPCHECK(dmalloc(&Q_, (size_t)mpad_ * D * es_));
    HIPCHECK(dmalloc(&K_, (size_t)mpad_ * D * es_));
    HIPCHECK(dmalloc(&Vt_, (size_t)mpad_ * D * es_));
    // rows past the last token are read (masked) by attention tiles: keep them finite
    HIPCHECK(hipMemsetAsync(Q_, 0, (size_t)mpad_ * D * es_, st_));
    HIPCHECK(hipMemsetAsync(K_, 0, (size_t)mpad_ * D * es_, st_));
    HIPCHECK(hipMemsetAsync(Vt_, 0, (size_t)mpad_ * D * es_, st_));
    HIPCHECK(hipMemsetAsync(X_, 0, (size_t)mcap_ * D * 4, st_));
    HIPCHECK(hipMemsetAsync(Y_, 0, (size_t)mcap_ * D * es_, st_));
    HIPCHECK(hipMemsetAsync(O_, 0, (size_t)mcap_ * D * es_, st_));
    HIPCHECK(hipStreamSynchronize(st_));
    if (fp8_) {
      HIPCHECK(dmalloc(&Y8_, (size_t)mcap_ * D));
      if (fp8_attn_) {
        // E4M3 q / k rows and their per-row scale bytes; rows past the tokens stay zero (finite)
        HIPCHECK(dmalloc(&Q8_, (size_t)mpad_ * D_));
        HIPCHECK(dmalloc(&K8_, (size_t)mpad_ * D_));
        HIPCHECK(dmalloc(&QE_, (size_t)mpad_ * H_));
        HIPCHECK(dmalloc(&KE_, (size_t)mpad_ * H_));
        HIPCHECK(hipMemsetAsync(Q8_, 0, (size_t)mpad_ * D_, st_));
        HIPCHECK(hipMemsetAsync(K8_, 0, (size_t)mpad_ * D_, st_));
        HIPCHECK(hipMemsetAsync(QE_, 0, (size_t)mpad_ * H_, st_));
        HIPCHECK(hipMemsetAsync(KE_, 0, (size_t)mpad_ * H_, st_));
        HIPCHECK(hipStreamSynchronize(st_));
      }
      HIPCHECK(dmalloc(&H8_, (size_t)mcap_ * F_));
      HIPCHECK(dmalloc(&srow_, (size_t)mcap_ * 4));
      HIPCHECK(dmalloc(&srow2_, (size_t)mcap_ * 4));
      HIPCHECK(dmalloc(&rowmax_, (size_t)mcap_ * 4));
      HIPCHECK(dmalloc(&amax_, (size_t)fcap_ * 4));
    }
    HIPCHECK(dmalloc(&camln_, (size_t)fcap_ * D * 4));
    HIPCHECK(dmalloc(&camg_, (size_t)fcap_ * D * 4));
    HIPCHECK(dmalloc(&pose9_, (size_t)fcap_ * 9 * 4));
    HIPCHECK(dmalloc(&tloc_, (size_t)fcap_ * 16 * 8));
    HIPCHECK(dmalloc(&res_, (size_t)fcap_ * sizeof(mf_focus)));
    HIPCHECK(dmalloc(&keys_, (size_t)fcap_ * 8));
    HIPCHECK(hipHostMalloc((void**)&res_host_, (size_t)fcap_ * sizeof(mf_focus), hipHostMallocDefault));
    return MF_OK;
  }

  void clear_graphs() {
    for (auto& kv : graphs_) {
      hipGraphExecDestroy(kv.second.exec);
      for (auto& e : kv.second.prof) {
        hipEventDestroy(e.a);
        hipEventDestroy(e.b);
      }
    }
    graphs_.clear();
  }

  mf_status ensure_tables(size_t bytes, std::string& err) {
    if (bytes <= tab_cap_) return MF_OK;
    clear_graphs();   // captured copies point at the old table buffers
    dfree(tab_dev_);
    tab_dev_ = nullptr;
    if (tab_host_) HIPCHECK(hipHostFree(tab_host_));
    tab_cap_ = align_up(bytes * 2, 1 << 20);
    HIPCHECK(dmalloc(&tab_dev_, tab_cap_));
    HIPCHECK(hipHostMalloc((void**)&tab_host_, tab_cap_, hipHostMallocDefault));
    return MF_OK;
  }

  // Partial sums of the map normaliser: one double per map job and render workgroup.  Grown before
  // a batch is captured or launched; a new buffer invalidates captured graphs.
  mf_status ensure_psum(size_t n, std::string& err) {
    if (n <= psum_cap_) return MF_OK;
    clear_graphs();
    dfree(psum_);
    psum_ = nullptr;
    psum_cap_ = std::max<size_t>(n, (size_t)fcap_ * 64);
    HIPCHECK(dmalloc(&psum_, psum_cap_ * sizeof(double)));
    return MF_OK;
  }

  // Position-code rows for a (gh, gw) grid: one table per resolution in a shared arena.
  // Opens of several streams may run at once on API threads (and a forward on the scheduler thread).
  mf_status pe_rows_for(int gh, int gw, int* base, std::string& err) {
    std::lock_guard<std::mutex> lk(pe_mu_);
    auto key = std::make_pair(gh, gw);
    auto it = pe_index_.find(key);
    if (it != pe_index_.end()) { *base = it->second; return MF_OK; }
    if (!pe_) {
      pe_cap_ = 32768;
      HIPCHECK(dmalloc(&pe_, (size_t)pe_cap_ * D_ * 4));
    }
    if (pe_rows_ + gh * gw > pe_cap_) { err = "too many distinct resolutions for the position-code arena"; return MF_ENOMEM; }
    HIPCHECK(make_pe(pe_ + (size_t)pe_rows_ * D_, gh, gw, D_, copy_));
    HIPCHECK(hipStreamSynchronize(copy_));
    *base = pe_rows_;
    pe_index_[key] = pe_rows_;
    pe_rows_ += gh * gw;
    return MF_OK;
  }

  // ------------------------------------------------------------------ batch planning
  // share: a frame that an earlier window of the batch holds too (consecutive windows of a stream
  // share their overlap frames, Sec. 2.2) takes that window's patch embedding instead of its own
  // im2col and GEMM rows; only the camera token (reference or not) differs.
  void add_window(Plan& p, const BatchWindow& w, bool share) const {
    const int H = w.cfg->height, W = w.cfg->width, gw = W / 14, P = (H / 14) * gw;
    const int n = P + 1, npad = rows_per_frame(H, W);
    const size_t fb = (size_t)3 * H * W;
    const int32_t base = (int32_t)p.mtot;
    for (int j = 0; j < w.size; ++j) {
      FrameDesc fd;
      const int64_t f = w.start + j;
      fd.px = (const float*)w.res->ring + (size_t)(f % w.res->ring_cap) * fb;
      fd.H = H; fd.W = W; fd.gw = gw; fd.P = P;
      fd.token_base = base + j * npad;
      fd.npad = npad;
      fd.first = j == 0;
      fd.pe_base = w.res->pe_base;
      fd.patch_base = (int32_t)p.patch_rows;
      fd.src_base = -1;
      if (share) {
        const auto key = std::make_pair(w.stream_id, f);
        const auto it = p.seen.find(key);
        if (it != p.seen.end()) {
          fd.patch_base = -1;
          fd.src_base = it->second;
          p.dups.push_back((int32_t)p.frames.size());
        } else {
          p.seen.emplace(key, fd.token_base);
        }
      }
      if (fd.patch_base >= 0) p.patch_rows += npad;
      p.frames.push_back(fd);
      p.cam_rows.push_back(fd.token_base);
      const int32_t si = (int32_t)p.fsegs.size();
      p.fsegs.push_back({fd.token_base, 1, n, npad});
      for (int q0 = 0; q0 < n; q0 += qt_) p.fwork.push_back({si, q0});
    }
    const int32_t gi = (int32_t)p.gsegs.size();
    p.gsegs.push_back({base, w.size, n, npad});
    for (int q0 = 0; q0 < w.size * npad; q0 += qt_) p.gwork.push_back({gi, q0});
    p.mtot += (int64_t)w.size * npad;
    p.max_npad = std::max(p.max_npad, npad);
    p.max_rows = std::max(p.max_rows, w.size * npad);
  }

  // ------------------------------------------------------------------ the network
  mf_status forward(const Plan& p, const FrameDesc* frames, const AttnSeg* fsegs, const AttnWork* fwork,
                    const AttnSeg* gsegs, const AttnWork* gwork, const int32_t* cam_rows, const int32_t* dups,
                    int layers, std::string& err) {
    const int M = (int)p.mtot, D = D_;
    HIPCHECK(im2col(dt_, frames, (int)p.frames.size(), p.max_npad, Hb_, KP, rowinfo_, rowframe_, prow_, pdst_, st_));
    GemmArgs g{};
    g.A = Hb_; g.lda = KP; g.Bt = Wp_; g.ldb = KP; g.M = (int)p.patch_rows; g.N = D; g.K = KP;
    g.bias = b_p_; g.C = X_; g.ldc = D; g.N = D;
    g.rowinfo = prow_; g.rowdst = pdst_; g.pe = pe_; g.c_ref = c_ref_; g.c_other = c_other_;
    HIPCHECK(run_gemm(EPI_PATCH, g, MF_STAGE_PATCH));
    if (!p.dups.empty()) {
      prof_begin();
      HIPCHECK(copy_embedded(frames, dups, (int)p.dups.size(), p.max_npad, X_, D, c_ref_, c_other_, st_));
      prof_end(MF_STAGE_PATCH);
    }
    // fp8: activations feeding the QKV and MLP GEMMs are quantised per window (dynamic scales)
    const int nwin = (int)p.gsegs.size();
    // (the LayerNorm outputs' window maxima come from its per-row maxima: rowmax non-null)
    auto quant = [&](const void* y, int C, unsigned char* q, float* srow, const float* rowmax) {
      prof_begin();
      const hipError_t r =
          rowmax ? window_quant_fp8_rows((const __bf16*)y, C, gsegs, nwin, p.max_rows, rowmax, amax_, q, srow, st_)
                 : window_quant_fp8((const __bf16*)y, C, gsegs, nwin, p.max_rows, amax_, q, srow, st_);
      prof_end(MF_STAGE_QUANT_FP8);
      return r;
    };
    auto ln = [&](const float* g_, const float* b_) {
      prof_begin();
      const hipError_t r = layernorm(dt_, X_, Y_, g_, b_, M, D, nullptr, st_, fp8_ ? rowmax_ : nullptr);
      prof_end(MF_STAGE_LAYERNORM);
      return r;
    };
    for (int l = 0; l < layers; ++l) {
      const LayerW& L = layers_[l];
      HIPCHECK(ln(L.ln1_g, L.ln1_b));
      GemmArgs q{};
      q.A = Y_; q.lda = D; q.Bt = L.Wqkv; q.ldb = D; q.M = M; q.N = 3 * D; q.K = D; q.bias = L.b_qkv;
      q.q = Q_; q.k = K_; q.vt = Vt_; q.heads = H_; q.hd = hd_; q.mpad = mpad_;
      q.qscale = attention_q_scale(hd_);
      if (fp8_attn_) { q.q8 = Q8_; q.k8 = K8_; q.qe8 = QE_; q.ke8 = KE_; }
      if (fp8_) {
        HIPCHECK(quant(Y_, D, Y8_, srow_, rowmax_));
        q.A = Y8_;
        q.ascale = srow_;
        q.bscale = wscale_ + 3 * l;
      }
      HIPCHECK(run_gemm(EPI_QKV, q, MF_STAGE_QKV, fp8_));
      const bool global = (l % 2) == 1;
      prof_begin();
      const AttnSeg* segs = global ? gsegs : fsegs;
      const AttnWork* wl = global ? gwork : fwork;
      const int nw = (int)(global ? p.gwork.size() : p.fwork.size());
      if (fp8_attn_)
        HIPCHECK(attention_fp8qk(Q8_, QE_, K8_, KE_, Vt_, O_, mpad_, H_, D, segs, wl, nw, st_));
      else
        HIPCHECK(attention(dt_, hd_, Q_, K_, Vt_, O_, mpad_, H_, D, segs, wl, nw, st_));
      prof_end(global ? MF_STAGE_ATTN_GLOBAL : MF_STAGE_ATTN_FRAME);
      GemmArgs o{};
      o.A = O_; o.lda = D; o.Bt = L.Wo; o.ldb = D; o.M = M; o.N = D; o.K = D; o.bias = L.b_o; o.C = X_; o.ldc = D;
      HIPCHECK(run_gemm(EPI_RESID, o, MF_STAGE_OUT_PROJ));
      HIPCHECK(ln(L.ln2_g, L.ln2_b));
      GemmArgs f1{};
      f1.A = Y_; f1.lda = D; f1.Bt = L.W1; f1.ldb = D; f1.M = M; f1.N = F_; f1.K = D; f1.bias = L.b_1;
      f1.C = Hb_; f1.ldc = F_;
      if (fp8_) {
        HIPCHECK(quant(Y_, D, Y8_, srow_, rowmax_));
        f1.A = Y8_;
        f1.ascale = srow_;
        f1.bscale = wscale_ + 3 * l + 1;
      }
      HIPCHECK(run_gemm(EPI_GELU, f1, MF_STAGE_FC1, fp8_));
      GemmArgs f2{};
      f2.A = Hb_; f2.lda = F_; f2.Bt = L.W2; f2.ldb = F_; f2.M = M; f2.N = D; f2.K = F_; f2.bias = L.b_2;
      f2.C = X_; f2.ldc = D;
      if (fp8_) {
        HIPCHECK(quant(Hb_, F_, H8_, srow2_, nullptr));
        f2.A = H8_;
        f2.ascale = srow2_;
        f2.bscale = wscale_ + 3 * l + 2;
      }
      HIPCHECK(run_gemm(EPI_RESID, f2, MF_STAGE_FC2, fp8_));
    }
    if (layers == depth_) {
      const int Fr = (int)p.frames.size();
      prof_begin();
      HIPCHECK(layernorm(DT_F32, X_, camln_, lnf_g_, lnf_b_, Fr, D, cam_rows, st_));
      GemmArgs h{};
      h.A = camln_; h.lda = D; h.Bt = H1t_; h.ldb = D; h.M = Fr; h.N = D; h.K = D; h.bias = h_1_;
      h.C = camg_; h.ldc = D;
      HIPCHECK(gemm(DT_F32, EPI_GELU, h, st_));
      HIPCHECK(pose_out(camg_, H_2_, h_2_, Fr, D, pose9_, tloc_, st_));
      prof_end(MF_STAGE_HEAD);
    }
    return MF_OK;
  }

  hipError_t run_gemm(Epi e, const GemmArgs& a, int stage, bool fp8 = false) {
    prof_begin();
    const hipError_t r = gemm(fp8 ? DT_FP8 : dt_, e, a, st_);
    prof_end(stage);
    return r;
  }

  // ------------------------------------------------------------------ optional per-kernel timing
  struct ProfEv { hipEvent_t a, b; int kind; };
  std::vector<ProfEv> prof_pool_;
  size_t prof_used_ = 0;
  void latch_profiling() {
    std::lock_guard<std::mutex> lk(prof_mu_);
    prof_batch_ = profiling_;
  }
  void prof_begin() {
    if (!prof_batch_) return;
    if (prof_target_) {   // capturing: the graph owns its events
      ProfEv e;
      hipEventCreate(&e.a);
      hipEventCreate(&e.b);
      e.kind = -1;
      prof_target_->push_back(e);
      hipEventRecord(e.a, st_);
      return;
    }
    if (prof_used_ == prof_pool_.size()) {
      ProfEv e;
      hipEventCreate(&e.a);
      hipEventCreate(&e.b);
      prof_pool_.push_back(e);
    }
    hipEventRecord(prof_pool_[prof_used_].a, st_);
  }
  void prof_end(int kind) {
    if (!prof_batch_) return;
    if (prof_target_) {
      prof_target_->back().kind = kind;
      hipEventRecord(prof_target_->back().b, st_);
      return;
    }
    hipEventRecord(prof_pool_[prof_used_].b, st_);
    prof_pool_[prof_used_].kind = kind;
    prof_used_++;
  }
  void account(const ProfEv& e) {
    float ms = 0.0f;
    hipEventSynchronize(e.b);
    hipEventElapsedTime(&ms, e.a, e.b);
    if (e.kind >= 0 && e.kind < MF_STAGE_COUNT) {
      prof_ms_[e.kind] += ms;
      prof_calls_[e.kind]++;
    }
  }
  void collect_profile(std::string&) {
    std::lock_guard<std::mutex> lk(prof_mu_);
    for (size_t i = 0; i < prof_used_; ++i) account(prof_pool_[i]);
    prof_used_ = 0;
    if (replayed_prof_ && prof_batch_)
      for (const ProfEv& e : *replayed_prof_) account(e);
    replayed_prof_ = nullptr;
  }

  void release() {
    hipSetDevice(device_);
    clear_graphs();
    auto F = [this](void* p) { dfree(p); };
    F(wdev_); F(Wp_); F(H1t_);
    for (auto& L : layers_) { F(L.Wqkv); F(L.Wo); F(L.W1); F(L.W2); }
    F(X_); F(Y_); F(O_); F(Hb_); F(rowinfo_); F(rowframe_); F(prow_); F(pdst_); F(win_scale_); F(Q_); F(K_); F(Vt_);
    F(Wd_); F(bd_);
    F(Y8_); F(H8_); F(srow_); F(srow2_); F(rowmax_); F(amax_); F(wscale_); F(wamax_); F(Q8_); F(K8_); F(QE_); F(KE_);
    F(camln_); F(camg_); F(pose9_); F(tloc_); F(res_); F(keys_); F(psum_); F(pe_); F(tab_dev_);
    if (res_host_) hipHostFree(res_host_);
    if (tab_host_) hipHostFree(tab_host_);
    for (auto& e : prof_pool_) { hipEventDestroy(e.a); hipEventDestroy(e.b); }
    if (ev0_) hipEventDestroy(ev0_);
    if (ev1_) hipEventDestroy(ev1_);
    if (copy_) hipStreamDestroy(copy_);
    if (own_stream_ && st_) hipStreamDestroy(st_);
  }

  // device memory: the caller's allocator when one was given, else hipMalloc
  template <typename T>
  hipError_t dmalloc(T** p, size_t bytes) {
    if (!ualloc_) return hipMalloc((void**)p, bytes);
    *p = (T*)ualloc_(bytes, uctx_);
    if (!*p && bytes) return hipErrorOutOfMemory;
    if (((uintptr_t)*p & 255) != 0) return hipErrorInvalidValue;
    return hipSuccess;
  }
  void dfree(void* p) {
    if (!p) return;
    if (ufree_) {
      // hipFree waits for the device; the caller's allocator may hand the memory out again at once
      hipDeviceSynchronize();
      ufree_(p, uctx_);
    } else {
      hipFree(p);
    }
  }
  void* (*ualloc_)(size_t, void*) = nullptr;
  void (*ufree_)(void*, void*) = nullptr;
  void* uctx_ = nullptr;

  mf_model_cfg m_{};
  int D_ = 0, H_ = 0, hd_ = 0, F_ = 0, depth_ = 0, device_ = 0, qt_ = 128;
  Dtype dt_ = DT_F32;
  size_t es_ = 4;
  hipStream_t st_ = nullptr, copy_ = nullptr;
  bool own_stream_ = false;
  uint64_t budget_ = 0;
  int64_t mcap_ = 0, mpad_ = 0, fcap_ = 0;
  float* wdev_ = nullptr;
  const float *b_p_ = nullptr, *c_ref_ = nullptr, *c_other_ = nullptr, *lnf_g_ = nullptr, *lnf_b_ = nullptr;
  const float *h_1_ = nullptr, *H_2_ = nullptr, *h_2_ = nullptr;
  void* Wp_ = nullptr;
  float* H1t_ = nullptr;
  std::vector<LayerW> layers_;
  float* X_ = nullptr;
  void *Y_ = nullptr, *O_ = nullptr, *Hb_ = nullptr, *Q_ = nullptr, *K_ = nullptr, *Vt_ = nullptr;
  int32_t* rowinfo_ = nullptr;
  int32_t* rowframe_ = nullptr;    // token row -> frame index of the batch (im2col)
  int32_t* prow_ = nullptr;        // patch matrix row -> rowinfo of its token row
  int32_t* pdst_ = nullptr;        // patch matrix row -> token row
  int64_t reused_ = 0;             // frames of the last batch that took an earlier window's embedding
  double* win_scale_ = nullptr;    // per chained window: the anchoring's translation scale factor
  bool depth_head_ = false;
  const float *lnd_g_ = nullptr, *lnd_b_ = nullptr;
  void* Wd_ = nullptr;             // depth head [DEPTH_N][D], compute type, rows >= DEPTH_OUT zero
  float* bd_ = nullptr;            // [DEPTH_N]
  float *camln_ = nullptr, *camg_ = nullptr, *pose9_ = nullptr;
  double* tloc_ = nullptr;
  mf_focus* res_ = nullptr;
  mf_focus* res_host_ = nullptr;
  unsigned long long* keys_ = nullptr;
  double* psum_ = nullptr;
  size_t psum_cap_ = 0;
  char* tab_dev_ = nullptr;
  char* tab_host_ = nullptr;
  size_t tab_cap_ = 0;
  float* pe_ = nullptr;
  int pe_rows_ = 0, pe_cap_ = 0;
  std::map<std::pair<int, int>, int> pe_index_;
  std::mutex pe_mu_;           // pe_, pe_rows_ and pe_index_
  hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
  std::mutex prof_mu_;         // profiling_ and the prof_*_ sums (mf_profile runs on API threads)
  bool profiling_ = false;     // the switch set by mf_profile
  bool prof_batch_ = false;    // the switch as the running batch read it when it started
  bool use_graphs_ = false;
  bool fp8_ = false;
  unsigned char *Y8_ = nullptr, *H8_ = nullptr;
  bool fp8_attn_ = false;
  unsigned char *Q8_ = nullptr, *K8_ = nullptr, *QE_ = nullptr, *KE_ = nullptr;
  float *srow_ = nullptr, *srow2_ = nullptr, *wscale_ = nullptr;
  float* rowmax_ = nullptr;        // fp8: max |Y| of each token row, written by the LayerNorm
  unsigned *amax_ = nullptr, *wamax_ = nullptr;
  struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    std::vector<ProfEv> prof;   // timing events recorded inside the graph (profiled shapes)
  };
  std::map<std::string, GraphEntry> graphs_;
  std::vector<ProfEv>* prof_target_ = nullptr;
  const std::vector<ProfEv>* replayed_prof_ = nullptr;
  double prof_ms_[MF_STAGE_COUNT] = {};     // summed event times per MF_STAGE_* since the last reset
  int64_t prof_calls_[MF_STAGE_COUNT] = {};
};

Executor* make_executor() { return new HipExecutor(); }

}  // namespace mf
