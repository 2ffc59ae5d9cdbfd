/* mf.h -- C ABI of the MI355X motion-focus library (libmfocus.so).
 *
 * The library turns video streams into per-frame camera poses and motion-focus points and
 * maps, following "Motion Focus Recognition in Fast-Moving Egocentric Video":
 *   - sliding-window ("sliding batch") inference of a multi-view ViT pose regressor over
 *     windows of L frames sharing O frames with their predecessor (Sec. 2.2);
 *   - incremental anchoring of each window's local poses to the previous trajectory at a
 *     shared frame, propagating only yaw and translation, in FP64; only frames not emitted
 *     before are emitted (Sec. 2.2);
 *   - the focus point: camera centre (Eq. 1), second difference (Eq. 2-3), rotation into
 *     the current camera (Eq. 4), pinhole projection with intrinsics K (Eq. 5-6);
 *   - the focus map: a normalised sum of Gaussians at the last N motion points (Eq. 7).
 *
 * Conventions
 *   - Poses are world-to-camera 4x4 row-major doubles, OpenCV axes (x right, y down,
 *     z forward).  The world frame is the first window's frame; gravity is its y axis.
 *   - Frames are fp32 RGB in [0,1), planar [n][3][H][W], H and W multiples of 14.
 *   - Intrinsics are in model-input pixels.
 *   - Every call returns an mf_status; 0 is success, negatives are errors.  No C++
 *     exception or abort crosses the ABI; mf_last_error() gives a thread-local message.
 *   - All calls on one engine are thread-safe.
 */
#ifndef MF_H
#define MF_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mf_status;
#define MF_OK 0
#define MF_EINVAL -1    /* bad argument, shape or call order */
#define MF_ENOMEM -2    /* does not fit the HBM budget, now or ever */
#define MF_EAGAIN -3    /* not now: nothing ready, ring full, or budget in use by other streams */
#define MF_ECLOSED -4   /* stream closed (end of stream reached) */
#define MF_EDEVICE -5   /* HIP error; see mf_last_error() */
#define MF_ENOTFOUND -6 /* unknown stream id */

/* precisions of the ViT forward (the chaining and focus stages are always FP64) */
#define MF_FP32 0       /* fp32 operands on fp32 MFMA */
#define MF_BF16 1       /* bf16 GEMM/attention operands, fp32 accumulation/softmax/LayerNorm */
#define MF_FP8 2        /* as MF_BF16, but the QKV and MLP GEMMs take OCP E4M3 operands: weights with
                           static per-tensor scales, activations with dynamic per-window scales */

/* anchoring modes */
#define MF_ANCHOR_YAW 0 /* lock pitch and roll, propagate yaw and translation (the paper) */
#define MF_ANCHOR_SE3 1 /* full rigid alignment (no lock) */
#define MF_ANCHOR_YAW_SCALE 2 /* MF_ANCHOR_YAW after rescaling the window's translations by the ratio
                                 of its shared frames' camera-centre distances to the anchor in the
                                 world chain and in the window (monocular windows carry their own
                                 scale; the paper's rigid chaining keeps it) */

/* Motion vector of the focus (Sec. 2.3), differences over s = diff_stride frames: */
#define MF_FOCUS_ACCEL 0    /* a_w = p_t - 2 p_{t-s} + p_{t-2s} (Eq. 3 at s = 1; the paper's focus) */
#define MF_FOCUS_VELOCITY 1 /* v = p_t - p_{t-s} (Eq. 2): the velocity-based projection the paper
                               contrasts with (focus of expansion) */

/* Normaliser Z of the focus map (Eq. 7): */
#define MF_MAP_MAX 0        /* Z = the map's largest value: the peak is 1 (the default) */
#define MF_MAP_SUM 1        /* Z = the map's sum over the pixel grid: M is a probability map */

/* push flags */
#define MF_EOS 1          /* these are the stream's last frames */
#define MF_DEVICE_PTR 2   /* the pointer is device memory (HIP) */
#define MF_POSES_LOCAL 4  /* mf_push_poses: poses of one window in its own local frame */

typedef struct mf_engine mf_engine;

typedef struct mf_model_cfg {
  int32_t depth;      /* transformer blocks, alternating frame-wise (even) / global (odd) */
  int32_t dim;        /* width D: 128, 256, 384, 512, 768 or 1024 */
  int32_t heads;      /* D / heads must be 32 or 64 */
  int32_t mlp;        /* MLP hidden width (multiple of 128) */
  int32_t patch;      /* must be 14 */
  int32_t precision;  /* MF_FP32, MF_BF16 or MF_FP8 */
  int32_t depth_head; /* 1: the blob also carries the depth head (below), so streams may emit the
                         depth maps {D_t} that Sec. 2.2's window forward predicts beside the poses */
} mf_model_cfg;

typedef struct mf_runtime_cfg {
  int32_t device;               /* HIP device ordinal */
  int32_t threaded;             /* 1: an internal scheduler thread runs batches as windows become
                                   ready; 0: batches run inside mf_engine_step / mf_engine_sync */
  int64_t max_tokens_per_batch; /* token rows of one fused batch (0: 262144) */
  uint64_t hbm_budget_bytes;    /* device memory the engine may use (0: 80% of free memory) */
  void* stream;                 /* hipStream_t to run on, or NULL for an engine-owned stream */
  int32_t use_graphs;           /* 1: each batch shape is captured once as a hipGraph and replayed */
  int32_t reserved;
  /* Optional device allocator (both or neither): every device buffer of the engine (weights,
     workspace, stream rings, tables) is taken from dev_alloc(bytes, alloc_ctx) and handed back
     with dev_free(ptr, alloc_ctx) instead of hipMalloc / hipFree, e.g. to share a framework's
     caching allocator.  Returned memory must be device memory of `device`, 256-byte aligned;
     NULL means out of memory (MF_EDEVICE).  Calls may come from the engine's scheduler thread. */
  void* (*dev_alloc)(size_t bytes, void* ctx);
  void (*dev_free)(void* ptr, void* ctx);
  void* alloc_ctx;
} mf_runtime_cfg;

typedef struct mf_stream_cfg {
  int32_t height, width;        /* model-input frame size, multiples of 14 */
  int32_t window, overlap;      /* L and O, 1 <= O < L: consecutive windows share O frames */
  double fx, fy, cx, cy;        /* pinhole intrinsics (Eq. 5) */
  int32_t n_points;             /* N of Eq. 7, 1..32 */
  int32_t anchor_mode;          /* MF_ANCHOR_YAW, MF_ANCHOR_SE3 or MF_ANCHOR_YAW_SCALE */
  double sigma;                 /* Eq. 7 scale: spread = clip(sigma * |a_w,i|, sigma_min, sigma_max) px */
  double sigma_min, sigma_max;  /* 0 => 0.5 and 4 * max(H, W) */
  int32_t emit_maps;            /* 1: render the focus map of every emitted frame */
  int32_t ring_frames;          /* device frame ring capacity (0: 2L + 8) */
  int32_t result_frames;        /* results (and maps) held until polled (0: 4L) */
  int32_t focus_mode;           /* MF_FOCUS_ACCEL (Eq. 3, the paper's) or MF_FOCUS_VELOCITY (Eq. 2) */
  int32_t diff_stride;          /* frames between the differenced centres, 1..64 (0: 1, the paper's) */
  int32_t map_mode;             /* MF_MAP_MAX or MF_MAP_SUM: the map normaliser Z of Eq. 7 */
  int32_t emit_depth;           /* 1: keep every emitted frame's depth map (model with depth_head) */
} mf_stream_cfg;

/* One emitted frame.  valid bit 0: focus point defined (t >= 2 s, or t >= s for velocity;
   |a_w| > 0; a_z not ~0); bit 1: the map is non-zero.  a_world / a_cam / s hold the motion
   vector of the stream's focus mode (the velocity in MF_FOCUS_VELOCITY). */
typedef struct mf_focus {
  int64_t frame;            /* frame index within the stream */
  int32_t window;           /* window that emitted it */
  int32_t valid;
  double T_w2c[16];         /* chained world-to-camera pose */
  float pose9[9];           /* raw head output (t3, quaternion xyzw, fov2); zeros for pushed poses */
  int32_t peak_x, peak_y;   /* argmax of the map (ties: smallest y*W + x) */
  float sigma_px;           /* this frame's own Gaussian spread of Eq. 7 in pixels,
                               clip(sigma * s, sigma_min, sigma_max); 0 without a focus point */
  double a_world[3];        /* Eq. 3 */
  double a_cam[3];          /* Eq. 4 */
  double u, v;              /* Eq. 6 */
  double s;                 /* |a_world|, the motion magnitude of Eq. 7 */
  double t_push, t_ready;   /* seconds since engine creation: frame pushed / result complete */
  double t_window;          /* the frame's window became complete (its last frame pushed; for the
                               tail or only window of a stream, also its end of stream) */
  double t_batch;           /* the batch that computed the window started: latency t_ready - t_push
                               = buffering (t_window - t_push) + queueing (t_batch - t_window) +
                               compute (t_ready - t_batch) */
} mf_focus;

typedef struct mf_stats {
  int64_t frames_pushed, frames_emitted, windows_run, batches_run;
  int64_t tokens_run;
  int32_t streams_open, streams_pending;
  uint64_t hbm_used_bytes, hbm_budget_bytes;
  double gpu_ms;            /* device time of all batches (HIP events) */
  int64_t frames_embed_shared; /* Sec. 2.2: frames of a window whose patch embedding was taken from an
                                  earlier window of the same stream in the same batch (the overlap
                                  frames of consecutive windows) instead of being computed again */
} mf_stats;

/* Sec. 2.2 (the per-window pose inference of the foundation model; here the seeded ViT whose sizes
 * the workloads fix).  Create an engine: copies the fp32 weight blob (caller keeps ownership) to the device,
 * allocates the per-batch workspace, creates the stream and (threaded) the scheduler.
 * Blob order: W_p[588,D] b_p c_ref c_other, per layer {ln1.g ln1.b W_qkv[D,3D] b_qkv W_o b_o
 * ln2.g ln2.b W_1[D,F] b_1 W_2[F,D] b_2}, lnf.g lnf.b H_1[D,D] h_1 H_2[D,9] h_2;
 * with depth_head, then lnd.g lnd.b W_d[D,196] b_d[196]: the depth of pixel (14 py + ky, 14 px + kx)
 * is exp of output ky*14 + kx of LN_d(patch token (py, px)) W_d + b_d, in the window's units;
 * linear layers stored [in, out].  n_floats must match exactly (MF_EINVAL otherwise). */
mf_status mf_engine_create(const mf_model_cfg* model, const float* weights, size_t n_floats,
                           const mf_runtime_cfg* rt, mf_engine** out);
/* Stop the scheduler, free every device allocation.  Safe on NULL.  (Resource management of the
 * boundary; no paper passage.) */
void mf_engine_destroy(mf_engine* e);

/* Admit a stream: the video {I_t} of Sec. 2.2 with its window L and overlap O (Sec. 2.2), the
 * intrinsics K of Eq. 5, and the map's N, sigma and normaliser (Eq. 7).  MF_EAGAIN: the HBM budget
 * is held by other streams now; MF_ENOMEM: it can never fit; MF_EINVAL: bad sizes or modes.
 * cfg is copied; stream_id receives the new id. */
mf_status mf_open_stream(mf_engine* e, const mf_stream_cfg* cfg, int32_t* stream_id);

/* Sec. 2.2: append frames of the stream {I_t}; a window of L frames runs once all of them are
 * here.  n frames [n][3][H][W] (host or, with MF_DEVICE_PTR, device memory) are copied before
 * return, so the caller may reuse rgb.  MF_EAGAIN: the frame ring is full (poll, then retry);
 * MF_ECLOSED after end of stream; MF_EINVAL on a stream that takes poses. */
mf_status mf_push_frames(mf_engine* e, int32_t stream_id, const float* rgb, int32_t n, int32_t flags);

/* The "any pose estimator" entry (Sec. 1, Sec. 2.3): push poses instead of frames.
 * Without MF_POSES_LOCAL: n world poses of frames first_frame .. first_frame+n-1, which must
 * continue the stream.  With MF_POSES_LOCAL: the n local poses of one window starting at
 * frame first_frame; the engine anchors them to the previous window at the last frame it
 * emitted (which the window must contain) and emits the frames not emitted before.
 * A stream takes either frames or poses, not both. */
mf_status mf_push_poses(mf_engine* e, int32_t stream_id, const double* T_w2c, int32_t n,
                        int64_t first_frame, int32_t flags);

/* Sec. 2.2 (each frame emitted once, by the first window that completes it, in order), Eq. 1-6
 * (the record's pose, motion vector and focus (u, v)) and Eq. 7 (the map).
 * Copy up to cap completed frames, in frame order, each exactly once.  maps (nullable):
 * [cap][H][W] fp32 host memory, or device memory with MF_DEVICE_PTR in maps_flags.
 * MF_EAGAIN: nothing ready now; MF_ECLOSED: closed and fully drained (the id is released). */
mf_status mf_poll_focus(mf_engine* e, int32_t stream_id, mf_focus* out, int32_t cap,
                        int32_t* n_out, float* maps, int32_t maps_flags);

/* Sec. 2.2 (the window forward predicts depth maps {D_t} beside the poses; only frames not emitted
 * before are emitted): mf_poll_focus, plus each returned frame's depth map into depth (nullable;
 * [cap][H][W] fp32, host, or device memory with MF_DEVICE_PTR in flags, which also applies to maps).
 * A frame's depth is that of the window that emits it, camera-relative, multiplied by the window's
 * anchoring scale under MF_ANCHOR_YAW_SCALE (1 otherwise).  MF_EINVAL if depth is given for a
 * stream opened without emit_depth. */
mf_status mf_poll_focus_depth(mf_engine* e, int32_t stream_id, mf_focus* out, int32_t cap, int32_t* n_out,
                              float* maps, float* depth, int32_t flags);

/* End of stream (Sec. 2.2's windows, with this library's tail window [N - L, N) for frames the
 * regular windows left out): no more pushes; the tail window is scheduled; results stay pollable. */
mf_status mf_close_stream(mf_engine* e, int32_t stream_id);

/* Sec. 2.2's sliding-batch inference, several streams' ready windows fused into one batch.
 * Non-threaded engines: run one batch of ready windows (n_windows may be NULL).
 * Threaded engines: MF_EINVAL. */
mf_status mf_engine_step(mf_engine* e, int32_t* n_windows);
/* Block until every ready window has been run and its results are pollable (Sec. 2.2's windows). */
mf_status mf_engine_sync(mf_engine* e);
/* Counters of the run (frames, windows, batches, HBM in use, device time); no paper passage. */
mf_status mf_engine_stats(mf_engine* e, mf_stats* out);

/* Error reporting of the boundary (no paper passage): the name of a status, and the thread-local
 * message of the last failed call on this thread (never NULL). */
const char* mf_status_str(mf_status s);
const char* mf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MF_H */
