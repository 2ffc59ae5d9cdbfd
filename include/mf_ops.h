/* mf_ops.h -- op-level entry points of libmfocus.so: single stages of the path, exposed so that
 * each can be checked and timed on its own.  Same status and error conventions as mf.h.
 *
 * Device layouts used below (T = float for MF_FP32, bfloat16 for MF_BF16):
 *   token rows  : a window of S frames occupies S * npad rows, frame f at rows f*npad ..;
 *                 row 0 of a frame is its camera token, rows 1..P its patches (grid row-major),
 *                 rows P+1 .. npad-1 padding; npad = P + 1 rounded up to a multiple of 8.
 *   Q, K        : head-major [heads][mpad][hd]
 *   Vt          : transposed [heads][hd][mpad]
 *   O           : [rows][dim], head h in columns h*hd .. h*hd+hd-1
 * mpad must exceed every row a segment can touch by 256 (rows beyond the data must hold
 * finite values: they are read and masked).
 */
#ifndef MF_OPS_H
#define MF_OPS_H
#include "mf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Rows per frame in the token layout (npad above) for an H x W frame. */
int32_t mf_rows_per_frame(int32_t height, int32_t width);

/* The ViT forward of one window (Sec. 2.2's per-window pose inference) on S frames already in
 * device memory ([S][3][H][W] fp32).  max_layers < 0 runs the whole network and writes
 * pose9 [S][9] (fp32) and T [S][16] (world(window)-to-camera, fp64); otherwise only the
 * patch embedding and the first max_layers blocks run.  tokens (nullable, host):
 * the residual stream [S * npad][dim] fp32 after the last block run.  Host outputs are
 * nullable.  MF_EAGAIN while the engine is running a batch. */
mf_status mf_forward_window(mf_engine* e, const float* frames_dev, int32_t S, int32_t height,
                            int32_t width, int32_t max_layers, float* pose9, double* T, float* tokens);

/* Diagnostics: copy the first `bytes` of an internal buffer, as left by the last batch or
 * mf_forward_window, to host memory.  which: 0 residual X (fp32 [rows][dim]), 1 LayerNorm output
 * ([rows][dim]), 2 Q (stored multiplied by log2(e)/sqrt(head_dim), the form the attention kernels
 * take), 3 K, 4 Vt (layouts above; mpad is max_tokens_per_batch rounded up to 8,
 * plus 256), 5 attention output O
 * ([rows][dim]), 6 MLP hidden / patch matrix ([rows][max(mlp, 640)]); element type T of the
 * engine's precision except X; MF_FP8 engines with head dim 64 keep their queries and keys only as
 * 7 the E4M3 queries and 8 keys ([heads][mpad][64] bytes) and 9, 10 their E8M0 row-scale bytes
 * ([heads][mpad]); their buffers 2 and 3 are not written.
 * MF_EINVAL beyond the buffer or for a buffer the engine does not keep. */
mf_status mf_debug_copy(mf_engine* e, int32_t which, void* host, size_t bytes);

/* Per-kernel timing (HIP events on the engine's stream, summed over batches since the last
 * reset).  enable: 1 start and reset, 0 stop and reset, -1 just read. */
mf_status mf_profile(mf_engine* e, int32_t enable, double* attn_global_ms, int64_t* attn_global_calls,
                     double* attn_frame_ms, double* gemm_ms);

/* Stages of the window forward (Sec. 2.2's per-window inference) timed by the same events. */
#define MF_STAGE_ATTN_GLOBAL 0  /* attention over every token of a window (odd blocks) */
#define MF_STAGE_ATTN_FRAME 1   /* attention within each frame (even blocks) */
#define MF_STAGE_QKV 2          /* LN1 output x W_qkv (head-major Q, K and transposed V) */
#define MF_STAGE_OUT_PROJ 3     /* attention output x W_o, added to the residual */
#define MF_STAGE_FC1 4          /* LN2 output x W_1, GELU */
#define MF_STAGE_FC2 5          /* hidden x W_2, added to the residual */
#define MF_STAGE_PATCH 6        /* patch-embedding GEMM (with position code and camera tokens) */
#define MF_STAGE_LAYERNORM 7    /* LN1 and LN2 of every block */
#define MF_STAGE_QUANT_FP8 8    /* per-window E4M3 activation quantisers (MF_FP8) */
#define MF_STAGE_HEAD 9         /* final LayerNorm of the camera tokens and the pose head */
#define MF_STAGE_COUNT 10
/* Per-stage sums of the timing mf_profile switches on: ms[k] milliseconds and calls[k] launches
 * of stage k since the last reset, for k < n (n <= MF_STAGE_COUNT is read; arrays host, nullable).
 * Launches replayed from hipGraphs are included when their batch was captured with timing on. */
mf_status mf_profile_stages(mf_engine* e, double* ms, int64_t* calls, int32_t n);

/* Attention softmax(Q K^T / sqrt(hd)) V per head within segments.  segs (host): nseg rows of
 * {base, nf, n, npad}: tokens base .. base + nf*npad - 1, frames of n valid tokens every npad
 * rows (keys in padding rows are masked).  Q, K, Vt, O: device, layouts above.
 * Frame-wise layers use nf = 1 per frame; global layers one segment per window. */
mf_status mf_op_attention(int32_t precision, int32_t head_dim, int32_t heads, int32_t dim,
                          const void* q, const void* k, const void* vt, void* o, int64_t mpad,
                          const int32_t* segs, int32_t nseg, void* stream);

/* The attention of mf_op_attention with its scores on E4M3 operands (the MF_FP8 precision, head
 * dim 64): q8, k8 [heads][mpad][64] E4M3 rows, qe, ke [heads][mpad] bytes: row r of head h stands for
 * q8[h][r] * 2^(qe[h][r] - 127) (E8M0), the queries already multiplied by log2(e)/sqrt(64); Vt bf16
 * and O bf16 in the layouts above; segs as for mf_op_attention.  S = q k^T is computed on E4M3 MFMA
 * with the row scales in the MFMA's scale operands; the softmax and P V are those of the bf16 path.
 * dim = 64 heads, mpad % 8 == 0; MF_EINVAL otherwise. */
mf_status mf_op_attention_fp8(int32_t heads, int32_t dim, const void* q8, const void* qe, const void* k8,
                              const void* ke, const void* vt, void* o, int64_t mpad, const int32_t* segs,
                              int32_t nseg, void* stream);

/* C[M][N] = A[M][K] Bt[N][K]^T + bias (fp32 out; bias nullable).  A, Bt in the precision's
 * type, device memory; N a multiple of 128; K a multiple of 64 (bf16) / 32 (fp32). */
mf_status mf_op_gemm(int32_t precision, const void* A, const void* Bt, const float* bias, float* C,
                     int32_t M, int32_t N, int32_t K, void* stream);

/* Low-precision variant of the window inference (the foundation-model stage of Sec. 2.2, which
 * the paper runs without fixing a precision): OCP E4M3 operands with per-tensor scales.
 *
 * FP8 GEMM: C[M][N] = (A[M][K] Bt[N][K]^T) * ascale[m] * bscale[0] + bias, fp32 out (bias nullable).
 * A, Bt: E4M3 bytes, device; ascale [M], bscale [1] fp32 device; N % 128 == 0, K % 128 == 0.
 * MF_EINVAL on other shapes or null operands; MF_EDEVICE on a launch error. */
mf_status mf_op_gemm_fp8(const void* A, const void* Bt, const float* ascale, const float* bscale, const float* bias,
                         float* C, int32_t M, int32_t N, int32_t K, void* stream);

/* q[i] = E4M3(x[i] * (1/scale)) (fp32 product), round to nearest even, saturating at +-448;
 * x fp32 device, q n bytes device, n % 4 == 0, scale > 0. */
mf_status mf_op_quantize_fp8(const float* x, int64_t n, float scale, void* q, void* stream);

/* Per-window dynamic activation scaling: for each window w of segs (host, nwin rows of
 * {base, nf, n, npad} as for attention), s_w = amax / 448 over the valid rows (the first n of
 * every npad) of y [rows][C] bf16 (s_w = 1 for an all-zero window); every row r of the window,
 * padding included, gets q[r][c] = E4M3(y[r][c] * (1/s_w)) and srow[r] = s_w.  y, q ([rows][C]
 * bytes), srow ([rows] fp32): device.  C % 16 == 0; windows must not overlap. */
mf_status mf_op_quantize_fp8_windows(const void* y, int32_t C, const int32_t* segs, int32_t nwin, void* q,
                                     float* srow, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): mf_op_quantize_fp8_windows with the same arguments and
 * results, calling no allocator.  Its window table and per-window amax counters live in a static
 * device array of the library, one copy per GPU, held until the process ends
 * (MF_NOALLOC_MAX_WINDOWS * 20 bytes); the counters are cleared on every call.  nwin above
 * MF_NOALLOC_MAX_WINDOWS -> MF_EINVAL.  Every call on one GPU uses that GPU's array: calls that
 * overlap on one GPU (other host threads or streams) race and must be serialised by the caller.
 * Returns after the quantiser has finished on `stream`. */
#define MF_NOALLOC_MAX_WINDOWS 4096
mf_status mf_op_quantize_fp8_windows_noalloc(const void* y, int32_t C, const int32_t* segs, int32_t nwin,
                                             void* q, float* srow, void* stream);

/* y = LayerNorm(x) * g + b over rows of dim (eps 1e-6), x fp32, y in the precision's type. */
mf_status mf_op_layernorm(int32_t precision, const float* x, void* y, const float* g, const float* b,
                          int64_t rows, int32_t dim, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MF_OPS_H */
