// Host-side launchers of the gfx950 kernels (internal interface of the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mf {

enum Dtype { DT_F32 = 0, DT_BF16 = 1, DT_FP8 = 2 };   // DT_FP8: OCP E4M3 bytes

// ---------------------------------------------------------------- GEMM  C = A Bt^T (+ epilogue)
enum Epi { EPI_RESID = 1, EPI_GELU = 2, EPI_QKV = 3, EPI_PATCH = 4, EPI_STORE = 5, EPI_DEPTH = 6 };

// EPI_DEPTH: one frame of a batch whose patch rows are written as a depth map
struct DepthFrame {
  float* dst;                      // [H][W] fp32 depth map of the frame, or null (frame not emitted)
  int32_t W, gw, pe_base;          // width, patch-grid width, first position-code row of its resolution
  int32_t win;                     // its window's index in the chain table (scale factor win_scale[win])
};

struct GemmArgs {
  const void* A; int64_t lda;      // [M, K] row-major, dtype
  const void* Bt; int64_t ldb;     // [N, K] row-major (the weight transposed), dtype
  int M, N, K;                     // K a multiple of the k-tile (64 bf16 / 32 fp32)
  const float* bias;               // [N] or null
  void* C; int64_t ldc;            // RESID: fp32 [M,N] (+=); GELU/STORE: dtype [M,N]; PATCH: fp32 X
  // EPI_QKV: Q, K head-major [H][mpad][hd], V transposed [H][hd][mpad]
  void* q; void* k; void* vt; int heads; int hd; int64_t mpad;
  int qkv_which0;                  // block (0 q, 1 k, 2 v) of column 0 of this launch (set internally)
  float qscale;                    // EPI_QKV: factor on the q block before its rounding (0 reads as 1)
  // fp8 operands: per-row scale of A [M] and the scale of B [1] (device); null otherwise
  const float* ascale; const float* bscale;
  // EPI_PATCH: per-row kind/PE row (rowinfo), PE table [rows][N] fp32, camera tokens; rowdst
  // (nullable): the X row each A row is written to
  const int32_t* rowinfo; const float* pe; const float* c_ref; const float* c_other; const int32_t* rowdst;
  // EPI_DEPTH: rowinfo as above, each row's frame in the batch, the frames' targets, and the windows'
  // scale factors; C = depth maps: dst[(14 py + n / 14) W + 14 px + n % 14] = scale exp(acc + bias)
  // for output columns n < 196 of a patch row (py, px)
  const int32_t* rowframe; const DepthFrame* dframes; const double* win_scale;
  // EPI_QKV, head dim 64, when q8 is set: the q and k blocks are written as OCP E4M3 rows (not to q / k)
  // [H][mpad][64] scaled per token and head by 2^-e (e the least integer with 448 2^e >= the row's
  // amax), with the E8M0 byte e + 127 in qe8 / ke8 [H][mpad]
  unsigned char *q8, *k8, *qe8, *ke8;
};
hipError_t gemm(Dtype dt, Epi epi, const GemmArgs& a, hipStream_t s);

// ---------------------------------------------------------------- attention over segments
struct AttnSeg { int32_t base, nf, n, npad; };   // tokens [base, base+nf*npad); frame stride npad, n valid
struct AttnWork { int32_t seg, q0; };             // a query tile of a segment (attention_q_tile queries)
int attention_q_tile(Dtype dt, int hd);
// The kernels take the queries pre-multiplied by attention_q_scale(hd) = log2(e) / sqrt(hd), so
// that a score is already the exponent of 2 of the softmax (the QKV epilogue applies the factor
// before rounding to the storage type).
float attention_q_scale(int hd);
// y[i] = x[i] * s in fp32, rounded to dt (bf16 or fp32); n elements.
hipError_t scale_copy(Dtype dt, const void* x, void* y, int64_t n, float s, hipStream_t st);
hipError_t attention(Dtype dt, int hd, const void* q, const void* k, const void* vt, void* o,
                     int64_t mpad, int heads, int dim, const AttnSeg* segs, const AttnWork* work,
                     int nwork, hipStream_t s);
// The same with the scores on E4M3 operands (head dim 64): q8 / k8 [H][mpad][64] E4M3 rows with
// E8M0 per-row scale bytes qe8 / ke8 [H][mpad] (queries pre-multiplied by attention_q_scale), V^T and
// O bf16; the work list is attention_q_tile(DT_BF16, 64) queries per item.
hipError_t attention_fp8qk(const unsigned char* q8, const unsigned char* qe8, const unsigned char* k8,
                           const unsigned char* ke8, const void* vt, void* o, int64_t mpad, int heads, int dim,
                           const AttnSeg* segs, const AttnWork* work, int nwork, hipStream_t s);

// ---------------------------------------------------------------- LayerNorm (fp32 in, dtype out)
// rows: optional gather table (out row i <- in row rows[i]); rowmax (optional): max |y| of every
// output row as stored, [nrows] fp32.
hipError_t layernorm(Dtype out_dt, const float* x, void* y, const float* g, const float* b,
                     int64_t nrows, int dim, const int32_t* rows, hipStream_t s, float* rowmax = nullptr);

// ---------------------------------------------------------------- patch embedding input
struct FrameDesc {
  const float* px;        // [3, H, W] fp32 pixels in [0,1)
  int32_t H, W, gw, P;    // grid width, patches
  int32_t token_base;     // row of the frame's camera token
  int32_t npad;           // rows reserved for the frame
  int32_t first;          // 1 for the first frame of its window (reference camera token)
  int32_t pe_base;        // first row of the frame's resolution in the PE arena
  int32_t patch_base;     // first row of its patch matrix rows, or -1: the frame is embedded already
  int32_t src_base;       // (patch_base -1) token row of the earlier occurrence whose rows it takes
};
// Writes rowinfo and (if not null) rowframe (the row's frame index in `frames`) for every token
// row, and for every frame with patch_base >= 0 its rows of the patch matrix A [rows, kpad] (dtype)
// at patch_base.., with prow (the rows' rowinfo) and pdst (the token row each patch row is for).
hipError_t im2col(Dtype dt, const FrameDesc* frames, int nframes, int max_npad, void* A, int kpad,
                  int32_t* rowinfo, int32_t* rowframe, int32_t* prow, int32_t* pdst, hipStream_t s);
// Frames embedded earlier in the batch (patch_base -1): token rows 1.. copied from src_base's rows
// (patch rows and padding, fp32 X [rows][dim]), row 0 set to the frame's own camera token.
hipError_t copy_embedded(const FrameDesc* frames, const int32_t* dups, int ndups, int max_npad, float* X, int dim,
                         const float* c_ref, const float* c_other, hipStream_t s);
hipError_t make_pe(float* pe, int gh, int gw, int dim, hipStream_t s);

// ---------------------------------------------------------------- weights
// out[c * ld_out + r] = w[r * cols + c]
hipError_t convert_transpose(Dtype dt, const float* w, int rows, int cols, void* out, int ld_out,
                             hipStream_t s);

// ---------------------------------------------------------------- FP8 (OCP E4M3) quantisation
// Per-window dynamic scales: q = E4M3(y / s_w), s_w = amax over window w's valid rows / 448; srow[m] =
// the scale of row m's window.  amax: [nwin] scratch (cleared here).  y [rows][C] bf16, C % 16 == 0.
hipError_t window_quant_fp8(const __bf16* y, int C, const AttnSeg* wins, int nwin, int max_rows, unsigned* amax,
                            unsigned char* q, float* srow, hipStream_t s);
// The same with the rows' maxima already known (the LayerNorm's rowmax output): the window amax is
// a reduction over [rows] floats instead of a pass over y.
hipError_t window_quant_fp8_rows(const __bf16* y, int C, const AttnSeg* wins, int nwin, int max_rows,
                                 const float* rowmax, unsigned* amax, unsigned char* q, float* srow, hipStream_t s);
// Static per-tensor weight scale: out[c * ld + r] = E4M3(w[r][c] / s), s = amax(|w|) / 448 -> *scale.
hipError_t quantize_weight_fp8(const float* w, int rows, int cols, unsigned char* out, int ld, unsigned* amax_tmp,
                               float* scale, hipStream_t s);
hipError_t quantize_plain_fp8(const float* x, int64_t n, float scale, unsigned char* q, hipStream_t s);

// ---------------------------------------------------------------- pose head tail
// g: [F, D] fp32 (after Linear-GELU), H2: [D, 9] fp32, h2: [9] -> pose9 [F, 9] fp32, T_loc [F,16] fp64
hipError_t pose_out(const float* g, const float* H2, const float* h2, int F, int dim, float* pose9,
                    double* T_loc, hipStream_t s);

}  // namespace mf

// ---------------------------------------------------------------- chaining, focus and maps (FP64)
#include "../../include/mf.h"
namespace mf {

struct FrameHist {            // per-stream device history entry (ring indexed by frame & mask)
  double T[16];               // world-to-camera pose
  double a_w[3];              // world motion vector (acceleration, Eq. 3, or velocity, Eq. 2)
  double s;                   // |a_w|
  int32_t valid;              // focus point defined
  int32_t pad;
};

struct StreamDev {            // per-stream constants of one batch
  FrameHist* hist; int32_t hist_mask; int32_t n_points;
  double fx, fy, cx, cy, sigma, sigma_min, sigma_max;
  int32_t anchor_mode, H, W, map_cap;
  float* maps;                // map ring [map_cap][H][W]
  int32_t focus_mode, stride; // MF_FOCUS_ACCEL / MF_FOCUS_VELOCITY, difference stride s
  int32_t map_mode;           // MF_MAP_MAX / MF_MAP_SUM: the normaliser Z of Eq. 7
  int32_t pad;
};

enum ChainMode { CHAIN_ANCHOR = 0, CHAIN_FIRST = 1, CHAIN_WORLD = 2 };

struct ChainWin {             // one window of one stream in this batch
  int32_t stream, mode, loc_off, window_id;
  int64_t start, emit_begin, emit_end;
  int32_t out_off, has_pose9;
};
struct ChainGroup { int32_t first_win, n_win; };   // the windows of one stream, in order

struct MapJob { int32_t stream, out; int64_t frame; };

// T_loc [rows][16] fp64 local poses, pose9 [rows][9] (nullable); out: result records; win_scale
// (nullable): [nwins] each window's translation scale factor (MF_ANCHOR_YAW_SCALE, else 1).
hipError_t chain_focus(const ChainGroup* groups, int ngroups, const ChainWin* wins,
                       const StreamDev* streams, const double* T_loc, const float* pose9,
                       mf_focus* out, double* win_scale, hipStream_t s);
// Rows of the map one render workgroup covers; the sum normaliser takes one partial per workgroup.
constexpr int MAP_ROWS = 8;
inline int map_row_blocks(int max_h) { return (max_h + MAP_ROWS - 1) / MAP_ROWS; }
// keys: [njobs] scratch (cleared here); psum: [njobs][map_row_blocks(max_h)] scratch (every entry
// written before it is read).  Renders every job's map into its stream's ring.
hipError_t focus_maps(const MapJob* jobs, int njobs, int max_h, int max_w, const StreamDev* streams,
                      mf_focus* out, unsigned long long* keys, double* psum, hipStream_t s);

}  // namespace mf
