// Row-wise kernels: LayerNorm, patch extraction with ImageNet normalisation, the 2-D sin-cos
// position table, weight conversion, and the tail of the camera-token pose head.
#include "device.h"
#include "kernels.h"

namespace mf {

// ------------------------------------------------------------------ LayerNorm, one wave per row
// (x - mean) / sqrt(var + 1e-6) * g + b with fp32 statistics (two passes over registers).
// rowmax (nullable): max |y| of each written row (the values as stored), for the fp8 window scales.
template <typename T, int VPL>
__global__ __launch_bounds__(256) void ln_kernel(const float* __restrict__ x, T* __restrict__ y,
                                                 const float* __restrict__ g,
                                                 const float* __restrict__ b, int64_t nrows,
                                                 const int32_t* __restrict__ rows, float* __restrict__ rowmax) {
  constexpr int D = VPL * 64;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= nrows) return;
  const int lane = threadIdx.x & 63;
  const int64_t src = rows ? rows[r] : r;
  const float* xr = x + src * D;
  float v[VPL];
#pragma unroll
  for (int i = 0; i < VPL; ++i) v[i] = xr[i * 64 + lane];
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < VPL; ++i) s += v[i];
  const float mean = wave_sum(s) * (1.0f / D);
  float q = 0.0f;
#pragma unroll
  for (int i = 0; i < VPL; ++i) {
    const float d = v[i] - mean;
    q += d * d;
  }
  const float rstd = rsqrtf(wave_sum(q) * (1.0f / D) + 1e-6f);
  T* yr = y + r * D;
  float mx = 0.0f;
#pragma unroll
  for (int i = 0; i < VPL; ++i) {
    const int c = i * 64 + lane;
    const T o = from_f32<T>((v[i] - mean) * rstd * g[c] + b[c]);
    yr[c] = o;
    mx = fmaxf(mx, fabsf(to_f32(o)));
  }
  if (rowmax) {
    mx = wave_max(mx);
    if (lane == 0) rowmax[r] = mx;
  }
}

template <typename T>
static hipError_t ln_launch(const float* x, void* y, const float* g, const float* b,
                            int64_t nrows, int dim, const int32_t* rows, float* rowmax, hipStream_t s) {
  const dim3 grid((unsigned)((nrows + 3) / 4));
  switch (dim) {
    case 128: hipLaunchKernelGGL((ln_kernel<T, 2>), grid, dim3(256), 0, s, x, (T*)y, g, b, nrows, rows, rowmax); break;
    case 256: hipLaunchKernelGGL((ln_kernel<T, 4>), grid, dim3(256), 0, s, x, (T*)y, g, b, nrows, rows, rowmax); break;
    case 384: hipLaunchKernelGGL((ln_kernel<T, 6>), grid, dim3(256), 0, s, x, (T*)y, g, b, nrows, rows, rowmax); break;
    case 512: hipLaunchKernelGGL((ln_kernel<T, 8>), grid, dim3(256), 0, s, x, (T*)y, g, b, nrows, rows, rowmax); break;
    case 768: hipLaunchKernelGGL((ln_kernel<T, 12>), grid, dim3(256), 0, s, x, (T*)y, g, b, nrows, rows, rowmax); break;
    case 1024: hipLaunchKernelGGL((ln_kernel<T, 16>), grid, dim3(256), 0, s, x, (T*)y, g, b, nrows, rows, rowmax); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t layernorm(Dtype out_dt, const float* x, void* y, const float* g, const float* b,
                     int64_t nrows, int dim, const int32_t* rows, hipStream_t s, float* rowmax) {
  if (nrows <= 0) return hipSuccess;
  return out_dt == DT_BF16 ? ln_launch<bf16>(x, y, g, b, nrows, dim, rows, rowmax, s)
                           : ln_launch<float>(x, y, g, b, nrows, dim, rows, rowmax, s);
}

// ------------------------------------------------------------------ patch matrix
// Block (x, f): token rows x*4 .. x*4+3 of frame f (one wave per row).  Row kinds: the
// camera token (row 0), patches (rows 1..P, grid row-major) and padding (P+1 .. npad-1).
// A patch row holds (pixel - mean_c) / std_c flattened (c, ky, kx), zero beyond 588.
template <typename T>
__global__ __launch_bounds__(256) void im2col_kernel(const FrameDesc* __restrict__ frames,
                                                     T* __restrict__ A, int kpad,
                                                     int32_t* __restrict__ rowinfo,
                                                     int32_t* __restrict__ rowframe,
                                                     int32_t* __restrict__ prow, int32_t* __restrict__ pdst) {
  const FrameDesc fd = frames[blockIdx.y];
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= fd.npad) return;
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)fd.token_base + j;
  const int p = j - 1;
  const int32_t info = (j == 0) ? (fd.first ? (1 << 30) : (2 << 30)) : (j > fd.P ? (3 << 30) : fd.pe_base + p);
  if (lane == 0) {
    rowinfo[row] = info;
    if (rowframe) rowframe[row] = (int32_t)blockIdx.y;
  }
  if (fd.patch_base < 0) return;                 // embedded already: its rows are copied afterwards
  const int64_t arow = (int64_t)fd.patch_base + j;
  if (lane == 0) {
    prow[arow] = info;
    pdst[arow] = (int32_t)row;
  }
  T* ar = A + arow * kpad;
  if (j == 0 || j > fd.P) {
    for (int k = lane; k < kpad; k += 64) ar[k] = from_f32<T>(0.0f);
    return;
  }
  const int py = p / fd.gw, px = p - py * fd.gw;
  const float mean[3] = {0.485f, 0.456f, 0.406f};
  const float istd[3] = {1.0f / 0.229f, 1.0f / 0.224f, 1.0f / 0.225f};
  for (int k = lane; k < kpad; k += 64) {
    float v = 0.0f;
    if (k < 588) {
      const int c = k / 196, rem = k - c * 196, ky = rem / 14, kx = rem - ky * 14;
      const float pix = fd.px[((int64_t)c * fd.H + py * 14 + ky) * fd.W + px * 14 + kx];
      v = (pix - mean[c]) * istd[c];
    }
    ar[k] = from_f32<T>(v);
  }
}

hipError_t im2col(Dtype dt, const FrameDesc* frames, int nframes, int max_npad, void* A, int kpad,
                  int32_t* rowinfo, int32_t* rowframe, int32_t* prow, int32_t* pdst, hipStream_t s) {
  if (nframes <= 0) return hipSuccess;
  const dim3 grid((unsigned)((max_npad + 3) / 4), (unsigned)nframes);
  if (dt == DT_BF16)
    hipLaunchKernelGGL((im2col_kernel<bf16>), grid, dim3(256), 0, s, frames, (bf16*)A, kpad, rowinfo, rowframe, prow,
                       pdst);
  else
    hipLaunchKernelGGL((im2col_kernel<float>), grid, dim3(256), 0, s, frames, (float*)A, kpad, rowinfo, rowframe, prow,
                       pdst);
  return hipGetLastError();
}

// Block (x, d): rows x*4 .. x*4+3 of duplicate frame dups[d] (one wave per row, dim / 64 floats per lane).
__global__ __launch_bounds__(256) void copy_embedded_kernel(const FrameDesc* __restrict__ frames,
                                                            const int32_t* __restrict__ dups, float* __restrict__ X,
                                                            int dim, const float* __restrict__ c_ref,
                                                            const float* __restrict__ c_other) {
  const FrameDesc fd = frames[dups[blockIdx.y]];
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= fd.npad) return;
  const int lane = threadIdx.x & 63;
  float* dst = X + ((int64_t)fd.token_base + j) * dim;
  const float* src = j == 0 ? (fd.first ? c_ref : c_other) : X + ((int64_t)fd.src_base + j) * dim;
  for (int c = lane * 4; c < dim; c += 256) *(f32x4*)(dst + c) = *(const f32x4*)(src + c);
}

hipError_t copy_embedded(const FrameDesc* frames, const int32_t* dups, int ndups, int max_npad, float* X, int dim,
                         const float* c_ref, const float* c_other, hipStream_t s) {
  if (ndups <= 0) return hipSuccess;
  if (dim % 4) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((max_npad + 3) / 4), (unsigned)ndups);
  hipLaunchKernelGGL(copy_embedded_kernel, grid, dim3(256), 0, s, frames, dups, X, dim, c_ref, c_other);
  return hipGetLastError();
}

// ------------------------------------------------------------------ sin-cos position table
// pe[y*gw + x][c]: c in quarter 0..3 -> sin(y w), cos(y w), sin(x w), cos(x w),
// w_i = 10000^(-i/(dim/4)); evaluated in double, stored fp32.
__global__ void pe_kernel(float* pe, int gh, int gw, int dim) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)gh * gw * dim) return;
  const int c = (int)(idx % dim);
  const int p = (int)(idx / dim);
  const int y = p / gw, x = p - y * gw;
  const int q = dim / 4, quarter = c / q, i = c - quarter * q;
  const double w = pow(10000.0, -(double)i / q);
  const double arg = (quarter < 2 ? y : x) * w;
  pe[idx] = (float)((quarter & 1) ? cos(arg) : sin(arg));
}

hipError_t make_pe(float* pe, int gh, int gw, int dim, hipStream_t s) {
  const int64_t n = (int64_t)gh * gw * dim;
  hipLaunchKernelGGL(pe_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pe, gh, gw, dim);
  return hipGetLastError();
}

// ------------------------------------------------------------------ weights: [rows, cols] fp32 -> [cols, rows] dtype
template <typename T>
__global__ void transpose_kernel(const float* __restrict__ w, int rows, int cols, T* __restrict__ out,
                                 int ld_out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)rows * cols) return;
  const int r = (int)(idx / cols), c = (int)(idx % cols);
  out[(int64_t)c * ld_out + r] = from_f32<T>(w[idx]);
}

hipError_t convert_transpose(Dtype dt, const float* w, int rows, int cols, void* out, int ld_out,
                             hipStream_t s) {
  const int64_t n = (int64_t)rows * cols;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (dt == DT_BF16)
    hipLaunchKernelGGL((transpose_kernel<bf16>), grid, dim3(256), 0, s, w, rows, cols, (bf16*)out, ld_out);
  else
    hipLaunchKernelGGL((transpose_kernel<float>), grid, dim3(256), 0, s, w, rows, cols, (float*)out, ld_out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ pose head tail
// One wave per frame: o = g H2 + h2 (fp32), then the world-to-camera pose [R(q) | t] in double:
// q = o[3:7] (x, y, z, w) normalised (identity below 1e-12), t = o[0:3].
__global__ __launch_bounds__(64) void pose_out_kernel(const float* __restrict__ g,
                                                      const float* __restrict__ H2,
                                                      const float* __restrict__ h2, int dim,
                                                      float* __restrict__ pose9,
                                                      double* __restrict__ T_loc) {
  const int f = blockIdx.x, lane = threadIdx.x;
  const float* gr = g + (int64_t)f * dim;
  float acc[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) acc[j] = 0.0f;
  for (int c = lane; c < dim; c += 64) {
    const float v = gr[c];
#pragma unroll
    for (int j = 0; j < 9; ++j) acc[j] = fmaf(v, H2[c * 9 + j], acc[j]);
  }
  float o[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) o[j] = wave_sum(acc[j]) + h2[j];
  if (lane != 0) return;
#pragma unroll
  for (int j = 0; j < 9; ++j) pose9[f * 9 + j] = o[j];
  double x = o[3], y = o[4], z = o[5], w = o[6];
  const double nrm = sqrt(x * x + y * y + z * z + w * w);
  double* T = T_loc + (int64_t)f * 16;
  if (nrm < 1e-12) {
    x = y = z = 0.0;
    w = 1.0;
  } else {
    x /= nrm; y /= nrm; z /= nrm; w /= nrm;
  }
  T[0] = 1 - 2 * (y * y + z * z); T[1] = 2 * (x * y - z * w);     T[2] = 2 * (x * z + y * w);     T[3] = o[0];
  T[4] = 2 * (x * y + z * w);     T[5] = 1 - 2 * (x * x + z * z); T[6] = 2 * (y * z - x * w);     T[7] = o[1];
  T[8] = 2 * (x * z - y * w);     T[9] = 2 * (y * z + x * w);     T[10] = 1 - 2 * (x * x + y * y); T[11] = o[2];
  T[12] = 0; T[13] = 0; T[14] = 0; T[15] = 1;
}

hipError_t pose_out(const float* g, const float* H2, const float* h2, int F, int dim, float* pose9,
                    double* T_loc, hipStream_t s) {
  if (F <= 0) return hipSuccess;
  hipLaunchKernelGGL(pose_out_kernel, dim3(F), dim3(64), 0, s, g, H2, h2, dim, pose9, T_loc);
  return hipGetLastError();
}

}  // namespace mf

// ------------------------------------------------------------------ FP8 (OCP E4M3) quantisation
namespace mf {

__global__ void fill_u32_kernel(unsigned* p, int n, unsigned v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Per-window amax of bf16 rows [rows][C] over the valid (non-padding) token rows of each window.
// Block (x, w) of gridDim.x per window: rows base + 16 x + 16 gridDim.x k of window w (16 threads
// per row), reduced in the block to one atomicMax: about a thousand atomics per launch instead of
// one per 16 rows.
__global__ __launch_bounds__(256) void window_amax_kernel(const bf16* __restrict__ y, int C,
                                                          const AttnSeg* __restrict__ wins,
                                                          unsigned* __restrict__ amax) {
  const AttnSeg w = wins[blockIdx.y];
  const int rows = w.nf * w.npad;
  float mx = 0.0f;
  for (int rel = blockIdx.x * 16 + (threadIdx.x >> 4); rel < rows; rel += gridDim.x * 16) {
    if ((rel % w.npad) < w.n) {
      const bf16* row = y + (int64_t)(w.base + rel) * C;
      for (int c = (threadIdx.x & 15) * 8; c < C; c += 128) {
        const bf16x8 v = *(const bf16x8*)(row + c);
#pragma unroll
        for (int e = 0; e < 8; ++e) mx = fmaxf(mx, fabsf((float)v[e]));
      }
    }
  }
  mx = wave_max(mx);
  __shared__ float red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    atomicMax(&amax[blockIdx.y], __float_as_uint(m));   // non-negative floats order as unsigned
  }
}

// q = E4M3(y / s), s = amax / 448 of the row's window (1 if the window is all zero); every row of
// the window (padding rows included) gets srow = s.  Block (x, w): 16 rows, 16 threads per row,
// each thread 16 consecutive columns per step (C a multiple of 16).
__global__ __launch_bounds__(256) void window_quant_kernel(const bf16* __restrict__ y, int C,
                                                           const AttnSeg* __restrict__ wins,
                                                           const unsigned* __restrict__ amax,
                                                           fp8* __restrict__ q, float* __restrict__ srow) {
  const AttnSeg w = wins[blockIdx.y];
  const int rel = blockIdx.x * 16 + (threadIdx.x >> 4);
  if (rel >= w.nf * w.npad) return;
  const float am = __uint_as_float(amax[blockIdx.y]);
  const float s = am > 0.0f ? am / 448.0f : 1.0f;
  const float inv = 1.0f / s;
  const int64_t r = w.base + rel;
  const bf16* row = y + r * C;
  fp8* qrow = q + r * C;
  for (int c = (threadIdx.x & 15) * 16; c < C; c += 256) {
    const bf16x8 v0 = *(const bf16x8*)(row + c);
    const bf16x8 v1 = *(const bf16x8*)(row + c + 8);
    u32x4 o;
    o.x = pack4_fp8((float)v0[0] * inv, (float)v0[1] * inv, (float)v0[2] * inv, (float)v0[3] * inv);
    o.y = pack4_fp8((float)v0[4] * inv, (float)v0[5] * inv, (float)v0[6] * inv, (float)v0[7] * inv);
    o.z = pack4_fp8((float)v1[0] * inv, (float)v1[1] * inv, (float)v1[2] * inv, (float)v1[3] * inv);
    o.w = pack4_fp8((float)v1[4] * inv, (float)v1[5] * inv, (float)v1[6] * inv, (float)v1[7] * inv);
    *(u32x4*)(qrow + c) = o;
  }
  if ((threadIdx.x & 15) == 0) srow[r] = s;
}

// amax[w] = the largest row maximum over window w's valid rows: one workgroup per window, so the
// value is written whole (nothing to clear first).
__global__ __launch_bounds__(1024) void window_amax_rows_kernel(const float* __restrict__ rowmax,
                                                                const AttnSeg* __restrict__ wins,
                                                                unsigned* __restrict__ amax) {
  const AttnSeg w = wins[blockIdx.x];
  const int rows = w.nf * w.npad;
  float mx = 0.0f;
  // four rows in flight per thread: the loop is bound by load latency, not bandwidth
  for (int rel0 = threadIdx.x; rel0 < rows; rel0 += 4 * 1024) {
    float v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int rel = rel0 + k * 1024;
      v[k] = (rel < rows && (rel % w.npad) < w.n) ? rowmax[w.base + rel] : 0.0f;
    }
    mx = fmaxf(mx, fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3])));
  }
  mx = wave_max(mx);
  __shared__ float red[16];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = red[0];
    for (int i = 1; i < 16; ++i) m = fmaxf(m, red[i]);
    amax[blockIdx.x] = __float_as_uint(m);
  }
}

hipError_t window_quant_fp8_rows(const bf16* y, int C, const AttnSeg* wins, int nwin, int max_rows,
                                 const float* rowmax, unsigned* amax, fp8* q, float* srow, hipStream_t s) {
  if (nwin <= 0) return hipSuccess;
  if (C % 16 != 0 || !rowmax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(window_amax_rows_kernel, dim3((unsigned)nwin), dim3(1024), 0, s, rowmax, wins, amax);
  const int xb = (max_rows + 15) / 16;
  hipLaunchKernelGGL(window_quant_kernel, dim3((unsigned)xb, (unsigned)nwin), dim3(256), 0, s, y, C, wins, amax, q,
                     srow);
  return hipGetLastError();
}

hipError_t window_quant_fp8(const bf16* y, int C, const AttnSeg* wins, int nwin, int max_rows, unsigned* amax,
                            fp8* q, float* srow, hipStream_t s) {
  if (nwin <= 0) return hipSuccess;
  if (C % 16 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((nwin + 255) / 256), dim3(256), 0, s, amax, nwin, 0u);
  const int xb = (max_rows + 15) / 16;
  const int per_win = 1024 / nwin > 16 ? 1024 / nwin : 16;
  hipLaunchKernelGGL(window_amax_kernel, dim3((unsigned)(xb < per_win ? xb : per_win), (unsigned)nwin), dim3(256),
                     0, s, y, C, wins, amax);
  hipLaunchKernelGGL(window_quant_kernel, dim3((unsigned)xb, (unsigned)nwin), dim3(256), 0, s, y, C, wins, amax, q,
                     srow);
  return hipGetLastError();
}

// Weights: amax of an fp32 tensor, then E4M3(w / s) transposed to [cols][rows] (ld), s = amax/448.
__global__ void amax_f32_kernel(const float* __restrict__ w, int64_t n, unsigned* __restrict__ out) {
  float mx = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    mx = fmaxf(mx, fabsf(w[i]));
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(mx));
}

__global__ void quant_transpose_kernel(const float* __restrict__ w, int rows, int cols, fp8* __restrict__ out,
                                       int ld, const unsigned* __restrict__ amax, float* __restrict__ scale) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // 4 consecutive rows per thread
  const int64_t n4 = (int64_t)(rows / 4) * cols;
  const float am = __uint_as_float(*amax);
  const float s = am > 0.0f ? am / 448.0f : 1.0f;
  if (idx == 0) *scale = s;
  if (idx >= n4) return;
  const int c = (int)(idx % cols), r = (int)(idx / cols) * 4;
  const float inv = 1.0f / s;
  const unsigned p = pack4_fp8(w[(int64_t)r * cols + c] * inv, w[(int64_t)(r + 1) * cols + c] * inv,
                               w[(int64_t)(r + 2) * cols + c] * inv, w[(int64_t)(r + 3) * cols + c] * inv);
  *(unsigned*)(out + (int64_t)c * ld + r) = p;
}

hipError_t quantize_weight_fp8(const float* w, int rows, int cols, fp8* out, int ld, unsigned* amax_tmp,
                               float* scale, hipStream_t s) {
  if (rows % 4 != 0 || ld % 4 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, s, amax_tmp, 1, 0u);
  hipLaunchKernelGGL(amax_f32_kernel, dim3(1024), dim3(256), 0, s, w, (int64_t)rows * cols, amax_tmp);
  const int64_t n4 = (int64_t)(rows / 4) * cols;
  hipLaunchKernelGGL(quant_transpose_kernel, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s, w, rows, cols, out,
                     ld, amax_tmp, scale);
  return hipGetLastError();
}

// Op-level: q[i] = E4M3(x[i] / scale) for fp32 x (n a multiple of 4).
__global__ void quant_plain_kernel(const float* __restrict__ x, int64_t n4, float inv, unsigned* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n4) return;
  const f32x4 v = *(const f32x4*)(x + 4 * i);
  q[i] = pack4_fp8(v[0] * inv, v[1] * inv, v[2] * inv, v[3] * inv);
}

hipError_t quantize_plain_fp8(const float* x, int64_t n, float scale, fp8* q, hipStream_t s) {
  if (n % 4 != 0 || !(scale > 0.0f)) return hipErrorInvalidValue;
  const int64_t n4 = n / 4;
  if (n4 == 0) return hipSuccess;
  hipLaunchKernelGGL(quant_plain_kernel, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s, x, n4, 1.0f / scale,
                     (unsigned*)q);
  return hipGetLastError();
}

// Op-level: y[i] = x[i] * s, the product in fp32 rounded to T (the attention op's query scaling).
template <typename T>
__global__ void scale_copy_kernel(const T* __restrict__ x, T* __restrict__ y, int64_t n, float s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (T)((float)x[i] * s);
}

hipError_t scale_copy(Dtype dt, const void* x, void* y, int64_t n, float s, hipStream_t st) {
  if (n < 0 || (dt != DT_BF16 && dt != DT_F32)) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (dt == DT_BF16)
    hipLaunchKernelGGL(scale_copy_kernel<bf16>, grid, dim3(256), 0, st, (const bf16*)x, (bf16*)y, n, s);
  else
    hipLaunchKernelGGL(scale_copy_kernel<float>, grid, dim3(256), 0, st, (const float*)x, (float*)y, n, s);
  return hipGetLastError();
}

}  // namespace mf
