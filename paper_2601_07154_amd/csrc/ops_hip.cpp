// Single-stage entry points (attention, GEMM, LayerNorm) over caller-provided device buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/mf_ops.h"
#include "kernels.h"

using namespace mf;

extern "C" {

int32_t mf_rows_per_frame(int32_t height, int32_t width) {
  const int32_t n = (height / 14) * (width / 14) + 1;
  return (n + 7) / 8 * 8;
}

mf_status mf_op_attention(int32_t precision, int32_t head_dim, int32_t heads, int32_t dim, const void* q,
                          const void* k, const void* vt, void* o, int64_t mpad, const int32_t* segs, int32_t nseg,
                          void* stream) {
  if (!q || !k || !vt || !o || !segs || nseg < 1 || heads < 1 || heads * head_dim != dim) return MF_EINVAL;
  if (head_dim != 32 && head_dim != 64) return MF_EINVAL;
  std::vector<AttnSeg> sg(nseg);
  std::vector<AttnWork> wk;
  for (int i = 0; i < nseg; ++i) {
    sg[i] = {segs[4 * i], segs[4 * i + 1], segs[4 * i + 2], segs[4 * i + 3]};
    const AttnSeg& s = sg[i];
    if (s.base < 0 || s.nf < 1 || s.n < 1 || s.npad < s.n || s.npad % 8 || s.base % 8) return MF_EINVAL;
    const int64_t end = (int64_t)s.base + (int64_t)s.nf * s.npad;
    if (end + 256 > mpad) return MF_EINVAL;
    const int qend = s.nf == 1 ? s.n : s.nf * s.npad;
    const int qt = attention_q_tile(precision == MF_BF16 ? DT_BF16 : DT_F32, head_dim);
    for (int q0 = 0; q0 < qend; q0 += qt) wk.push_back({i, q0});
  }
  hipStream_t st = (hipStream_t)stream;
  const Dtype dt = precision == MF_BF16 ? DT_BF16 : DT_F32;
  // the kernels take the queries multiplied by log2(e)/sqrt(hd): a scaled copy of q goes first
  const int64_t nq = (int64_t)heads * mpad * head_dim;
  const size_t qb = ((size_t)nq * (dt == DT_BF16 ? 2 : 4) + 255) / 256 * 256;
  void* dev = nullptr;
  const size_t sb = sg.size() * sizeof(AttnSeg), wb = wk.size() * sizeof(AttnWork);
  if (hipMalloc(&dev, qb + sb + wb) != hipSuccess) return MF_EDEVICE;
  char* tabs = (char*)dev + qb;
  hipError_t r = hipMemcpyAsync(tabs, sg.data(), sb, hipMemcpyHostToDevice, st);
  if (r == hipSuccess) r = hipMemcpyAsync(tabs + sb, wk.data(), wb, hipMemcpyHostToDevice, st);
  if (r == hipSuccess) r = scale_copy(dt, q, dev, nq, attention_q_scale(head_dim), st);
  if (r == hipSuccess)
    r = attention(dt, head_dim, dev, k, vt, o, mpad, heads, dim, (const AttnSeg*)tabs,
                  (const AttnWork*)(tabs + sb), (int)wk.size(), st);
  const hipError_t rs = hipStreamSynchronize(st);   // the host tables and the copy must outlive the launches
  if (r == hipSuccess) r = rs;
  hipFree(dev);
  return r == hipSuccess ? MF_OK : MF_EDEVICE;
}

mf_status mf_op_attention_fp8(int32_t heads, int32_t dim, const void* q8, const void* qe, const void* k8,
                              const void* ke, const void* vt, void* o, int64_t mpad, const int32_t* segs, int32_t nseg,
                              void* stream) {
  if (!q8 || !qe || !k8 || !ke || !vt || !o || !segs || nseg < 1 || heads < 1 || dim != heads * 64) return MF_EINVAL;
  std::vector<AttnSeg> sg(nseg);
  std::vector<AttnWork> wk;
  const int qt = attention_q_tile(DT_BF16, 64);
  for (int i = 0; i < nseg; ++i) {
    sg[i] = {segs[4 * i], segs[4 * i + 1], segs[4 * i + 2], segs[4 * i + 3]};
    const AttnSeg& s = sg[i];
    if (s.base < 0 || s.nf < 1 || s.n < 1 || s.npad < s.n || s.npad % 8 || s.base % 8) return MF_EINVAL;
    if ((int64_t)s.base + (int64_t)s.nf * s.npad + 256 > mpad) return MF_EINVAL;
    const int qend = s.nf == 1 ? s.n : s.nf * s.npad;
    for (int q0 = 0; q0 < qend; q0 += qt) wk.push_back({i, q0});
  }
  if (mpad % 8) return MF_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  void* dev = nullptr;
  const size_t sb = sg.size() * sizeof(AttnSeg), wb = wk.size() * sizeof(AttnWork);
  if (hipMalloc(&dev, sb + wb) != hipSuccess) return MF_EDEVICE;
  hipError_t r = hipMemcpyAsync(dev, sg.data(), sb, hipMemcpyHostToDevice, st);
  if (r == hipSuccess) r = hipMemcpyAsync((char*)dev + sb, wk.data(), wb, hipMemcpyHostToDevice, st);
  if (r == hipSuccess)
    r = attention_fp8qk((const unsigned char*)q8, (const unsigned char*)qe, (const unsigned char*)k8,
                        (const unsigned char*)ke, vt, o, mpad, heads, dim, (const AttnSeg*)dev,
                        (const AttnWork*)((char*)dev + sb), (int)wk.size(), st);
  const hipError_t rs = hipStreamSynchronize(st);
  if (r == hipSuccess) r = rs;
  hipFree(dev);
  return r == hipSuccess ? MF_OK : MF_EDEVICE;
}

mf_status mf_op_gemm(int32_t precision, const void* A, const void* Bt, const float* bias, float* C, int32_t M,
                     int32_t N, int32_t K, void* stream) {
  if (!A || !Bt || !C || M < 0 || N % 128 || K <= 0) return MF_EINVAL;
  if (K % (precision == MF_BF16 ? 64 : 32)) return MF_EINVAL;
  GemmArgs a{};
  a.A = A; a.lda = K; a.Bt = Bt; a.ldb = K; a.M = M; a.N = N; a.K = K; a.bias = bias; a.C = C; a.ldc = N;
  // fp32 output: the STORE epilogue of the fp32 instantiation writes float; for bf16 operands
  // the accumulator is stored through the residual epilogue onto a zeroed C.
  hipError_t r;
  if (precision == MF_BF16) {
    r = hipMemsetAsync(C, 0, (size_t)M * N * 4, (hipStream_t)stream);
    if (r == hipSuccess) r = gemm(DT_BF16, EPI_RESID, a, (hipStream_t)stream);
  } else {
    r = gemm(DT_F32, EPI_STORE, a, (hipStream_t)stream);
  }
  if (r == hipSuccess) r = hipStreamSynchronize((hipStream_t)stream);
  return r == hipSuccess ? MF_OK : MF_EDEVICE;
}

mf_status mf_op_gemm_fp8(const void* A, const void* Bt, const float* ascale, const float* bscale, const float* bias,
                         float* C, int32_t M, int32_t N, int32_t K, void* stream) {
  if (!A || !Bt || !C || !ascale || !bscale || M < 0 || N % 128 || K <= 0 || K % 128) return MF_EINVAL;
  GemmArgs a{};
  a.A = A; a.lda = K; a.Bt = Bt; a.ldb = K; a.M = M; a.N = N; a.K = K; a.bias = bias; a.C = C; a.ldc = N;
  a.ascale = ascale; a.bscale = bscale;
  hipError_t r = hipMemsetAsync(C, 0, (size_t)M * N * 4, (hipStream_t)stream);
  if (r == hipSuccess) r = gemm(DT_FP8, EPI_RESID, a, (hipStream_t)stream);
  if (r == hipSuccess) r = hipStreamSynchronize((hipStream_t)stream);
  return r == hipSuccess ? MF_OK : MF_EDEVICE;
}

mf_status mf_op_quantize_fp8(const float* x, int64_t n, float scale, void* q, void* stream) {
  if (!x || !q || n < 0 || n % 4 || !(scale > 0.0f)) return MF_EINVAL;
  hipError_t r = quantize_plain_fp8(x, n, scale, (unsigned char*)q, (hipStream_t)stream);
  if (r == hipSuccess) r = hipStreamSynchronize((hipStream_t)stream);
  return r == hipSuccess ? MF_OK : MF_EDEVICE;
}

mf_status mf_op_quantize_fp8_windows(const void* y, int32_t C, const int32_t* segs, int32_t nwin, void* q,
                                     float* srow, void* stream) {
  if (!y || !q || !srow || !segs || nwin < 1 || C <= 0 || C % 16) return MF_EINVAL;
  std::vector<AttnSeg> sg(nwin);
  int max_rows = 0;
  for (int i = 0; i < nwin; ++i) {
    sg[i] = {segs[4 * i], segs[4 * i + 1], segs[4 * i + 2], segs[4 * i + 3]};
    const AttnSeg& s = sg[i];
    if (s.base < 0 || s.nf < 1 || s.n < 1 || s.npad < s.n) return MF_EINVAL;
    max_rows = std::max(max_rows, s.nf * s.npad);
  }
  hipStream_t st = (hipStream_t)stream;
  void* dev = nullptr;
  const size_t sb = sg.size() * sizeof(AttnSeg);
  if (hipMalloc(&dev, sb + (size_t)nwin * 4) != hipSuccess) return MF_EDEVICE;
  hipError_t r = hipMemcpyAsync(dev, sg.data(), sb, hipMemcpyHostToDevice, st);
  if (r == hipSuccess)
    r = window_quant_fp8((const __bf16*)y, C, (const AttnSeg*)dev, nwin, max_rows, (unsigned*)((char*)dev + sb),
                         (unsigned char*)q, srow, st);
  hipStreamSynchronize(st);
  hipFree(dev);
  return r == hipSuccess ? MF_OK : MF_EDEVICE;
}

mf_status mf_op_layernorm(int32_t precision, const float* x, void* y, const float* g, const float* b, int64_t rows,
                          int32_t dim, void* stream) {
  if (!x || !y || !g || !b || rows < 0) return MF_EINVAL;
  hipError_t r = layernorm(precision == MF_BF16 ? DT_BF16 : DT_F32, x, y, g, b, rows, dim, nullptr,
                           (hipStream_t)stream);
  if (r == hipSuccess) r = hipStreamSynchronize((hipStream_t)stream);
  return r == hipSuccess ? MF_OK : MF_EDEVICE;
}

}  // extern "C"
