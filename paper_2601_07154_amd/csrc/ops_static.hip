// Allocation-free variant of the per-window fp8 activation quantiser: the window table and the
// per-window amax counters live in a static device array of the library instead of a buffer
// allocated per call.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mf_ops.h"
#include "kernels.h"

using namespace mf;

namespace {

constexpr size_t kTableBytes = (size_t)MF_NOALLOC_MAX_WINDOWS * sizeof(AttnSeg);
constexpr size_t kAmaxBytes = (size_t)MF_NOALLOC_MAX_WINDOWS * sizeof(unsigned);
static_assert(sizeof(AttnSeg) == 4 * sizeof(int32_t), "window rows are copied as four int32");

// One copy per GPU, held until the process ends: [window table | amax counters].
static __device__ __align__(256) unsigned char scratch[kTableBytes + kAmaxBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];   // device address of `scratch` on each GPU, resolved once per device

// The device address of this GPU's copy of `scratch` (the array's name is only a host stand-in).
hipError_t scratch_ptr(void** out) {
  int dev = -1;
  hipError_t r = hipGetDevice(&dev);
  if (r != hipSuccess) return r;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    r = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (r != hipSuccess) return r;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" mf_status mf_op_quantize_fp8_windows_noalloc(const void* y, int32_t C, const int32_t* segs, int32_t nwin,
                                                        void* q, float* srow, void* stream) {
  if (!y || !q || !srow || !segs || nwin < 1 || C <= 0 || C % 16) return MF_EINVAL;
  if (nwin > MF_NOALLOC_MAX_WINDOWS) return MF_EINVAL;
  int max_rows = 0;
  for (int i = 0; i < nwin; ++i) {
    const int32_t* s = segs + 4 * i;   // {base, nf, n, npad}
    if (s[0] < 0 || s[1] < 1 || s[2] < 1 || s[3] < s[2]) return MF_EINVAL;
    const int64_t rows = (int64_t)s[1] * s[3];
    if (rows > INT32_MAX) return MF_EINVAL;
    if (rows > max_rows) max_rows = (int)rows;
  }
  void* base = nullptr;
  hipError_t r = scratch_ptr(&base);
  if (r != hipSuccess) return MF_EDEVICE;
  hipStream_t st = (hipStream_t)stream;
  AttnSeg* wins = (AttnSeg*)base;
  unsigned* amax = (unsigned*)((unsigned char*)base + kTableBytes);
  // the amax counters are cleared by a fill kernel inside window_quant_fp8 (no memset)
  r = hipMemcpyAsync(wins, segs, (size_t)nwin * sizeof(AttnSeg), hipMemcpyHostToDevice, st);
  if (r == hipSuccess)
    r = window_quant_fp8((const __bf16*)y, C, wins, nwin, max_rows, amax, (unsigned char*)q, srow, st);
  const hipError_t rs = hipStreamSynchronize(st);   // the caller's segs must outlive the copy
  if (r == hipSuccess) r = rs;
  return r == hipSuccess ? MF_OK : MF_EDEVICE;
}
