// Device-side helpers shared by the gfx950 kernels of the motion-focus library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef __bf16 bf16;
typedef unsigned char fp8;   // OCP E4M3 storage byte
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
// Native vector types for 16- and 8-byte fragments.  (HIP's uint4/uint2 are structs with
// unions; arrays of them kept across loop iterations were demoted to scratch memory.)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

#define MF_DEV __device__ __forceinline__

// Map a linear workgroup id so that the ids handled by one XCD are contiguous: the
// hardware deals workgroups round-robin over the 8 XCDs, each with its own L2.
MF_DEV int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  const int base = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  return base + (b >> 3);
}

MF_DEV float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
MF_DEV float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
MF_DEV double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T> MF_DEV T from_f32(float x);
template <> MF_DEV float from_f32<float>(float x) { return x; }
template <> MF_DEV bf16 from_f32<bf16>(float x) { return (bf16)x; }
template <typename T> MF_DEV float to_f32(T x) { return (float)x; }

MF_DEV float gelu_erf(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

// erf by Abramowitz & Stegun, Handbook of Mathematical Functions, formula 7.1.26:
// erf(x) = 1 - (a1 t + a2 t^2 + a3 t^3 + a4 t^4 + a5 t^5) exp(-x^2), t = 1 / (1 + p x), x >= 0,
// |error| <= 1.5e-7.  Used where the result is rounded to bf16 (relative step 2^-8).
MF_DEV float erf_as7126(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
  float poly = fmaf(1.061405429f, t, -1.453152027f);
  poly = fmaf(poly, t, 1.421413741f);
  poly = fmaf(poly, t, -0.284496736f);
  poly = fmaf(poly, t, 0.254829592f);
  poly *= t;
  const float e = __builtin_amdgcn_exp2f(-ax * ax * 1.4426950408889634f);
  return copysignf(fmaf(-poly, e, 1.0f), x);
}
MF_DEV float gelu_erf_fast(float z) { return 0.5f * z * (1.0f + erf_as7126(z * 0.70710678118654752f)); }

// fp32 -> OCP E4M3 with round-to-nearest-even, saturating at +-448 (the scale maps the amax to 448).
MF_DEV unsigned pack4_fp8(float a, float b, float c, float d) {
  a = fminf(fmaxf(a, -448.0f), 448.0f);
  b = fminf(fmaxf(b, -448.0f), 448.0f);
  c = fminf(fmaxf(c, -448.0f), 448.0f);
  d = fminf(fmaxf(d, -448.0f), 448.0f);
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
  return (unsigned)w;
}

// The least integer e with 448 * 2^e >= amax, from the bits of amax = m 2^E (m in [1, 2)):
// amax / 448 = (m / 1.75) 2^(E - 8) and m / 1.75 lies in (0.5, 1] for m <= 1.75, so e = E - 8 there and
// E - 7 above (mantissa field beyond 0x600000).  0 for amax = 0; normal amax only (the E4M3 operands
// this scales have amax >= 2^-126 or are zero rows).
MF_DEV int e4m3_row_exponent(float amax) {
  const unsigned u = __float_as_uint(amax);
  if (!(amax > 0.0f)) return 0;
  const int E = (int)((u >> 23) & 255u) - 127;
  const int e = E - 8 + ((u & 0x7fffffu) > 0x600000u ? 1 : 0);
  return e < -127 ? -127 : (e > 126 ? 126 : e);   // the E8M0 range with 2^-e a normal fp32
}
