// MFMA GEMM for gfx950 with fused epilogues: C = A Bt^T + bias, then store / += residual /
// erf-GELU / scatter into head-major Q, K and transposed V / patch-embedding assembly.
//
// Workgroup: 256 threads = 2 x 2 waves; each wave owns a (32 WM) x (32 WN) block of 32x32
// MFMA tiles (256 x 128 tiles of 128 x 64 per wave for large grids, else 128 x 128).  Two main
// loops feed the same epilogue:
//  - gemm_kernel_dma (bf16, fp32): 64-byte k-slices streamed by direct-to-LDS loads into two LDS
//    stages, chunks XOR-swizzled by (row >> 2) & 3;
//  - gemm_kernel (fp8): 128-byte k-slices through one LDS stage, the next slice prefetched into
//    registers, chunks XOR-swizzled by (row >> 1) & 7.
// Both swizzles make the 8-lane groups of a fragment read hit distinct 16-byte bank slots.
//   bf16: v_mfma_f32_32x32x16_bf16, one 16-byte fragment (8 k) per lane per MFMA
//   fp32: v_mfma_f32_32x32x2_f32, the same 16-byte fragment feeds 4 MFMAs
//   fp8:  v_mfma_scale_f32_32x32x64_f8f6f4, two 16-byte fragments (32 k) per lane per MFMA
// A and B use the same (lane group, register) -> k assignment, so the contraction is
// over every k exactly once whatever order the hardware sums in.
#include "device.h"
#include "kernels.h"

namespace mf {

// One MFMA over a lane's NCH 16-byte k-fragments of A and B.
template <typename T> struct Mma;
template <> struct Mma<bf16> {
  static constexpr int NCH = 1;
  static MF_DEV void run(const u32x4* a, const u32x4* b, f32x16& c) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*(const bf16x8*)a, *(const bf16x8*)b, c, 0, 0, 0);
  }
};
template <> struct Mma<float> {
  static constexpr int NCH = 1;
  static MF_DEV void run(const u32x4* a, const u32x4* b, f32x16& c) {
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a->x), __uint_as_float(b->x), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a->y), __uint_as_float(b->y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a->z), __uint_as_float(b->z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a->w), __uint_as_float(b->w), c, 0, 0, 0);
  }
};
// OCP E4M3 operands: v_mfma_scale_f32_32x32x64_f8f6f4 (format 0 = E4M3 for A and B), block scales
// 127 (2^0: the per-tensor scales are applied in the epilogue); 32 bytes of k per lane.
template <> struct Mma<fp8> {
  static constexpr int NCH = 2;
  static MF_DEV void run(const u32x4* a, const u32x4* b, f32x16& c) {
    const i32x8 av = {(int)a[0].x, (int)a[0].y, (int)a[0].z, (int)a[0].w, (int)a[1].x, (int)a[1].y, (int)a[1].z, (int)a[1].w};
    const i32x8 bv = {(int)b[0].x, (int)b[0].y, (int)b[0].z, (int)b[0].w, (int)b[1].x, (int)b[1].y, (int)b[1].z, (int)b[1].w};
    c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, c, 0, 0, 0, 127, 0, 127);
  }
};
template <typename T> struct OutT { using type = T; };
template <> struct OutT<fp8> { using type = bf16; };   // fp8 GEMMs write bf16 (or fp32 residuals)

// TC = 1 computes each 32x32 tile transposed (the weight fragment as the MFMA's A operand), so
// that a lane holds one output row and 4 consecutive columns per register group: every
// epilogue access is a 16-byte (fp32) or 8-byte (bf16) vector.  TC = 0 (lane = one column, 4
// consecutive rows per group) is used for the transposed V store of the QKV projection.
// Epilogue of one BM x BN tile: scales, bias, then the EPI-specific store (see the kernel).  smem:
// at least 4 x 64 x 36 floats of LDS that no wave reads any more.
template <typename T, int WM, int WN, int EPI, int TC>
MF_DEV void gemm_epilogue(const GemmArgs& a, f32x16 (&acc)[WM][WN], int m0, int n0, u32x4* smem) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int g = lane >> 5, l32 = lane & 31;
  // ------------------------------------------------------------------------------ epilogue
  // The q / k / v block of a QKV tile is uniform (the block width D is a multiple of BN):
  // resolve it once per workgroup.
  using To = typename OutT<T>::type;   // element type of the q/k/v, GELU and STORE outputs
  // fp8 operands carry per-tensor scales: a per-row scale of A (its window's) and one of B
  const float bs = a.ascale ? a.bscale[0] : 1.0f;
  int which = 0, nbase = 0;
  To* dst = nullptr;
  float qs = 1.0f;   // QKV: the q block's factor (the attention kernels take scaled queries)
  if constexpr (EPI == EPI_QKV) {
    const int D = a.heads * a.hd;
    which = a.qkv_which0 + n0 / D;
    nbase = (n0 / D) * D;
    dst = (To*)(which == 0 ? a.q : (which == 1 ? a.k : a.vt));
    if (which == 0 && a.qscale != 0.0f) qs = a.qscale;
  }
  static_assert(WN % 2 == 0, "the staged epilogue takes a wave's columns 64 at a time");
  if constexpr (EPI == EPI_DEPTH) {
    // depth maps: a lane holds one token row and 4 consecutive columns per register group; patch
    // rows of frames with a target write scale * exp(value) to the pixel of each column < 196
    static_assert(TC == 1, "depth rows are row-major tiles");
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      const int m = m0 + wr * 32 * WM + i * 32 + l32;
      if (m >= a.M) continue;
      const int32_t ri = a.rowinfo[m];
      if ((ri >> 30) & 3) continue;                      // camera token or padding row
      const DepthFrame df = a.dframes[a.rowframe[m]];
      if (!df.dst) continue;                             // frame not emitted by this window
      const int p = (ri & 0x3fffffff) - df.pe_base;
      const int py = p / df.gw, px = p - py * df.gw;
      const float sc = (float)a.win_scale[df.win];
      float* base = df.dst + (int64_t)(py * 14) * df.W + px * 14;
#pragma unroll
      for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int rg = 0; rg < 4; ++rg)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int n = n0 + wc * 32 * WN + j * 32 + 8 * rg + 4 * g + e;
            if (n < 196) {
              const int ky = n / 14, kx = n - ky * 14;
              base[(int64_t)ky * df.W + kx] = sc * expf(acc[i][j][4 * rg + e] + a.bias[n]);
            }
          }
    }
  } else if constexpr (EPI == EPI_PATCH) {
    // once per batch: direct stores. rowinfo bits 30-31: 0 patch, 1 reference camera, 2 other
    // camera, 3 padding; low bits the position-code row
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      const int m = m0 + wr * 32 * WM + i * 32 + l32;
      if (m >= a.M) continue;
      const int32_t ri = a.rowinfo[m];
      const int kind = (ri >> 30) & 3;
      float* crow = (float*)a.C + (a.rowdst ? (int64_t)a.rowdst[m] : (int64_t)m) * a.ldc;
#pragma unroll
      for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) {
          const int n = n0 + wc * 32 * WN + j * 32 + 4 * g + 8 * rg;
          const f32x4 v = {acc[i][j][4 * rg], acc[i][j][4 * rg + 1], acc[i][j][4 * rg + 2], acc[i][j][4 * rg + 3]};
          f32x4 o;
          if (kind == 0) o = v + *(const f32x4*)(a.bias + n) + *(const f32x4*)(a.pe + (int64_t)(ri & 0x3fffffff) * a.N + n);
          else if (kind == 1) o = *(const f32x4*)(a.c_ref + n);
          else if (kind == 2) o = *(const f32x4*)(a.c_other + n);
          else o = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
          *(f32x4*)(crow + n) = o;
        }
    }
  } else if constexpr (TC) {
    // Row-major outputs.  A lane's accumulators hold one row and 4-column groups; written as they
    // are, a wave store would touch 32 rows with 16 bytes each.  Each wave's 32 x 64 block of a
    // chunk i is staged through LDS instead and read back so that 16 lanes cover one row's 64
    // consecutive columns: every global access is a row-contiguous run of 128 B (bf16) or 256 B.
    constexpr int SR = 68;   // floats per staged row: 16-byte aligned, rows 4 banks apart
    float* stage = (float*)smem + wave * (32 * SR);
    const int rr = lane >> 4, c4 = (lane & 15) * 4;
#pragma unroll
    for (int jh = 0; jh < WN / 2; ++jh) {
    const int nb = n0 + wc * 32 * WN + jh * 64 + c4;
    f32x4 bias4 = {0.0f, 0.0f, 0.0f, 0.0f};
    if (a.bias) bias4 = *(const f32x4*)(a.bias + nb);
    int64_t qoff = 0;   // QKV: head-major offset of column nb (4 columns stay within one head)
    if constexpr (EPI == EPI_QKV) {
      const int nn = nb - nbase;
      const int h = nn / a.hd, d = nn - h * a.hd;
      qoff = (int64_t)h * a.mpad * a.hd + d;
    }
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int rg = 0; rg < 4; ++rg)
          *(f32x4*)(stage + l32 * SR + j * 32 + 8 * rg + 4 * g) =
              (f32x4){acc[i][2 * jh + j][4 * rg], acc[i][2 * jh + j][4 * rg + 1], acc[i][2 * jh + j][4 * rg + 2],
                      acc[i][2 * jh + j][4 * rg + 3]};
      __syncthreads();
      // fp8 operands: the chunk's row scales are loaded before its first store (loads and stores
      // share one in-order counter: a load issued after a store waits for that store)
      float rsc[8];
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        rsc[p] = 1.0f;
        if constexpr (sizeof(T) == 1) rsc[p] = a.ascale[min(m0 + wr * 32 * WM + i * 32 + rr + 4 * p, a.M - 1)] * bs;
      }
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int r = rr + 4 * p;
        const int m = m0 + wr * 32 * WM + i * 32 + r;
        if constexpr (EPI == EPI_QKV) {
          // E4M3 copy of a q / k row for the fp8 attention scores: the 16 lanes of this row hold its
          // 64 columns (one head), so the row's amax is a reduction over those 16 lanes (run by every
          // lane: inactive rows contribute 0)
          if (a.q8 && which < 2) {
            const bool ok = m < a.M;
            f32x4 v = *(const f32x4*)(stage + r * SR + c4);
            v = (v * rsc[p] + bias4) * qs;
            float mx = ok ? fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3]))) : 0.0f;
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
            const int e = e4m3_row_exponent(mx);
            const float inv = __uint_as_float((unsigned)(127 - e) << 23);   // 2^-e, exact
            const unsigned pk = pack4_fp8(v[0] * inv, v[1] * inv, v[2] * inv, v[3] * inv);
            if (ok) {
              const int64_t hrow = qoff / a.hd;   // h * mpad (qoff = h mpad hd + d, d < hd)
              *(unsigned*)((which == 0 ? a.q8 : a.k8) + qoff + (int64_t)m * a.hd) = pk;
              if ((lane & 15) == 0) (which == 0 ? a.qe8 : a.ke8)[hrow + m] = (unsigned char)(e + 127);
            }
            continue;   // the attention reads these rows only in E4M3: no bf16 copy
          }
        }
        if (m < a.M) {
          f32x4 v = *(const f32x4*)(stage + r * SR + c4);
          v = v * rsc[p] + bias4;
          if constexpr (EPI == EPI_QKV) v = v * qs;
          if constexpr (EPI == EPI_RESID) {
            f32x4* c = (f32x4*)((float*)a.C + (int64_t)m * a.ldc + nb);
            *c = *c + v;
          } else {
            if constexpr (EPI == EPI_GELU) {
#pragma unroll
              for (int e = 0; e < 4; ++e) v[e] = sizeof(To) == 2 ? gelu_erf_fast(v[e]) : gelu_erf(v[e]);
            }
            To* out;
            if constexpr (EPI == EPI_QKV) out = dst + qoff + (int64_t)m * a.hd;
            else out = (To*)a.C + (int64_t)m * a.ldc + nb;
            if constexpr (sizeof(To) == 2) {
              bf16x4 o;
#pragma unroll
              for (int e = 0; e < 4; ++e) o[e] = (bf16)v[e];
              *(bf16x4*)out = o;
            } else {
              *(f32x4*)out = v;
            }
          }
        }
      }
    }
    }
  } else {
    // V^T of the QKV projection (lane = column, 4 consecutive rows per register group): staged
    // transposed, [column][row], so that 8 lanes read one column's 32 consecutive rows = keys.
    static_assert(EPI == EPI_QKV, "untransposed tiles are used for the V^T store only");
    constexpr int SV = 36;   // floats per staged column: 16-byte aligned, 4-bank-group spread
    float* stage = (float*)smem + wave * (64 * SV);
    const int cc = lane >> 3, r4 = (lane & 7) * 4;
#pragma unroll
    for (int jh = 0; jh < WN / 2; ++jh)
#pragma unroll
    for (int i = 0; i < WM; ++i) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int rg = 0; rg < 4; ++rg)
          *(f32x4*)(stage + (j * 32 + l32) * SV + 8 * rg + 4 * g) =
              (f32x4){acc[i][2 * jh + j][4 * rg], acc[i][2 * jh + j][4 * rg + 1], acc[i][2 * jh + j][4 * rg + 2],
                      acc[i][2 * jh + j][4 * rg + 3]};
      __syncthreads();
      const int mb = m0 + wr * 32 * WM + i * 32 + r4;
      // loads before stores (one in-order counter for both): row scales (fp8), the columns' biases
      float sc[4], bnv[8];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        sc[e] = 1.0f;
        if constexpr (sizeof(T) == 1) sc[e] = a.ascale[min(mb + e, a.M - 1)] * bs;
      }
#pragma unroll
      for (int p = 0; p < 8; ++p) bnv[p] = a.bias[n0 + wc * 32 * WN + jh * 64 + cc + 8 * p];
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const int c = cc + 8 * p;
        const int n = n0 + wc * 32 * WN + jh * 64 + c;
        const int nn = n - nbase;
        const int h = nn / a.hd, d = nn - h * a.hd;
        const float bn = bnv[p];
        const f32x4 v = *(const f32x4*)(stage + c * SV + r4);
        To* row = dst + ((int64_t)h * a.hd + d) * a.mpad;
        if (mb + 3 < a.M) {
          if constexpr (sizeof(To) == 2) {
            bf16x4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = (bf16)(v[e] * sc[e] + bn);
            *(bf16x4*)(row + mb) = o;
          } else {
            f32x4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = v[e] * sc[e] + bn;
            *(f32x4*)(row + mb) = o;
          }
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (mb + e < a.M) row[mb + e] = from_f32<To>(v[e] * sc[e] + bn);
        }
      }
    }
  }
}

template <typename T, int WM, int WN, int EPI, int TC>
__global__ __launch_bounds__(256, 2) void gemm_kernel(GemmArgs a) {
  constexpr int BM = 64 * WM, BN = 64 * WN;
  constexpr int EPC = 16 / sizeof(T);   // elements per 16-byte chunk
  constexpr int BK = 8 * EPC;           // elements per 128-byte row slice
  constexpr int ACH = BM * 8 / 256, BCH = BN * 8 / 256;   // chunks per thread
  // one LDS stage: the next k-slice is prefetched into registers while this one is consumed
  // main loop: A and B k-slices; epilogue: per-wave staging (4 x 64 x 36 floats at most)
  constexpr int SMEM = (BM + BN) * 8 > 2304 ? (BM + BN) * 8 : 2304;
  __shared__ u32x4 smem[SMEM];
  u32x4* const sA = smem;
  u32x4* const sB = smem + BM * 8;

  const int tilesN = a.N / BN;
  const int tilesM = (a.M + BM - 1) / BM;
  const int nb = tilesM * tilesN;
  const int bid = xcd_remap(blockIdx.x, nb);
  const int tm = bid / tilesN, tn = bid - tm * tilesN;
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int g = lane >> 5, l32 = lane & 31;

  const T* A = (const T*)a.A;
  const T* B = (const T*)a.Bt;
  const T* aptr[ACH];
  const T* bptr[BCH];
  int aoff[ACH], boff[BCH];
#pragma unroll
  for (int i = 0; i < ACH; ++i) {
    const int c = tid + i * 256, row = c >> 3, col = c & 7;
    const int gm = min(m0 + row, a.M - 1);
    aptr[i] = A + (int64_t)gm * a.lda + col * EPC;
    aoff[i] = row * 8 + (col ^ ((row >> 1) & 7));
  }
#pragma unroll
  for (int i = 0; i < BCH; ++i) {
    const int c = tid + i * 256, row = c >> 3, col = c & 7;
    bptr[i] = B + (int64_t)(n0 + row) * a.ldb + col * EPC;
    boff[i] = row * 8 + (col ^ ((row >> 1) & 7));
  }

  f32x16 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  u32x4 ra[ACH], rb[BCH];
#pragma unroll
  for (int i = 0; i < ACH; ++i) ra[i] = *(const u32x4*)aptr[i];
#pragma unroll
  for (int i = 0; i < BCH; ++i) rb[i] = *(const u32x4*)bptr[i];

  const int nk = a.K / BK;
  for (int kt = 0; kt < nk; ++kt) {
#pragma unroll
    for (int i = 0; i < ACH; ++i) sA[aoff[i]] = ra[i];
#pragma unroll
    for (int i = 0; i < BCH; ++i) sB[boff[i]] = rb[i];
    __syncthreads();
    {   // prefetch the next k-slice (the last iteration re-reads its own: no conditional registers)
      const int64_t kn = (int64_t)min(kt + 1, nk - 1) * BK;
#pragma unroll
      for (int i = 0; i < ACH; ++i) ra[i] = *(const u32x4*)(aptr[i] + kn);
#pragma unroll
      for (int i = 0; i < BCH; ++i) rb[i] = *(const u32x4*)(bptr[i] + kn);
    }
    // keep the prefetch ahead of the MFMAs: without this fence the scheduler sinks the loads to
    // the end of the iteration, right before the wait that consumes them
    __builtin_amdgcn_sched_barrier(0);
    constexpr int NCH = Mma<T>::NCH, KK = 4 / NCH;
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
      u32x4 fa[WM][NCH], fb[WN][NCH];
#pragma unroll
      for (int q = 0; q < NCH; ++q) {
        const int ch = NCH == 1 ? 2 * kk + g : 4 * kk + 2 * g + q;
#pragma unroll
        for (int i = 0; i < WM; ++i) {
          const int row = wr * 32 * WM + i * 32 + l32;
          fa[i][q] = sA[row * 8 + (ch ^ ((row >> 1) & 7))];
        }
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          const int row = wc * 32 * WN + j * 32 + l32;
          fb[j][q] = sB[row * 8 + (ch ^ ((row >> 1) & 7))];
        }
      }
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          if constexpr (TC) Mma<T>::run(fb[j], fa[i], acc[i][j]);
          else Mma<T>::run(fa[i], fb[j], acc[i][j]);
        }
    }
    __syncthreads();
  }

  gemm_epilogue<T, WM, WN, EPI, TC>(a, acc, m0, n0, smem);
}

// Main loop with direct-to-LDS loads: k-slices of 64 bytes per row (4 chunks), two LDS stages
// filled by global_load_lds_dwordx4 (lane l of a wave instruction writes LDS slot base + l, so the
// XOR swizzle (row >> 2) & 3 of the chunk index is applied to the global address), one barrier per
// slice: the next slice streams into the other stage while this one is consumed.  No staging
// registers.
template <typename T, int WM, int WN, int EPI, int TC>
__global__ __launch_bounds__(256, 2) void gemm_kernel_dma(GemmArgs a) {
  constexpr int BM = 64 * WM, BN = 64 * WN;
  constexpr int EPC = 16 / sizeof(T);      // elements per 16-byte chunk
  constexpr int CPR = 4;                   // chunks per row of a slice
  constexpr int BK = CPR * EPC;            // elements per slice
  constexpr int STAGE = (BM + BN) * CPR;   // 16-byte slots per stage
  constexpr int AI = BM * CPR / 256, BI = BN * CPR / 256;   // DMA instructions per wave per slice
  // stages: NST - 1 slices in flight.  Two measured best: three or four stages (72 / 96 KB of LDS
  // at 256 x 128) lose a resident workgroup per CU and run slower
  constexpr int NST = 2;
  constexpr int SMEM = NST * STAGE > 2304 ? NST * STAGE : 2304;
  __shared__ u32x4 smem[SMEM];

  const int tilesN = a.N / BN;
  const int tilesM = (a.M + BM - 1) / BM;
  const int nb = tilesM * tilesN;
  const int bid = xcd_remap(blockIdx.x, nb);
  const int tm = bid / tilesN, tn = bid - tm * tilesN;
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int g = lane >> 5, l32 = lane & 31;

  // per-lane sources: instruction i of this wave fills slots (4 i + wave) * 64 + lane
  const T* asrc[AI];
  const T* bsrc[BI];
#pragma unroll
  for (int i = 0; i < AI; ++i) {
    const int row = (4 * i + wave) * 16 + (lane >> 2), col = (lane & 3) ^ ((row >> 2) & 3);
    asrc[i] = (const T*)a.A + (int64_t)min(m0 + row, a.M - 1) * a.lda + col * EPC;
  }
#pragma unroll
  for (int i = 0; i < BI; ++i) {
    const int row = (4 * i + wave) * 16 + (lane >> 2), col = (lane & 3) ^ ((row >> 2) & 3);
    bsrc[i] = (const T*)a.Bt + (int64_t)(n0 + row) * a.ldb + col * EPC;
  }
  auto issue = [&](int kt, int stage) {
    const int64_t ko = (int64_t)kt * BK;
    u32x4* base = smem + stage * STAGE;
#pragma unroll
    for (int i = 0; i < AI; ++i)
      __builtin_amdgcn_global_load_lds((const void*)(asrc[i] + ko),
                                       (__attribute__((address_space(3))) void*)(base + (4 * i + wave) * 64), 16, 0, 0);
#pragma unroll
    for (int i = 0; i < BI; ++i)
      __builtin_amdgcn_global_load_lds((const void*)(bsrc[i] + ko),
                                       (__attribute__((address_space(3))) void*)(base + BM * CPR + (4 * i + wave) * 64),
                                       16, 0, 0);
  };

  f32x16 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  const int nk = a.K / BK;
  constexpr unsigned VM_ONE = 0x0f70u | (unsigned)(AI + BI);   // vmcnt(AI + BI): one later slice may be in flight
  constexpr unsigned VM_TWO = 0x0f70u | (unsigned)(2 * (AI + BI));
#pragma unroll
  for (int st = 0; st < NST - 1; ++st)
    if (st < nk) issue(st, st);
  for (int kt = 0; kt < nk; ++kt) {
    // this thread's loads of slice kt have landed once at most the later slices are outstanding
    const int later = min(NST - 2, nk - 1 - kt);
    if (NST >= 4 && later >= 2) __builtin_amdgcn_s_waitcnt(VM_TWO);
    else if (NST >= 3 && later >= 1) __builtin_amdgcn_s_waitcnt(VM_ONE);
    else __builtin_amdgcn_s_waitcnt(0x0f70);
    __syncthreads();   // everyone's slice kt has landed; every wave is done with slice kt - 1
    if (kt + NST - 1 < nk) issue(kt + NST - 1, (kt + NST - 1) % NST);
    const u32x4* sA = smem + (kt % NST) * STAGE;
    const u32x4* sB = sA + BM * CPR;
    constexpr int NCH = Mma<T>::NCH, KK = CPR / (2 * NCH);
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
      u32x4 fa[WM][NCH], fb[WN][NCH];
#pragma unroll
      for (int q = 0; q < NCH; ++q) {
        const int ch = NCH == 1 ? 2 * kk + g : 2 * g + q;
#pragma unroll
        for (int i = 0; i < WM; ++i) {
          const int row = wr * 32 * WM + i * 32 + l32;
          fa[i][q] = sA[row * CPR + (ch ^ ((row >> 2) & 3))];
        }
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          const int row = wc * 32 * WN + j * 32 + l32;
          fb[j][q] = sB[row * CPR + (ch ^ ((row >> 2) & 3))];
        }
      }
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          if constexpr (TC) Mma<T>::run(fb[j], fa[i], acc[i][j]);
          else Mma<T>::run(fa[i], fb[j], acc[i][j]);
        }
    }
  }
  __syncthreads();   // the last stage is read by every wave before the epilogue reuses the LDS
  gemm_epilogue<T, WM, WN, EPI, TC>(a, acc, m0, n0, smem);
}

template <typename T, int EPI, int WM, int WN, int TC>
static hipError_t launch_tile(const GemmArgs& a, hipStream_t s) {
  constexpr int BM = 64 * WM, BN = 64 * WN;
  if (a.M <= 0 || a.N <= 0) return hipSuccess;
  if (a.N % BN != 0) return hipErrorInvalidValue;
  // the epilogue resolves the q / k / v destination once per tile: a tile must not straddle blocks
  if constexpr (EPI == EPI_QKV)
    if ((a.heads * a.hd) % BN != 0) return hipErrorInvalidValue;
  const int nb = ((a.M + BM - 1) / BM) * (a.N / BN);
  // bf16 / fp32: direct-to-LDS main loop; fp8: register-staged (measured faster for E4M3)
  if constexpr (sizeof(T) == 1) hipLaunchKernelGGL((gemm_kernel<T, WM, WN, EPI, TC>), dim3(nb), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((gemm_kernel_dma<T, WM, WN, EPI, TC>), dim3(nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T, int EPI, int TC>
static hipError_t launch_shape(const GemmArgs& a, hipStream_t s) {
  // 256 x 128 tiles (waves of 128 x 64: fewer LDS bytes per MFMA) once there are enough of them;
  // E4M3 products narrower than 768 columns run faster on 128 x 128 tiles (measured: 12% on
  // N = 384, K = 1536)
  const bool wide = sizeof(T) == 2 || a.N >= 768;
  if (sizeof(T) <= 2 && wide && (int64_t)((a.M + 255) / 256) * (a.N / 128) >= 512)
    return launch_tile<T, EPI, 4, 2, TC>(a, s);
  return launch_tile<T, EPI, 2, 2, TC>(a, s);
}

template <typename T, int EPI>
static hipError_t launch(const GemmArgs& a, hipStream_t s) {
  constexpr int BK = 128 / sizeof(T);
  if (a.M <= 0) return hipSuccess;
  if (a.N % 128 != 0 || a.K % BK != 0 || a.K <= 0) return hipErrorInvalidValue;
  if constexpr (EPI == EPI_QKV) {
    const int D = a.heads * a.hd;
    if (D % 128 != 0 || a.N != 3 * D || !a.bias || a.hd % 4 != 0) return hipErrorInvalidValue;
    // q and k columns (row-contiguous stores) transposed tiles; v columns (V^T stores) plain
    GemmArgs qk = a;
    qk.N = 2 * D;
    qk.qkv_which0 = 0;
    hipError_t e = launch_shape<T, EPI, 1>(qk, s);
    if (e != hipSuccess) return e;
    GemmArgs v = a;
    v.N = D;
    v.Bt = (const T*)a.Bt + (int64_t)2 * D * a.ldb;
    v.bias = a.bias + 2 * D;
    v.qkv_which0 = 2;
    return launch_shape<T, EPI, 0>(v, s);
  } else {
    return launch_shape<T, EPI, 1>(a, s);
  }
}

template <typename T>
static hipError_t dispatch(Epi epi, const GemmArgs& a, hipStream_t s) {
  switch (epi) {
    case EPI_RESID: return launch<T, EPI_RESID>(a, s);
    case EPI_GELU: return launch<T, EPI_GELU>(a, s);
    case EPI_QKV: return launch<T, EPI_QKV>(a, s);
    case EPI_PATCH: return launch<T, EPI_PATCH>(a, s);
    case EPI_STORE: return launch<T, EPI_STORE>(a, s);
    case EPI_DEPTH: return launch<T, EPI_DEPTH>(a, s);
  }
  return hipErrorInvalidValue;
}

// The pointers each epilogue dereferences: a launch without them is refused on the host (the
// kernels would otherwise fault on the device).
static bool epilogue_args_ok(Epi epi, const GemmArgs& a) {
  if (!a.A || !a.Bt) return false;
  switch (epi) {
    case EPI_RESID: case EPI_GELU: case EPI_STORE: return a.C != nullptr;
    case EPI_QKV: return a.q && a.k && a.vt && a.heads > 0 && a.hd > 0 && a.mpad > 0;
    case EPI_PATCH: return a.C && a.rowinfo && a.pe && a.c_ref && a.c_other && a.bias;
    case EPI_DEPTH: return a.rowinfo && a.rowframe && a.dframes && a.win_scale && a.bias;
  }
  return false;
}

hipError_t gemm(Dtype dt, Epi epi, const GemmArgs& a, hipStream_t s) {
  if (!epilogue_args_ok(epi, a)) return hipErrorInvalidValue;
  if (dt == DT_FP8) {
    if (epi == EPI_PATCH || epi == EPI_STORE || epi == EPI_DEPTH) return hipErrorInvalidValue;   // not used with fp8
    if (!a.ascale || !a.bscale) return hipErrorInvalidValue;
    return dispatch<fp8>(epi, a, s);
  }
  return dt == DT_BF16 ? dispatch<bf16>(epi, a, s) : dispatch<float>(epi, a, s);
}

}  // namespace mf
