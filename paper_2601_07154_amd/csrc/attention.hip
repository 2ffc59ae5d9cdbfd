// Fused flash attention for gfx950 over token segments (frame-wise and global layers).
//
// A segment is nf frames of n valid tokens stored every npad rows (npad = n rounded up to 8,
// so every frame starts 16-byte aligned in the transposed V layout).  Frame-wise layers use
// one segment per frame, global layers one segment per window; keys in the padding rows
// between frames are masked.  softmax(Q K^T / sqrt(hd)) V is computed per head with the
// running-max rescaling of flash attention: scores never leave registers.  The queries arrive
// multiplied by log2(e)/sqrt(hd) (the QKV projection applies the factor before rounding), so a
// score is directly the base-2 exponent of its unnormalised probability.
//
// attn_kernel (fp32, and bf16 with hd 32): each workgroup (4 waves) takes 128 queries of one
// segment and one head; each wave owns 32 queries.  attn_kernel_v3 (bf16, hd 64) doubles the
// queries per wave (below).  Scores are computed transposed, S^T = K Q^T, so that each lane holds one query
// column: the row max is a reduction over the lane's 16 values plus one exchange between
// the two lane halves.  The probabilities feed O^T = V^T P^T directly from registers as the
// B operand (their k order, {4g..4g+3, 8+4g..8+4g+3}, is matched by the V^T fragments read
// from LDS).  K tiles [64 keys][hd] and V^T tiles [hd][64 keys] are staged in LDS with
// XOR-swizzled 16-byte chunks, double-buffered.
#include "device.h"
#include "kernels.h"

namespace mf {


// Validity bits of the 16 keys a lane holds in a 32-key sub-tile starting at key kb0 + 4g:
// keys kb0 + 4g + 8j + i (j, i < 4) -> bit 4j + i.  A key is valid if it lies in the segment and
// not in the padding rows of its frame (frames every npad >= 8 rows, n valid).  One modulo per
// sub-tile; the rest walks the frame offset incrementally (no per-key division).
MF_DEV unsigned key_mask(int kb0, int g, int key_end, int npad, int n) {
  const int k0 = kb0 + 4 * g;
  int rel = k0 % npad;
  unsigned bits = 0u;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (j) {
      rel += 8;
      rel = rel >= npad ? rel - npad : rel;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int ri = rel + i;
      ri = ri >= npad ? ri - npad : ri;
      const bool ok = (k0 + 8 * j + i < key_end) & (ri < n);
      bits |= (ok ? 1u : 0u) << (4 * j + i);
    }
  }
  return bits;
}

template <typename T, int HD>
struct AttnCfg {
  static constexpr int BK = 64;                          // keys per tile
  static constexpr int KCPR = HD * (int)sizeof(T) / 16;  // 16-byte chunks per K row
  static constexpr int VCPR = BK * (int)sizeof(T) / 16;  // 16-byte chunks per V^T row
  static constexpr int KCH = BK * KCPR;                  // chunks per K tile
  static constexpr int VCH = HD * VCPR;                  // chunks per V^T tile
  static constexpr int QF = HD * (int)sizeof(T) / 32;    // 16-byte Q fragments per lane
  static constexpr int DT = HD / 32;                     // 32-row tiles of O^T
};

// S^T (32 keys x 32 queries) += K_frag x Q^T_frag over the head dimension.
template <typename T, int HD>
MF_DEV void qk_tile(const u32x4* sK, int key_row, const u32x4* qf, int g, f32x16& s) {
  using C = AttnCfg<T, HD>;
#pragma unroll
  for (int f = 0; f < C::QF; ++f) {
    const int ch = 2 * f + g;
    const u32x4 kf = sK[key_row * C::KCPR + (ch ^ (key_row % C::KCPR))];
    if constexpr (sizeof(T) == 2) {
      s = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*(const bf16x8*)&kf, *(const bf16x8*)&qf[f], s, 0, 0, 0);
    } else {
      s = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(kf.x), __uint_as_float(qf[f].x), s, 0, 0, 0);
      s = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(kf.y), __uint_as_float(qf[f].y), s, 0, 0, 0);
      s = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(kf.z), __uint_as_float(qf[f].z), s, 0, 0, 0);
      s = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(kf.w), __uint_as_float(qf[f].w), s, 0, 0, 0);
    }
  }
}

// O^T (32 d x 32 queries) += V^T (rows d, keys of sub-tile kb) x P^T (from the score registers).
template <typename T, int HD>
MF_DEV void pv_tile(const u32x4* sV, int d_row, int kb, int g, const f32x16& p, f32x16& o) {
  using C = AttnCfg<T, HD>;
  const int sw = d_row % C::VCPR;
  if constexpr (sizeof(T) == 2) {
#pragma unroll
    for (int j2 = 0; j2 < 2; ++j2) {
      // keys kb*32 + 16*j2 + {4g..4g+3} (chunk c0, half g) and + 8 (chunk c0+1, half g)
      const int c0 = 4 * kb + 2 * j2;
      const u32x2* row = (const u32x2*)(sV + d_row * C::VCPR);
      const u32x2 lo = row[2 * (c0 ^ sw) + g];
      const u32x2 hi = row[2 * ((c0 + 1) ^ sw) + g];
      u32x4 vf = {lo.x, lo.y, hi.x, hi.y};
      bf16x8 pf;
#pragma unroll
      for (int r = 0; r < 8; ++r) pf[r] = (bf16)p[8 * j2 + r];
      o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*(const bf16x8*)&vf, pf, o, 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      // keys kb*32 + 8*jj + 4g + {0..3}: chunk 8kb + 2jj + g
      const u32x4 vf = sV[d_row * C::VCPR + ((8 * kb + 2 * jj + g) ^ sw)];
      o = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(vf.x), p[4 * jj + 0], o, 0, 0, 0);
      o = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(vf.y), p[4 * jj + 1], o, 0, 0, 0);
      o = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(vf.z), p[4 * jj + 2], o, 0, 0, 0);
      o = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(vf.w), p[4 * jj + 3], o, 0, 0, 0);
    }
  }
}

template <typename T, int HD>
__global__ __launch_bounds__(256) void attn_kernel(const T* __restrict__ Q, const T* __restrict__ K,
                                                   const T* __restrict__ Vt, T* __restrict__ O,
                                                   int64_t mpad, int heads, int dim,
                                                   const AttnSeg* __restrict__ segs,
                                                   const AttnWork* __restrict__ work, int nwork) {
  using C = AttnCfg<T, HD>;
  constexpr int BK = C::BK;
  __shared__ u32x4 sK[2][C::KCH];
  __shared__ u32x4 sV[2][C::VCH];

  const int nb = nwork * heads;
  const int bid = xcd_remap(blockIdx.x, nb);
  // head-major: the query tiles of one segment and head are consecutive, so the workgroups an XCD
  // runs together share that head's K and V in its L2
  const int h = bid / nwork, wi = bid - h * nwork;
  const AttnWork wk = work[wi];
  const AttnSeg sg = segs[wk.seg];
  const int seg_len = sg.nf * sg.npad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 5, l32 = lane & 31;
  const int qrow = wk.q0 + wave * 32 + l32;   // this lane's query (segment-relative)

  const T* Qh = Q + ((int64_t)h * mpad + sg.base) * HD;
  const T* Kh = K + ((int64_t)h * mpad + sg.base) * HD;
  const T* Vh = Vt + (int64_t)h * HD * mpad + sg.base;

  // Q^T fragments (B operand): lane (query l32, group g) holds chunks 2f+g of its query row.
  u32x4 qf[C::QF];
  {
    const u32x4* qr = (const u32x4*)(Qh + (int64_t)qrow * HD);
#pragma unroll
    for (int f = 0; f < C::QF; ++f) qf[f] = qr[2 * f + g];
  }

  // Tile loaders: chunk c of the K tile is (row c / KCPR, col c % KCPR); of the V^T tile
  // (d row c / VCPR, key chunk c % VCPR).
  constexpr int KPT = C::KCH / 256, VPT = C::VCH / 256;
  u32x4 rk[KPT], rv[VPT];
  auto load_tile = [&](int kt) {
#pragma unroll
    for (int i = 0; i < KPT; ++i) {
      const int c = tid + i * 256, row = c / C::KCPR, col = c % C::KCPR;
      rk[i] = *(const u32x4*)(Kh + (int64_t)(kt + row) * HD + col * (16 / sizeof(T)));
    }
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int c = tid + i * 256, row = c / C::VCPR, col = c % C::VCPR;
      rv[i] = *(const u32x4*)(Vh + (int64_t)row * mpad + kt + col * (16 / sizeof(T)));
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int i = 0; i < KPT; ++i) {
      const int c = tid + i * 256, row = c / C::KCPR, col = c % C::KCPR;
      sK[buf][row * C::KCPR + (col ^ (row % C::KCPR))] = rk[i];
    }
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int c = tid + i * 256, row = c / C::VCPR, col = c % C::VCPR;
      sV[buf][row * C::VCPR + (col ^ (row % C::VCPR))] = rv[i];
    }
  };

  f32x16 o[C::DT];
#pragma unroll
  for (int t = 0; t < C::DT; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) o[t][r] = 0.0f;
  float m_run = -INFINITY, l_run = 0.0f;

  const int key_end = sg.nf == 1 ? sg.n : seg_len;
  const int ntiles = (key_end + BK - 1) / BK;
  load_tile(0);
  store_tile(0);
  __syncthreads();

  for (int it = 0; it < ntiles; ++it) {
    const int cur = it & 1, kt = it * BK;
    load_tile(it + 1 < ntiles ? kt + BK : kt);   // unconditional: the registers stay plain values

    f32x16 s[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) s[kb][r] = 0.0f;
      qk_tile<T, HD>(sK[cur], kb * 32 + l32, qf, g, s[kb]);
    }
    // mask keys outside the segment or in the padding rows between frames
    const int f0 = kt / sg.npad;
    const bool full = kt + BK <= (f0 * sg.npad + sg.n) && kt + BK <= key_end;
    if (!full) {   // branch-free select: no divergent control flow around the scores
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const unsigned bits = key_mask(kt + kb * 32, g, key_end, sg.npad, sg.n);
#pragma unroll
        for (int r = 0; r < 16; ++r) s[kb][r] = ((bits >> r) & 1u) ? s[kb][r] : -INFINITY;
      }
    }
    float mx = -INFINITY;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int r = 0; r < 16; ++r) mx = fmaxf(mx, s[kb][r]);
    mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
    const float m_new = fmaxf(m_run, mx);
    const float alpha = exp2f(m_run - m_new);
    m_run = m_new;
    float ls = 0.0f;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float p = exp2f(s[kb][r] - m_new);
        s[kb][r] = p;
        ls += p;
      }
    l_run = l_run * alpha + ls;
#pragma unroll
    for (int t = 0; t < C::DT; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) o[t][r] *= alpha;
#pragma unroll
    for (int t = 0; t < C::DT; ++t)
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) pv_tile<T, HD>(sV[cur], t * 32 + l32, kb, g, s[kb], o[t]);

    if (it + 1 < ntiles) {
      __syncthreads();
      store_tile(cur ^ 1);
      __syncthreads();
    }
  }

  const float l_tot = l_run + __shfl_xor(l_run, 32, 64);
  const float inv = 1.0f / l_tot;
  if (qrow < seg_len) {
    T* orow = O + (int64_t)(sg.base + qrow) * dim + h * HD;
#pragma unroll
    for (int t = 0; t < C::DT; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int d = t * 32 + 8 * j + 4 * g;
        if constexpr (sizeof(T) == 2) {
          bf16x4 v;
#pragma unroll
          for (int i = 0; i < 4; ++i) v[i] = (bf16)(o[t][4 * j + i] * inv);
          *(bf16x4*)(orow + d) = v;
        } else {
          f32x4 v;
#pragma unroll
          for (int i = 0; i < 4; ++i) v[i] = o[t][4 * j + i] * inv;
          *(f32x4*)(orow + d) = v;
        }
      }
  }
}


// ------------------------------------------------------------------ bf16, hd 64 (attn_kernel_v3)
// Each wave owns two 32-query blocks that share every K and V^T fragment read from LDS (half
// the LDS traffic per flop of one block per wave); a workgroup covers 256 queries.  Keys are
// staged in LDS tiles of 128 (double-buffered, one barrier per tile; the next tile passes
// through 16 registers per thread, K during the first steps, V after) and consumed in 32-key
// steps, unrolled four to a tile so every LDS offset is a constant.  Per step:
//  - S^T = K Q^T is accumulated onto -m (m the query's reference), so the MFMA result is the
//    exp2 argument itself: no VALU work per score before the exp (the -m block is rewritten
//    only when m changes);
//  - m is set from the query's first-step maximum and raised only when a step's probabilities
//    grow large (a lane's partial row sum above 2^12, which also catches an overflow to inf);
//    no per-step maximum is computed otherwise, and the O rescale is rare;
//  - the two query blocks finish one after the other (softmax, then PV), so the PV MFMAs of one
//    block can overlap the softmax of the other;
//  - row sums are taken from the bf16-rounded probabilities that the PV product uses (v_dot2),
//    so numerator and denominator see the same weights.
// V^T tiles are stored with the keys of each 16-key group reordered [0-3, 8-11, 4-7, 12-15] so
// that a lane's PV fragment, in the key order of its probabilities, is one 16-byte LDS read.
namespace v3 {
constexpr int HD = 64, KT = 128, KS = 32, QW = 64, QT = 256;
constexpr int KCPR = 8;    // 16-byte chunks per K row (64 d)
constexpr int VCPR = 16;   // 16-byte chunks per V^T row (128 keys)
constexpr float GROW = 4096.0f;
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

MF_DEV float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// v and the value of lane l ^ 32, combined (identically in both lanes)
MF_DEV float pair_max(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}
MF_DEV float pair_sum(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// p = exp2(s - d) as bf16 pairs (the B operand of PV, keys 4g.., 8+4g.. per 16-key half) and the
// lane's partial row sum over those probabilities; s already holds the exponent relative to the
// reference, d is a further shift (a raised reference), used only when `shift` is set
MF_DEV void probs(const f32x16& s, float d, u32x4 (&pf)[2], float& ls, bool shift) {
  const bf16x2_t ones = {(bf16)1.0f, (bf16)1.0f};
  float acc = 0.0f;
#pragma unroll
  for (int j2 = 0; j2 < 2; ++j2)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float a0 = shift ? s[8 * j2 + 2 * q] - d : s[8 * j2 + 2 * q];
      const float a1 = shift ? s[8 * j2 + 2 * q + 1] - d : s[8 * j2 + 2 * q + 1];
      const f32x2 e = {fast_exp2(a0), fast_exp2(a1)};
      const bf16x2_t pr = __builtin_convertvector(e, bf16x2_t);
      acc = __builtin_amdgcn_fdot2_f32_bf16(pr, ones, acc, false);
      pf[j2][q] = __builtin_bit_cast(unsigned, pr);
    }
  ls = acc;
}

__global__ __launch_bounds__(256, 2) void attn_kernel_v3(const bf16* __restrict__ Q, const bf16* __restrict__ K,
                                                         const bf16* __restrict__ Vt, bf16* __restrict__ O,
                                                         int64_t mpad, int heads, int dim,
                                                         const AttnSeg* __restrict__ segs,
                                                         const AttnWork* __restrict__ work, int nwork) {
  __shared__ u32x4 sK[2][KT * KCPR];
  __shared__ u32x4 sV[2][HD * VCPR];
  const int nb = nwork * heads;
  const int bid = xcd_remap(blockIdx.x, nb);
  // head-major: the query tiles of one segment and head are consecutive, so the workgroups an XCD
  // runs together share that head's K and V in its L2
  const int h = bid / nwork, wi = bid - h * nwork;
  const AttnWork wk = work[wi];
  const AttnSeg sg = segs[wk.seg];
  const int seg_len = sg.nf * sg.npad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 5, l32 = lane & 31;
  const int qbase = wk.q0 + wave * QW;            // this wave's first query (segment-relative)

  const bf16* Qh = Q + ((int64_t)h * mpad + sg.base) * HD;
  const bf16* Kh = K + ((int64_t)h * mpad + sg.base) * HD;
  const bf16* Vh = Vt + (int64_t)h * HD * mpad + sg.base;

  u32x4 qf[2][4];
#pragma unroll
  for (int hb = 0; hb < 2; ++hb) {
    const u32x4* qr = (const u32x4*)(Qh + (int64_t)(qbase + hb * 32 + l32) * HD);
#pragma unroll
    for (int f = 0; f < 4; ++f) qf[hb][f] = qr[2 * f + g];
  }

  // K tile: thread -> row tid/2, chunks 4 (tid%2) .. +3.  V^T tile: thread -> row tid/4, keys
  // 32 (tid%4) .. +31 (two 16-key groups), stored with keys 4-7 and 8-11 of every group swapped,
  // the order of a lane's probabilities.
  // The next tile is staged through 16 registers per thread, K first then V: the buffer it goes to
  // was last read in the previous tile, which every wave has finished (one barrier per tile).
  u32x4 rt[4];
  auto load_k = [&](int kt) {
    const u32x4* ksrc = (const u32x4*)(Kh + (int64_t)(kt + (tid >> 1)) * HD) + 4 * (tid & 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) rt[i] = ksrc[i];
  };
  auto load_v = [&](int kt) {
    const u32x4* vsrc = (const u32x4*)(Vh + (int64_t)(tid >> 2) * mpad + kt + (tid & 3) * 32);
#pragma unroll
    for (int i = 0; i < 4; ++i) rt[i] = vsrc[i];
  };
  auto store_k = [&](int buf) {
    const int krow = tid >> 1, ksw = (krow >> 1) & 7;
#pragma unroll
    for (int i = 0; i < 4; ++i) sK[buf][krow * KCPR + ((4 * (tid & 1) + i) ^ ksw)] = rt[i];
  };
  auto store_v = [&](int buf) {
    const u32x4* rv = rt;
    const int vrow = tid >> 2, sw = vrow & 15;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int ch = 4 * (tid & 3) + 2 * p;
      const u32x4 lo = {rv[2 * p].x, rv[2 * p].y, rv[2 * p + 1].x, rv[2 * p + 1].y};   // keys 0-3 | 8-11
      const u32x4 hi = {rv[2 * p].z, rv[2 * p].w, rv[2 * p + 1].z, rv[2 * p + 1].w};   // keys 4-7 | 12-15
      sV[buf][vrow * VCPR + (ch ^ sw)] = lo;
      sV[buf][vrow * VCPR + ((ch + 1) ^ sw)] = hi;
    }
  };

  f32x16 o[2][2];
#pragma unroll
  for (int hb = 0; hb < 2; ++hb)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) o[hb][t][r] = 0.0f;
  float l_run[2] = {0.0f, 0.0f};
  float m_cur[2] = {0.0f, 0.0f};   // reference per query (log2 units), set on the first step
  f32x16 mneg[2];                  // -m_cur in all 16 registers, the value S^T accumulates onto
#pragma unroll
  for (int hb = 0; hb < 2; ++hb)
#pragma unroll
    for (int r = 0; r < 16; ++r) mneg[hb][r] = 0.0f;

  const int key_end = sg.nf == 1 ? sg.n : seg_len;
  const int nsteps = (key_end + KS - 1) / KS;
  const int ntiles = (nsteps + 3) / 4;

  // K fragments of step `sub` of an LDS tile (row l32 of the step's 32 keys, k-group g)
  auto load_kf = [&](int cur, int sub, u32x4 (&kf)[4]) {
    const int krow = sub * KS + l32;
#pragma unroll
    for (int f = 0; f < 4; ++f) kf[f] = sK[cur][krow * KCPR + ((2 * f + g) ^ ((krow >> 1) & 7))];
  };
  // one 32-key step: S^T, mask, then per query block softmax and PV
  auto step = [&](int cur, int sub, int st) {
    const int k0 = st * KS;
    u32x4 kf[4];
    load_kf(cur, sub, kf);
    f32x16 s[2];
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
      s[hb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*(const bf16x8*)&kf[0], *(const bf16x8*)&qf[hb][0], mneg[hb],
                                                      0, 0, 0);
#pragma unroll
      for (int f = 1; f < 4; ++f)
        s[hb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*(const bf16x8*)&kf[f], *(const bf16x8*)&qf[hb][f], s[hb],
                                                        0, 0, 0);
    }
    // mask keys outside the segment or in the padding rows between frames
    const int f0 = k0 / sg.npad;
    const bool full = k0 + KS <= (f0 * sg.npad + sg.n) && k0 + KS <= key_end;
    if (!full) {   // branch-free select: no divergent control flow around the scores
      const unsigned bits = key_mask(k0, g, key_end, sg.npad, sg.n);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const bool ok = (bits >> r) & 1u;
        s[0][r] = ok ? s[0][r] : -INFINITY;
        s[1][r] = ok ? s[1][r] : -INFINITY;
      }
    }
    // V^T fragments of the step, shared by both query blocks
    u32x4 vf[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int drow = t * 32 + l32;
#pragma unroll
      for (int j2 = 0; j2 < 2; ++j2) vf[t][j2] = sV[cur][drow * VCPR + ((4 * sub + 2 * j2 + g) ^ (drow & 15))];
    }
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
      u32x4 pf[2];
      float ls;
      probs(s[hb], 0.0f, pf, ls, false);
      // (re)establish the reference on the first step, or when the probabilities grew large
      if (__any(st == 0 || !(ls <= GROW))) {
        float mx = s[hb][0];
#pragma unroll
        for (int r = 1; r < 16; ++r) mx = fmaxf(mx, s[hb][r]);
        const float m_old = m_cur[hb];
        mx = pair_max(mx) + m_old;
        float m_new = st == 0 ? mx : fmaxf(m_old, mx);
        m_new = m_new > -INFINITY ? m_new : 0.0f;   // a step with every key masked keeps a finite m
        const float alpha = st == 0 ? 1.0f : fast_exp2(m_old - m_new);
        m_cur[hb] = m_new;
#pragma unroll
        for (int r = 0; r < 16; ++r) mneg[hb][r] = -m_new;
        l_run[hb] *= alpha;
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int r = 0; r < 16; ++r) o[hb][t][r] *= alpha;
        probs(s[hb], m_new - m_old, pf, ls, true);
      }
      l_run[hb] += ls;
      // O^T += V^T P^T for this block
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j2 = 0; j2 < 2; ++j2)
          o[hb][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*(const bf16x8*)&vf[t][j2], *(const bf16x8*)&pf[j2],
                                                             o[hb][t], 0, 0, 0);
    }
  };

  load_k(0);
  store_k(0);
  load_v(0);
  store_v(0);
  // The Q fragments must have landed before the loop: left pending, they make the compiler wait
  // on vmcnt before each S^T MFMA inside the loop, which (loads retire in order) also waits for
  // the next tile's K/V prefetch.  The empty asm consumes them here.
#pragma unroll
  for (int hb = 0; hb < 2; ++hb)
#pragma unroll
    for (int f = 0; f < 4; ++f) asm volatile("" : : "v"(qf[hb][f]));
  __syncthreads();
  for (int tile = 0; tile < ntiles; ++tile) {
    const int cur = tile & 1, st0 = tile * 4;
    const bool more = tile + 1 < ntiles;
    const int kt_next = (tile + 1) * KT;
    if (more) load_k(kt_next);
#pragma unroll
    for (int sub = 0; sub < 4; ++sub) {
      if (st0 + sub < nsteps) step(cur, sub, st0 + sub);
      if (sub == 1 && more) {
        store_k(cur ^ 1);
        load_v(kt_next);
      }
    }
    if (more) {
      store_v(cur ^ 1);
      __syncthreads();
    }
  }

#pragma unroll
  for (int hb = 0; hb < 2; ++hb) {
    const int qrow = qbase + hb * 32 + l32;
    const float inv = 1.0f / pair_sum(l_run[hb]);
    if (qrow < seg_len) {
      bf16* orow = O + (int64_t)(sg.base + qrow) * dim + h * HD;
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          bf16x4 v;
#pragma unroll
          for (int i = 0; i < 4; ++i) v[i] = (bf16)(o[hb][t][4 * j + i] * inv);
          *(bf16x4*)(orow + t * 32 + 8 * j + 4 * g) = v;
        }
    }
  }
}
}  // namespace v3

// attn_kernel_f8qk: attn_kernel_v3 with the scores on E4M3 operands.  Queries and keys arrive as
// E4M3 rows with one E8M0 scale per row (per token and head); S^T = K Q^T is one
// v_mfma_scale_f32_32x32x64_f8f6f4 per 32 keys and query block, the per-row scales riding in the
// MFMA's scale operands (lane (row, k-half) supplies its row's exponent), so the product is already
// in base-2 exponent units and accumulates onto -m as in v3.  K tiles are 64 bytes per key in LDS
// (chunks XOR-swizzled by (row >> 2) & 3), with their scale bytes beside them; the softmax, the
// bf16 probabilities and O^T += V^T P^T are v3's.
namespace f8qk {
using v3::HD; using v3::KT; using v3::KS; using v3::QW; using v3::QT; using v3::VCPR; using v3::GROW;
using v3::fast_exp2; using v3::pair_max; using v3::pair_sum; using v3::probs;
constexpr int K8CPR = 4;   // 16-byte chunks per E4M3 K row (64 d)

__global__ __launch_bounds__(256, 2) void attn_kernel_f8qk(const unsigned char* __restrict__ Q8,
                                                           const unsigned char* __restrict__ Qe,
                                                           const unsigned char* __restrict__ K8,
                                                           const unsigned char* __restrict__ Ke,
                                                           const bf16* __restrict__ Vt, bf16* __restrict__ O,
                                                           int64_t mpad, int heads, int dim,
                                                           const AttnSeg* __restrict__ segs,
                                                           const AttnWork* __restrict__ work, int nwork) {
  __shared__ u32x4 sK[2][KT * K8CPR];
  __shared__ unsigned sKe[2][KT / 4];
  __shared__ u32x4 sV[2][HD * VCPR];
  const int nb = nwork * heads;
  const int bid = xcd_remap(blockIdx.x, nb);
  const int h = bid / nwork, wi = bid - h * nwork;
  const AttnWork wk = work[wi];
  const AttnSeg sg = segs[wk.seg];
  const int seg_len = sg.nf * sg.npad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 5, l32 = lane & 31;
  const int qbase = wk.q0 + wave * QW;

  const int64_t hrow = (int64_t)h * mpad + sg.base;   // row of the segment's first token in [H][mpad]
  const unsigned char* Qh = Q8 + hrow * HD;
  const unsigned char* Kh = K8 + hrow * HD;
  const unsigned char* Keh = Ke + hrow;
  const bf16* Vh = Vt + (int64_t)h * HD * mpad + sg.base;

  // query block hb: lane (query l32, k-half g) holds bytes 32 g .. 32 g + 31 of its row
  i32x8 qf[2];
  int qsc[2];
#pragma unroll
  for (int hb = 0; hb < 2; ++hb) {
    const int row = qbase + hb * 32 + l32;
    const u32x4* qr = (const u32x4*)(Qh + (int64_t)row * HD);
    const u32x4 c0 = qr[2 * g], c1 = qr[2 * g + 1];
    qf[hb] = (i32x8){(int)c0.x, (int)c0.y, (int)c0.z, (int)c0.w, (int)c1.x, (int)c1.y, (int)c1.z, (int)c1.w};
    qsc[hb] = (int)Qe[hrow + row];
  }

  // K tile: thread -> row tid/2, chunks 2 (tid%2) .. +1; scale bytes: threads 0..31, 4 rows each.
  // V^T tile as in v3.  The next tile goes through registers (K first, then V).
  u32x4 rk[2];
  unsigned rks = 0u;
  u32x4 rv[4];
  auto load_k = [&](int kt) {
    const u32x4* ksrc = (const u32x4*)(Kh + (int64_t)(kt + (tid >> 1)) * HD) + 2 * (tid & 1);
    rk[0] = ksrc[0];
    rk[1] = ksrc[1];
    if (tid < KT / 4) rks = *(const unsigned*)(Keh + kt + 4 * tid);
  };
  auto load_v = [&](int kt) {
    const u32x4* vsrc = (const u32x4*)(Vh + (int64_t)(tid >> 2) * mpad + kt + (tid & 3) * 32);
#pragma unroll
    for (int i = 0; i < 4; ++i) rv[i] = vsrc[i];
  };
  auto store_k = [&](int buf) {
    const int krow = tid >> 1, ksw = (krow >> 2) & 3;
#pragma unroll
    for (int i = 0; i < 2; ++i) sK[buf][krow * K8CPR + ((2 * (tid & 1) + i) ^ ksw)] = rk[i];
    if (tid < KT / 4) sKe[buf][tid] = rks;
  };
  auto store_v = [&](int buf) {
    const int vrow = tid >> 2, sw = vrow & 15;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int ch = 4 * (tid & 3) + 2 * p;
      const u32x4 lo = {rv[2 * p].x, rv[2 * p].y, rv[2 * p + 1].x, rv[2 * p + 1].y};
      const u32x4 hi = {rv[2 * p].z, rv[2 * p].w, rv[2 * p + 1].z, rv[2 * p + 1].w};
      sV[buf][vrow * VCPR + (ch ^ sw)] = lo;
      sV[buf][vrow * VCPR + ((ch + 1) ^ sw)] = hi;
    }
  };

  f32x16 o[2][2];
#pragma unroll
  for (int hb = 0; hb < 2; ++hb)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) o[hb][t][r] = 0.0f;
  float l_run[2] = {0.0f, 0.0f};
  float m_cur[2] = {0.0f, 0.0f};
  f32x16 mneg[2];
#pragma unroll
  for (int hb = 0; hb < 2; ++hb)
#pragma unroll
    for (int r = 0; r < 16; ++r) mneg[hb][r] = 0.0f;

  const int key_end = sg.nf == 1 ? sg.n : seg_len;
  const int nsteps = (key_end + KS - 1) / KS;
  const int ntiles = (nsteps + 3) / 4;

  auto step = [&](int cur, int sub, int st) {
    const int k0 = st * KS;
    const int krow = sub * KS + l32, ksw = (krow >> 2) & 3;
    const u32x4 c0 = sK[cur][krow * K8CPR + ((2 * g) ^ ksw)];
    const u32x4 c1 = sK[cur][krow * K8CPR + ((2 * g + 1) ^ ksw)];
    const i32x8 kf = {(int)c0.x, (int)c0.y, (int)c0.z, (int)c0.w, (int)c1.x, (int)c1.y, (int)c1.z, (int)c1.w};
    const int ksc = (int)((sKe[cur][krow >> 2] >> (8 * (krow & 3))) & 255u);
    f32x16 s[2];
#pragma unroll
    for (int hb = 0; hb < 2; ++hb)
      s[hb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(kf, qf[hb], mneg[hb], 0, 0, 0, ksc, 0, qsc[hb]);
    const int f0 = k0 / sg.npad;
    const bool full = k0 + KS <= (f0 * sg.npad + sg.n) && k0 + KS <= key_end;
    if (!full) {
      const unsigned bits = key_mask(k0, g, key_end, sg.npad, sg.n);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const bool ok = (bits >> r) & 1u;
        s[0][r] = ok ? s[0][r] : -INFINITY;
        s[1][r] = ok ? s[1][r] : -INFINITY;
      }
    }
    u32x4 vf[2][2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int drow = t * 32 + l32;
#pragma unroll
      for (int j2 = 0; j2 < 2; ++j2) vf[t][j2] = sV[cur][drow * VCPR + ((4 * sub + 2 * j2 + g) ^ (drow & 15))];
    }
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
      u32x4 pf[2];
      float ls;
      probs(s[hb], 0.0f, pf, ls, false);
      if (__any(st == 0 || !(ls <= GROW))) {
        float mx = s[hb][0];
#pragma unroll
        for (int r = 1; r < 16; ++r) mx = fmaxf(mx, s[hb][r]);
        const float m_old = m_cur[hb];
        mx = pair_max(mx) + m_old;
        float m_new = st == 0 ? mx : fmaxf(m_old, mx);
        m_new = m_new > -INFINITY ? m_new : 0.0f;
        const float alpha = st == 0 ? 1.0f : fast_exp2(m_old - m_new);
        m_cur[hb] = m_new;
#pragma unroll
        for (int r = 0; r < 16; ++r) mneg[hb][r] = -m_new;
        l_run[hb] *= alpha;
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int r = 0; r < 16; ++r) o[hb][t][r] *= alpha;
        probs(s[hb], m_new - m_old, pf, ls, true);
      }
      l_run[hb] += ls;
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j2 = 0; j2 < 2; ++j2)
          o[hb][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*(const bf16x8*)&vf[t][j2], *(const bf16x8*)&pf[j2],
                                                             o[hb][t], 0, 0, 0);
    }
  };

  load_k(0);
  store_k(0);
  load_v(0);
  store_v(0);
#pragma unroll
  for (int hb = 0; hb < 2; ++hb) asm volatile("" : : "v"(qf[hb]), "v"(qsc[hb]));
  __syncthreads();
  for (int tile = 0; tile < ntiles; ++tile) {
    const int cur = tile & 1, st0 = tile * 4;
    const bool more = tile + 1 < ntiles;
    const int kt_next = (tile + 1) * KT;
    if (more) load_k(kt_next);
#pragma unroll
    for (int sub = 0; sub < 4; ++sub) {
      if (st0 + sub < nsteps) step(cur, sub, st0 + sub);
      if (sub == 1 && more) {
        store_k(cur ^ 1);
        load_v(kt_next);
      }
    }
    if (more) {
      store_v(cur ^ 1);
      __syncthreads();
    }
  }

#pragma unroll
  for (int hb = 0; hb < 2; ++hb) {
    const int qrow = qbase + hb * 32 + l32;
    const float inv = 1.0f / pair_sum(l_run[hb]);
    if (qrow < seg_len) {
      bf16* orow = O + (int64_t)(sg.base + qrow) * dim + h * HD;
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          bf16x4 v;
#pragma unroll
          for (int i = 0; i < 4; ++i) v[i] = (bf16)(o[hb][t][4 * j + i] * inv);
          *(bf16x4*)(orow + t * 32 + 8 * j + 4 * g) = v;
        }
    }
  }
}
}  // namespace f8qk

template <typename T, int HD>
static hipError_t launch(const void* q, const void* k, const void* vt, void* o, int64_t mpad,
                         int heads, int dim, const AttnSeg* segs, const AttnWork* work, int nwork,
                         hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  hipLaunchKernelGGL((attn_kernel<T, HD>), dim3(nwork * heads), dim3(256), 0, s, (const T*)q,
                     (const T*)k, (const T*)vt, (T*)o, mpad, heads, dim, segs, work, nwork);
  return hipGetLastError();
}

int attention_q_tile(Dtype dt, int hd) { return (dt == DT_BF16 && hd == 64) ? v3::QT : 128; }

float attention_q_scale(int hd) { return (float)(1.4426950408889634 / sqrt((double)hd)); }

hipError_t attention_fp8qk(const unsigned char* q8, const unsigned char* qe8, const unsigned char* k8,
                           const unsigned char* ke8, const void* vt, void* o, int64_t mpad, int heads, int dim,
                           const AttnSeg* segs, const AttnWork* work, int nwork, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  if (dim != heads * 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(f8qk::attn_kernel_f8qk, dim3(nwork * heads), dim3(256), 0, s, q8, qe8, k8, ke8, (const bf16*)vt,
                     (bf16*)o, mpad, heads, dim, segs, work, nwork);
  return hipGetLastError();
}

hipError_t attention(Dtype dt, int hd, const void* q, const void* k, const void* vt, void* o,
                     int64_t mpad, int heads, int dim, const AttnSeg* segs, const AttnWork* work,
                     int nwork, hipStream_t s) {
  if (dt == DT_BF16) {
    if (hd == 64) {
      if (nwork <= 0) return hipSuccess;
      hipLaunchKernelGGL(v3::attn_kernel_v3, dim3(nwork * heads), dim3(256), 0, s, (const bf16*)q, (const bf16*)k,
                         (const bf16*)vt, (bf16*)o, mpad, heads, dim, segs, work, nwork);
      return hipGetLastError();
    }
    if (hd == 32) return launch<bf16, 32>(q, k, vt, o, mpad, heads, dim, segs, work, nwork, s);
  } else {
    if (hd == 64) return launch<float, 64>(q, k, vt, o, mpad, heads, dim, segs, work, nwork, s);
    if (hd == 32) return launch<float, 32>(q, k, vt, o, mpad, heads, dim, segs, work, nwork, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace mf
