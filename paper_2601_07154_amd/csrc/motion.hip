// FP64 window anchoring, motion focus (Eq. 1-6) and the Gaussian focus map (Eq. 7).
//
// chain_focus: one workgroup per stream, walking that stream's windows of the batch in order
// (window k's anchor needs window k-1's world pose).  For each window: the alignment A from
// the anchor frame (the last frame the previous window emitted, shared by both windows);
// world poses T_w(t) = T_loc(t) A of the new frames; then per new frame the camera centre
// p_t = -R_t^T t_t, a_w = p_t - 2 p_{t-s} + p_{t-2s} (or v = p_t - p_{t-s} in velocity mode),
// a_c = R_t a_w and the pinhole focus.
//
// focus_maps: per emitted frame, the last N valid accelerations rotated by the frame's
// rotation and projected are the Gaussian centres; spread clip(sigma |a_w,i|); the map is
// normalised by its maximum, or by its sum over the pixel grid (MF_MAP_SUM); zero map when the
// normaliser is below 1e-30.
#include "device.h"
#include "kernels.h"

namespace mf {

MF_DEV void centre(const double* T, double* p) {   // -R^T t
  for (int i = 0; i < 3; ++i) p[i] = -(T[0 + i] * T[3] + T[4 + i] * T[7] + T[8 + i] * T[11]);
}

MF_DEV void mat4_mul(const double* A, const double* B, double* C) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += A[i * 4 + k] * B[k * 4 + j];
      C[i * 4 + j] = s;
    }
}

MF_DEV void rigid_inv(const double* T, double* Ti) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Ti[i * 4 + j] = T[j * 4 + i];
  for (int i = 0; i < 3; ++i)
    Ti[i * 4 + 3] = -(T[0 + i] * T[3] + T[4 + i] * T[7] + T[8 + i] * T[11]);
  Ti[12] = Ti[13] = Ti[14] = 0.0;
  Ti[15] = 1.0;
}

// World -> window-local alignment at the anchor frame: the full rigid A = T_loc^-1 T_w, or its
// yaw about y (atan2(A02, A22)) with the translation that keeps the anchor's centre fixed.
MF_DEV void alignment(const double* Tl, const double* Tw, int mode, double* A) {
  double Ti[16];
  rigid_inv(Tl, Ti);
  mat4_mul(Ti, Tw, A);
  if (mode == MF_ANCHOR_SE3) return;
  const double s = A[2], c = A[10];
  const double psi = (s * s + c * c >= 1e-24) ? atan2(s, c) : 0.0;
  const double cp = cos(psi), sp = sin(psi);
  double cl[3], cw[3];
  centre(Tl, cl);
  centre(Tw, cw);
  const double R[9] = {cp, 0.0, sp, 0.0, 1.0, 0.0, -sp, 0.0, cp};
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) A[i * 4 + j] = R[i * 3 + j];
    A[i * 4 + 3] = cl[i] - (R[i * 3 + 0] * cw[0] + R[i * 3 + 1] * cw[1] + R[i * 3 + 2] * cw[2]);
  }
  A[12] = A[13] = A[14] = 0.0;
  A[15] = 1.0;
}

__global__ __launch_bounds__(64) void chain_focus_kernel(const ChainGroup* __restrict__ groups,
                                                         const ChainWin* __restrict__ wins,
                                                         const StreamDev* __restrict__ streams,
                                                         const double* __restrict__ T_loc,
                                                         const float* __restrict__ pose9,
                                                         mf_focus* __restrict__ out,
                                                         double* __restrict__ win_scale) {
  __shared__ double A[16];
  __shared__ double rho;   // scale of the window's translations (MF_ANCHOR_YAW_SCALE), else 1
  const ChainGroup gr = groups[blockIdx.x];
  for (int wi = gr.first_win; wi < gr.first_win + gr.n_win; ++wi) {
    const ChainWin w = wins[wi];
    const StreamDev sd = streams[w.stream];
    FrameHist* hist = sd.hist;
    const int mask = sd.hist_mask;
    if (threadIdx.x == 0) {
      rho = 1.0;
      if (w.mode == CHAIN_ANCHOR) {
        const int64_t a = w.emit_begin - 1;
        const double* Tla = T_loc + (int64_t)(w.loc_off + (a - w.start)) * 16;
        if (sd.anchor_mode == MF_ANCHOR_YAW_SCALE) {
          // summed centre distances to the anchor over the shared frames, world over window
          double cwa[3], cla[3], num = 0.0, den = 0.0;
          centre(hist[a & mask].T, cwa);
          centre(Tla, cla);
          for (int64_t i = w.start; i < w.emit_begin; ++i) {
            double cw[3], cl[3];
            centre(hist[i & mask].T, cw);
            centre(T_loc + (int64_t)(w.loc_off + (i - w.start)) * 16, cl);
            num += sqrt((cw[0] - cwa[0]) * (cw[0] - cwa[0]) + (cw[1] - cwa[1]) * (cw[1] - cwa[1]) +
                        (cw[2] - cwa[2]) * (cw[2] - cwa[2]));
            den += sqrt((cl[0] - cla[0]) * (cl[0] - cla[0]) + (cl[1] - cla[1]) * (cl[1] - cla[1]) +
                        (cl[2] - cla[2]) * (cl[2] - cla[2]));
          }
          if (den > 1e-12) rho = num / den;
          double Ts[16];
          for (int i = 0; i < 16; ++i) Ts[i] = Tla[i];
          Ts[3] *= rho;
          Ts[7] *= rho;
          Ts[11] *= rho;
          alignment(Ts, hist[a & mask].T, MF_ANCHOR_YAW, A);
        } else {
          alignment(Tla, hist[a & mask].T, sd.anchor_mode, A);
        }
      } else {
        for (int i = 0; i < 16; ++i) A[i] = (i % 5 == 0) ? 1.0 : 0.0;
      }
      if (win_scale) win_scale[wi] = rho;
    }
    __syncthreads();
    const int64_t n_emit = w.emit_end - w.emit_begin;
    for (int64_t j = threadIdx.x; j < n_emit; j += 64) {
      const int64_t t = w.emit_begin + j;
      const double* Tl = T_loc + (int64_t)(w.loc_off + (t - w.start)) * 16;
      FrameHist& h = hist[t & mask];
      if (w.mode == CHAIN_WORLD) {
        for (int i = 0; i < 16; ++i) h.T[i] = Tl[i];
      } else {
        double Ts[16], Tw[16];
        for (int i = 0; i < 16; ++i) Ts[i] = Tl[i];
        Ts[3] *= rho;
        Ts[7] *= rho;
        Ts[11] *= rho;
        mat4_mul(Ts, A, Tw);
        for (int i = 0; i < 16; ++i) h.T[i] = Tw[i];
      }
    }
    __syncthreads();
    for (int64_t j = threadIdx.x; j < n_emit; j += 64) {
      const int64_t t = w.emit_begin + j;
      FrameHist& h = hist[t & mask];
      mf_focus& r = out[w.out_off + j];
      r.frame = t;
      r.window = w.window_id;
      for (int i = 0; i < 16; ++i) r.T_w2c[i] = h.T[i];
      for (int i = 0; i < 9; ++i)
        r.pose9[i] = w.has_pose9 ? pose9[(int64_t)(w.loc_off + (t - w.start)) * 9 + i] : 0.0f;
      r.peak_x = -1;
      r.peak_y = -1;
      double aw[3] = {0.0, 0.0, 0.0}, ac[3] = {0.0, 0.0, 0.0}, u = 0.0, v = 0.0, s = 0.0;
      int valid = 0;
      const int ds = sd.stride;
      const bool velocity = sd.focus_mode == MF_FOCUS_VELOCITY;
      if (t >= (velocity ? ds : 2 * ds)) {
        double p0[3], p1[3], p2[3] = {0.0, 0.0, 0.0};
        centre(h.T, p0);
        centre(hist[(t - ds) & mask].T, p1);
        if (!velocity) centre(hist[(t - 2 * ds) & mask].T, p2);
        for (int i = 0; i < 3; ++i) aw[i] = velocity ? p0[i] - p1[i] : (p0[i] - p1[i]) - (p1[i] - p2[i]);
        for (int i = 0; i < 3; ++i) ac[i] = h.T[i * 4 + 0] * aw[0] + h.T[i * 4 + 1] * aw[1] + h.T[i * 4 + 2] * aw[2];
        s = sqrt(aw[0] * aw[0] + aw[1] * aw[1] + aw[2] * aw[2]);
        const double np = sqrt(p0[0] * p0[0] + p0[1] * p0[1] + p0[2] * p0[2]);
        const double nac = sqrt(ac[0] * ac[0] + ac[1] * ac[1] + ac[2] * ac[2]);
        if (s > 1e-12 * fmax(1.0, np) && fabs(ac[2]) > 1e-6 * nac) {
          valid = 1;
          u = sd.cx + sd.fx * ac[0] / ac[2];
          v = sd.cy + sd.fy * ac[1] / ac[2];
        }
      }
      for (int i = 0; i < 3; ++i) {
        h.a_w[i] = aw[i];
        r.a_world[i] = aw[i];
        r.a_cam[i] = ac[i];
      }
      h.s = s;
      h.valid = valid;
      r.sigma_px = valid ? (float)fmin(fmax(sd.sigma * s, sd.sigma_min), sd.sigma_max) : 0.0f;
      r.s = s;
      r.u = u;
      r.v = v;
      r.valid = valid;
      r.t_push = 0.0;
      r.t_ready = 0.0;
      r.t_window = 0.0;
      r.t_batch = 0.0;
    }
    __syncthreads();
  }
}

hipError_t chain_focus(const ChainGroup* groups, int ngroups, const ChainWin* wins,
                       const StreamDev* streams, const double* T_loc, const float* pose9,
                       mf_focus* out, double* win_scale, hipStream_t s) {
  if (ngroups <= 0) return hipSuccess;
  hipLaunchKernelGGL(chain_focus_kernel, dim3(ngroups), dim3(64), 0, s, groups, wins, streams,
                     T_loc, pose9, out, win_scale);
  return hipGetLastError();
}

// ------------------------------------------------------------------ focus maps
constexpr int MAX_POINTS = 32;

__global__ void clear_keys_kernel(unsigned long long* keys, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) keys[i] = 0ull;
}

// Unnormalised map G of job blockIdx.y, rows blockIdx.x*8 .., plus the running max key
// (G bits << 32 | ~index) so the maximum and its smallest index come out of one atomic, and the
// workgroup's partial sum of G (summed in double in a fixed order: the normaliser is the same
// whatever else shares the launch).
__global__ __launch_bounds__(256) void map_render_kernel(const MapJob* __restrict__ jobs,
                                                         const StreamDev* __restrict__ streams,
                                                         unsigned long long* __restrict__ keys,
                                                         double* __restrict__ psum) {
  __shared__ double pu[MAX_POINTS], pv[MAX_POINTS], pk[MAX_POINTS];
  __shared__ int pok[MAX_POINTS];
  __shared__ unsigned long long red[4];
  __shared__ double sred[4];
  const MapJob job = jobs[blockIdx.y];
  const StreamDev sd = streams[job.stream];
  const int y0 = blockIdx.x * MAP_ROWS;
  if (y0 >= sd.H) {   // rows beyond this stream's frame: nothing to render, a zero partial sum
    if (threadIdx.x == 0) psum[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = 0.0;
    return;
  }
  const int tid = threadIdx.x;
  const int N = sd.n_points;
  const FrameHist* hist = sd.hist;
  if (tid < N) {
    const int64_t i = job.frame - N + 1 + tid;
    int ok = 0;
    if (i >= 0) {
      const FrameHist& hi = hist[i & sd.hist_mask];
      const double* T = hist[job.frame & sd.hist_mask].T;
      if (hi.valid) {
        double a[3];
        for (int r = 0; r < 3; ++r) a[r] = T[r * 4 + 0] * hi.a_w[0] + T[r * 4 + 1] * hi.a_w[1] + T[r * 4 + 2] * hi.a_w[2];
        const double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        if (fabs(a[2]) > 1e-6 * na) {
          ok = 1;
          pu[tid] = sd.cx + sd.fx * a[0] / a[2];
          pv[tid] = sd.cy + sd.fy * a[1] / a[2];
          const double sig = fmin(fmax(sd.sigma * hi.s, sd.sigma_min), sd.sigma_max);
          pk[tid] = 1.0 / (2.0 * sig * sig);
        }
      }
    }
    pok[tid] = ok;
  }
  __syncthreads();
  float* G = sd.maps + (int64_t)(job.frame % sd.map_cap) * sd.H * sd.W;
  unsigned long long best = 0ull;
  double part = 0.0;
  const int y1 = min(y0 + MAP_ROWS, sd.H);
  for (int idx = tid; idx < (y1 - y0) * sd.W; idx += 256) {
    const int y = y0 + idx / sd.W, x = idx - (idx / sd.W) * sd.W;
    float acc = 0.0f;
    for (int i = 0; i < N; ++i) {
      if (!pok[i]) continue;
      const double dx = x - pu[i], dy = y - pv[i];
      acc += expf(-(float)((dx * dx + dy * dy) * pk[i]));
    }
    const int64_t pix = (int64_t)y * sd.W + x;
    G[pix] = acc;
    part += (double)acc;
    const unsigned long long key = ((unsigned long long)__float_as_uint(acc) << 32) |
                                   (unsigned long long)(0xFFFFFFFFu - (unsigned)pix);
    best = key > best ? key : best;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long other = __shfl_xor(best, o, 64);
    best = other > best ? other : best;
    part += __shfl_xor(part, o, 64);
  }
  if ((tid & 63) == 0) {
    red[tid >> 6] = best;
    sred[tid >> 6] = part;
  }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 4; ++w) best = red[w] > best ? red[w] : best;
    best = red[0] > best ? red[0] : best;
    atomicMax(&keys[blockIdx.y], best);
    psum[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = ((sred[0] + sred[1]) + sred[2]) + sred[3];
  }
}

__global__ __launch_bounds__(256) void map_normalise_kernel(const MapJob* __restrict__ jobs,
                                                            const StreamDev* __restrict__ streams,
                                                            const unsigned long long* __restrict__ keys,
                                                            const double* __restrict__ psum, int nrb,
                                                            mf_focus* __restrict__ out) {
  const MapJob job = jobs[blockIdx.y];
  const StreamDev sd = streams[job.stream];
  const unsigned long long key = keys[blockIdx.y];
  const float zmax = __uint_as_float((unsigned)(key >> 32));
  float* G = sd.maps + (int64_t)(job.frame % sd.map_cap) * sd.H * sd.W;
  const int64_t npix = (int64_t)sd.H * sd.W;
  bool zero;
  if (sd.map_mode == MF_MAP_SUM) {
    // the render workgroups' partial sums, added in their row order by every workgroup alike
    double Z = 0.0;
    for (int b = 0; b < nrb; ++b) Z += psum[(int64_t)blockIdx.y * nrb + b];
    zero = !(Z >= 1e-30);
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < npix; p += (int64_t)gridDim.x * 256)
      G[p] = zero ? 0.0f : (float)((double)G[p] / Z);
  } else {
    zero = !(zmax >= 1e-30f);
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < npix; p += (int64_t)gridDim.x * 256)
      G[p] = zero ? 0.0f : G[p] / zmax;
  }
  // the argmax is the same under both normalisers (the largest G, ties to the smallest index)
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    mf_focus& r = out[job.out];
    if (zero) {
      r.peak_x = 0;
      r.peak_y = 0;
    } else {
      const unsigned pix = 0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull);
      r.peak_y = (int)(pix / (unsigned)sd.W);
      r.peak_x = (int)(pix % (unsigned)sd.W);
      r.valid |= 2;
    }
  }
}

hipError_t focus_maps(const MapJob* jobs, int njobs, int max_h, int max_w, const StreamDev* streams,
                      mf_focus* out, unsigned long long* keys, double* psum, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  const int nrb = map_row_blocks(max_h);
  hipLaunchKernelGGL(clear_keys_kernel, dim3((njobs + 255) / 256), dim3(256), 0, s, keys, njobs);
  hipLaunchKernelGGL(map_render_kernel, dim3(nrb, njobs), dim3(256), 0, s, jobs, streams, keys, psum);
  const int chunks = (int)(((int64_t)max_h * max_w + 256 * 8 - 1) / (256 * 8));
  hipLaunchKernelGGL(map_normalise_kernel, dim3(chunks, njobs), dim3(256), 0, s, jobs, streams, keys, psum, nrb,
                     out);
  return hipGetLastError();
}

}  // namespace mf
