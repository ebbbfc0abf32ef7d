// HIP kernels (gfx950) of the GFST operator pair and the sparse solver.
//
// Pipeline of L (Algorithm 1 of Section 3.1, factorisation of Section 4):
//   k_model_r2c     rows (b,j,l): stretch S, deapodise, real DFT along tau'   (steps 1-2)
//   k_nufft_interp  tiles (b, frequency tile): q-grid FFT + kernel interpolation
//                   at k_q = f' h^2 and linear azimuth weights                 (step 3)
//   k_data_c2r      traces: inverse real DFT, unstretch S^-1                   (steps 4-5)
// L^T runs the transposes in reverse order (k_data_r2c, k_nufft_spread,
// k_model_c2r).  The solver fuses the residual into the data-side kernels and
// the soft-threshold/momentum update into the model-side inverse DFT, which then
// carries the new y through steps 1-2 for the next iteration: an iteration is
// k_nufft_interp, k_residual_r2c, k_nufft_spread, k_model_c2r_update.
//
// This file: the row kernels (one model row or one trace per workgroup) and their launchers.
#include <hip/hip_runtime.h>

#include "kernel_common.hpp"

namespace aahrt {

// ------------------------------------------------------------------ model side
// Steps 1-2 of L: M'(tau') = S M, times the deapodisation of its curvature
// index, real DFT of length N, bins 0..N/2-1 stored as mhat[row][f].
template <int IP>
__global__ __launch_bounds__(kBlock) void k_model_r2c(const float* __restrict__ m,
                                                      float2* __restrict__ mhat, Tables tb, Dims dm,
                                                      FftPlan fp) {
  extern __shared__ float2 lds[];
  float2* A = lds;
  float2* B = lds + dm.nhp;
  float* row = reinterpret_cast<float*>(B);
  const size_t rid = blockIdx.x;
  const int l = (int)(rid % dm.nq);
  const float* src = m + rid * dm.ntau;
  const auto twb = row_twiddles<IP>(tb);
  for (int i = threadIdx.x; i < dm.ntau; i += kBlock) row[i] = src[i];
  __syncthreads();
  stretch_pack(A, row, tb.deapod[l], tb, dm);
  __syncthreads();
  const float2* X = row_fft<false, IP>(A, B, fp, tb, dm, twb);
  store_real_spectrum(X, mhat + rid * dm.nf, tb, dm);
}

template <int IP>
__global__ __launch_bounds__(kBlock) void k_model_c2r(const float2* __restrict__ mhat,
                                                      float* __restrict__ m, Tables tb, Dims dm,
                                                      FftPlan fp) {
  extern __shared__ float2 lds[];
  const size_t rid = blockIdx.x;
  const int l = (int)(rid % dm.nq);
  const auto twb = row_twiddles<IP>(tb);
  const float* xs = model_c2r_core<IP>(mhat, lds, lds + dm.nhp, tb, dm, fp, rid, twb);
  const float sc = tb.deapod[l] / (float)dm.nfft;
  float* dst = m + rid * dm.ntau;
  for (int i = threadIdx.x; i < dm.ntau; i += kBlock) {
    store_nt(dst + i, sc * stretch_transpose(i, tb.s_start, tb.s_w, xs));
  }
}

// Same transpose, fused with one forward-backward step on the row:
//   x_new = soft(y + gamma g, gamma lambda); y <- x_new + beta (x_new - x_old); x <- x_new
// (ISTA: y <- x_new).  l1[row] receives sum |x_new| when l1 is not null.  NEXT: the
// row then goes on through steps 1-2 of L for the next iteration, S y_new -> R2C,
// written over its own spectrum row (each row is read and written by one block).
template <int IP, bool NEXT>
__global__ __launch_bounds__(kBlock) void k_model_c2r_update(float2* __restrict__ mhat,
                                                             float* __restrict__ y,
                                                             float* __restrict__ x, Tables tb,
                                                             Dims dm, FftPlan fp,
                                                             const float* __restrict__ gam,
                                                             const float* __restrict__ lam,
                                                             float beta, int ista,
                                                             float* __restrict__ l1) {
  extern __shared__ float2 lds[];
  __shared__ float red[kBlock / 64];
  const size_t rid = blockIdx.x;
  const int l = (int)(rid % dm.nq);
  const int b = (int)(rid / ((size_t)dm.nq * dm.ntheta));
  float2* A = lds;
  float2* B = lds + dm.nhp;
  float* yr = y + rid * dm.ntau;
  float* xr = x + rid * dm.ntau;
  // the first kPrefetch samples of this thread's y and x are loaded before the
  // transform, so that their latency overlaps it
  float yv[kPrefetch], xv[kPrefetch];
#pragma unroll
  for (int k = 0; k < kPrefetch; ++k) {
    const int i = threadIdx.x + k * kBlock;
    yv[k] = i < dm.ntau ? yr[i] : 0.f;
    xv[k] = i < dm.ntau ? xr[i] : 0.f;
  }
  const auto twb = row_twiddles<IP>(tb);
  const float* xs = model_c2r_core<IP>(mhat, A, B, tb, dm, fp, rid, twb);
  // the new y row is staged after A (in place) or in the buffer not holding xs
  float* stage = IP ? reinterpret_cast<float*>(B)
                    : reinterpret_cast<float*>(xs == reinterpret_cast<const float*>(A) ? B : A);
  const float sc = tb.deapod[l] / (float)dm.nfft;
  const float g = gam[b];
  const float thr = g * lam[b];
  float s1 = 0.f;
  bool nonzero = false;
  auto step = [&](int i, float yo, float xo) {
    const float v = yo + g * (sc * stretch_transpose(i, tb.s_start, tb.s_w, xs));
    const float a = fabsf(v) - thr;
    const float xn = a > 0.f ? copysignf(a, v) : 0.f;
    const float yn = ista ? xn : xn + beta * (xn - xo);
    store_nt(yr + i, yn);
    store_nt(xr + i, xn);
    if (NEXT) stage[i] = yn;
    nonzero |= yn != 0.f;
    s1 += fabsf(xn);
  };
#pragma unroll
  for (int k = 0; k < kPrefetch; ++k) {
    const int i = threadIdx.x + k * kBlock;
    if (i < dm.ntau) step(i, yv[k], xv[k]);
  }
  for (int i = threadIdx.x + kPrefetch * kBlock; i < dm.ntau; i += kBlock) step(i, yr[i], xr[i]);
  if (l1) {
    const float t = block_sum<kBlock>(s1, red);
    if (threadIdx.x == 0) l1[rid] = t;
  }
  if (NEXT) {
    // S^T reads of xs done, new row staged; a row of y that the shrinkage left all zero has
    // a zero spectrum, written without the transform (most rows of a sparse cube are)
    if (!__syncthreads_or(nonzero ? 1 : 0)) {
      float2* dst = mhat + rid * dm.nf;
      for (int k = threadIdx.x; k < dm.nf; k += kBlock) store_nt(dst + k, make_float2(0.f, 0.f));
      return;
    }
    float2* in = IP ? A : (stage == reinterpret_cast<float*>(A) ? B : A);
    float2* other = IP ? B : reinterpret_cast<float2*>(stage);
    stretch_pack(in, stage, tb.deapod[l], tb, dm);
    __syncthreads();
    const float2* X = row_fft<false, IP>(in, other, fp, tb, dm, twb);
    store_real_spectrum(X, mhat + rid * dm.nf, tb, dm);
  }
}

// ------------------------------------------------------------------ data side
// Deconvolutive AAHRT (Section 4): with a wavelet set (WAV), the data side of L ends
// with W, the linear convolution of every trace with the wavelet taps w[0..nw-1]
// (origin wc, samples outside the trace zero), and the data side of L^T starts with
// W^T, the correlation:
//   (W v)[s] = sum_j w[j] v[s - j + wc],   (W^T r)[s] = sum_j w[j] r[s + j - wc].
__device__ __forceinline__ float wav_conv(const float* v, int s, const Tables& tb, const Dims& dm) {
  const int jlo = max(0, s + dm.wc - dm.nt + 1), jhi = min(dm.nw - 1, s + dm.wc);
  float acc = 0.f;
  for (int j = jlo; j <= jhi; ++j) acc = fmaf(tb.wav[j], v[s - j + dm.wc], acc);
  return acc;
}

__device__ __forceinline__ float wav_corr(const float* r, int s, const Tables& tb, const Dims& dm) {
  const int jlo = max(0, dm.wc - s), jhi = min(dm.nw - 1, dm.nt - 1 - s + dm.wc);
  float acc = 0.f;
  for (int j = jlo; j <= jhi; ++j) acc = fmaf(tb.wav[j], r[s + j - dm.wc], acc);
  return acc;
}

// Steps 4-5 of L: inverse real DFT of Dh[n][0..N/2-1], unstretch (then W).
template <int IP, bool WAV>
__global__ __launch_bounds__(kBlock) void k_data_c2r(const float2* __restrict__ dhat,
                                                     float* __restrict__ d, Tables tb, Dims dm,
                                                     FftPlan fp) {
  extern __shared__ float2 lds[];
  float2* A = lds;
  float2* B = lds + dm.nhp;
  const size_t n = blockIdx.x;
  const auto twb = row_twiddles<IP>(tb);
  load_packed_c2r_pairs(A, dhat + n * dm.nf, tb, dm);
  __syncthreads();
  const float2* X = row_fft<true, IP>(A, B, fp, tb, dm, twb);
  const float* xs = reinterpret_cast<const float*>(X);
  const float invN = 1.0f / (float)dm.nfft;
  float* dst = d + n * dm.nt;
  if (!WAV) {
#pragma unroll 4
    for (int s = threadIdx.x; s < dm.nt; s += kBlock) {
      const Tap t = tb.u_tap[s];
      store_nt(dst + s, invN * (t.w0 * xs[t.i0] + t.w1 * xs[t.i1]));
    }
  } else {
    float* v = reinterpret_cast<float*>(X == A ? B : A);  // IP: the staging area after A
    for (int s = threadIdx.x; s < dm.nt; s += kBlock) {
      const Tap t = tb.u_tap[s];
      v[s] = invN * (t.w0 * xs[t.i0] + t.w1 * xs[t.i1]);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < dm.nt; s += kBlock) store_nt(dst + s, wav_conv(v, s, tb, dm));
  }
}

// (W^T, then) transpose of step 5, then the forward real DFT (the data side of L^T).
// tr_bound[n] = max_f (|Re Dh[n,f]| + |Im Dh[n,f]|) (the spreading scale bound).
template <int IP, bool WAV>
__global__ __launch_bounds__(kBlock) void k_data_r2c(const float* __restrict__ d,
                                                     float2* __restrict__ dhat,
                                                     float* __restrict__ tr_bound, Tables tb, Dims dm,
                                                     FftPlan fp) {
  extern __shared__ float2 lds[];
  __shared__ float red[kBlock / 64];
  float2* A = lds;
  float2* B = lds + dm.nhp;
  float* g = reinterpret_cast<float*>(B);
  const size_t n = blockIdx.x;
  const float* src = d + n * dm.nt;
  const auto twb = row_twiddles<IP>(tb);
  if (!WAV) {
    for (int s = threadIdx.x; s < dm.nt; s += kBlock) g[s] = src[s];
  } else {
    float* r = reinterpret_cast<float*>(A);
    for (int s = threadIdx.x; s < dm.nt; s += kBlock) r[s] = src[s];
    __syncthreads();
    for (int s = threadIdx.x; s < dm.nt; s += kBlock) g[s] = wav_corr(r, s, tb, dm);
  }
  __syncthreads();
  pack_transpose(A, g, tb, dm.nts, dm.nh);
  __syncthreads();
  const float2* X = row_fft<false, IP>(A, B, fp, tb, dm, twb);
  const float mx = block_max<kBlock>(store_real_spectrum(X, dhat + n * dm.nf, tb, dm), red);
  if (threadIdx.x == 0) tr_bound[n] = mx;
}

// Solver data side, in place on dhat[n]: r = d_obs - (W) S^-1 F1^-1 Dh (steps 4-5),
// then the data side of L^T applied to r.  rss[n] = sum r^2 when not null.
template <int IP, bool WAV>
__global__ __launch_bounds__(kBlock) void k_residual_r2c(float2* __restrict__ dhat,
                                                         const float* __restrict__ dobs,
                                                         float* __restrict__ rss,
                                                         float* __restrict__ tr_bound, Tables tb,
                                                         Dims dm, FftPlan fp) {
  extern __shared__ float2 lds[];
  __shared__ float red[kBlock / 64];
  float2* A = lds;
  float2* B = lds + dm.nhp;
  const size_t n = blockIdx.x;
  const float* ob = dobs + n * dm.nt;
  float ov[kPrefetch];  // observed samples loaded before the transform
#pragma unroll
  for (int k = 0; k < kPrefetch; ++k) {
    const int s = threadIdx.x + k * kBlock;
    ov[k] = (!WAV && s < dm.nt) ? ob[s] : 0.f;
  }
  const auto twb = row_twiddles<IP>(tb);
  load_packed_c2r(A, dhat + n * dm.nf, tb, dm);
  __syncthreads();
  float2* X = row_fft<true, IP>(A, B, fp, tb, dm, twb);
  float2* Y = (X == A) ? B : A;      // IP: the staging area after A
  const float* xs = reinterpret_cast<const float*>(X);
  float* g = reinterpret_cast<float*>(Y);
  const float invN = 1.0f / (float)dm.nfft;
  float ss = 0.f;
  if (!WAV) {
    auto res = [&](int s, float o) {
      const Tap t = tb.u_tap[s];
      const float v = invN * (t.w0 * xs[t.i0] + t.w1 * xs[t.i1]);
      const float r = o - v;
      g[s] = r;
      ss += r * r;
    };
#pragma unroll
    for (int k = 0; k < kPrefetch; ++k) {
      const int s = threadIdx.x + k * kBlock;
      if (s < dm.nt) res(s, ov[k]);
    }
    for (int s = threadIdx.x + kPrefetch * kBlock; s < dm.nt; s += kBlock) res(s, ob[s]);
  } else {
    // v = S^-1 F1^-1 Dh into g; r = d_obs - W v into X (its spectrum is consumed); g = W^T r
    for (int s = threadIdx.x; s < dm.nt; s += kBlock) {
      const Tap t = tb.u_tap[s];
      g[s] = invN * (t.w0 * xs[t.i0] + t.w1 * xs[t.i1]);
    }
    __syncthreads();
    float* rr = reinterpret_cast<float*>(X);
    for (int s = threadIdx.x; s < dm.nt; s += kBlock) {
      const float r = ob[s] - wav_conv(g, s, tb, dm);
      rr[s] = r;
      ss += r * r;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < dm.nt; s += kBlock) g[s] = wav_corr(rr, s, tb, dm);
  }
  __syncthreads();
  pack_transpose(X, g, tb, dm.nts, dm.nh);
  __syncthreads();
  const float2* Z = row_fft<false, IP>(X, Y, fp, tb, dm, twb);
  const float mx = block_max<kBlock>(store_real_spectrum(Z, dhat + n * dm.nf, tb, dm), red);
  if (threadIdx.x == 0) tr_bound[n] = mx;
  if (rss) {
    const float t = block_sum<kBlock>(ss, red);
    if (threadIdx.x == 0) rss[n] = t;
  }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_model_r2c(const Plan& p, const float* m, float2* mhat, hipStream_t s) {
  const Dims& dm = p.dm;
  return launch_row(AAHRT_ROWK(k_model_r2c), dm, dm.ntau, model_rows(dm), s, m, mhat, p.tb, dm,
                    p.fft_half);
}

hipError_t launch_rows_r2c(const Dims& dm, const Tables& tb, const FftPlan& fp, const float* in, float2* out,
                           unsigned nrows, hipStream_t s) {
  return launch_row(AAHRT_ROWK(k_model_r2c), dm, dm.ntau, nrows, s, in, out, tb, dm, fp);
}

hipError_t launch_model_c2r(const Plan& p, const float2* mhat, float* m, hipStream_t s) {
  const Dims& dm = p.dm;
  return launch_row(AAHRT_ROWK(k_model_c2r), dm, 0, model_rows(dm), s, mhat, m, p.tb, dm,
                    p.fft_half);
}

hipError_t launch_model_c2r_update(const Plan& p, float2* mhat, float* y, float* x, const float* gam,
                                   const float* lam, float beta, int ista, float* l1, bool next,
                                   hipStream_t s) {
  const Dims& dm = p.dm;
  if (next)
    return launch_row(AAHRT_ROWK(k_model_c2r_update, true), dm, dm.ntau,
                      model_rows(dm), s, mhat, y, x, p.tb, dm, p.fft_half, gam, lam, beta, ista, l1);
  return launch_row(AAHRT_ROWK(k_model_c2r_update, false), dm, 0, model_rows(dm), s,
                    mhat, y, x, p.tb, dm, p.fft_half, gam, lam, beta, ista, l1);
}

hipError_t launch_data_c2r(const Plan& p, const float2* dhat, float* d, hipStream_t s) {
  const Dims& dm = p.dm;
  if (dm.nw > 0)
    return launch_row(AAHRT_ROWK(k_data_c2r, true), dm, dm.nt, (unsigned)dm.ntr, s, dhat, d,
                      p.tb, dm, p.fft_half);
  return launch_row(AAHRT_ROWK(k_data_c2r, false), dm, 0, (unsigned)dm.ntr, s, dhat, d, p.tb,
                    dm, p.fft_half);
}

hipError_t launch_data_r2c(const Plan& p, const float* d, float2* dhat, float* tr_bound, hipStream_t s) {
  const Dims& dm = p.dm;
  if (dm.nw > 0)
    return launch_row(AAHRT_ROWK(k_data_r2c, true), dm, dm.nt, (unsigned)dm.ntr, s, d, dhat,
                      tr_bound, p.tb, dm, p.fft_half);
  return launch_row(AAHRT_ROWK(k_data_r2c, false), dm, dm.nt, (unsigned)dm.ntr, s, d, dhat,
                    tr_bound, p.tb, dm, p.fft_half);
}

hipError_t launch_residual_r2c(const Plan& p, float2* dhat, const float* dobs, float* rss,
                               hipStream_t s) {
  const Dims& dm = p.dm;
  if (dm.nw > 0)
    return launch_row(AAHRT_ROWK(k_residual_r2c, true), dm, dm.nt, (unsigned)dm.ntr, s,
                      dhat, dobs, rss, p.tr_bound, p.tb, dm, p.fft_half);
  return launch_row(AAHRT_ROWK(k_residual_r2c, false), dm, dm.nt, (unsigned)dm.ntr, s,
                    dhat, dobs, rss, p.tr_bound, p.tb, dm, p.fft_half);
}

}  // namespace aahrt
