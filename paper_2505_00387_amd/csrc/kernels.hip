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
#include <hip/hip_runtime.h>

#include "aahrt_internal.hpp"
#include "fft_lds.hpp"

namespace aahrt {

// ------------------------------------------------------------------ helpers
template <int NT>
__device__ __forceinline__ float block_sum(float v, float* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  float s = 0.f;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NT / 64; ++i) s += red[i];
  }
  return s;  // valid on thread 0
}

template <int NT>
__device__ __forceinline__ float block_max(float v, float* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  float s = 0.f;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NT / 64; ++i) s = fmaxf(s, red[i]);
  }
  return s;
}

// Spectrum of a real sequence of length N from the FFT Z of the packed
// complex sequence z[p] = x[2p] + i x[2p+1] (length N/2), bins k < N/2.
// Returns this thread's max over its bins of |Re| + |Im|.
__device__ __forceinline__ float store_real_spectrum(const float2* buf, float2* __restrict__ dst,
                                                     const Tables& tb, const Dims& dm) {
  float mx = 0.f;
#pragma unroll 4
  for (int k = threadIdx.x; k < dm.nf; k += kBlock) {
    const float2 z = buf[k];
    float2 zc = buf[k == 0 ? 0 : dm.nh - k];
    zc.y = -zc.y;
    const float2 ze = make_float2(0.5f * (z.x + zc.x), 0.5f * (z.y + zc.y));
    const float2 dz = make_float2(0.5f * (z.x - zc.x), 0.5f * (z.y - zc.y));
    const float2 zo = make_float2(dz.y, -dz.x);  // dz / i
    const float2 X = cadd(ze, cmul(tb.tw_real[k], zo));
    dst[k] = X;
    mx = fmaxf(mx, fabsf(X.x) + fabsf(X.y));
  }
  return mx;
}

// Packed spectrum Z for the inverse real DFT of X[0..N/2-1] (Im X[0] and the
// Nyquist bin taken as zero): Z[k] = (X[k] + conj X[N/2-k]) + i e^{2 pi i k/N}(X[k] - conj X[N/2-k]).
__device__ __forceinline__ void load_packed_c2r(float2* buf, const float2* __restrict__ src,
                                                const Tables& tb, const Dims& dm) {
#pragma unroll 4
  for (int k = threadIdx.x; k < dm.nh; k += kBlock) {
    float2 X = src[k];
    float2 Xm = make_float2(0.f, 0.f);
    if (k == 0) X.y = 0.f;
    else Xm = src[dm.nh - k];
    const float2 Xc = make_float2(Xm.x, -Xm.y);
    const float2 Xe = cadd(X, Xc);
    float2 t = tb.tw_real[k];
    t.y = -t.y;
    const float2 Xo = cmul(csub(X, Xc), t);
    buf[k] = make_float2(Xe.x - Xo.y, Xe.y + Xo.x);
  }
}

// Transpose of a monotone two-tap interpolator at output i (inputs r with lower tap
// lo(r), non-decreasing in r, weights w[r] = (w0, w1) on lo and lo + 1):
//   y[i] = sum_{lo(r) = i-1} w1[r] x[r] + sum_{lo(r) = i} w0[r] x[r],
// where start[i] is the first input whose lower tap is >= i, so both sums run over
// one contiguous range of inputs.  Loads are issued four at a time.
__device__ __forceinline__ float lerp_transpose(int i, const int* __restrict__ start, const float2* __restrict__ w,
                                                const float* x) {
  const int b = start[i], c = start[i + 1];
  const int a = i > 0 ? start[i - 1] : b;
  float acc = 0.f;
  for (int r0 = a; r0 < c; r0 += 4) {
    float2 wv[4];
    float xv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = r0 + k;
      wv[k] = r < c ? w[r] : make_float2(0.f, 0.f);
      xv[k] = r < c ? x[r] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) acc = fmaf(r0 + k < b ? wv[k].y : wv[k].x, xv[k], acc);
  }
  return acc;
}

// Pack x[r] = (U^T g)[r] (r < nts, zero beyond) as z[p] = x[2p] + i x[2p+1], i.e. x
// written in order over the floats of buf.  One output per thread and pass: the
// first outputs gather the most inputs (t' = t^2 is flat near t = 0).
__device__ __forceinline__ void pack_transpose(float2* buf, const float* g, const Tables& tb, int nts, int nh) {
  float* xf = reinterpret_cast<float*>(buf);
  for (int r = threadIdx.x; r < 2 * nh; r += kBlock)
    xf[r] = r < nts ? lerp_transpose(r, tb.u_start, tb.u_w, g) : 0.f;
}

// ------------------------------------------------------------------ model side
// Row kernels transform one row (or trace) per workgroup in LDS.  IP = true:
// one buffer of N/2 (padded) complex values, transformed in place, plus a
// staging area after it for a real input row; IP = false (long rows whose FFT
// passes have more butterflies than threads): two ping-pong buffers, the staged
// input row aliasing the second one before the first pass.
template <bool INV, int IP>
__device__ __forceinline__ float2* row_fft(float2* A, float2* B, const FftPlan& fp, const Tables& tb,
                                           const Dims& dm) {
  if constexpr (IP == 1) {
    fft_lds_ip<INV, kBlock>(A, fp, 1, 0, tb.tw_half);
    return A;
  } else if constexpr (IP == 2) {
    fft_lds_ipk<INV, kBlock>(A, fp, tb.tw_half);
    return A;
  }
  return fft_lds<INV, kBlock>(A, B, fp, 1, dm.nh, tb.tw_half);
}

// Stretch S of a staged model row, times sc, packed as z[p] = M'[2p] + i M'[2p+1]
// (zero beyond nt').
__device__ __forceinline__ void stretch_pack(float2* A, const float* row, float sc, const Tables& tb,
                                             const Dims& dm) {
#pragma unroll 4
  for (int p = threadIdx.x; p < dm.nh; p += kBlock) {
    const int r0 = 2 * p, r1 = 2 * p + 1;
    float a = 0.f, b = 0.f;
    if (r0 < dm.nts) {
      const Tap t = tb.s_tap[r0];
      a = sc * (t.w0 * row[t.i0] + t.w1 * row[t.i1]);
    }
    if (r1 < dm.nts) {
      const Tap t = tb.s_tap[r1];
      b = sc * (t.w0 * row[t.i0] + t.w1 * row[t.i1]);
    }
    A[p] = make_float2(a, b);
  }
}

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
  for (int i = threadIdx.x; i < dm.ntau; i += kBlock) row[i] = src[i];
  __syncthreads();
  stretch_pack(A, row, tb.deapod[l], tb, dm);
  __syncthreads();
  const float2* X = row_fft<false, IP>(A, B, fp, tb, dm);
  store_real_spectrum(X, mhat + rid * dm.nf, tb, dm);
}

// Transpose of steps 1-2: inverse real DFT (1/N, doubled positive bins), first
// nt' samples, times the deapodisation, then S^T.
template <int IP>
__device__ __forceinline__ const float* model_c2r_core(const float2* mhat, float2* A,
                                                       float2* B, const Tables& tb, const Dims& dm,
                                                       const FftPlan& fp, size_t rid) {
  load_packed_c2r(A, mhat + rid * dm.nf, tb, dm);
  __syncthreads();
  return reinterpret_cast<const float*>(row_fft<true, IP>(A, B, fp, tb, dm));
}

template <int IP>
__global__ __launch_bounds__(kBlock) void k_model_c2r(const float2* __restrict__ mhat,
                                                      float* __restrict__ m, Tables tb, Dims dm,
                                                      FftPlan fp) {
  extern __shared__ float2 lds[];
  const size_t rid = blockIdx.x;
  const int l = (int)(rid % dm.nq);
  const float* xs = model_c2r_core<IP>(mhat, lds, lds + dm.nhp, tb, dm, fp, rid);
  const float sc = tb.deapod[l] / (float)dm.nfft;
  float* dst = m + rid * dm.ntau;
  for (int i = threadIdx.x; i < dm.ntau; i += kBlock) {
    dst[i] = sc * lerp_transpose(i, tb.s_start, tb.s_w, xs);
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
  const float* xs = model_c2r_core<IP>(mhat, A, B, tb, dm, fp, rid);
  // the new y row is staged after A (in place) or in the buffer not holding xs
  float* stage = IP ? reinterpret_cast<float*>(B)
                    : reinterpret_cast<float*>(xs == reinterpret_cast<const float*>(A) ? B : A);
  const float sc = tb.deapod[l] / (float)dm.nfft;
  const float g = gam[b];
  const float thr = g * lam[b];
  float s1 = 0.f;
  auto step = [&](int i, float yo, float xo) {
    const float v = yo + g * (sc * lerp_transpose(i, tb.s_start, tb.s_w, xs));
    const float a = fabsf(v) - thr;
    const float xn = a > 0.f ? copysignf(a, v) : 0.f;
    const float yn = ista ? xn : xn + beta * (xn - xo);
    yr[i] = yn;
    xr[i] = xn;
    if (NEXT) stage[i] = yn;
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
    __syncthreads();  // S^T reads of xs done, new row staged
    float2* in = IP ? A : (stage == reinterpret_cast<float*>(A) ? B : A);
    float2* other = IP ? B : reinterpret_cast<float2*>(stage);
    stretch_pack(in, stage, tb.deapod[l], tb, dm);
    __syncthreads();
    const float2* X = row_fft<false, IP>(in, other, fp, tb, dm);
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
  load_packed_c2r(A, dhat + n * dm.nf, tb, dm);
  __syncthreads();
  const float2* X = row_fft<true, IP>(A, B, fp, tb, dm);
  const float* xs = reinterpret_cast<const float*>(X);
  const float invN = 1.0f / (float)dm.nfft;
  float* dst = d + n * dm.nt;
  if (!WAV) {
#pragma unroll 4
    for (int s = threadIdx.x; s < dm.nt; s += kBlock) {
      const Tap t = tb.u_tap[s];
      dst[s] = invN * (t.w0 * xs[t.i0] + t.w1 * xs[t.i1]);
    }
  } else {
    float* v = reinterpret_cast<float*>(X == A ? B : A);  // IP: the staging area after A
    for (int s = threadIdx.x; s < dm.nt; s += kBlock) {
      const Tap t = tb.u_tap[s];
      v[s] = invN * (t.w0 * xs[t.i0] + t.w1 * xs[t.i1]);
    }
    __syncthreads();
    for (int s = threadIdx.x; s < dm.nt; s += kBlock) dst[s] = wav_conv(v, s, tb, dm);
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
  const float2* X = row_fft<false, IP>(A, B, fp, tb, dm);
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
  load_packed_c2r(A, dhat + n * dm.nf, tb, dm);
  __syncthreads();
  float2* X = row_fft<true, IP>(A, B, fp, tb, dm);
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
  const float2* Z = row_fft<false, IP>(X, Y, fp, tb, dm);
  const float mx = block_max<kBlock>(store_real_spectrum(Z, dhat + n * dm.nf, tb, dm), red);
  if (threadIdx.x == 0) tr_bound[n] = mx;
  if (rss) {
    const float t = block_sum<kBlock>(ss, red);
    if (threadIdx.x == 0) rss[n] = t;
  }
}

// ------------------------------------------------------------------ GFST stage
// Each workgroup owns one gather b and a tile of ft consecutive frequencies.
// The oversampled q-grid of one azimuth slice for all ft frequencies lives in
// LDS as ft rows of ldr complex cells: mg grid cells, then w-1 ghost cells that
// repeat the first w-1 cells (periodic extension, so a kernel footprint never
// wraps), then padding to an odd row length (rows of one access fall in
// distinct LDS banks).  Slices are visited in azimuth order; traces are grouped
// by their lower azimuth bin j_n, so bin j needs slices j and j+1 (mod ntheta).
// The (trace, frequency) items of a bin run with the frequency fastest across
// threads; the per-trace tables are read straight from memory (the lanes of one
// trace share the cache line), so a bin needs no barrier of its own.
//
// Phases use 0.64 fixed point: frac(f b) for an integer frequency index f is the
// wrapped 64-bit product, of which only the top 32 bits are formed
// (f * b_hi + umulhi(f, b_lo)); the grid position u = mg * frac(f b) keeps 32
// fractional bits before its conversion to FP32.

struct KernelPoint {
  int base;   // first grid cell of the footprint, in [0, mg)
  float z0;   // 2 d0 / w, d0 = distance from the point to the first cell
};

template <int W>
__device__ __forceinline__ KernelPoint kernel_point(unsigned f, unsigned long long bfix, int mg) {
  const unsigned t32 = f * (unsigned)(bfix >> 32) + __umulhi(f, (unsigned)bfix);
  const unsigned long long u = (unsigned long long)t32 * (unsigned)mg;
  const int ui = (int)(u >> 32);
  const float uf = (float)(unsigned)u * 2.3283064365386963e-10f;
  int off;
  if (W % 2 == 0) off = -W / 2;
  else off = uf < 0.5f ? -(W + 1) / 2 : -(W - 1) / 2;
  KernelPoint kp;
  int base = ui + off + 1;
  kp.base = base < 0 ? base + mg : base;
  kp.z0 = (uf - (float)(off + 1)) * (2.0f / (float)W);
  return kp;
}

// exp(-2 pi i frac(f a)) (SIGN = -1) or its conjugate (SIGN = +1), with the
// hardware sine and cosine, whose argument is in revolutions.
template <int SIGN>
__device__ __forceinline__ float2 pre_phase(unsigned f, unsigned long long afix) {
  const unsigned p32 = f * (unsigned)(afix >> 32) + __umulhi(f, (unsigned)afix);
  float rev = (float)(p32 >> 8) * 5.9604644775390625e-08f;  // 24 bits, 2^-24
  if (rev >= 0.5f) rev -= 1.0f;
  return make_float2(__builtin_amdgcn_cosf(rev), (float)SIGN * __builtin_amdgcn_sinf(rev));
}

// Exponential-of-semicircle kernel at normalised distance z = 2 d / w:
// exp(beta (sqrt(1 - z^2) - 1)) = exp2(cbeta sqrt(1 - z^2) - cbeta), cbeta = beta log2(e).
__device__ __forceinline__ float es_tap(float z, float cbeta) {
  const float q = fmaxf(fmaf(-z, z, 1.0f), 0.0f);
  return __builtin_amdgcn_exp2f(fmaf(cbeta, __builtin_amdgcn_sqrtf(q), -cbeta));
}

// Interpolation weight of a tap at normalised distance z: the exponential of
// semicircle for W >= 3; W = 2 is the linear interpolation of the paper's step 3
// (Section 3.4), weight 1 - |z| between the two neighbouring grid cells.
template <int W>
__device__ __forceinline__ float grid_tap(float z, float cbeta) {
  if (W == 2) return fmaxf(1.0f - fabsf(z), 0.0f);
  return es_tap(z, cbeta);
}

// Logical tile index with consecutive tiles (same gather) on one XCD: the
// hardware deals workgroup i to XCD i mod 8.
__device__ __forceinline__ int xcd_tile(int id, int n) {
  const int q = n >> 3, r = n & 7;
  const int x = id & 7, loc = id >> 3;
  return x < r ? x * (q + 1) + loc : r * (q + 1) + (x - r) * q + loc;
}

// q-coefficients of one slice for the tile, c[l][fl] = Mh[b][s][l][f0 + fl], kCoefRegs
// per thread.
constexpr int kCoefRegs = 4;
static_assert(kCoefRegs * kBlockG >= kPrefetchCells, "coefficient prefetch capacity");

__device__ __forceinline__ void load_coefs(float2* cr, const float2* __restrict__ mhat_slice, int f0,
                                           const Dims& dm, int ftl) {
#pragma unroll
  for (int k = 0; k < kCoefRegs; ++k) {
    const int it = threadIdx.x + k * kBlockG;
    cr[k] = make_float2(0.f, 0.f);
    if (it < dm.nq * dm.ft) {
      const int f = f0 + (it & (dm.ft - 1));
      if (f < dm.nf) cr[k] = mhat_slice[(size_t)(it >> ftl) * dm.nf + f];
    }
  }
}

// Forward q-grid of one slice from its coefficients: g[f][m] = sum_k c_k exp(-2 pi i k m/mg),
// transformed in place, then the ghost cells g[f][mg + t] = g[f][t], t < W - 1.
template <int W>
__device__ __forceinline__ void build_grid(float2* G, const float2* cr, const float2* twl, const Dims& dm,
                                           const FftPlan& fpg, int ftl) {
  const int ldr = dm.ldr;
  const int ft = dm.ft;
  const int nz = dm.mg - dm.nq;  // zero-padded cells [nq - qhalf, mg - qhalf) of each row
  for (int i = threadIdx.x; i < ft * nz; i += kBlockG) {
    const int fl = i / nz;
    G[fl * ldr + dm.nq - dm.qhalf + (i - fl * nz)] = make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int k = 0; k < kCoefRegs; ++k) {
    const int it = threadIdx.x + k * kBlockG;
    if (it < dm.nq * ft) {
      const int l = it >> ftl;
      int m = l - dm.qhalf;
      if (m < 0) m += dm.mg;
      G[(it & (ft - 1)) * ldr + m] = cr[k];
    }
  }
  __syncthreads();
  fft_lds_ip<false, kBlockG>(G, fpg, ft, ldr, twl);
  for (int i = threadIdx.x; i < ft * (W - 1); i += kBlockG) {
    const int fl = i / (W - 1), t = i - fl * (W - 1);
    G[fl * ldr + dm.mg + t] = G[fl * ldr + t];
  }
  __syncthreads();
}

// Storage of the forward q-grid.  GD = AAHRT_GRID_F32: the FP32 grid itself;
// GD = AAHRT_GRID_F16 / AAHRT_GRID_BF16: one 32-bit cell holds (Re, Im) as two
// 16-bit floats (rounded to nearest even), built by an FP32 transform and read
// back into FP32 for the interpolation, which accumulates in FP32.
template <int GD>
struct GridCell {
  using T = unsigned;
};
template <>
struct GridCell<AAHRT_GRID_F32> {
  using T = float2;
};

template <int GD>
__device__ __forceinline__ typename GridCell<GD>::T enc_cell(float2 v) {
  if constexpr (GD == AAHRT_GRID_F32) {
    return v;
  } else if constexpr (GD == AAHRT_GRID_F16) {
    const _Float16 a = (_Float16)v.x, b = (_Float16)v.y;
    return (unsigned)__builtin_bit_cast(unsigned short, a) | ((unsigned)__builtin_bit_cast(unsigned short, b) << 16);
  } else {
    unsigned a = __float_as_uint(v.x), b = __float_as_uint(v.y);
    a = (a + 0x7FFFu + ((a >> 16) & 1u)) >> 16;
    b = (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
    return a | (b << 16);
  }
}

template <int GD>
__device__ __forceinline__ float2 dec_cell(typename GridCell<GD>::T c) {
  if constexpr (GD == AAHRT_GRID_F32) {
    return c;
  } else if constexpr (GD == AAHRT_GRID_F16) {
    const _Float16 a = __builtin_bit_cast(_Float16, (unsigned short)(c & 0xFFFFu));
    const _Float16 b = __builtin_bit_cast(_Float16, (unsigned short)(c >> 16));
    return make_float2((float)a, (float)b);
  } else {
    return make_float2(__uint_as_float(c << 16), __uint_as_float(c & 0xFFFF0000u));
  }
}

// Forward GFST map (type-2 nonuniform FFT in q plus the azimuth weights) for one
// gather and a tile of ft frequencies.  Two slots hold the q-grids of slices j
// and j+1 while bin j is interpolated; slice j+2 (mod ntheta, so slice 0 is
// built again for the last bin) then replaces slice j.
// Registers are capped for six waves per SIMD: with two 32-frequency slots (46 KB of LDS)
// three workgroups then fit a CU instead of two (measured 8-11% faster, same results).
template <int W, int GD>
__global__ __launch_bounds__(kBlockG) __attribute__((amdgpu_waves_per_eu(6))) void k_nufft_interp(const float2* __restrict__ mhat,
                                                          float2* __restrict__ dhat, Tables tb,
                                                          Dims dm, FftPlan fpg, int ftl) {
  using Cell = typename GridCell<GD>::T;
  extern __shared__ float2 lds[];
  const int ldr = dm.ldr;
  const int ft = dm.ft;
  const int slot_sz = ft * ldr;
  Cell* slots = reinterpret_cast<Cell*>(lds);
  float2* work = lds + interp_slots_f2(ft, ldr, dm.ntheta, GD);  // 16-bit grids: FP32 transform buffer
  float2* twl = GD == AAHRT_GRID_F32 ? work : work + slot_sz;  // q-grid twiddles
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int b = tile / dm.nftile;
  const int f0 = (tile - b * dm.nftile) * ft;
  const int* bp = tb.bin_ptr + (size_t)b * (dm.ntheta + 1);
  const size_t slice_stride = (size_t)dm.nq * dm.nf;
  const float2* mb = mhat + (size_t)b * dm.ntheta * slice_stride;
  if (bp[dm.ntheta] == bp[0]) return;  // empty gather: nothing to write
  for (int i = threadIdx.x; i < dm.mg; i += kBlockG) twl[i] = tb.tw_grid[i];
  const int nt = dm.ntheta;

  // step -2 and -1 build slices 0 and 1; step j >= 0 interpolates bin j, then builds
  // slice (j + 2) mod ntheta into the slot of slice j (while j + 2 <= ntheta).  The
  // coefficients are loaded just before the build (holding them across the
  // interpolation costs registers, hence resident waves, for little overlap).
  float2 cr[kCoefRegs];
  for (int j = -2; j < nt; ++j) {
    const int sb = j + 2;
    const bool build = sb < 2 ? sb < nt : sb <= nt;
    const int sbm = sb >= nt ? sb - nt : sb;
    if (j >= 0) {
      const Cell* G0 = slots + (nt == 1 ? 0 : (j & 1)) * slot_sz;
      const Cell* G1 = slots + (nt == 1 ? 0 : ((j + 1) & 1)) * slot_sz;
      const int c0 = bp[j];
      const int cnt = bp[j + 1] - c0;
      for (int it = threadIdx.x; it < cnt * ft; it += kBlockG) {
        const int n = c0 + (it >> ftl);
        const int fl = it & (ft - 1);
        const unsigned f = (unsigned)(f0 + fl);
        if (f >= (unsigned)dm.nf) continue;
        const KernelPoint kp = kernel_point<W>(f, tb.tr_b[n], dm.mg);
        const Cell* g0 = G0 + fl * ldr + kp.base;
        const Cell* g1 = G1 + fl * ldr + kp.base;
        float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
#pragma unroll
        for (int t = 0; t < W; ++t) {
          const float ph = grid_tap<W>(fmaf((float)t, -2.0f / (float)W, kp.z0), dm.cbeta);
          const float2 v0 = dec_cell<GD>(g0[t]), v1 = dec_cell<GD>(g1[t]);
          a0.x = fmaf(ph, v0.x, a0.x);
          a0.y = fmaf(ph, v0.y, a0.y);
          a1.x = fmaf(ph, v1.x, a1.x);
          a1.y = fmaf(ph, v1.y, a1.y);
        }
        const float alpha = tb.tr_alpha[n];
        const float2 v = make_float2(fmaf(alpha, a1.x - a0.x, a0.x), fmaf(alpha, a1.y - a0.y, a0.y));
        dhat[(size_t)tb.tr_row[n] * dm.nf + f] = cmul(v, pre_phase<-1>(f, tb.tr_a[n]));
      }
      __syncthreads();
    }
    if (build) {
      load_coefs(cr, mb + (size_t)sbm * slice_stride, f0, dm, ftl);
      if (sb >= 2 && nt == 2 && sbm == 0) {
        // two slices: slice 0 is still in its slot
      } else if constexpr (GD == AAHRT_GRID_F32) {
        build_grid<W>(slots + (sb & 1) * slot_sz, cr, twl, dm, fpg, ftl);
      } else {
        build_grid<W>(work, cr, twl, dm, fpg, ftl);
        Cell* G = slots + (sb & 1) * slot_sz;
        for (int i = threadIdx.x; i < slot_sz; i += kBlockG) G[i] = enc_cell<GD>(work[i]);
        __syncthreads();
      }
    }
  }
}

// Type-1 spreading accumulates in LDS in fixed point: a complex contribution c
// is added as one 64-bit integer round(S Re c) + 2^32 round(S Im c).  Integer
// addition is exact and order independent (deterministic results), and the
// two 32-bit fields can be read back exactly while each partial sum stays
// below 2^31 in magnitude, which the scale guarantees.  Each azimuth slice s
// has its own scale S_s = 0.99 (2^31 - 1)/B_s, where B_s sums, over the only
// traces that reach the slice (bin s with weight 1 - alpha, bin s-1 mod ntheta
// with weight alpha), the weight times max_f (|Re Dh| + |Im Dh|) of the trace:
// an upper bound of every cell sum of the slice, the kernel being <= 1.
__device__ __forceinline__ unsigned long long pack_fix(float x, float y) {
  const int a = __float2int_rn(x), b = __float2int_rn(y);
  return (unsigned long long)(long long)a + ((unsigned long long)(unsigned)b << 32);
}

__device__ __forceinline__ float2 unpack_fix(unsigned long long v, float inv_s) {
  const int lo = (int)(unsigned)v;
  const int hi = (int)(unsigned)((v - (unsigned long long)(long long)lo) >> 32);
  return make_float2((float)lo * inv_s, (float)hi * inv_s);
}

// Scale S_s of every (gather, slice): one block per pair, fixed summation order.
__global__ __launch_bounds__(kBlock) void k_slice_scales(const float* __restrict__ tr_bound, Tables tb,
                                                         int ntheta, float* __restrict__ scale) {
  __shared__ float red[kBlock / 64];
  const int b = blockIdx.x / ntheta;
  const int s = blockIdx.x - b * ntheta;
  const int* bp = tb.bin_ptr + (size_t)b * (ntheta + 1);
  const int sb = s == 0 ? ntheta - 1 : s - 1;
  float part = 0.f;
  for (int pos = bp[s] + threadIdx.x; pos < bp[s + 1]; pos += kBlock)
    part += (1.0f - tb.tr_alpha[pos]) * tr_bound[tb.tr_row[pos]];
  for (int pos = bp[sb] + threadIdx.x; pos < bp[sb + 1]; pos += kBlock)
    part += tb.tr_alpha[pos] * tr_bound[tb.tr_row[pos]];
  const float sum = block_sum<kBlock>(part, red);
  if (threadIdx.x == 0) scale[blockIdx.x] = sum > 0.f ? 0.99f * 2147483647.0f / sum : 1.0f;
}

// One azimuth bin into the slots lo (weight 1 - alpha, slice j, scale S_lo) and hi
// (weight alpha, slice j+1, scale S_hi); HAS_LO / HAS_HI say which slots take part.
template <int W, bool HAS_LO, bool HAS_HI>
__device__ __forceinline__ void spread_bin(unsigned long long* lo, unsigned long long* hi, int c_begin, int c_end,
                                           const float2* __restrict__ dhat, int f0, float S_lo,
                                           float S_hi, const Tables& tb, const Dims& dm, int ftl) {
  const int ldr = dm.ldr;
  const int ft = dm.ft;
  const int cnt = c_end - c_begin;
  for (int it = threadIdx.x; it < cnt * ft; it += kBlockG) {
    const int n = c_begin + (it >> ftl);
    const int fl = it & (ft - 1);
    const unsigned f = (unsigned)(f0 + fl);
    if (f >= (unsigned)dm.nf) continue;
    const float2 dv = dhat[(size_t)tb.tr_row[n] * dm.nf + f];
    const float2 s = cmul(dv, pre_phase<1>(f, tb.tr_a[n]));
    const KernelPoint kp = kernel_point<W>(f, tb.tr_b[n], dm.mg);
    const float alpha = tb.tr_alpha[n];
    const float2 s1 = cscale(s, alpha * S_hi);
    const float2 s0 = cscale(s, (1.0f - alpha) * S_lo);
    unsigned long long* g0 = HAS_LO ? lo + fl * ldr + kp.base : nullptr;
    unsigned long long* g1 = HAS_HI ? hi + fl * ldr + kp.base : nullptr;
#pragma unroll
    for (int t = 0; t < W; ++t) {
      const float ph = grid_tap<W>(fmaf((float)t, -2.0f / (float)W, kp.z0), dm.cbeta);
      if (HAS_LO) atomicAdd(g0 + t, pack_fix(ph * s0.x, ph * s0.y));
      if (HAS_HI) atomicAdd(g1 + t, pack_fix(ph * s1.x, ph * s1.y));
    }
  }
  __syncthreads();
}

// Fold the ghost cells back, decode the slot in place to FP32, inverse q-grid
// FFT in place: H[k] = sum_m G[m] exp(+2 pi i k m/mg) for the nq modes, written to
// Mh[b][s][k + nq/2][f0 + f]; the slot is cleared afterwards.
template <int W>
__device__ __forceinline__ void finish_slot(unsigned long long* slot, float2* __restrict__ out_slice, int f0,
                                            float inv_s, const float2* twl, const Dims& dm, const FftPlan& fpg,
                                            int ftl) {
  const int ldr = dm.ldr;
  const int ft = dm.ft;
  for (int i = threadIdx.x; i < ft * (W - 1); i += kBlockG) {
    const int fl = i / (W - 1), t = i - fl * (W - 1);
    slot[fl * ldr + t] += slot[fl * ldr + dm.mg + t];
  }
  __syncthreads();
  float2* P = reinterpret_cast<float2*>(slot);
  for (int i = threadIdx.x; i < ft * ldr; i += kBlockG) P[i] = unpack_fix(slot[i], inv_s);
  __syncthreads();
  fft_lds_ip<true, kBlockG>(P, fpg, ft, ldr, twl);
  for (int it = threadIdx.x; it < dm.nq * ft; it += kBlockG) {
    const int l = it >> ftl;
    const int fl = it & (ft - 1);
    const int f = f0 + fl;
    int m = l - dm.qhalf;
    if (m < 0) m += dm.mg;
    if (f < dm.nf) out_slice[(size_t)l * dm.nf + f] = P[fl * ldr + m];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ft * ldr; i += kBlockG) slot[i] = 0ull;
  __syncthreads();
}

// Transpose of k_nufft_interp.  Two fixed-point slots: slice s lives in slot
// s & 1.  The wrap bin ntheta-1 is spread twice, its upper part into slice 0
// before the sweep and its lower part into slice ntheta-1 at the end, so no
// slice has to stay resident across the whole sweep.
template <int W>
__global__ __launch_bounds__(kBlockG) void k_nufft_spread(const float2* __restrict__ dhat,
                                                          const float* __restrict__ slice_scale,
                                                          float2* __restrict__ mhat, Tables tb,
                                                          Dims dm, FftPlan fpg, int ftl) {
  extern __shared__ float2 lds[];
  const int ft = dm.ft;
  const int slot_sz = ft * dm.ldr;
  unsigned long long* slot0 = reinterpret_cast<unsigned long long*>(lds);
  unsigned long long* slot1 = slot0 + slot_sz;
  float2* twl = lds + 2 * slot_sz;  // q-grid twiddles
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int b = tile / dm.nftile;
  const int f0 = (tile - b * dm.nftile) * ft;
  const int* bp = tb.bin_ptr + (size_t)b * (dm.ntheta + 1);
  const size_t slice_stride = (size_t)dm.nq * dm.nf;
  float2* mb = mhat + (size_t)b * dm.ntheta * slice_stride;

  for (int i = threadIdx.x; i < 2 * slot_sz; i += kBlockG) slot0[i] = 0ull;
  for (int i = threadIdx.x; i < dm.mg; i += kBlockG) twl[i] = tb.tw_grid[i];
  __syncthreads();
  const int last = dm.ntheta - 1;
  float S_prev = 1.0f;  // scale of the slice finished at this step

  // step 0: upper part of the wrap bin into slice 0; step s = 1..last: bin s-1 into slices
  // s-1 and s, then slice s-1 is complete; step last+1: lower part of the wrap bin into slice last
  for (int step = 0; step <= last + 1; ++step) {
    const int bin = (step == 0 || step == last + 1) ? last : step - 1;
    unsigned long long* lo = step == 0 ? nullptr : (((step - 1) & 1) ? slot1 : slot0);
    unsigned long long* hi = step == last + 1 ? nullptr : ((step & 1) ? slot1 : slot0);
    const float S_hi = step <= last ? slice_scale[(size_t)b * dm.ntheta + step] : 1.0f;
    if (step == 0)
      spread_bin<W, false, true>(lo, hi, bp[bin], bp[bin + 1], dhat, f0, S_prev, S_hi, tb, dm, ftl);
    else if (step == last + 1)
      spread_bin<W, true, false>(lo, hi, bp[bin], bp[bin + 1], dhat, f0, S_prev, S_hi, tb, dm, ftl);
    else
      spread_bin<W, true, true>(lo, hi, bp[bin], bp[bin + 1], dhat, f0, S_prev, S_hi, tb, dm, ftl);
    if (step >= 1)
      finish_slot<W>(lo, mb + (size_t)(step - 1) * slice_stride, f0, 1.0f / S_prev, twl, dm, fpg, ftl);
    S_prev = S_hi;
  }
}

// ------------------------------------------------------------------ small kernels
__global__ void k_fill(float* p, float v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_copy(float* __restrict__ dst, const float* __restrict__ src, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Counter-based uniform(-1,1) start vector for the power iteration (splitmix64 of the index).
__global__ void k_seed(float* v, size_t n, unsigned seed) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    unsigned long long z = (unsigned long long)i + 0x9E3779B97F4A7C15ull * (seed + 1ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    v[i] = (float)(z >> 40) * (2.0f / 16777216.0f) - 1.0f;
  }
}

// Per-gather reduction over model-sized arrays: stage 1 writes one partial per
// (gather, block); stage 2 combines them in a fixed order (deterministic).
__global__ __launch_bounds__(kBlock) void k_reduce_stage1(const float* __restrict__ x, size_t per,
                                                          int nblk, int op, float* __restrict__ part) {
  __shared__ float red[kBlock / 64];
  const int b = blockIdx.x / nblk;
  const int k = blockIdx.x - b * nblk;
  const float* xb = x + (size_t)b * per;
  const size_t chunk = (per + nblk - 1) / nblk;
  const size_t lo = k * chunk;
  const size_t hi = lo + chunk < per ? lo + chunk : per;
  float acc = 0.f;
  for (size_t i = lo + threadIdx.x; i < hi; i += kBlock) {
    const float v = xb[i];
    if (op == RED_SUMSQ) acc += v * v;
    else if (op == RED_MAXABS) acc = fmaxf(acc, fabsf(v));
    else acc += fabsf(v);
  }
  const float r = (op == RED_MAXABS) ? block_max<kBlock>(acc, red) : block_sum<kBlock>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void k_reduce_stage2(const float* __restrict__ part, int nblk, int nseg, int op,
                                float* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nseg) return;
  float acc = 0.f;
  for (int k = 0; k < nblk; ++k) {
    const float v = part[(size_t)b * nblk + k];
    acc = (op == RED_MAXABS) ? fmaxf(acc, v) : acc + v;
  }
  out[b] = acc;
}

__global__ void k_scale_per_gather(float* __restrict__ x, size_t per, int batch,
                                   const float* __restrict__ norms) {
  const int b = blockIdx.y;
  const float nv = norms[b];
  const float s = nv > 0.f ? 1.0f / nv : 0.f;
  float* xb = x + (size_t)b * per;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < per; i += (size_t)gridDim.x * blockDim.x)
    xb[i] *= s;
}

__global__ void k_gather_scalar(int batch, int op, const float* __restrict__ a, float* __restrict__ out,
                                float c) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const float v = a[b];
  if (op == GS_STEP) out[b] = v > 0.f ? 1.0f / (c * v) : 0.f;  // gamma = 1/(c ||L||^2)
  else if (op == GS_LAMBDA) out[b] = c * v;
  else out[b] = sqrtf(v);
}

// objective[b] = 0.5 sum_{traces of b} rss + lambda_b sum_{rows of b} l1
__global__ void k_objective(const float* __restrict__ rss, const int64_t* __restrict__ trace_ptr,
                            const float* __restrict__ l1, int rows_per, const float* __restrict__ lam,
                            int batch, float* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  float r = 0.f;
  for (int64_t n = trace_ptr[b]; n < trace_ptr[b + 1]; ++n) r += rss[n];
  float s = 0.f;
  for (int k = 0; k < rows_per; ++k) s += l1[(size_t)b * rows_per + k];
  out[b] = 0.5f * r + lam[b] * s;
}

// Automatic anisotropic velocity estimate (Section 3): for every gather b, azimuth j
// and intercept i, qbar = sum_l q_l |m| / sum_l |m| over the curvature samples
// (0 where the cube holds no energy) and v = qbar^(-1/2) (0 where qbar <= 0).  One
// thread per intercept; the curvature loop reads rows of the model, coalesced in tau.
__global__ __launch_bounds__(kBlock) void k_velocity(const float* __restrict__ m, float* __restrict__ qbar,
                                                     float* __restrict__ vel, int nq, int ntau, float q_min,
                                                     float dq) {
  const size_t bj = blockIdx.y;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= ntau) return;
  const float* src = m + bj * (size_t)nq * ntau + i;
  float num = 0.f, den = 0.f;
  for (int l = 0; l < nq; ++l) {
    const float a = fabsf(src[(size_t)l * ntau]);
    den += a;
    num = fmaf(fmaf((float)l, dq, q_min), a, num);
  }
  const float qb = den > 0.f ? num / den : 0.f;
  qbar[bj * ntau + i] = qb;
  vel[bj * ntau + i] = qb > 0.f ? 1.0f / sqrtf(qb) : 0.f;
}

// Conventional time-domain adjoint (the direct summation the paper compares against
// in Section 5): for every output (b, j, l, i) the Riemann sum over the traces that
// reach azimuth j (bin j with weight 1 - alpha, bin j-1 mod ntheta with weight alpha)
// of the trace sample at t = sqrt(tau_i^2 + q_l h^2), linearly interpolated in time
// (taps at or beyond nt dropped).  Positions in FP64; one thread per intercept, the
// per-trace values are uniform across the block.
__global__ __launch_bounds__(kBlock) void k_direct_adjoint(const float* __restrict__ d, float* __restrict__ m,
                                                           Tables tb, Dims dm, double dtau, double dt,
                                                           double q_min, double dq) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= dm.ntau) return;
  const int l = blockIdx.y;
  const int bj = blockIdx.z;
  const int b = bj / dm.ntheta;
  const int j = bj - b * dm.ntheta;
  const int* bp = tb.bin_ptr + (size_t)b * (dm.ntheta + 1);
  const int jm = j == 0 ? dm.ntheta - 1 : j - 1;  // ntheta = 1: both passes run over bin 0
  const double tau = i * dtau;
  const double tau2 = tau * tau;
  const double q = q_min + l * dq;
  const double inv_dt = 1.0 / dt;
  float acc = 0.f;
  for (int pass = 0; pass < 2; ++pass) {
    const int lo = pass == 0 ? bp[j] : bp[jm];
    const int hi = pass == 0 ? bp[j + 1] : bp[jm + 1];
    for (int n = lo; n < hi; ++n) {
      const double arg = tau2 + q * tb.tr_h2[n];
      if (arg < 0.0) continue;
      const double tt = sqrt(arg) * inv_dt;
      const double sf = floor(tt);
      if (sf >= (double)dm.nt) continue;
      const int s = (int)sf;
      const float a = (float)(tt - sf);
      const float* row = d + (size_t)tb.tr_row[n] * dm.nt;
      float v = (1.0f - a) * row[s];
      if (s + 1 < dm.nt) v = fmaf(a, row[s + 1], v);
      const float al = tb.tr_alpha[n];
      acc = fmaf(pass == 0 ? 1.0f - al : al, v, acc);
    }
  }
  m[((size_t)bj * dm.nq + l) * dm.ntau + i] = acc;
}

// ------------------------------------------------------------------ Algorithm 2 (Section 3.2)
// Step 3 and the k-half of step 4 on a regular offset grid.  Workgroup (f tile, j, b):
// for every bin f of the tile and every k_p, the data spectrum is read at the offset
//   x = sqrt(k_p / f') cos(theta_j),  y = sqrt(k_p / f') sin(theta_j)
// by the bilinear coefficients B1..B4 of Section 3.4 (0 for k_p < 0, f = 0 or outside the
// grid), times exp(2 pi i k_p q_min) / nq; an inverse DFT over k in LDS then gives the
// q_l = q_min + l dq rows of the model spectrum.  Positions are computed in FP64.
__global__ __launch_bounds__(kBlock) void k_grid_polar(const float2* __restrict__ dhat,
                                                       float2* __restrict__ mhat, GridTables gt,
                                                       Dims dm, FftPlan fq, int ft, int ftl) {
  extern __shared__ float2 lds[];
  const int nq = dm.nq;
  const int ld = pad16(nq - 1) + 1;
  float2* A = lds;
  float2* B = lds + ft * ld;
  const int f0 = blockIdx.x * ft;
  const int j = blockIdx.y;
  const int b = blockIdx.z;
  const GridGather G = gt.g[b];
  const double2 cs = gt.cs[j];
  for (int it = threadIdx.x; it < nq * ft; it += kBlock) {
    const int p = it >> ftl;
    const int fl = it & (ft - 1);
    const int f = f0 + fl;
    float2 v = make_float2(0.f, 0.f);
    const double kp = gt.kp[p];
    if (f >= 1 && f < dm.nf && kp >= 0.0 && G.mx >= 2 && G.my >= 2) {
      const double r = sqrt(kp / ((double)f * gt.fscale));
      const double u = (r * cs.x - G.x0) / G.dx;
      const double w = (r * cs.y - G.y0) / G.dy;
      if (u >= 0.0 && u <= (double)(G.mx - 1) && w >= 0.0 && w <= (double)(G.my - 1)) {
        const int m = min((int)u, G.mx - 2);
        const int n = min((int)w, G.my - 2);
        const float a = (float)(u - m);
        const float c = (float)(w - n);
        const int* nd = gt.node + G.node0 + m * G.my + n;
        const float2 d00 = dhat[(size_t)nd[0] * dm.nf + f];
        const float2 d01 = dhat[(size_t)nd[1] * dm.nf + f];
        const float2 d10 = dhat[(size_t)nd[G.my] * dm.nf + f];
        const float2 d11 = dhat[(size_t)nd[G.my + 1] * dm.nf + f];
        const float b00 = (1.f - a) * (1.f - c), b01 = (1.f - a) * c, b10 = a * (1.f - c), b11 = a * c;
        v.x = b00 * d00.x + b01 * d01.x + b10 * d10.x + b11 * d11.x;
        v.y = b00 * d00.y + b01 * d01.y + b10 * d10.y + b11 * d11.y;
        v = cmul(v, gt.phase[p]);
      }
    }
    A[fl * ld + p] = v;
  }
  __syncthreads();
  const float2* R = fft_lds<true, kBlock>(A, B, fq, ft, ld, gt.tw);
  float2* out = mhat + ((size_t)b * dm.ntheta + j) * nq * dm.nf;
  for (int it = threadIdx.x; it < nq * ft; it += kBlock) {
    const int l = it >> ftl;
    const int fl = it & (ft - 1);
    const int f = f0 + fl;
    if (f < dm.nf) out[(size_t)l * dm.nf + f] = R[fl * ld + l];
  }
}

// The f'-half of step 4 (inverse real DFT, 1/N) and step 5, the unstretch by
// interpolation M(tau_i) = M'(tau_i^2).
template <int IP>
__global__ __launch_bounds__(kBlock) void k_model_c2r_grid(const float2* __restrict__ mhat,
                                                           float* __restrict__ m, Tables tb, Dims dm,
                                                           FftPlan fp, const Tap* __restrict__ vtap) {
  extern __shared__ float2 lds[];
  const size_t rid = blockIdx.x;
  const float* xs = model_c2r_core<IP>(mhat, lds, lds + dm.nhp, tb, dm, fp, rid);
  const float sc = 1.0f / (float)dm.nfft;
  float* dst = m + rid * dm.ntau;
  for (int i = threadIdx.x; i < dm.ntau; i += kBlock) {
    const Tap t = vtap[i];
    dst[i] = sc * (t.w0 * xs[t.i0] + t.w1 * xs[t.i1]);
  }
}

// ------------------------------------------------------------------ launchers

static size_t interp_lds_bytes(const Dims& dm) {
  return interp_lds_f2(dm.ft, dm.ldr, dm.ntheta, dm.mg, dm.gdt) * sizeof(float2);
}

static size_t spread_lds_bytes(const Dims& dm) { return spread_lds_f2(dm.ft, dm.ldr, dm.mg) * sizeof(float2); }

static int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

template <typename K>
static hipError_t set_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Launch one row kernel: in place (every FFT pass fits the block) with `stage`
// real samples of staging after the buffer, else the two-buffer form.
// kip: in place, one butterfly per thread per pass; kipk: in place, several; kpp: ping-pong.
template <typename KIP, typename KIPK, typename KPP, typename... Args>
static hipError_t launch_row(KIP kip, KIPK kipk, KPP kpp, const Dims& dm, int stage, unsigned grid, hipStream_t s,
                             Args... args) {
  if (grid == 0) return hipSuccess;
  if (dm.row_ip == 1) {
    const size_t lds = ((size_t)dm.nhp + (size_t)(stage + 5) / 2) * sizeof(float2);  // staging + 4 spare
    hipError_t e = set_lds(kip, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kip, dim3(grid), dim3(kBlock), lds, s, args...);
  } else if (dm.row_ip == 2) {
    const size_t lds = ((size_t)dm.nhp + (size_t)(stage + 5) / 2) * sizeof(float2);
    hipError_t e = set_lds(kipk, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kipk, dim3(grid), dim3(kBlock), lds, s, args...);
  } else {
    const size_t lds = 2 * (size_t)dm.nhp * sizeof(float2);
    hipError_t e = set_lds(kpp, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kpp, dim3(grid), dim3(kBlock), lds, s, args...);
  }
  return hipGetLastError();
}

static unsigned model_rows(const Dims& dm) { return (unsigned)((size_t)dm.batch * dm.ntheta * dm.nq); }

hipError_t launch_model_r2c(const Plan& p, const float* m, float2* mhat, hipStream_t s) {
  const Dims& dm = p.dm;
  return launch_row(k_model_r2c<1>, k_model_r2c<2>, k_model_r2c<0>, dm, dm.ntau, model_rows(dm), s, m, mhat, p.tb, dm,
                    p.fft_half);
}

hipError_t launch_model_c2r(const Plan& p, const float2* mhat, float* m, hipStream_t s) {
  const Dims& dm = p.dm;
  return launch_row(k_model_c2r<1>, k_model_c2r<2>, k_model_c2r<0>, dm, 0, model_rows(dm), s, mhat, m, p.tb, dm,
                    p.fft_half);
}

hipError_t launch_model_c2r_update(const Plan& p, float2* mhat, float* y, float* x, const float* gam,
                                   const float* lam, float beta, int ista, float* l1, bool next,
                                   hipStream_t s) {
  const Dims& dm = p.dm;
  if (next)
    return launch_row(k_model_c2r_update<1, true>, k_model_c2r_update<2, true>, k_model_c2r_update<0, true>, dm, dm.ntau,
                      model_rows(dm), s, mhat, y, x, p.tb, dm, p.fft_half, gam, lam, beta, ista, l1);
  return launch_row(k_model_c2r_update<1, false>, k_model_c2r_update<2, false>, k_model_c2r_update<0, false>, dm, 0, model_rows(dm), s,
                    mhat, y, x, p.tb, dm, p.fft_half, gam, lam, beta, ista, l1);
}

hipError_t launch_data_c2r(const Plan& p, const float2* dhat, float* d, hipStream_t s) {
  const Dims& dm = p.dm;
  if (dm.nw > 0)
    return launch_row(k_data_c2r<1, true>, k_data_c2r<2, true>, k_data_c2r<0, true>, dm, dm.nt, (unsigned)dm.ntr, s, dhat, d,
                      p.tb, dm, p.fft_half);
  return launch_row(k_data_c2r<1, false>, k_data_c2r<2, false>, k_data_c2r<0, false>, dm, 0, (unsigned)dm.ntr, s, dhat, d, p.tb,
                    dm, p.fft_half);
}

hipError_t launch_data_r2c(const Plan& p, const float* d, float2* dhat, hipStream_t s) {
  const Dims& dm = p.dm;
  if (dm.nw > 0)
    return launch_row(k_data_r2c<1, true>, k_data_r2c<2, true>, k_data_r2c<0, true>, dm, dm.nt, (unsigned)dm.ntr, s, d, dhat,
                      p.tr_bound, p.tb, dm, p.fft_half);
  return launch_row(k_data_r2c<1, false>, k_data_r2c<2, false>, k_data_r2c<0, false>, dm, dm.nt, (unsigned)dm.ntr, s, d, dhat,
                    p.tr_bound, p.tb, dm, p.fft_half);
}

hipError_t launch_residual_r2c(const Plan& p, float2* dhat, const float* dobs, float* rss,
                               hipStream_t s) {
  const Dims& dm = p.dm;
  if (dm.nw > 0)
    return launch_row(k_residual_r2c<1, true>, k_residual_r2c<2, true>, k_residual_r2c<0, true>, dm, dm.nt, (unsigned)dm.ntr, s,
                      dhat, dobs, rss, p.tr_bound, p.tb, dm, p.fft_half);
  return launch_row(k_residual_r2c<1, false>, k_residual_r2c<2, false>, k_residual_r2c<0, false>, dm, dm.nt, (unsigned)dm.ntr, s,
                    dhat, dobs, rss, p.tr_bound, p.tb, dm, p.fft_half);
}

#define AAHRT_W_CASES(MACRO) \
  MACRO(2) MACRO(3) MACRO(4) MACRO(5) MACRO(6) MACRO(7) MACRO(8) MACRO(9) MACRO(10) MACRO(11) MACRO(12)

// Dims of a GFST launch with the kernel's own frequency tile.
static Dims tile_dims(const Dims& d0, int ft) {
  Dims dm = d0;
  dm.ft = ft;
  dm.nftile = (dm.nf + ft - 1) / ft;
  return dm;
}

hipError_t launch_nufft_interp(const Plan& p, const float2* mhat, float2* dhat, hipStream_t s) {
  const Dims dm = tile_dims(p.dm, p.ft_interp);
  if (dm.ntr == 0) return hipSuccess;
  const size_t lds = interp_lds_bytes(dm);
  const dim3 grid((unsigned)dm.batch * dm.nftile), block(kBlockG);
  const int ftl = ilog2(dm.ft);
  switch (dm.w) {
#define AAHRT_LAUNCH_INTERP(WW, GG)                                                               \
  {                                                                                               \
    hipError_t e = set_lds(k_nufft_interp<WW, GG>, lds);                                          \
    if (e != hipSuccess) return e;                                                                \
    hipLaunchKernelGGL((k_nufft_interp<WW, GG>), grid, block, lds, s, mhat, dhat, p.tb, dm, p.fft_grid, ftl); \
  }
#define AAHRT_CASE(WW)                                                                       \
  case WW: {                                                                                 \
    if (dm.gdt == AAHRT_GRID_F16) AAHRT_LAUNCH_INTERP(WW, AAHRT_GRID_F16)                    \
    else if (dm.gdt == AAHRT_GRID_BF16) AAHRT_LAUNCH_INTERP(WW, AAHRT_GRID_BF16)             \
    else AAHRT_LAUNCH_INTERP(WW, AAHRT_GRID_F32)                                             \
    break;                                                                                   \
  }
    AAHRT_W_CASES(AAHRT_CASE)
#undef AAHRT_CASE
#undef AAHRT_LAUNCH_INTERP
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_nufft_spread(const Plan& p, const float2* dhat, float2* mhat, hipStream_t s) {
  const Dims dm = tile_dims(p.dm, p.ft_spread);
  const size_t lds = spread_lds_bytes(dm);
  const dim3 grid((unsigned)dm.batch * dm.nftile), block(kBlockG);
  const int ftl = ilog2(dm.ft);
  hipLaunchKernelGGL(k_slice_scales, dim3((unsigned)dm.batch * dm.ntheta), dim3(kBlock), 0, s, p.tr_bound, p.tb,
                     dm.ntheta, p.slice_scale);
  switch (dm.w) {
#define AAHRT_CASE(WW)                                                                       \
  case WW: {                                                                                 \
    hipError_t e = set_lds(k_nufft_spread<WW>, lds);                                         \
    if (e != hipSuccess) return e;                                                           \
    hipLaunchKernelGGL(k_nufft_spread<WW>, grid, block, lds, s, dhat, p.slice_scale, mhat, \
                       p.tb, dm, p.fft_grid, ftl);                                           \
    break;                                                                                   \
  }
    AAHRT_W_CASES(AAHRT_CASE)
#undef AAHRT_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static unsigned ew_blocks(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  if (b == 0) b = 1;
  return (unsigned)b;
}

hipError_t launch_fill(float* ptr, float v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(ew_blocks(n)), dim3(kBlock), 0, s, ptr, v, n);
  return hipGetLastError();
}

hipError_t launch_copy(float* dst, const float* src, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(ew_blocks(n)), dim3(kBlock), 0, s, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_seed_vector(float* v, size_t n, unsigned seed, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_seed, dim3(ew_blocks(n)), dim3(kBlock), 0, s, v, n, seed);
  return hipGetLastError();
}

hipError_t launch_gather_reduce(const Plan& p, const float* x, int op, float* out, hipStream_t s) {
  const Dims& dm = p.dm;
  const size_t per = (size_t)dm.ntheta * dm.nq * dm.ntau;
  const int nblk = p.red_blocks_model;
  hipLaunchKernelGGL(k_reduce_stage1, dim3((unsigned)dm.batch * nblk), dim3(kBlock), 0, s, x, per,
                     nblk, op, p.red);
  hipLaunchKernelGGL(k_reduce_stage2, dim3((dm.batch + 63) / 64), dim3(64), 0, s, p.red, nblk,
                     dm.batch, op, out);
  return hipGetLastError();
}

hipError_t launch_scale_per_gather(const Plan& p, float* x, const float* norms, hipStream_t s) {
  const Dims& dm = p.dm;
  const size_t per = (size_t)dm.ntheta * dm.nq * dm.ntau;
  size_t bx = (per + kBlock - 1) / kBlock;
  if (bx > 256) bx = 256;
  hipLaunchKernelGGL(k_scale_per_gather, dim3((unsigned)bx, dm.batch), dim3(kBlock), 0, s, x, per,
                     dm.batch, norms);
  return hipGetLastError();
}

hipError_t launch_gather_scalar(const Plan& p, int op, const float* a, float* out, float c,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_gather_scalar, dim3((p.dm.batch + 63) / 64), dim3(64), 0, s, p.dm.batch, op, a,
                     out, c);
  return hipGetLastError();
}

hipError_t launch_objective(const Plan& p, const float* rss, const int64_t* trace_ptr_dev,
                            const float* l1, const float* lam, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_objective, dim3((p.dm.batch + 63) / 64), dim3(64), 0, s, rss, trace_ptr_dev, l1,
                     p.dm.ntheta * p.dm.nq, lam, p.dm.batch, out);
  return hipGetLastError();
}

hipError_t launch_velocity(const Plan& p, const float* m, float* qbar, float* vel, hipStream_t s) {
  const Dims& dm = p.dm;
  const double dq = (p.prm.q_max - p.prm.q_min) / (dm.nq - 1);
  const dim3 grid((unsigned)((dm.ntau + kBlock - 1) / kBlock), (unsigned)(dm.batch * dm.ntheta));
  hipLaunchKernelGGL(k_velocity, grid, dim3(kBlock), 0, s, m, qbar, vel, dm.nq, dm.ntau, (float)p.prm.q_min,
                     (float)dq);
  return hipGetLastError();
}

hipError_t launch_direct_adjoint(const Plan& p, const float* d, float* m, hipStream_t s) {
  const Dims& dm = p.dm;
  const double dq = (p.prm.q_max - p.prm.q_min) / (dm.nq - 1);
  const dim3 grid((unsigned)((dm.ntau + kBlock - 1) / kBlock), (unsigned)dm.nq, (unsigned)(dm.batch * dm.ntheta));
  hipLaunchKernelGGL(k_direct_adjoint, grid, dim3(kBlock), 0, s, d, m, p.tb, dm, p.prm.dtau, p.prm.dt, p.prm.q_min,
                     dq);
  return hipGetLastError();
}

// Algorithm 2: steps 1-2 through the model-side row kernel (data rows of nt samples,
// interpolation taps of the data stretch, unit scale), then the polar interpolation with
// the k-transform, then the f'-transform with the unstretch.
hipError_t launch_grid_adjoint(const Plan& p, const float* d, float* m, hipStream_t s) {
  Dims dd = p.dm;
  dd.ntau = p.dm.nt;
  dd.nq = 1;
  Tables td = p.tb;
  td.s_tap = p.gt.dtap;
  td.deapod = p.gt.one;
  hipError_t e = launch_row(k_model_r2c<1>, k_model_r2c<2>, k_model_r2c<0>, dd, dd.ntau, (unsigned)p.dm.ntr, s, d, p.dhat,
                            td, dd, p.fft_half);
  if (e != hipSuccess) return e;
  const Dims& dm = p.dm;
  const int ft = p.grid_ft;
  int ftl = 0;
  while ((1 << ftl) < ft) ++ftl;
  const size_t lds = 2 * (size_t)ft * (pad16(dm.nq - 1) + 1) * sizeof(float2);
  e = set_lds(k_grid_polar, lds);
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)((dm.nf + ft - 1) / ft), (unsigned)dm.ntheta, (unsigned)dm.batch);
  hipLaunchKernelGGL(k_grid_polar, grid, dim3(kBlock), lds, s, p.dhat, p.mhat, p.gt, dm, p.fft_q, ft, ftl);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_row(k_model_c2r_grid<1>, k_model_c2r_grid<2>, k_model_c2r_grid<0>, dm, 0, model_rows(dm), s, p.mhat, m, p.tb,
                    dm, p.fft_half, p.gt.vtap);
}

}  // namespace aahrt
