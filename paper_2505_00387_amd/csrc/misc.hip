// HIP kernels (gfx950) beside the operator pair: fills, reductions over gathers, the
// objective, the velocity estimate of Section 3, the time-domain direct-sum adjoint of
// Section 5 and Algorithm 2 of Section 3.2, with their launchers.
#include <hip/hip_runtime.h>

#include "kernel_common.hpp"

namespace aahrt {

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
  const auto twb = row_twiddles<IP>(tb);
  const float* xs = model_c2r_core<IP>(mhat, lds, lds + dm.nhp, tb, dm, fp, rid, twb);
  const float sc = 1.0f / (float)dm.nfft;
  float* dst = m + rid * dm.ntau;
  for (int i = threadIdx.x; i < dm.ntau; i += kBlock) {
    const Tap t = vtap[i];
    dst[i] = sc * (t.w0 * xs[t.i0] + t.w1 * xs[t.i1]);
  }
}

// ------------------------------------------------------------------ launchers
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
  hipError_t e = launch_rows_r2c(dd, td, p.fft_half, d, p.dhat, (unsigned)p.dm.ntr, s);
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
  return launch_row(AAHRT_ROWK(k_model_c2r_grid), dm, 0, model_rows(dm), s, p.mhat, m, p.tb,
                    dm, p.fft_half, p.gt.vtap);
}

}  // namespace aahrt
