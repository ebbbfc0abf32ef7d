// HIP kernels (gfx950) of step 3 of Algorithm 1 and its transpose, resident-slice form, and
// their launchers.
#include <hip/hip_runtime.h>

#include "gfst_common.hpp"

namespace aahrt {

// ------------------------------------------------------------------ resident-slice variant
// The same map and its transpose with every azimuth slice of a frequency tile resident in
// LDS ([ntheta][ft][ldr] cells), for q-grids of 64, 128 or 256 cells in FP32.  A workgroup
// first builds (interpolation) or clears (spreading) all slices, then runs over all the
// gather's traces with no barrier per azimuth bin: a trace of bin j reads or feeds slices j
// and j + 1 (mod ntheta).  Each q-grid row (slice, frequency) is transformed in registers by
// a group of L lanes (mg = R1 L): lane t holds x[t + L r], r < R1, transforms them (DFT of
// length R1), applies the twiddles exp(-+2 pi i t k1/mg), exchanges through the row's own
// LDS cells, and finishes with DFTs of length L (Cooley-Tukey, mg = R1 x L).  The L lanes of
// a row belong to one wavefront, so the exchange needs wavefront ordering only.

// Orders this wavefront's LDS accesses before and after (a compiler and memory fence for
// the wavefront; its lanes execute in lockstep).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exchange position of element (k1, t) in a row: k1 L + t + k1 / (R1/L).  The padding term
// puts the L reads of one second-pass input in distinct LDS banks; positions stay below
// mg + L - 1, which the row length of the resident layout provides.
template <int R1, int L>
__device__ __forceinline__ int xch_pos(int k1, int t) {
  return k1 * L + t + k1 / (R1 / L);
}

// One mg = R1 L point DFT (INV: exp(+...)) by the L lanes of a group.  In: lane t holds
// v[r] = x[t + L r].  Out: v[i L + k2] = X[(t C + i) + R1 k2], C = R1/L, i < C, k2 < L.
// xch: mg + L - 1 cells of LDS private to the group.
template <int R1, int L, bool INV>
__device__ __forceinline__ void row_dft_lanes(float2 (&v)[R1], int t, float2* xch, const float2* twl) {
  constexpr int C = R1 / L;
  Dft<R1, INV>::run(v);
  apply_twiddles<R1, INV>(v, twl, t);
  wave_sync();
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) xch[xch_pos<R1, L>(k1, t)] = v[k1];
  wave_sync();
#pragma unroll
  for (int i = 0; i < C; ++i) {
    float2 u[L];
    const int k1 = t * C + i;
#pragma unroll
    for (int tp = 0; tp < L; ++tp) u[tp] = xch[xch_pos<R1, L>(k1, tp)];
    Dft<L, INV>::run(u);
#pragma unroll
    for (int k2 = 0; k2 < L; ++k2) v[i * L + k2] = u[k2];
  }
  wave_sync();
}

// Curvature row l of grid cell m (mode k = m for m < nq - nq/2, k = m - mg for m >= mg - nq/2,
// l = k + nq/2), or -1 for the zero-padded cells.
__device__ __forceinline__ int mode_row(int m, const Dims& dm) {
  if (m < dm.nq - dm.qhalf) return m + dm.qhalf;
  if (m >= dm.mg - dm.qhalf) return m - dm.mg + dm.qhalf;
  return -1;
}

// HALF (mg = 2 nq, nq even): cell m = t + L r of lane t holds a mode exactly when r < R1/4
// (l = m + mg/4) or r >= 3 R1/4 (l = m - 3 mg/4), and output m = t C + i + R1 k2 is a kept mode
// exactly when k2 < L/4 or k2 >= 3 L/4: the zero inputs and the dropped outputs are then
// known at compile time and their arithmetic disappears.
template <int R1, int L, bool HALF>
__device__ __forceinline__ int mode_row_of(int t, int r, const Dims& dm) {
  if constexpr (HALF) {
    constexpr int mg = R1 * L;
    if (r < R1 / 4) return t + L * r + mg / 4;
    if (r >= 3 * R1 / 4) return t + L * r - 3 * mg / 4;
    return -1;
  } else {
    return mode_row(t + L * r, dm);
  }
}
template <int R1, int L, bool HALF>
__device__ __forceinline__ int kept_mode_row(int t, int i, int k2, const Dims& dm) {
  constexpr int C = R1 / L;
  if constexpr (HALF) {
    constexpr int mg = R1 * L;
    const int m = t * C + i + R1 * k2;
    if (k2 < L / 4) return m + mg / 4;
    if (k2 >= 3 * L / 4) return m - 3 * mg / 4;
    return -1;
  } else {
    return mode_row(t * C + i + R1 * k2, dm);
  }
}

// Forward GFST map with resident slices (see above).
template <int W, int R1, int L, bool POLY, int NT, bool HALF>
__global__ __launch_bounds__(NT) void k_nufft_interp_res(const float2* __restrict__ mhat,
                                                              float2* __restrict__ dhat, Tables tb, Dims dm,
                                                              int ftl) {
  extern __shared__ float2 lds[];
  constexpr int C = R1 / L;
  const int ldr = dm.ldr, ft = dm.ft, nt = dm.ntheta, mg = dm.mg;
  const int slab = ft * ldr;
  float2* slots = lds;                                   // [nt][ft][ldr]
  float2* twl = lds + (size_t)nt * slab;                 // [mg]
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int b = tile / dm.nftile;
  const int f0 = (tile - b * dm.nftile) * ft;
  const int* bp = tb.bin_ptr + (size_t)b * (nt + 1);
  const int c0 = bp[0], ntr = bp[nt] - bp[0];
  if (ntr == 0) return;  // empty gather: nothing to write
  for (int i = threadIdx.x; i < mg; i += NT) twl[i] = tb.tw_grid[i];
  __syncthreads();

  // q-grids of every (slice, frequency) row: modes from the model spectrum, DFT to the grid,
  // the first W - 1 cells repeated after the last (ghost cells)
  // Offsets within a slice use 24-bit products (l < 256, and nf < 2^14 since a row transform
  // fits LDS), which issue at the full
  // VALU rate where 32- and 64-bit integer products take four times as long.
  const int t = threadIdx.x % L;
  const float2* msrc = mhat + (size_t)b * nt * dm.nq * dm.nf;
  const unsigned qn = (unsigned)dm.nq * (unsigned)dm.nf;
  for (int row = threadIdx.x / L; row < nt * ft; row += NT / L) {
    const int sl = row >> ftl, fl = row & (ft - 1);
    const int f = f0 + fl;
    // a row past the last frequency is built from the last one's modes and never read
    const float2* src = msrc + (size_t)sl * qn + min(f, dm.nf - 1);
    float2 v[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      const int l = mode_row_of<R1, L, HALF>(t, r, dm);
      const float2 x = src[__umul24((unsigned)max(l, 0), (unsigned)dm.nf)];
      v[r] = l >= 0 ? x : make_float2(-0.f, -0.f);  // -0: the additive identity, folded away
    }
    float2* cell = slots + (size_t)row * ldr;
    row_dft_lanes<R1, L, false>(v, t, cell, twl);
#pragma unroll
    for (int i = 0; i < C; ++i) {
#pragma unroll
      for (int k2 = 0; k2 < L; ++k2) {
        const int m = t * C + i + R1 * k2;
        cell[m] = v[i * L + k2];
        if (m < W - 1) cell[mg + m] = v[i * L + k2];
      }
    }
  }
  __syncthreads();

  // every trace of the gather, kFptI consecutive frequencies per thread item (one)
  const int gpt = ft >= kFptI ? ft / kFptI : 1;
  const int gpl = ft >= kFptI ? ftl - kFptILog : 0;
  for (int it = threadIdx.x; it < ntr * gpt; it += NT) {
    const int n = c0 + (it >> gpl);
    const unsigned f1 = (unsigned)((f0 & ~(kFptI - 1)) + (it & (gpt - 1)) * kFptI);
    const int fl0 = (int)f1 - f0;
    if (f1 >= (unsigned)dm.nf) continue;
    const int j = tb.tr_bin[n];
    const int j1 = j + 1 == nt ? 0 : j + 1;
    const float2* G0 = slots + __umul24((unsigned)j, (unsigned)slab);
    const float2* G1 = slots + __umul24((unsigned)j1, (unsigned)slab);
    const unsigned long long bfix = tb.tr_b[n];
    unsigned long long tt = fix_mul(f1, bfix);
    const float2 rot = tb.tr_rot[n];
    float2 pre = pre_phase<-1>(f1, tb.tr_a[n]);
    const float alpha = tb.tr_alpha[n];
    float2* dst = dhat + (size_t)tb.tr_row[n] * dm.nf + f1;
#pragma unroll
    for (int k = 0; k < kFptI; ++k) {
      if (fl0 + k >= 0 && fl0 + k < ft && f1 + k < (unsigned)dm.nf) {
        const KernelPoint kp = kernel_point<W>((unsigned)(tt >> 32), R1 * L);
        const float2* g0 = G0 + __umul24((unsigned)(fl0 + k), (unsigned)ldr) + kp.base;
        const float2* g1 = G1 + __umul24((unsigned)(fl0 + k), (unsigned)ldr) + kp.base;
        float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
        float ph[W];
        kernel_taps<W, POLY>(kp.z0, dm.cbeta, ph);
#pragma unroll
        for (int tp = 0; tp < W; ++tp) {
          const float2 v0 = g0[tp], v1 = g1[tp];
          a0.x = fmaf(ph[tp], v0.x, a0.x);
          a0.y = fmaf(ph[tp], v0.y, a0.y);
          a1.x = fmaf(ph[tp], v1.x, a1.x);
          a1.y = fmaf(ph[tp], v1.y, a1.y);
        }
        const float2 v = make_float2(fmaf(alpha, a1.x - a0.x, a0.x), fmaf(alpha, a1.y - a0.y, a0.y));
        dst[k] = cmul(v, pre);
      }
      pre = cmul(pre, rot);
      tt += bfix;
    }
  }
}

// Transpose of k_nufft_interp_res: every slice cleared, every trace spread into its two
// slices in fixed point (scale per slice, as k_nufft_spread), then per row: ghost cells
// folded back, decoded, inverse DFT, the nq kept modes written to Mh[b][s][l][f].
template <int W, int R1, int L, bool POLY, int NT, bool HALF>
__global__ __launch_bounds__(NT) void k_nufft_spread_res(const float2* __restrict__ dhat,
                                                              const float* __restrict__ slice_scale,
                                                              float2* __restrict__ mhat, Tables tb, Dims dm,
                                                              int ftl) {
  extern __shared__ float2 lds[];
  constexpr int C = R1 / L;
  const int ldr = dm.ldr, ft = dm.ft, nt = dm.ntheta, mg = dm.mg;
  const int slab = ft * ldr;
  unsigned long long* slots = reinterpret_cast<unsigned long long*>(lds);   // [nt][ft][ldr]
  float2* twl = lds + (size_t)nt * slab;                                    // [mg]
  float2* sc = twl + mg;                                                    // [nt]: (scale, 1/scale)
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int b = tile / dm.nftile;
  const int f0 = (tile - b * dm.nftile) * ft;
  const int* bp = tb.bin_ptr + (size_t)b * (nt + 1);
  const int c0 = bp[0], ntr = bp[nt] - bp[0];
  for (int i = threadIdx.x; i < nt * slab; i += NT) slots[i] = 0ull;
  for (int i = threadIdx.x; i < mg; i += NT) twl[i] = tb.tw_grid[i];
  for (int i = threadIdx.x; i < nt; i += NT) {
    const float v = slice_scale[(size_t)b * nt + i];
    sc[i] = make_float2(v, 1.0f / v);
  }
  __syncthreads();

  const int ld = dm.ldr;
  const int gpt = ft >= kFptS ? ft / kFptS : 1;
  const int gpl = ft >= kFptS ? ftl - kFptSLog : 0;
  for (int it = threadIdx.x; it < ntr * gpt; it += NT) {
    const int n = c0 + (it >> gpl);
    const unsigned f1 = (unsigned)((f0 & ~(kFptS - 1)) + (it & (gpt - 1)) * kFptS);
    const int fl0 = (int)f1 - f0;
    if (f1 >= (unsigned)dm.nf) continue;
    const int j = tb.tr_bin[n];
    const int j1 = j + 1 == nt ? 0 : j + 1;
    const float2* src = dhat + (size_t)tb.tr_row[n] * dm.nf + f1;
    float2 dv[kFptS];
#pragma unroll
    for (int k = 0; k < kFptS; ++k)
      dv[k] = (fl0 + k >= 0 && fl0 + k < ft && f1 + k < (unsigned)dm.nf) ? src[k] : make_float2(0.f, 0.f);
    const unsigned long long bfix = tb.tr_b[n];
    unsigned long long tt = fix_mul(f1, bfix);
    const float2 r = tb.tr_rot[n];
    const float2 rot = make_float2(r.x, -r.y);
    float2 pre = pre_phase<1>(f1, tb.tr_a[n]);
    const float alpha = tb.tr_alpha[n];
    const float sh = alpha * sc[j1].x, sl = (1.0f - alpha) * sc[j].x;
    unsigned long long* lo = slots + __umul24((unsigned)j, (unsigned)slab);
    unsigned long long* hi = slots + __umul24((unsigned)j1, (unsigned)slab);
#pragma unroll
    for (int k = 0; k < kFptS; ++k) {
      if (fl0 + k >= 0 && fl0 + k < ft && f1 + k < (unsigned)dm.nf) {
        const float2 sv = cmul(dv[k], pre);
        const KernelPoint kp = kernel_point<W>((unsigned)(tt >> 32), R1 * L);
        const float2 s1 = cscale(sv, sh);
        const float2 s0 = cscale(sv, sl);
        unsigned long long* g0 = lo + __umul24((unsigned)(fl0 + k), (unsigned)ld) + kp.base;
        unsigned long long* g1 = hi + __umul24((unsigned)(fl0 + k), (unsigned)ld) + kp.base;
        float ph[W];
        kernel_taps<W, POLY>(kp.z0, dm.cbeta, ph);
#pragma unroll
        for (int tp = 0; tp < W; ++tp) {
          atomicAdd(g0 + tp, pack_fix(ph[tp] * s0.x, ph[tp] * s0.y));
          atomicAdd(g1 + tp, pack_fix(ph[tp] * s1.x, ph[tp] * s1.y));
        }
      }
      pre = cmul(pre, rot);
      tt += bfix;
    }
  }
  __syncthreads();

  const int t = threadIdx.x % L;
  float2* mdst = mhat + (size_t)b * nt * dm.nq * dm.nf;
  const unsigned qn = (unsigned)dm.nq * (unsigned)dm.nf;
  for (int row = threadIdx.x / L; row < nt * ft; row += NT / L) {
    const int s = row >> ftl, fl = row & (ft - 1);
    const int f = f0 + fl;
    unsigned long long* cell = slots + (size_t)row * ldr;
    const float inv = sc[s].y;
    float2 v[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      const int m = t + L * r;
      unsigned long long c = cell[m];
      if (m < W - 1) c += cell[mg + m];
      v[r] = unpack_fix(c, inv);
    }
    row_dft_lanes<R1, L, true>(v, t, reinterpret_cast<float2*>(cell), twl);
    if (f < dm.nf) {
      float2* dst = mdst + (size_t)s * qn + f;
#pragma unroll
      for (int i = 0; i < C; ++i) {
#pragma unroll
        for (int k2 = 0; k2 < L; ++k2) {
          const int l = kept_mode_row<R1, L, HALF>(t, i, k2, dm);
          if (l >= 0) dst[__umul24((unsigned)l, (unsigned)dm.nf)] = v[i * L + k2];
        }
      }
    }
  }
}

// ------------------------------------------------------------------ launchers
// Lane split of the q-grid transform by grid length (64 = 8 x 8, 128 = 16 x 8, 256 = 16 x 16)
// and kernel taps by polynomial for widths of 5 and more at the sigma = 2 shape.
template <int W, int R1, int L, int NT, bool HALF>
static hipError_t launch_interp_res_w(const Plan& p, const Dims& dm, const float2* mhat, float2* dhat,
                                      hipStream_t s) {
  const size_t lds = res_lds_f2(dm.ft, dm.ldr, dm.ntheta, dm.mg) * sizeof(float2);
  const dim3 grid((unsigned)dm.batch * dm.nftile), block(NT);
  const int ftl = ilog2(dm.ft);
  if constexpr (W >= 5) {
    if (dm.poly) {
      hipError_t e = set_lds(k_nufft_interp_res<W, R1, L, true, NT, HALF>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_nufft_interp_res<W, R1, L, true, NT, HALF>), grid, block, lds, s, mhat, dhat, p.tb, dm, ftl);
      return hipGetLastError();
    }
  }
  hipError_t e = set_lds(k_nufft_interp_res<W, R1, L, false, NT, HALF>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_nufft_interp_res<W, R1, L, false, NT, HALF>), grid, block, lds, s, mhat, dhat, p.tb, dm, ftl);
  return hipGetLastError();
}

template <int W, int R1, int L, int NT, bool HALF>
static hipError_t launch_spread_res_w(const Plan& p, const Dims& dm, const float2* dhat, const float* slice_scale,
                                      float2* mhat, hipStream_t s) {
  const size_t lds = res_lds_f2(dm.ft, dm.ldr, dm.ntheta, dm.mg) * sizeof(float2) + dm.ntheta * sizeof(float2);
  const dim3 grid((unsigned)dm.batch * dm.nftile), block(NT);
  const int ftl = ilog2(dm.ft);
  if constexpr (W >= 5) {
    if (dm.poly) {
      hipError_t e = set_lds(k_nufft_spread_res<W, R1, L, true, NT, HALF>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_nufft_spread_res<W, R1, L, true, NT, HALF>), grid, block, lds, s, dhat, slice_scale, mhat, p.tb,
                         dm, ftl);
      return hipGetLastError();
    }
  }
  hipError_t e = set_lds(k_nufft_spread_res<W, R1, L, false, NT, HALF>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_nufft_spread_res<W, R1, L, false, NT, HALF>), grid, block, lds, s, dhat, slice_scale, mhat, p.tb,
                     dm, ftl);
  return hipGetLastError();
}

template <int W, int R1, int L, int NT>
static hipError_t interp_res_half(const Plan& p, const Dims& dm, const float2* mhat, float2* dhat, hipStream_t s) {
  if (2 * dm.nq == R1 * L && dm.nq % 2 == 0) return launch_interp_res_w<W, R1, L, NT, true>(p, dm, mhat, dhat, s);
  return launch_interp_res_w<W, R1, L, NT, false>(p, dm, mhat, dhat, s);
}

template <int W, int R1, int L, int NT>
static hipError_t spread_res_half(const Plan& p, const Dims& dm, const float2* dhat, const float* slice_scale,
                                  float2* mhat, hipStream_t s) {
  if (2 * dm.nq == R1 * L && dm.nq % 2 == 0)
    return launch_spread_res_w<W, R1, L, NT, true>(p, dm, dhat, slice_scale, mhat, s);
  return launch_spread_res_w<W, R1, L, NT, false>(p, dm, dhat, slice_scale, mhat, s);
}

template <int W, int NT>
static hipError_t interp_res_mg(const Plan& p, const Dims& dm, const float2* mhat, float2* dhat, hipStream_t s) {
  if (dm.mg == 64) return interp_res_half<W, 8, 8, NT>(p, dm, mhat, dhat, s);
  if (dm.mg == 128) return interp_res_half<W, 16, 8, NT>(p, dm, mhat, dhat, s);
  if (dm.mg == 256) return interp_res_half<W, 16, 16, NT>(p, dm, mhat, dhat, s);
  return hipErrorInvalidValue;
}

template <int W, int NT>
static hipError_t spread_res_mg(const Plan& p, const Dims& dm, const float2* dhat, const float* slice_scale,
                                float2* mhat, hipStream_t s) {
  if (dm.mg == 64) return spread_res_half<W, 8, 8, NT>(p, dm, dhat, slice_scale, mhat, s);
  if (dm.mg == 128) return spread_res_half<W, 16, 8, NT>(p, dm, dhat, slice_scale, mhat, s);
  if (dm.mg == 256) return spread_res_half<W, 16, 16, NT>(p, dm, dhat, slice_scale, mhat, s);
  return hipErrorInvalidValue;
}

// Workgroups of 512, 768 or 1024 threads (dm.bsz): the larger ones keep more wavefronts per
// CU when the tile's slices take most of the LDS.
template <int W>
static hipError_t interp_res_bs(const Plan& p, const Dims& dm, const float2* mhat, float2* dhat, hipStream_t s) {
  if (dm.bsz == 512) return interp_res_mg<W, 512>(p, dm, mhat, dhat, s);
  if (dm.bsz == 768) return interp_res_mg<W, 768>(p, dm, mhat, dhat, s);
  if (dm.bsz == 1024) return interp_res_mg<W, 1024>(p, dm, mhat, dhat, s);
  return hipErrorInvalidValue;
}

template <int W>
static hipError_t spread_res_bs(const Plan& p, const Dims& dm, const float2* dhat, const float* slice_scale,
                                float2* mhat, hipStream_t s) {
  if (dm.bsz == 512) return spread_res_mg<W, 512>(p, dm, dhat, slice_scale, mhat, s);
  if (dm.bsz == 768) return spread_res_mg<W, 768>(p, dm, dhat, slice_scale, mhat, s);
  if (dm.bsz == 1024) return spread_res_mg<W, 1024>(p, dm, dhat, slice_scale, mhat, s);
  return hipErrorInvalidValue;
}

hipError_t launch_interp_res(const Plan& p, const Dims& dm, const float2* mhat, float2* dhat, hipStream_t s) {
  switch (dm.w) {
#define AAHRT_CASE(WW) \
  case WW:             \
    return interp_res_bs<WW>(p, dm, mhat, dhat, s);
    AAHRT_W_CASES(AAHRT_CASE)
#undef AAHRT_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_spread_res(const Plan& p, const Dims& dm, const float2* dhat, const float* slice_scale,
                             float2* mhat, hipStream_t s) {
  switch (dm.w) {
#define AAHRT_CASE(WW) \
  case WW:             \
    return spread_res_bs<WW>(p, dm, dhat, slice_scale, mhat, s);
    AAHRT_W_CASES(AAHRT_CASE)
#undef AAHRT_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace aahrt
