// HIP kernels (gfx950) of step 3 of Algorithm 1 and its transpose, slice-sweep form: the
// per-frequency GFST map as a type-2 nonuniform FFT in q with the linear azimuth weights
// (k_nufft_interp) and the type-1 spreading that is its exact transpose (k_nufft_spread),
// with the launchers of both forms (the resident-slice form lives in gfst_res.hip).
#include <hip/hip_runtime.h>

#include "gfst_common.hpp"

namespace aahrt {

// Forward GFST map (type-2 nonuniform FFT in q plus the azimuth weights) for one
// gather and a tile of ft frequencies.  Two slots hold the q-grids of slices j
// and j+1 while bin j is interpolated; slice j+2 (mod ntheta, so slice 0 is
// built again for the last bin) then replaces slice j.
// Registers are capped for six waves per SIMD: with two 32-frequency slots (46 KB of LDS)
// three workgroups then fit a CU instead of two (measured 8-11% faster, same results).
template <int W, int GD, bool POLY>
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
  // thread items: kFptI consecutive frequencies of one trace (all ft when ft < kFptI)
  const int gpt = ft >= kFptI ? ft / kFptI : 1;
  const int gpl = ft >= kFptI ? ftl - kFptILog : 0;

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
      for (int it = threadIdx.x; it < cnt * gpt; it += kBlockG) {
        const int n = c0 + (it >> gpl);
        const unsigned f1 = (unsigned)((f0 & ~(kFptI - 1)) + (it & (gpt - 1)) * kFptI);
        const int fl0 = (int)f1 - f0;
        if (f1 >= (unsigned)dm.nf) continue;
        const unsigned long long bfix = tb.tr_b[n];
        unsigned long long t = fix_mul(f1, bfix);
        const float2 rot = tb.tr_rot[n];
        float2 pre = pre_phase<-1>(f1, tb.tr_a[n]);
        const float alpha = tb.tr_alpha[n];
        float2* dst = dhat + (size_t)tb.tr_row[n] * dm.nf + f1;
#pragma unroll
        for (int k = 0; k < kFptI; ++k) {
          if (fl0 + k >= 0 && fl0 + k < ft && f1 + k < (unsigned)dm.nf) {
            const KernelPoint kp = kernel_point<W>((unsigned)(t >> 32), dm.mg);
            const Cell* g0 = G0 + (fl0 + k) * ldr + kp.base;
            const Cell* g1 = G1 + (fl0 + k) * ldr + kp.base;
            float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
            float ph[W];
            kernel_taps<W, POLY>(kp.z0, dm.cbeta, ph);
#pragma unroll
            for (int tp = 0; tp < W; ++tp) {
              const float2 v0 = dec_cell<GD>(g0[tp]), v1 = dec_cell<GD>(g1[tp]);
              a0.x = fmaf(ph[tp], v0.x, a0.x);
              a0.y = fmaf(ph[tp], v0.y, a0.y);
              a1.x = fmaf(ph[tp], v1.x, a1.x);
              a1.y = fmaf(ph[tp], v1.y, a1.y);
            }
            const float2 v = make_float2(fmaf(alpha, a1.x - a0.x, a0.x), fmaf(alpha, a1.y - a0.y, a0.y));
            dst[k] = cmul(v, pre);
          }
          pre = cmul(pre, rot);
          t += bfix;
        }
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
template <int W, bool POLY, bool HAS_LO, bool HAS_HI>
__device__ __forceinline__ void spread_bin(unsigned long long* lo, unsigned long long* hi, int c_begin, int c_end,
                                           const float2* __restrict__ dhat, int f0, float S_lo,
                                           float S_hi, const Tables& tb, const Dims& dm, int ftl) {
  const int ldr = dm.ldr;
  const int ft = dm.ft;
  const int cnt = c_end - c_begin;
  const int gpt = ft >= kFptS ? ft / kFptS : 1;
  const int gpl = ft >= kFptS ? ftl - kFptSLog : 0;
  for (int it = threadIdx.x; it < cnt * gpt; it += kBlockG) {
    const int n = c_begin + (it >> gpl);
    const unsigned f1 = (unsigned)((f0 & ~(kFptS - 1)) + (it & (gpt - 1)) * kFptS);
    const int fl0 = (int)f1 - f0;
    if (f1 >= (unsigned)dm.nf) continue;
    const float2* src = dhat + (size_t)tb.tr_row[n] * dm.nf + f1;
    float2 dv[kFptS];
#pragma unroll
    for (int k = 0; k < kFptS; ++k)
      dv[k] = (fl0 + k >= 0 && fl0 + k < ft && f1 + k < (unsigned)dm.nf) ? src[k] : make_float2(0.f, 0.f);
    const unsigned long long bfix = tb.tr_b[n];
    unsigned long long t = fix_mul(f1, bfix);
    const float2 r = tb.tr_rot[n];
    const float2 rot = make_float2(r.x, -r.y);
    float2 pre = pre_phase<1>(f1, tb.tr_a[n]);
    const float alpha = tb.tr_alpha[n];
    const float sh = alpha * S_hi, sl = (1.0f - alpha) * S_lo;
#pragma unroll
    for (int k = 0; k < kFptS; ++k) {
      if (fl0 + k >= 0 && fl0 + k < ft && f1 + k < (unsigned)dm.nf) {
        const float2 sv = cmul(dv[k], pre);
        const KernelPoint kp = kernel_point<W>((unsigned)(t >> 32), dm.mg);
        const float2 s1 = cscale(sv, sh);
        const float2 s0 = cscale(sv, sl);
        unsigned long long* g0 = HAS_LO ? lo + (fl0 + k) * ldr + kp.base : nullptr;
        unsigned long long* g1 = HAS_HI ? hi + (fl0 + k) * ldr + kp.base : nullptr;
        float ph[W];
        kernel_taps<W, POLY>(kp.z0, dm.cbeta, ph);
#pragma unroll
        for (int tp = 0; tp < W; ++tp) {
          if (HAS_LO) atomicAdd(g0 + tp, pack_fix(ph[tp] * s0.x, ph[tp] * s0.y));
          if (HAS_HI) atomicAdd(g1 + tp, pack_fix(ph[tp] * s1.x, ph[tp] * s1.y));
        }
      }
      pre = cmul(pre, rot);
      t += bfix;
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
template <int W, bool POLY>
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
      spread_bin<W, POLY, false, true>(lo, hi, bp[bin], bp[bin + 1], dhat, f0, S_prev, S_hi, tb, dm, ftl);
    else if (step == last + 1)
      spread_bin<W, POLY, true, false>(lo, hi, bp[bin], bp[bin + 1], dhat, f0, S_prev, S_hi, tb, dm, ftl);
    else
      spread_bin<W, POLY, true, true>(lo, hi, bp[bin], bp[bin + 1], dhat, f0, S_prev, S_hi, tb, dm, ftl);
    if (step >= 1)
      finish_slot<W>(lo, mb + (size_t)(step - 1) * slice_stride, f0, 1.0f / S_prev, twl, dm, fpg, ftl);
    S_prev = S_hi;
  }
}

// ------------------------------------------------------------------ launchers
// Kernel taps by polynomial for widths of 5 and more at the sigma = 2 shape, else by the kernel.
template <int W, int GD>
static hipError_t launch_interp_w(const Plan& p, const Dims& dm, const float2* mhat, float2* dhat, hipStream_t s) {
  const size_t lds = interp_lds_bytes(dm);
  const dim3 grid((unsigned)dm.batch * dm.nftile), block(kBlockG);
  const int ftl = ilog2(dm.ft);
  if constexpr (W >= 5) {
    if (dm.poly) {
      hipError_t e = set_lds(k_nufft_interp<W, GD, true>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_nufft_interp<W, GD, true>), grid, block, lds, s, mhat, dhat, p.tb, dm, p.fft_grid, ftl);
      return hipGetLastError();
    }
  }
  hipError_t e = set_lds(k_nufft_interp<W, GD, false>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_nufft_interp<W, GD, false>), grid, block, lds, s, mhat, dhat, p.tb, dm, p.fft_grid, ftl);
  return hipGetLastError();
}

template <int W>
static hipError_t launch_spread_w(const Plan& p, const Dims& dm, const float2* dhat, const float* slice_scale,
                                  float2* mhat, hipStream_t s) {
  const size_t lds = spread_lds_bytes(dm);
  const dim3 grid((unsigned)dm.batch * dm.nftile), block(kBlockG);
  const int ftl = ilog2(dm.ft);
  if constexpr (W >= 5) {
    if (dm.poly) {
      hipError_t e = set_lds(k_nufft_spread<W, true>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_nufft_spread<W, true>), grid, block, lds, s, dhat, slice_scale, mhat, p.tb, dm, p.fft_grid,
                         ftl);
      return hipGetLastError();
    }
  }
  hipError_t e = set_lds(k_nufft_spread<W, false>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_nufft_spread<W, false>), grid, block, lds, s, dhat, slice_scale, mhat, p.tb, dm, p.fft_grid, ftl);
  return hipGetLastError();
}

hipError_t launch_nufft_interp(const Plan& p, const float2* mhat, float2* dhat, hipStream_t s) {
  const Dims dm = tile_dims(p.dm, p.ft_interp, p.bs_interp);
  if (dm.ntr == 0) return hipSuccess;
  if (dm.res) return launch_interp_res(p, dm, mhat, dhat, s);
  switch (dm.w) {
#define AAHRT_CASE(WW)                                                                         \
  case WW:                                                                                     \
    if (dm.gdt == AAHRT_GRID_F16) return launch_interp_w<WW, AAHRT_GRID_F16>(p, dm, mhat, dhat, s);   \
    if (dm.gdt == AAHRT_GRID_BF16) return launch_interp_w<WW, AAHRT_GRID_BF16>(p, dm, mhat, dhat, s); \
    return launch_interp_w<WW, AAHRT_GRID_F32>(p, dm, mhat, dhat, s);
    AAHRT_W_CASES(AAHRT_CASE)
#undef AAHRT_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_nufft_spread(const Plan& p, const float2* dhat, const float* tr_bound, float* slice_scale,
                               float2* mhat, hipStream_t s) {
  const Dims dm = tile_dims(p.dm, p.ft_spread, p.bs_spread);
  hipLaunchKernelGGL(k_slice_scales, dim3((unsigned)dm.batch * dm.ntheta), dim3(kBlock), 0, s, tr_bound, p.tb,
                     dm.ntheta, slice_scale);
  if (dm.res) return launch_spread_res(p, dm, dhat, slice_scale, mhat, s);
  switch (dm.w) {
#define AAHRT_CASE(WW) \
  case WW:             \
    return launch_spread_w<WW>(p, dm, dhat, slice_scale, mhat, s);
    AAHRT_W_CASES(AAHRT_CASE)
#undef AAHRT_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace aahrt
