// HIP kernels (gfx950) of step 3 of Algorithm 1 and its transpose: the per-frequency GFST
// map as a type-2 nonuniform FFT in q with the linear azimuth weights (k_nufft_interp), and
// the type-1 spreading that is its exact transpose (k_nufft_spread), with their launchers.
#include <hip/hip_runtime.h>

#include "kernel_common.hpp"

namespace aahrt {

// ------------------------------------------------------------------ GFST stage
// Each workgroup owns one gather b and a tile of ft consecutive frequencies.
// The oversampled q-grid of one azimuth slice for all ft frequencies lives in
// LDS as ft rows of ldr complex cells: mg grid cells, then w-1 ghost cells that
// repeat the first w-1 cells (periodic extension, so a kernel footprint never
// wraps), then padding to an odd row length (rows of one access fall in
// distinct LDS banks).  Slices are visited in azimuth order; traces are grouped
// by their lower azimuth bin j_n, so bin j needs slices j and j+1 (mod ntheta).
// The (trace, frequency) items of a bin run with the frequency fastest across
// threads, kFpt consecutive frequencies per thread; the per-trace tables are read
// straight from memory (the lanes of one trace share the cache line), so a bin needs
// no barrier of its own.
//
// Phases use 0.64 fixed point: frac(f b) for an integer frequency index f is the
// wrapped 64-bit product, of which only the top 32 bits are formed
// (f * b_hi + umulhi(f, b_lo)); the grid position u = mg * frac(f b) keeps 32
// fractional bits before its conversion to FP32.

struct KernelPoint {
  int base;   // first grid cell of the footprint, in [0, mg)
  float z0;   // 2 d0 / w, d0 = distance from the point to the first cell
};

// frac(f b) of a 0.64 fixed-point b for an integer frequency index f: the wrapped 64-bit
// product f b, formed from 32-bit multiplies.
__device__ __forceinline__ unsigned long long fix_mul(unsigned f, unsigned long long bfix) {
  const unsigned lo = f * (unsigned)bfix;
  const unsigned hi = f * (unsigned)(bfix >> 32) + __umulhi(f, (unsigned)bfix);
  return ((unsigned long long)hi << 32) | lo;
}

// Footprint of the point at grid position u = mg frac(f b), from the top 32 bits t32 of
// the 0.64 phase (32 fractional bits of u are kept before the FP32 fraction is taken).
template <int W>
__device__ __forceinline__ KernelPoint kernel_point(unsigned t32, int mg) {
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

// Consecutive frequencies per thread in the GFST kernels.  A thread takes kFpt neighbouring
// frequencies of one trace: the per-trace tables are read once for all of them, the grid
// position steps by the exact 64-bit increment b, and the pre-phase steps by the trace's
// rotation exp(-+2 pi i frac(a)) from one exact start (at most kFpt - 1 FP32 products).
constexpr int kFpt = 4;

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
  // thread items: kFpt consecutive frequencies of one trace (all ft when ft < kFpt)
  const int fpt = ft >= kFpt ? kFpt : ft;
  const int gpt = ft / fpt;
  const int gpl = ft >= kFpt ? ftl - 2 : 0;

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
        const int fl0 = (it & (gpt - 1)) * fpt;
        const unsigned f1 = (unsigned)(f0 + fl0);
        if (f1 >= (unsigned)dm.nf) continue;
        const unsigned long long bfix = tb.tr_b[n];
        unsigned long long t = fix_mul(f1, bfix);
        float2 pre = pre_phase<-1>(f1, tb.tr_a[n]);
        const float2 rot = tb.tr_rot[n];
        const float alpha = tb.tr_alpha[n];
        float2* dst = dhat + (size_t)tb.tr_row[n] * dm.nf + f1;
#pragma unroll
        for (int k = 0; k < kFpt; ++k) {
          if (k < fpt && f1 + k < (unsigned)dm.nf) {
            const KernelPoint kp = kernel_point<W>((unsigned)(t >> 32), dm.mg);
            const Cell* g0 = G0 + (fl0 + k) * ldr + kp.base;
            const Cell* g1 = G1 + (fl0 + k) * ldr + kp.base;
            float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
#pragma unroll
            for (int tp = 0; tp < W; ++tp) {
              const float ph = grid_tap<W>(fmaf((float)tp, -2.0f / (float)W, kp.z0), dm.cbeta);
              const float2 v0 = dec_cell<GD>(g0[tp]), v1 = dec_cell<GD>(g1[tp]);
              a0.x = fmaf(ph, v0.x, a0.x);
              a0.y = fmaf(ph, v0.y, a0.y);
              a1.x = fmaf(ph, v1.x, a1.x);
              a1.y = fmaf(ph, v1.y, a1.y);
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

// Type-1 spreading accumulates in LDS in fixed point: a complex contribution c
// is added as one 64-bit integer round(S Re c) + 2^32 round(S Im c).  Integer
// addition is exact and order independent (deterministic results), and the
// two 32-bit fields can be read back exactly while each partial sum stays
// below 2^31 in magnitude, which the scale guarantees.  Each azimuth slice s
// has its own scale S_s = 0.99 (2^31 - 1)/B_s, where B_s sums, over the only
// traces that reach the slice (bin s with weight 1 - alpha, bin s-1 mod ntheta
// with weight alpha), the weight times max_f (|Re Dh| + |Im Dh|) of the trace:
// an upper bound of every cell sum of the slice, the kernel being <= 1.
//
// The rounding is floor(x + 1/2) (one v_cvt_rpi_i32_f32), and the sign extension of the low
// field is folded into the high field: (hi, lo) = (b + (a >> 31), a) is the 64-bit value
// sext(a) + 2^32 b.
__device__ __forceinline__ int round_half_up(float x) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

__device__ __forceinline__ unsigned long long pack_fix(float x, float y) {
  const int a = round_half_up(x), b = round_half_up(y);
  const unsigned hi = (unsigned)b + (unsigned)(a >> 31);
  return ((unsigned long long)hi << 32) | (unsigned)a;
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
  const int fpt = ft >= kFpt ? kFpt : ft;
  const int gpt = ft / fpt;
  const int gpl = ft >= kFpt ? ftl - 2 : 0;
  for (int it = threadIdx.x; it < cnt * gpt; it += kBlockG) {
    const int n = c_begin + (it >> gpl);
    const int fl0 = (it & (gpt - 1)) * fpt;
    const unsigned f1 = (unsigned)(f0 + fl0);
    if (f1 >= (unsigned)dm.nf) continue;
    const float2* src = dhat + (size_t)tb.tr_row[n] * dm.nf + f1;
    float2 dv[kFpt];
#pragma unroll
    for (int k = 0; k < kFpt; ++k)
      dv[k] = (k < fpt && f1 + k < (unsigned)dm.nf) ? src[k] : make_float2(0.f, 0.f);
    const unsigned long long bfix = tb.tr_b[n];
    unsigned long long t = fix_mul(f1, bfix);
    float2 pre = pre_phase<1>(f1, tb.tr_a[n]);
    const float2 r = tb.tr_rot[n];
    const float2 rot = make_float2(r.x, -r.y);
    const float alpha = tb.tr_alpha[n];
    const float sh = alpha * S_hi, sl = (1.0f - alpha) * S_lo;
#pragma unroll
    for (int k = 0; k < kFpt; ++k) {
      if (k < fpt && f1 + k < (unsigned)dm.nf) {
        const float2 sv = cmul(dv[k], pre);
        const KernelPoint kp = kernel_point<W>((unsigned)(t >> 32), dm.mg);
        const float2 s1 = cscale(sv, sh);
        const float2 s0 = cscale(sv, sl);
        unsigned long long* g0 = HAS_LO ? lo + (fl0 + k) * ldr + kp.base : nullptr;
        unsigned long long* g1 = HAS_HI ? hi + (fl0 + k) * ldr + kp.base : nullptr;
#pragma unroll
        for (int tp = 0; tp < W; ++tp) {
          const float ph = grid_tap<W>(fmaf((float)tp, -2.0f / (float)W, kp.z0), dm.cbeta);
          if (HAS_LO) atomicAdd(g0 + tp, pack_fix(ph * s0.x, ph * s0.y));
          if (HAS_HI) atomicAdd(g1 + tp, pack_fix(ph * s1.x, ph * s1.y));
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

// ------------------------------------------------------------------ launchers
static size_t interp_lds_bytes(const Dims& dm) {
  return interp_lds_f2(dm.ft, dm.ldr, dm.ntheta, dm.mg, dm.gdt) * sizeof(float2);
}

static size_t spread_lds_bytes(const Dims& dm) { return spread_lds_f2(dm.ft, dm.ldr, dm.mg) * sizeof(float2); }

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

hipError_t launch_nufft_spread(const Plan& p, const float2* dhat, const float* tr_bound, float* slice_scale,
                               float2* mhat, hipStream_t s) {
  const Dims dm = tile_dims(p.dm, p.ft_spread);
  const size_t lds = spread_lds_bytes(dm);
  const dim3 grid((unsigned)dm.batch * dm.nftile), block(kBlockG);
  const int ftl = ilog2(dm.ft);
  hipLaunchKernelGGL(k_slice_scales, dim3((unsigned)dm.batch * dm.ntheta), dim3(kBlock), 0, s, tr_bound, p.tb,
                     dm.ntheta, slice_scale);
  switch (dm.w) {
#define AAHRT_CASE(WW)                                                                       \
  case WW: {                                                                                 \
    hipError_t e = set_lds(k_nufft_spread<WW>, lds);                                         \
    if (e != hipSuccess) return e;                                                           \
    hipLaunchKernelGGL(k_nufft_spread<WW>, grid, block, lds, s, dhat, slice_scale, mhat,   \
                       p.tb, dm, p.fft_grid, ftl);                                           \
    break;                                                                                   \
  }
    AAHRT_W_CASES(AAHRT_CASE)
#undef AAHRT_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace aahrt
