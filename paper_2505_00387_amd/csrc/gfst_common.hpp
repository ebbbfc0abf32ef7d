// Device helpers shared by the two forms of the GFST kernels (slice sweep, resident slices):
// fixed-point phases and kernel footprints, the centring pre-phase, the kernel taps, the
// fixed-point packing of the spreading, the sweep's q-grid build and its 16-bit grid cells.
#pragma once

#include <hip/hip_runtime.h>

#include "es_poly.hpp"
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

// Consecutive frequencies per thread in the GFST kernels.  A thread takes kFpt{I,S} neighbouring
// frequencies of one trace: the per-trace tables are read once for all of them, the grid
// position steps by the exact 64-bit increment b, and the pre-phase steps by the trace's
// rotation exp(-+2 pi i frac(a)) from one exact start (at most kFpt - 1 FP32 products).
// Interpolation takes one frequency per thread item (its loads and phase are cheap next to its
// latency-bound LDS reads; measured faster), spreading four.
constexpr int kFptILog = 0;
constexpr int kFptI = 1 << kFptILog;
constexpr int kFptSLog = 2;
constexpr int kFptS = 1 << kFptSLog;

// Thread runs start at multiples of the run length R: run g of a tile starting at f0 (ft >= R)
// begins at fb = f0 + g R; a tile narrower than a run lies inside the aligned run
// fb = f0 - f0 % R, of which only the tile's frequencies are active.  A frequency f thus always
// sits at position f % R of its run and gets the same arithmetic (phase started exactly at fb
// and stepped), so the tile changes no result.

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

// Kernel values at the W taps of a point whose first tap is at normalised distance z0.
// POLY (w >= 5 with the sigma = 2 shape): the per-tap polynomials of es_poly.hpp in
// y = 2x - 1, x = z0 w/2 - w/2 + 1 the point's fraction of a cell (Horner, literal
// coefficients); else the kernel itself (square root and exponential per tap).
template <int W, bool POLY>
__device__ __forceinline__ void kernel_taps(float z0, float cbeta, float (&ph)[W]) {
  if constexpr (POLY) {
    // taps t and W-1-t from the even and odd parts of one polynomial: E(y^2) +- y O(y^2)
    const float y = fmaf(z0, (float)W, 1.0f - (float)W);
    const float y2 = y * y;
#pragma unroll
    for (int t = 0; t < (W + 1) / 2; ++t) {
      float e = EsPoly<W>::e[t][0];
#pragma unroll
      for (int k = 1; k <= EsPoly<W>::DE; ++k) e = fmaf(e, y2, EsPoly<W>::e[t][k]);
      if (2 * t + 1 == W) {
        ph[t] = e;
      } else {
        float o = EsPoly<W>::o[t][0];
#pragma unroll
        for (int k = 1; k <= EsPoly<W>::DO; ++k) o = fmaf(o, y2, EsPoly<W>::o[t][k]);
        ph[t] = fmaf(y, o, e);
        ph[W - 1 - t] = fmaf(-y, o, e);
      }
    }
  } else {
#pragma unroll
    for (int t = 0; t < W; ++t) ph[t] = grid_tap<W>(fmaf((float)t, -2.0f / (float)W, z0), cbeta);
  }
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

inline size_t interp_lds_bytes(const Dims& dm) {
  return interp_lds_f2(dm.ft, dm.ldr, dm.ntheta, dm.mg, dm.gdt) * sizeof(float2);
}

inline size_t spread_lds_bytes(const Dims& dm) { return spread_lds_f2(dm.ft, dm.ldr, dm.mg) * sizeof(float2); }

#define AAHRT_W_CASES(MACRO) \
  MACRO(2) MACRO(3) MACRO(4) MACRO(5) MACRO(6) MACRO(7) MACRO(8) MACRO(9) MACRO(10) MACRO(11) MACRO(12)

// Launchers of the resident-slice kernels (gfst_res.hip); dm carries the launch's tile.
hipError_t launch_interp_res(const Plan& p, const Dims& dm, const float2* mhat, float2* dhat, hipStream_t s);
hipError_t launch_spread_res(const Plan& p, const Dims& dm, const float2* dhat, const float* slice_scale,
                             float2* mhat, hipStream_t s);

// Dims of a GFST launch with the kernel's own frequency tile.
inline Dims tile_dims(const Dims& d0, int ft, int bsz) {
  Dims dm = d0;
  dm.ft = ft;
  dm.bsz = bsz;
  dm.nftile = (dm.nf + ft - 1) / ft;
  return dm;
}


}  // namespace aahrt
