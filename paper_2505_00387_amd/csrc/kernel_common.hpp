// Device helpers and launch helpers shared by the kernel translation units: block
// reductions, the real-spectrum packing of the row transforms, the transposed stretch
// interpolation, the in-LDS row FFT and the row-kernel launcher.
#pragma once

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

// Stores of row outputs that no later step of the same kernel reads (spectra, model and data
// rows, the iterates): nontemporal, so that they do not displace the tables and inputs the
// other workgroups still read from L2 (1-4% faster row kernels).  The GFST kernels keep
// ordinary stores: theirs cover 32-64 bytes of a line and rely on L2 combining them.
typedef float v2f_nt __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_nt(float2* p, float2 x) {
  v2f_nt v;
  v.x = x.x;
  v.y = x.y;
  __builtin_nontemporal_store(v, reinterpret_cast<v2f_nt*>(p));
}
__device__ __forceinline__ void store_nt(float* p, float x) { __builtin_nontemporal_store(x, p); }

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
    store_nt(dst + k, X);
    mx = fmaxf(mx, fabsf(X.x) + fabsf(X.y));
  }
  return mx;
}

// Packed spectrum Z for the inverse real DFT of X[0..N/2-1] (Im X[0] and the
// Nyquist bin taken as zero): Z[k] = (X[k] + conj X[N/2-k]) + i e^{2 pi i k/N}(X[k] - conj X[N/2-k]).
__device__ __forceinline__ float2 packed_bin(float2 X, float2 Xm, float2 t) {
  const float2 Xc = make_float2(Xm.x, -Xm.y);
  const float2 Xe = cadd(X, Xc);
  const float2 Xo = cmul(csub(X, Xc), t);
  return make_float2(Xe.x - Xo.y, Xe.y + Xo.x);
}
__device__ __forceinline__ void load_packed_c2r(float2* buf, const float2* __restrict__ src,
                                                const Tables& tb, const Dims& dm) {
#pragma unroll 4
  for (int k = threadIdx.x; k < dm.nh; k += kBlock) {
    float2 X = src[k];
    float2 Xm = make_float2(0.f, 0.f);
    if (k == 0) X.y = 0.f;
    else Xm = src[dm.nh - k];
    float2 t = tb.tw_real[k];
    t.y = -t.y;
    buf[k] = packed_bin(X, Xm, t);
  }
}

// The same, with bins k and N/2 - k formed by one thread, so that each spectrum value and
// twiddle is read once (the twiddle of bin N/2 - k, exp(-2 pi i (N/2 - k)/N) = (-c, s), follows
// from that of bin k, (c, s)).  It measured faster in the data-side C2R kernel and slower in
// the model-side and fused kernels, which keep the form above.
__device__ __forceinline__ void load_packed_c2r_pairs(float2* buf, const float2* __restrict__ src,
                                                      const Tables& tb, const Dims& dm) {
#pragma unroll 2
  for (int k = threadIdx.x; 2 * k <= dm.nh; k += kBlock) {
    const int km = dm.nh - k;
    float2 X = src[k];
    const float2 Xm = k == 0 ? make_float2(0.f, 0.f) : src[km];
    if (k == 0) X.y = 0.f;
    const float2 t = tb.tw_real[k];
    buf[k] = packed_bin(X, Xm, make_float2(t.x, -t.y));
    if (k > 0 && km != k) buf[km] = packed_bin(Xm, X, make_float2(-t.x, -t.y));
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
  if (c - a <= 2) {
    // most outputs have at most two inputs: the same products in the same order, unmasked
    if (a < c) acc = fmaf(a < b ? w[a].y : w[a].x, x[a], acc);
    if (a + 1 < c) acc = fmaf(a + 1 < b ? w[a + 1].y : w[a + 1].x, x[a + 1], acc);
    return acc;
  }
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

// The same output from its record: one 16-byte load where at most two inputs reach it (the same
// products in the same order as above), the general gather otherwise.
__device__ __forceinline__ float lerp_transpose(int i, const LerpRec* __restrict__ rec, const int* __restrict__ start,
                                                const float2* __restrict__ w, const float* x) {
  const LerpRec r = rec[i];
  if (r.n < 0) return lerp_transpose(i, start, w, x);
  float acc = 0.f;
  if (r.n > 0) acc = fmaf(r.w0, x[r.a], acc);
  if (r.n > 1) acc = fmaf(r.w1, x[r.a + 1], acc);
  return acc;
}

// S^T output i as X_i + Y_{i-1}: X_j and Y_j sum the lower- and upper-tap weights of the inputs
// whose lower tap is j (those of [start[j], start[j+1])), so every input is read once.  The
// lanes of a wavefront hold consecutive outputs (i = threadIdx.x + k kBlock): Y_{i-1} comes
// from the lane before, and the first lane of the wavefront sums it itself.  All lanes of a
// wavefront that hold an output call this together.
static_assert(kBlock % 64 == 0, "row workgroups are whole wavefronts");
__device__ __forceinline__ float stretch_transpose(int i, const int* __restrict__ start, const float2* __restrict__ w,
                                                   const float* x) {
  const int b = start[i], c = start[i + 1];
  float xs = 0.f, ys = 0.f;
  for (int r = b; r < c; ++r) {
    const float2 wr = w[r];
    const float v = x[r];
    xs = fmaf(wr.x, v, xs);
    ys = fmaf(wr.y, v, ys);
  }
  float yp = __shfl_up(ys, 1);
  if ((threadIdx.x & 63) == 0) {
    yp = 0.f;
    if (i > 0)
      for (int r = start[i - 1]; r < b; ++r) yp = fmaf(w[r].y, x[r], yp);
  }
  return xs + yp;
}

// Pack x[r] = (U^T g)[r] (r < nts, zero beyond) as z[p] = x[2p] + i x[2p+1], i.e. x
// written in order over the floats of buf.  One output per thread and pass: the
// first outputs gather the most inputs (t' = t^2 is flat near t = 0).
__device__ __forceinline__ void pack_transpose(float2* buf, const float* g, const Tables& tb, int nts, int nh) {
  float* xf = reinterpret_cast<float*>(buf);
  for (int r = threadIdx.x; r < 2 * nh; r += kBlock)
    xf[r] = r < nts ? lerp_transpose(r, tb.u_rec, tb.u_start, tb.u_w, g) : 0.f;
}

// ------------------------------------------------------------------ model side
// Row kernels transform one row (or trace) per workgroup in LDS.  IP = true:
// one buffer of N/2 (padded) complex values, transformed in place, plus a
// staging area after it for a real input row; IP = false (long rows whose FFT
// passes have more butterflies than threads): two ping-pong buffers, the staged
// input row aliasing the second one before the first pass.
// Per-thread twiddle bases a row kernel loads at its start for the compiled plans (IP >= 3);
// nothing for the plans read at run time.
struct NoRowTwiddles {
  __device__ __forceinline__ void load(const float2*) {}
};
template <int IP>
struct RowTw {
  using type = NoRowTwiddles;
};
template <>
struct RowTw<3> {
  using type = RowTwiddles<StaticRowPlan<3>::type>;
};
template <>
struct RowTw<4> {
  using type = RowTwiddles<StaticRowPlan<4>::type>;
};
template <int IP>
__device__ __forceinline__ typename RowTw<IP>::type row_twiddles(const Tables& tb) {
  typename RowTw<IP>::type t;
  t.load(tb.tw_half);
  return t;
}

template <bool INV, int IP>
__device__ __forceinline__ float2* row_fft(float2* A, float2* B, const FftPlan& fp, const Tables& tb,
                                           const Dims& dm, const typename RowTw<IP>::type& twb) {
  if constexpr (IP >= 3) {
    fft_row_static<INV, kBlock>(A, twb);
    return A;
  } else if constexpr (IP == 1) {
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

// Transpose of steps 1-2: inverse real DFT (1/N, doubled positive bins), first
// nt' samples, times the deapodisation, then S^T.
template <int IP>
__device__ __forceinline__ const float* model_c2r_core(const float2* mhat, float2* A,
                                                       float2* B, const Tables& tb, const Dims& dm,
                                                       const FftPlan& fp, size_t rid,
                                                       const typename RowTw<IP>::type& twb) {
  load_packed_c2r(A, mhat + rid * dm.nf, tb, dm);
  __syncthreads();
  return reinterpret_cast<const float*>(row_fft<true, IP>(A, B, fp, tb, dm, twb));
}

// ------------------------------------------------------------------ launch helpers
inline int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

template <typename K>
hipError_t set_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// The five instantiations of a row kernel, indexed by Dims::row_ip.
template <typename K>
struct RowKernels {
  K k[kRowKinds];
};
template <typename K>
RowKernels<K> row_kernels(K k0, K k1, K k2, K k3, K k4) {
  return RowKernels<K>{{k0, k1, k2, k3, k4}};
}
// AAHRT_ROWK(k_data_c2r, true) -> the kernels k_data_c2r<IP, true> for IP = 0..4
#define AAHRT_ROWK(K, ...) \
  row_kernels(&K<0, ##__VA_ARGS__>, &K<1, ##__VA_ARGS__>, &K<2, ##__VA_ARGS__>, &K<3, ##__VA_ARGS__>, &K<4, ##__VA_ARGS__>)

// Launch one row kernel: in place (every FFT pass fits the block) with `stage` real samples
// of staging after the buffer, else the two-buffer form.
template <typename K, typename... Args>
hipError_t launch_row(const RowKernels<K>& ks, const Dims& dm, int stage, unsigned grid, hipStream_t s,
                      Args... args) {
  if (grid == 0) return hipSuccess;
  if (dm.row_ip < 0 || dm.row_ip >= kRowKinds) return hipErrorInvalidValue;
  const K k = ks.k[dm.row_ip];
  const size_t lds = dm.row_ip == 0 ? 2 * (size_t)dm.nhp * sizeof(float2)
                                    : ((size_t)dm.nhp + (size_t)(stage + 5) / 2) * sizeof(float2);  // staging + 4 spare
  hipError_t e = set_lds(k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kBlock), lds, s, args...);
  return hipGetLastError();
}

inline unsigned model_rows(const Dims& dm) { return (unsigned)((size_t)dm.batch * dm.ntheta * dm.nq); }

}  // namespace aahrt
