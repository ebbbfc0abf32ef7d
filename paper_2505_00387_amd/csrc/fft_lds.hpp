// Batched complex FFTs in LDS: Stockham autosort, radices 2/3/4/5/8/9/15/16.
//
// A workgroup of NT threads transforms `nbatch` sequences of length n stored at
// buf + b*bstride.  Passes alternate between two LDS buffers (ping-pong), so a
// butterfly is loaded, transformed and stored without holding other
// butterflies in registers.  Twiddles come from a table tw[t] = exp(-2 pi i t/n)
// built in FP64 on the host; INV selects the +i sign (unnormalised inverse).
// Index arithmetic uses host-built multiply-shift division constants.
#pragma once

#include <hip/hip_runtime.h>

#include "aahrt_internal.hpp"

namespace aahrt {

__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward sign) or +i (inverse sign)
template <bool INV>
__host__ __device__ __forceinline__ float2 mul_i(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// multiply by exp(-+ i pi/4) and exp(-+ 3 i pi/4)
template <bool INV>
__host__ __device__ __forceinline__ float2 mul_w8(float2 a) {
  const float r = 0.70710678118654752440f;
  return INV ? make_float2(r * (a.x - a.y), r * (a.x + a.y)) : make_float2(r * (a.x + a.y), r * (a.y - a.x));
}
template <bool INV>
__host__ __device__ __forceinline__ float2 mul_w8_3(float2 a) {
  const float r = 0.70710678118654752440f;
  return INV ? make_float2(-r * (a.x + a.y), r * (a.x - a.y)) : make_float2(r * (a.y - a.x), -r * (a.x + a.y));
}

__device__ __forceinline__ unsigned fdiv(unsigned x, const FastDiv& d) {
  return d.d == 1 ? x : (__umulhi(x, d.m) + x) >> d.s;
}

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  __host__ __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<3, INV> {
  __host__ __device__ __forceinline__ static void run(float2* v) {
    const float s = 0.86602540378443864676f;
    float2 a = v[0];
    float2 s1 = cadd(v[1], v[2]);
    float2 s2 = csub(v[1], v[2]);
    float2 t = make_float2(a.x - 0.5f * s1.x, a.y - 0.5f * s1.y);
    float2 u = mul_i<INV>(cscale(s2, s));
    v[0] = cadd(a, s1);
    v[1] = cadd(t, u);
    v[2] = csub(t, u);
  }
};

template <bool INV>
struct Dft<4, INV> {
  __host__ __device__ __forceinline__ static void run(float2* v) {
    float2 s0 = cadd(v[0], v[2]), s1 = csub(v[0], v[2]);
    float2 s2 = cadd(v[1], v[3]), s3 = mul_i<INV>(csub(v[1], v[3]));
    v[0] = cadd(s0, s2);
    v[2] = csub(s0, s2);
    v[1] = cadd(s1, s3);
    v[3] = csub(s1, s3);
  }
};

template <bool INV>
struct Dft<5, INV> {
  __host__ __device__ __forceinline__ static void run(float2* v) {
    const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
    const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;
    float2 x0 = v[0];
    float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    float2 a1 = make_float2(x0.x + c1 * t1.x + c2 * t2.x, x0.y + c1 * t1.y + c2 * t2.y);
    float2 a2 = make_float2(x0.x + c2 * t1.x + c1 * t2.x, x0.y + c2 * t1.y + c1 * t2.y);
    float2 b1 = make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
    float2 b2 = make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
    float2 ib1 = mul_i<INV>(b1), ib2 = mul_i<INV>(b2);
    v[0] = make_float2(x0.x + t1.x + t2.x, x0.y + t1.y + t2.y);
    v[1] = cadd(a1, ib1);
    v[4] = csub(a1, ib1);
    v[2] = cadd(a2, ib2);
    v[3] = csub(a2, ib2);
  }
};

template <bool INV>
struct Dft<8, INV> {
  __host__ __device__ __forceinline__ static void run(float2* v) {
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    const float2 w1 = mul_w8<INV>(o[1]);
    const float2 w2 = mul_i<INV>(o[2]);
    const float2 w3 = mul_w8_3<INV>(o[3]);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], w1);
    v[5] = csub(e[1], w1);
    v[2] = cadd(e[2], w2);
    v[6] = csub(e[2], w2);
    v[3] = cadd(e[3], w3);
    v[7] = csub(e[3], w3);
  }
};

// 16 = 4 x 4: DFT-4 over stride-4 inputs, twiddles W16^(a k1), DFT-4 across.
template <bool INV>
struct Dft<16, INV> {
  __host__ __device__ __forceinline__ static void run(float2* v) {
    const float c = 0.92387953251128675613f, s = 0.38268343236508977173f;
    float2 sub[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
      for (int b = 0; b < 4; ++b) sub[a][b] = v[a + 4 * b];
      Dft<4, INV>::run(sub[a]);
    }
    // twiddle W16^(a*k1): a = 1: k1 = 1,2,3 -> W^1, W^2, W^3; a = 2: W^2, W^4, W^6; a = 3: W^3, W^6, W^9
    const float sg = INV ? 1.f : -1.f;
    const float2 w1 = make_float2(c, sg * s), w3 = make_float2(s, sg * c);
    sub[1][1] = cmul(sub[1][1], w1);
    sub[1][2] = mul_w8<INV>(sub[1][2]);
    sub[1][3] = cmul(sub[1][3], w3);
    sub[2][1] = mul_w8<INV>(sub[2][1]);
    sub[2][2] = mul_i<INV>(sub[2][2]);
    sub[2][3] = mul_w8_3<INV>(sub[2][3]);
    sub[3][1] = cmul(sub[3][1], w3);
    sub[3][2] = mul_w8_3<INV>(sub[3][2]);
    sub[3][3] = cmul(sub[3][3], make_float2(-c, -sg * s));  // W^9 = -W^1
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 t[4] = {sub[0][k1], sub[1][k1], sub[2][k1], sub[3][k1]};
      Dft<4, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
  }
};

// 9 = 3 x 3: DFT-3 over stride-3 inputs, twiddles W9^(a k1), DFT-3 across.
template <bool INV>
struct Dft<9, INV> {
  __host__ __device__ __forceinline__ static void run(float2* v) {
    const float c1 = 0.766044443118978f, s1 = 0.6427876096865393f;   // W9^1
    const float c2 = 0.17364817766693041f, s2 = 0.984807753012208f;  // W9^2
    const float c4 = -0.9396926207859083f, s4 = 0.3420201433256689f; // W9^4
    const float sg = INV ? 1.f : -1.f;
    float2 sub[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int b = 0; b < 3; ++b) sub[a][b] = v[a + 3 * b];
      Dft<3, INV>::run(sub[a]);
    }
    sub[1][1] = cmul(sub[1][1], make_float2(c1, sg * s1));
    sub[1][2] = cmul(sub[1][2], make_float2(c2, sg * s2));
    sub[2][1] = cmul(sub[2][1], make_float2(c2, sg * s2));
    sub[2][2] = cmul(sub[2][2], make_float2(c4, sg * s4));
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      float2 t[3] = {sub[0][k1], sub[1][k1], sub[2][k1]};
      Dft<3, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < 3; ++k2) v[k1 + 3 * k2] = t[k2];
    }
  }
};

// 15 = 3 x 5 by the prime-factor (Good-Thomas) map: inputs x[(5 n1 + 3 n2) mod 15],
// DFT-3 over n1, DFT-5 over n2, outputs X[(10 k1 + 6 k2) mod 15]; no twiddles.
template <bool INV>
struct Dft<15, INV> {
  __host__ __device__ __forceinline__ static void run(float2* v) {
    float2 a[3][5];
#pragma unroll
    for (int n2 = 0; n2 < 5; ++n2) {
      float2 t[3];
#pragma unroll
      for (int n1 = 0; n1 < 3; ++n1) t[n1] = v[(5 * n1 + 3 * n2) % 15];
      Dft<3, INV>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 3; ++k1) a[k1][n2] = t[k1];
    }
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      Dft<5, INV>::run(a[k1]);
#pragma unroll
      for (int k2 = 0; k2 < 5; ++k2) v[(10 * k1 + 6 * k2) % 15] = a[k1][k2];
    }
  }
};

// Twiddles w^r = exp(-+2 pi i r k / (ns R)) for r = 1..R-1: w^1 and every w^(4a) are read
// from the table, the others are w^(4a) * w^b with b < 4 (at most three roundings).
template <int R, bool INV>
__device__ __forceinline__ void apply_twiddles(float2* v, const float2* __restrict__ tw, int step) {
  float2 w1 = tw[step];
  if (INV) w1.y = -w1.y;
  float2 wb[4];
  wb[0] = make_float2(1.f, 0.f);
  wb[1] = w1;
  wb[2] = cmul(w1, w1);
  wb[3] = cmul(wb[2], w1);
  float2 w4a = make_float2(1.f, 0.f);
#pragma unroll
  for (int r = 1; r < R; ++r) {
    if ((r & 3) == 0) {
      w4a = tw[r * step];
      if (INV) w4a.y = -w4a.y;
      v[r] = cmul(v[r], w4a);
    } else if (r < 4) {
      v[r] = cmul(v[r], wb[r]);
    } else {
      v[r] = cmul(v[r], cmul(w4a, wb[r & 3]));
    }
  }
}

// apply_twiddles with its table reads done ahead: base[0] = tw[step], base[a] = tw[4 a step].
template <int R, bool INV>
__device__ __forceinline__ void apply_twiddle_bases(float2* v, const float2* base) {
  float2 w1 = base[0];
  if (INV) w1.y = -w1.y;
  float2 wb[4];
  wb[0] = make_float2(1.f, 0.f);
  wb[1] = w1;
  wb[2] = cmul(w1, w1);
  wb[3] = cmul(wb[2], w1);
  float2 w4a = make_float2(1.f, 0.f);
#pragma unroll
  for (int r = 1; r < R; ++r) {
    if ((r & 3) == 0) {
      w4a = base[r >> 2];
      if (INV) w4a.y = -w4a.y;
      v[r] = cmul(v[r], w4a);
    } else if (r < 4) {
      v[r] = cmul(v[r], wb[r]);
    } else {
      v[r] = cmul(v[r], cmul(w4a, wb[r & 3]));
    }
  }
}
template <int R>
__host__ __device__ constexpr int twiddle_bases() {
  return 1 + (R - 1) / 4;
}

// Index of element i in a padded buffer: one spare cell after every 16, so
// the stride-R writes of a first pass (Ns = 1) spread over the LDS banks.
__host__ __device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }

// One out-of-place Stockham pass of radix R; PIN/POUT read/write padded buffers.
template <int R, bool INV, int NT, bool PIN, bool POUT>
__device__ __forceinline__ void fft_pass(const float2* __restrict__ src, float2* __restrict__ dst,
                                         const FftPass& ps, int nbatch, int bstride,
                                         const float2* __restrict__ tw) {
  const int nb = ps.nb;
  const int total = nb * nbatch;
  for (int b = threadIdx.x; b < total; b += NT) {
    int fb = 0, j = b;
    if (nbatch > 1) {
      fb = (int)fdiv((unsigned)b, ps.dnb);
      j = b - fb * nb;
    }
    const int jq = (int)fdiv((unsigned)j, ps.dns);
    const int k = j - jq * ps.ns;
    float2 v[R];
    const float2* x = src + fb * bstride;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = j + r * nb;
      v[r] = x[PIN ? pad16(i) : i];
    }
    if (ps.ns > 1) apply_twiddles<R, INV>(v, tw, k * ps.stride);
    Dft<R, INV>::run(v);
    float2* y = dst + fb * bstride;
    const int o = jq * ps.ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = o + r * ps.ns;
      y[POUT ? pad16(i) : i] = v[r];
    }
  }
  __syncthreads();
}

template <int R, bool INV, int NT>
__device__ __forceinline__ void fft_pass_sel(const float2* src, float2* dst, const FftPass& ps, int nbatch,
                                             int bstride, const float2* tw, int mode) {
  if (mode == 1) fft_pass<R, INV, NT, false, true>(src, dst, ps, nbatch, bstride, tw);
  else if (mode == 2) fft_pass<R, INV, NT, true, false>(src, dst, ps, nbatch, bstride, tw);
  else fft_pass<R, INV, NT, false, false>(src, dst, ps, nbatch, bstride, tw);
}

// Full transform of the data in `a` (the caller synchronises before calling).
// Returns the buffer (a or b) holding the result.  With two or more passes the
// first pass writes b padded (pad16) and the second reads it so; b must hold
// pad16(n - 1) + 1 cells per sequence.  Input and result are unpadded.
template <bool INV, int NT>
__device__ __forceinline__ float2* fft_lds(float2* a, float2* b, const FftPlan& pl, int nbatch, int bstride,
                           const float2* __restrict__ tw) {
  float2* src = a;
  float2* dst = b;
  for (int s = 0; s < pl.npass; ++s) {
    const FftPass& ps = pl.pass[s];
    const int mode = pl.npass < 2 ? 0 : (s == 0 ? 1 : (s == 1 ? 2 : 0));
    switch (ps.r) {
      case 2: fft_pass_sel<2, INV, NT>(src, dst, ps, nbatch, bstride, tw, mode); break;
      case 3: fft_pass_sel<3, INV, NT>(src, dst, ps, nbatch, bstride, tw, mode); break;
      case 4: fft_pass_sel<4, INV, NT>(src, dst, ps, nbatch, bstride, tw, mode); break;
      case 5: fft_pass_sel<5, INV, NT>(src, dst, ps, nbatch, bstride, tw, mode); break;
      case 8: fft_pass_sel<8, INV, NT>(src, dst, ps, nbatch, bstride, tw, mode); break;
      case 9: fft_pass_sel<9, INV, NT>(src, dst, ps, nbatch, bstride, tw, mode); break;
      case 15: fft_pass_sel<15, INV, NT>(src, dst, ps, nbatch, bstride, tw, mode); break;
      default: fft_pass_sel<16, INV, NT>(src, dst, ps, nbatch, bstride, tw, mode); break;
    }
    float2* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// In-place pass over nbatch sequences (stride bstride) whose butterflies, over all
// sequences, number at most NT: every thread reads its butterfly, the block
// synchronises, then writes it back to its Stockham output positions.  Needs half
// the LDS of the ping-pong form.
template <int R, bool INV, int NT, bool PIN, bool POUT>
__device__ __forceinline__ void fft_pass_ip(float2* buf, const FftPass& ps, int nbatch, int bstride,
                                            const float2* __restrict__ tw) {
  const int bt = threadIdx.x;
  const bool act = bt < ps.nb * nbatch;
  float2 v[R];
  int o = 0, fb = 0;
  if (act) {
    int j = bt;
    if (nbatch > 1) {
      fb = (int)fdiv((unsigned)bt, ps.dnb);
      j = bt - fb * ps.nb;
    }
    const int jq = (int)fdiv((unsigned)j, ps.dns);
    const int k = j - jq * ps.ns;
    const float2* x = buf + fb * bstride;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = j + r * ps.nb;
      v[r] = x[PIN ? pad16(i) : i];
    }
    if (ps.ns > 1) apply_twiddles<R, INV>(v, tw, k * ps.stride);
    Dft<R, INV>::run(v);
    o = jq * ps.ns * R + k;
  }
  __syncthreads();
  if (act) {
    float2* y = buf + fb * bstride;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = o + r * ps.ns;
      y[POUT ? pad16(i) : i] = v[r];
    }
  }
  __syncthreads();
}

template <int R, bool INV, int NT>
__device__ __forceinline__ void fft_pass_ip_sel(float2* buf, const FftPass& ps, int nbatch, int bstride,
                                                const float2* tw, int mode) {
  if (mode == 1) fft_pass_ip<R, INV, NT, false, true>(buf, ps, nbatch, bstride, tw);
  else if (mode == 2) fft_pass_ip<R, INV, NT, true, false>(buf, ps, nbatch, bstride, tw);
  else fft_pass_ip<R, INV, NT, false, false>(buf, ps, nbatch, bstride, tw);
}

// In-place transform of nbatch sequences at buf + b*bstride (every pass with at
// most NT butterflies in total; the caller synchronises before calling).  Each
// sequence holds pad16(n - 1) + 1 cells; input and result are unpadded.
template <bool INV, int NT>
__device__ __forceinline__ void fft_lds_ip(float2* buf, const FftPlan& pl, int nbatch, int bstride,
                                           const float2* __restrict__ tw) {
  for (int s = 0; s < pl.npass; ++s) {
    const FftPass& ps = pl.pass[s];
    const int mode = pl.npass < 2 ? 0 : (s == 0 ? 1 : (s == 1 ? 2 : 0));
    switch (ps.r) {
      case 2: fft_pass_ip_sel<2, INV, NT>(buf, ps, nbatch, bstride, tw, mode); break;
      case 3: fft_pass_ip_sel<3, INV, NT>(buf, ps, nbatch, bstride, tw, mode); break;
      case 4: fft_pass_ip_sel<4, INV, NT>(buf, ps, nbatch, bstride, tw, mode); break;
      case 5: fft_pass_ip_sel<5, INV, NT>(buf, ps, nbatch, bstride, tw, mode); break;
      case 8: fft_pass_ip_sel<8, INV, NT>(buf, ps, nbatch, bstride, tw, mode); break;
      case 9: fft_pass_ip_sel<9, INV, NT>(buf, ps, nbatch, bstride, tw, mode); break;
      case 15: fft_pass_ip_sel<15, INV, NT>(buf, ps, nbatch, bstride, tw, mode); break;
      default: fft_pass_ip_sel<16, INV, NT>(buf, ps, nbatch, bstride, tw, mode); break;
    }
  }
}

// In-place transform of one sequence of length N with radices Rs... fixed at compile time:
// the pass of fft_lds_ip with every count, stride and divisor a constant, so the index
// arithmetic folds into LDS offsets.  Same butterflies and twiddle products as
// fft_lds_ip, hence the same results.  Passes with a multiple of 16 between the
// elements of a butterfly address the padded buffer as pad16(first) + r * (step + step/16).
// HALF: inputs at and past N/2 of a forward transform are zero, outputs at and past N/2 of
// an inverse transform are not needed: in the first forward pass the elements r with
// r NB >= N/2 are not loaded (zero), in the last inverse pass those with r NS >= N/2 are
// not stored, and the arithmetic feeding only them disappears.
template <bool INV, int NT, int N, int NPASS, int S, int NS, bool HALF, int R, int... Rest>
__device__ __forceinline__ void fft_static(float2* buf, const float2* twb) {
  constexpr int NB = N / R;
  constexpr bool PIN = NPASS >= 2 && S == 1;
  constexpr bool POUT = NPASS >= 2 && S == 0;
  constexpr bool ZIN = HALF && !INV && S == 0;            // first pass of a forward transform
  constexpr bool DROP = HALF && INV && S == NPASS - 1;    // last pass of an inverse transform
  static_assert(NB <= NT && N % R == 0, "one butterfly per thread");
  const int j = threadIdx.x;
  const bool act = NB == NT || j < NB;
  float2 v[R];
  int o = 0;
  if (act) {
    const int jq = j / NS;
    const int k = j - jq * NS;
    if constexpr (PIN && NB % 16 == 0) {
      const float2* x = buf + pad16(j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = x[r * (NB + NB / 16)];
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = j + r * NB;
        v[r] = (ZIN && r * NB >= N / 2) ? make_float2(0.f, 0.f) : buf[PIN ? pad16(i) : i];
      }
    }
    if constexpr (NS > 1) apply_twiddle_bases<R, INV>(v, twb);
    Dft<R, INV>::run(v);
    o = jq * NS * R + k;
  }
  __syncthreads();
  if (act) {
    if constexpr (POUT && NS == 1 && R == 16) {
      float2* y = buf + 17 * j;  // o = 16 j: pad16(o + r) = 17 j + r
#pragma unroll
      for (int r = 0; r < R; ++r) y[r] = v[r];
    } else if constexpr (POUT && NS % 16 == 0) {
      float2* y = buf + pad16(o);
#pragma unroll
      for (int r = 0; r < R; ++r) y[r * (NS + NS / 16)] = v[r];
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = o + r * NS;
        if (!(DROP && r * NS >= N / 2)) buf[POUT ? pad16(i) : i] = v[r];
      }
    }
  }
  __syncthreads();
  if constexpr (sizeof...(Rest) > 0)
    fft_static<INV, NT, N, NPASS, S + 1, NS * R, HALF, Rest...>(buf, twb + (NS > 1 ? twiddle_bases<R>() : 0));
}

template <int N, bool HALF, int... Rs>
struct RowPlan {};

template <int IP>
struct StaticRowPlan;
template <>
struct StaticRowPlan<3> {
  using type = RowPlan<2160, true, 16, 15, 9>;
};
template <>
struct StaticRowPlan<4> {
  using type = RowPlan<480, false, 16, 15, 2>;
};

// Twiddle bases of one thread for every pass of a compiled plan (the passes after the
// first), read from the table once, ahead of both transforms of a row kernel (the forward
// and inverse transforms use the same bases, conjugated for the inverse).
template <int N, int NS, int R, int... Rest>
__host__ __device__ constexpr int plan_bases() {
  constexpr int here = NS > 1 ? twiddle_bases<R>() : 0;
  if constexpr (sizeof...(Rest) > 0) return here + plan_bases<N, NS * R, Rest...>();
  else return here;
}

template <int N, int NS, int R, int... Rest>
__device__ __forceinline__ void load_plan_bases(float2* b, const float2* __restrict__ tw, int j) {
  if constexpr (NS > 1) {
    constexpr int NB = N / R, STRIDE = N / (NS * R);
    const int step = (j % NS) * STRIDE;
    const bool act = NB >= 256 || j < NB;  // 256 = kBlock, the threads of a row workgroup
#pragma unroll
    for (int a = 0; a < twiddle_bases<R>(); ++a) b[a] = act ? tw[(a == 0 ? 1 : 4 * a) * step] : make_float2(1.f, 0.f);
  }
  if constexpr (sizeof...(Rest) > 0) load_plan_bases<N, NS * R, Rest...>(b + (NS > 1 ? twiddle_bases<R>() : 0), tw, j);
}

template <typename P>
struct RowTwiddles;
template <int N, bool HALF, int... Rs>
struct RowTwiddles<RowPlan<N, HALF, Rs...>> {
  static constexpr int count = plan_bases<N, 1, Rs...>();
  float2 b[count > 0 ? count : 1];
  __device__ __forceinline__ void load(const float2* __restrict__ tw) {
    load_plan_bases<N, 1, Rs...>(b, tw, threadIdx.x);
  }
};

template <bool INV, int NT, int N, bool HALF, int... Rs>
__device__ __forceinline__ void fft_row_static(float2* buf, const RowTwiddles<RowPlan<N, HALF, Rs...>>& twb) {
  fft_static<INV, NT, N, (int)sizeof...(Rs), 0, 1, HALF, Rs...>(buf, twb.b);
}

// The compiled plans agree with the host's table.
template <int IP, int N, bool HALF, int... Rs>
constexpr bool static_row_matches(RowPlan<N, HALF, Rs...>) {
  constexpr int rs[] = {Rs...};
  const StaticRowSpec& sp = kStaticRows[IP - 3];
  if (sp.ip != IP || sp.n != N || sp.npass != (int)sizeof...(Rs) || sp.half != (HALF ? 1 : 0)) return false;
  for (int i = 0; i < (int)sizeof...(Rs); ++i)
    if (sp.r[i] != rs[i]) return false;
  return true;
}
static_assert(static_row_matches<3>(StaticRowPlan<3>::type{}) && static_row_matches<4>(StaticRowPlan<4>::type{}),
              "compiled row plans match kStaticRows");

// In-place pass of one sequence in which a thread owns K butterflies (j = thread + k NT).
// Level k reads and transforms butterfly k into registers of its own, then the next level
// runs; the innermost level synchronises the block, and each level writes on the way back.
template <int R, bool INV, int NT, bool PIN, bool POUT, int KK, int K>
__device__ __forceinline__ void fft_pass_ipk_level(float2* buf, const FftPass& ps, const float2* __restrict__ tw) {
  float2 v[R];
  const int j = threadIdx.x + KK * NT;
  const bool act = j < ps.nb;
  int o = 0;
  if (act) {
    const int jq = (int)fdiv((unsigned)j, ps.dns);
    const int k = j - jq * ps.ns;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = j + r * ps.nb;
      v[r] = buf[PIN ? pad16(i) : i];
    }
    if (ps.ns > 1) apply_twiddles<R, INV>(v, tw, k * ps.stride);
    Dft<R, INV>::run(v);
    o = jq * ps.ns * R + k;
  }
  if constexpr (KK + 1 < K) fft_pass_ipk_level<R, INV, NT, PIN, POUT, KK + 1, K>(buf, ps, tw);
  else __syncthreads();
  if (act) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = o + r * ps.ns;
      buf[POUT ? pad16(i) : i] = v[r];
    }
  }
}

template <int R, bool INV, int NT, bool PIN, bool POUT, int K>
__device__ __forceinline__ void fft_pass_ipk(float2* buf, const FftPass& ps, const float2* __restrict__ tw) {
  fft_pass_ipk_level<R, INV, NT, PIN, POUT, 0, K>(buf, ps, tw);
  __syncthreads();
}

template <int R, bool INV, int NT, bool PIN, bool POUT>
__device__ __forceinline__ void fft_pass_ipk_k(float2* buf, const FftPass& ps, const float2* tw) {
  const int K = (ps.nb + NT - 1) / NT;  // at most row_kmax(R), by the plan
  if (K <= 1) {
    fft_pass_ip<R, INV, NT, PIN, POUT>(buf, ps, 1, 0, tw);
    return;
  }
  if constexpr (row_kmax(R) >= 2) {
    if (K == 2) {
      fft_pass_ipk<R, INV, NT, PIN, POUT, 2>(buf, ps, tw);
      return;
    }
  }
  if constexpr (row_kmax(R) >= 3) {
    if (K == 3) {
      fft_pass_ipk<R, INV, NT, PIN, POUT, 3>(buf, ps, tw);
      return;
    }
  }
  if constexpr (row_kmax(R) >= 4) {
    if (K == 4) {
      fft_pass_ipk<R, INV, NT, PIN, POUT, 4>(buf, ps, tw);
      return;
    }
  }
  if constexpr (row_kmax(R) >= 5) fft_pass_ipk<R, INV, NT, PIN, POUT, 5>(buf, ps, tw);
}

template <int R, bool INV, int NT>
__device__ __forceinline__ void fft_pass_ipk_sel(float2* buf, const FftPass& ps, const float2* tw, int mode) {
  if (mode == 1) fft_pass_ipk_k<R, INV, NT, false, true>(buf, ps, tw);
  else if (mode == 2) fft_pass_ipk_k<R, INV, NT, true, false>(buf, ps, tw);
  else fft_pass_ipk_k<R, INV, NT, false, false>(buf, ps, tw);
}

// In-place transform of one sequence whose passes may have more butterflies than
// threads, up to row_kmax(radix) per thread (the plan guarantees it).
template <bool INV, int NT>
__device__ __forceinline__ void fft_lds_ipk(float2* buf, const FftPlan& pl, const float2* __restrict__ tw) {
  for (int s = 0; s < pl.npass; ++s) {
    const FftPass ps = pl.pass[s];  // by value: keeps the plan argument out of private memory
    const int mode = pl.npass < 2 ? 0 : (s == 0 ? 1 : (s == 1 ? 2 : 0));
    switch (ps.r) {
      case 2: fft_pass_ipk_sel<2, INV, NT>(buf, ps, tw, mode); break;
      case 3: fft_pass_ipk_sel<3, INV, NT>(buf, ps, tw, mode); break;
      case 4: fft_pass_ipk_sel<4, INV, NT>(buf, ps, tw, mode); break;
      case 5: fft_pass_ipk_sel<5, INV, NT>(buf, ps, tw, mode); break;
      case 8: fft_pass_ipk_sel<8, INV, NT>(buf, ps, tw, mode); break;
      case 9: fft_pass_ipk_sel<9, INV, NT>(buf, ps, tw, mode); break;
      case 15: fft_pass_ipk_sel<15, INV, NT>(buf, ps, tw, mode); break;
      default: fft_pass_ipk_sel<16, INV, NT>(buf, ps, tw, mode); break;
    }
  }
}

}  // namespace aahrt
