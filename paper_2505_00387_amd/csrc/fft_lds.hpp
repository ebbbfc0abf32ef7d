// Batched complex FFTs held in LDS, Stockham autosort, radices 2/3/4/5/8.
//
// One workgroup of kBlock threads transforms `nbatch` sequences of length n
// stored at buf + b*bstride.  Each pass loads every butterfly's R inputs into
// registers, synchronises, then writes the R outputs in autosort order, so a
// single LDS buffer is transformed in place.  Twiddles come from a table
// tw[t] = exp(-2 pi i t/n) built in FP64 on the host.  INV selects the sign
// +i (unnormalised inverse).
#pragma once

#include <hip/hip_runtime.h>

#include "aahrt_internal.hpp"

namespace aahrt {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward sign) or +i (inverse sign)
template <bool INV>
__device__ __forceinline__ float2 mul_i(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<3, INV> {
  __device__ __forceinline__ static void run(float2* v) {
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
  __device__ __forceinline__ static void run(float2* v) {
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
  __device__ __forceinline__ static void run(float2* v) {
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
  __device__ __forceinline__ static void run(float2* v) {
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    const float r = 0.70710678118654752440f;
    float2 o1 = o[1], o2 = o[2], o3 = o[3];
    float2 w1, w2, w3;
    if (!INV) {
      w1 = make_float2(r * (o1.x + o1.y), r * (o1.y - o1.x));
      w2 = make_float2(o2.y, -o2.x);
      w3 = make_float2(r * (o3.y - o3.x), -r * (o3.x + o3.y));
    } else {
      w1 = make_float2(r * (o1.x - o1.y), r * (o1.x + o1.y));
      w2 = make_float2(-o2.y, o2.x);
      w3 = make_float2(-r * (o3.x + o3.y), r * (o3.x - o3.y));
    }
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

// One Stockham pass of radix R; MAXB butterflies per thread at most.
template <int R, int MAXB, bool INV>
__device__ __forceinline__ void fft_pass(float2* buf, int n, int nbatch, int bstride, int Ns,
                                         const float2* __restrict__ tw) {
  const int nb = n / R;
  const int total = nb * nbatch;
  const int stride = n / (Ns * R);
  float2 v[MAXB][R];
  int jj[MAXB], bb[MAXB];
#pragma unroll
  for (int t = 0; t < MAXB; ++t) {
    const int b = threadIdx.x + t * kBlock;
    jj[t] = -1;
    bb[t] = 0;
    if (b < total) {
      const int fb = b / nb;
      const int j = b - fb * nb;
      jj[t] = j;
      bb[t] = fb;
      const float2* x = buf + fb * bstride + j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[t][r] = x[r * nb];
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < MAXB; ++t) {
    const int j = jj[t];
    if (j >= 0) {
      const int k = j % Ns;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[r * k * stride];
          if (INV) w.y = -w.y;
          v[t][r] = cmul(v[t][r], w);
        }
      }
      Dft<R, INV>::run(v[t]);
      float2* y = buf + bb[t] * bstride + (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) y[r * Ns] = v[t][r];
    }
  }
  __syncthreads();
}

template <int R, bool INV>
__device__ __forceinline__ void fft_pass_dispatch(float2* buf, int n, int nbatch, int bstride,
                                                  int Ns, const float2* tw) {
  const int total = (n / R) * nbatch;
  const int mb = (total + kBlock - 1) / kBlock;
  if (mb <= 1) fft_pass<R, 1, INV>(buf, n, nbatch, bstride, Ns, tw);
  else if (mb <= 2) fft_pass<R, 2, INV>(buf, n, nbatch, bstride, Ns, tw);
  else if (mb <= 4) fft_pass<R, 4, INV>(buf, n, nbatch, bstride, Ns, tw);
  else if constexpr (fft_max_bpt(R) >= 8) {
    if (mb <= 8) fft_pass<R, 8, INV>(buf, n, nbatch, bstride, Ns, tw);
    else if constexpr (fft_max_bpt(R) >= 16) fft_pass<R, 16, INV>(buf, n, nbatch, bstride, Ns, tw);
  }
}

// Full transform; the caller synchronises before the first pass.
template <bool INV>
__device__ void fft_lds(float2* buf, const FftPlan& pl, int nbatch, int bstride,
                        const float2* __restrict__ tw) {
  int Ns = 1;
  for (int s = 0; s < pl.nrad; ++s) {
    const int R = pl.rad[s];
    switch (R) {
      case 2: fft_pass_dispatch<2, INV>(buf, pl.n, nbatch, bstride, Ns, tw); break;
      case 3: fft_pass_dispatch<3, INV>(buf, pl.n, nbatch, bstride, Ns, tw); break;
      case 4: fft_pass_dispatch<4, INV>(buf, pl.n, nbatch, bstride, Ns, tw); break;
      case 5: fft_pass_dispatch<5, INV>(buf, pl.n, nbatch, bstride, Ns, tw); break;
      default: fft_pass_dispatch<8, INV>(buf, pl.n, nbatch, bstride, Ns, tw); break;
    }
    Ns *= R;
  }
}

}  // namespace aahrt
