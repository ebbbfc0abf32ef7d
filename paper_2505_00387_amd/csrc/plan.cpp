// Host side of the library: parameter validation, FP64 plan tables, device
// allocation, and the C ABI entry points declared in include/aahrt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <vector>

#include "aahrt_internal.hpp"

namespace aahrt {
hipError_t launch_objective(const Plan& p, const float* rss, const int64_t* trace_ptr_dev,
                            const float* l1, const float* lam, float* out, hipStream_t s);
}

using namespace aahrt;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(AAHRT_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)

bool smooth235(long n) {
  if (n <= 0) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

int next_smooth_even(long n) {
  if (n < 2) n = 2;
  while (!(n % 2 == 0 && smooth235(n))) ++n;
  return (int)n;
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// exponential-of-semicircle kernel in grid units, support |t| <= w/2
double es_kernel_host(double t, int w, double beta) {
  double z = 2.0 * t / w;
  double q = 1.0 - z * z;
  if (q < 0.0) q = 0.0;
  return std::exp(beta * (std::sqrt(q) - 1.0));
}

// Phi(xi) = integral of phi(t) exp(i xi t) dt = 2 int_0^{w/2} phi(t) cos(xi t) dt
double es_transform(double xi, int w, double beta) {
  static thread_local std::vector<double> gx, gw;
  if (gx.empty()) gauss_legendre(256, gx, gw);
  const double h = 0.25 * w;  // [0, w/2] mapped from [-1, 1]
  double s = 0.0;
  for (size_t i = 0; i < gx.size(); ++i) {
    const double t = h * (gx[i] + 1.0);
    s += gw[i] * es_kernel_host(t, w, beta) * std::cos(xi * t);
  }
  return 2.0 * h * s;
}

uint64_t to_fix64(double v) {
  double f = v - std::floor(v);
  if (!(f >= 0.0) || f >= 1.0) f = 0.0;
  const double s = f * 4294967296.0;
  const double hi = std::floor(s);
  const double lo = std::floor((s - hi) * 4294967296.0);
  return ((uint64_t)hi << 32) | (uint64_t)lo;
}

FastDiv make_fastdiv(unsigned d) {
  FastDiv f{1u, 0u, 0u};
  if (d <= 1) return f;
  unsigned s = 0;
  while ((1u << s) < d) ++s;
  f.d = d;
  f.s = s;
  f.m = (unsigned)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
  return f;
}

// Radix schedule for a length-n Stockham FFT, fewest passes first: 16s, then 15 and 9,
// then 8/4/2, 5, 3.
bool make_fft_plan(int n, FftPlan& pl) {
  pl.n = n;
  pl.npass = 0;
  int m = n;
  int ns = 1;
  while (m > 1) {
    int R = 0;
    if (m % 16 == 0) R = 16;
    else if (m % 15 == 0) R = 15;
    else if (m % 9 == 0) R = 9;
    else if (m % 8 == 0) R = 8;
    else if (m % 4 == 0) R = 4;
    else if (m % 2 == 0) R = 2;
    else if (m % 5 == 0) R = 5;
    else if (m % 3 == 0) R = 3;
    if (R == 0 || pl.npass >= kMaxPasses) return false;
    FftPass& ps = pl.pass[pl.npass++];
    ps.r = R;
    ps.nb = n / R;
    ps.ns = ns;
    ps.stride = n / (ns * R);
    ps.dnb = make_fastdiv((unsigned)ps.nb);
    ps.dns = make_fastdiv((unsigned)ps.ns);
    ns *= R;
    m /= R;
  }
  return true;
}

// Fill the passes of a plan for a given radix order.
void fill_fft_plan(int n, const std::vector<int>& radices, FftPlan& pl) {
  pl.n = n;
  pl.npass = (int)radices.size();
  int ns = 1;
  for (int i = 0; i < pl.npass; ++i) {
    FftPass& ps = pl.pass[i];
    const int R = radices[i];
    ps.r = R;
    ps.nb = n / R;
    ps.ns = ns;
    ps.stride = n / (ns * R);
    ps.dnb = make_fastdiv((unsigned)ps.nb);
    ps.dns = make_fastdiv((unsigned)ps.ns);
    ns *= R;
  }
}

// Radix order of the q-grid transform, which runs in place (one butterfly per thread
// per pass over all rows): the fewest butterflies in the busiest pass, then the fewest
// passes; ties keep the order of make_fft_plan.
bool make_grid_fft_plan(int n, FftPlan& pl) {
  if (!make_fft_plan(n, pl)) return false;
  int best_nb = 0;
  for (int i = 0; i < pl.npass; ++i) best_nb = std::max(best_nb, pl.pass[i].nb);
  int best_np = pl.npass;
  std::vector<int> best, cur;
  const int radices[] = {16, 15, 9, 8, 5, 4, 3, 2};
  std::function<void(int)> search = [&](int m) {
    if ((int)cur.size() > kMaxPasses) return;
    if (m == 1) {
      int mx = 0;
      for (int r : cur) mx = std::max(mx, n / r);
      if (mx < best_nb || (mx == best_nb && (int)cur.size() < best_np)) {
        best_nb = mx;
        best_np = (int)cur.size();
        best = cur;
      }
      return;
    }
    for (int r : radices)
      if (m % r == 0) {
        cur.push_back(r);
        search(m / r);
        cur.pop_back();
      }
  };
  search(n);
  if (!best.empty()) fill_fft_plan(n, best, pl);
  return true;
}

// Row transforms run in place when every pass fits the threads of a row workgroup:
// 1 = one butterfly per thread, 2 = up to row_kmax(radix) per thread, 0 = ping-pong.
int row_plan_kind(const FftPlan& pl) {
  int kind = 1;
  for (int i = 0; i < pl.npass; ++i) {
    const int k = (pl.pass[i].nb + kBlock - 1) / kBlock;
    if (k > row_kmax(pl.pass[i].r)) return 0;
    if (k > 1) kind = 2;
  }
  return kind;
}

// A radix order for a long row transform that runs in place: the fewest passes, then the
// fewest butterflies per thread in the busiest pass.  False if there is none.
bool make_row_fft_plan(int n, FftPlan& pl) {
  std::vector<int> best, cur;
  int best_np = kMaxPasses + 1, best_k = 1 << 30;
  const int radices[] = {16, 15, 9, 8, 5, 4, 3, 2};
  std::function<void(int)> search = [&](int m) {
    if ((int)cur.size() >= best_np && m > 1) return;
    if (m == 1) {
      int kmax = 0;
      for (int r : cur) kmax = std::max(kmax, (n / r + kBlock - 1) / kBlock);
      if ((int)cur.size() < best_np || kmax < best_k) {
        best_np = (int)cur.size();
        best_k = kmax;
        best = cur;
      }
      return;
    }
    for (int r : radices)
      if (m % r == 0 && (n / r + kBlock - 1) / kBlock <= row_kmax(r)) {
        cur.push_back(r);
        search(m / r);
        cur.pop_back();
      }
  };
  search(n);
  if (best.empty()) return false;
  fill_fft_plan(n, best, pl);
  return true;
}

template <typename T>
int upload(Plan& p, const std::vector<T>& h, const T** out) {
  void* d = nullptr;
  const size_t bytes = std::max<size_t>(h.size(), 1) * sizeof(T);
  if (hipMalloc(&d, bytes) != hipSuccess) return fail(AAHRT_E_NOMEM, "hipMalloc of a plan table failed");
  p.allocations.push_back(d);
  if (!h.empty()) HIP_TRY(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  *out = static_cast<const T*>(d);
  return AAHRT_OK;
}

template <typename T>
int alloc(Plan& p, size_t count, T** out) {
  void* d = nullptr;
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  if (hipMalloc(&d, bytes) != hipSuccess)
    return fail(AAHRT_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " workspace bytes failed");
  p.allocations.push_back(d);
  p.workspace_bytes += bytes;
  *out = static_cast<T*>(d);
  return AAHRT_OK;
}

#define TRY(expr)              \
  do {                         \
    int rc_ = (expr);          \
    if (rc_ != AAHRT_OK) {     \
      return rc_;              \
    }                          \
  } while (0)

void free_plan(Plan* p) {
  if (!p) return;
  if (p->wav_dev) (void)hipFree(p->wav_dev);
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (void* a : p->allocations) (void)hipFree(a);
  delete p;
}

int validate_params(const aahrt_params& q) {
  auto bad = [](const char* m) { return fail(AAHRT_E_INVALID, m); };
  if (q.nt < 2) return bad("nt must be >= 2");
  if (!(q.dt > 0.0) || !std::isfinite(q.dt)) return bad("dt must be finite and > 0");
  if (q.ntau < 1) return bad("ntau must be >= 1");
  if (!(q.dtau > 0.0) || !std::isfinite(q.dtau)) return bad("dtau must be finite and > 0");
  if (q.nq < 2) return bad("nq must be >= 2");
  if (!std::isfinite(q.q_min) || !std::isfinite(q.q_max) || !(q.q_min < q.q_max))
    return bad("need finite q_min < q_max");
  if (q.ntheta < 1) return bad("ntheta must be >= 1");
  if (q.stretch < 0 || q.stretch > 16) return bad("stretch must be in 0..16");
  const long nts = (long)(q.stretch == 0 ? 2 : q.stretch) * q.nt;
  if (q.nfft != 0 && (q.nfft < nts || q.nfft % 2 || !smooth235(q.nfft)))
    return bad("nfft must be 0 or even, 2^a3^b5^c and >= nt'");
  if (q.nufft_tol < 0.0 || !std::isfinite(q.nufft_tol)) return bad("nufft_tol must be >= 0");
  if (q.sigma != 0.0 && !(q.sigma >= 1.25 && q.sigma <= 4.0)) return bad("sigma must be 0 or in [1.25, 4]");
  if (q.kernel_width != 0 && (q.kernel_width < 2 || q.kernel_width > 12))
    return bad("kernel_width must be 0 or in 2..12");
  if (q.freq_tile != 0 && (q.freq_tile < 1 || q.freq_tile > 64 || (q.freq_tile & (q.freq_tile - 1))))
    return bad("freq_tile must be 0 or a power of two in 1..64");
  if (q.grid_dtype != AAHRT_GRID_F32 && q.grid_dtype != AAHRT_GRID_F16 && q.grid_dtype != AAHRT_GRID_BF16)
    return bad("grid_dtype must be 0, 1 or 2");
  if (q.gfst_kind < 0 || q.gfst_kind > 1) return bad("gfst_kind must be 0 or 1");
  if (q.block_threads != 0 && q.block_threads != 512 && q.block_threads != 768 && q.block_threads != 1024)
    return bad("block_threads must be 0, 512, 768 or 1024");
  if (q.freq_tile_adjoint != 0 &&
      (q.freq_tile_adjoint < 1 || q.freq_tile_adjoint > 64 || (q.freq_tile_adjoint & (q.freq_tile_adjoint - 1))))
    return bad("freq_tile_adjoint must be 0 or a power of two in 1..64");
  if (q.block_threads_adjoint != 0 && q.block_threads_adjoint != 512 && q.block_threads_adjoint != 768 &&
      q.block_threads_adjoint != 1024)
    return bad("block_threads_adjoint must be 0, 512, 768 or 1024");
  return AAHRT_OK;
}

// LDS bytes of the larger of the two GFST kernels for a tile of ft frequencies.
size_t grid_lds(int ft, int ldr, int ntheta, int mg, int gdt) {
  const size_t a = interp_lds_f2(ft, ldr, ntheta, mg, gdt), b = spread_lds_f2(ft, ldr, mg);
  return (a > b ? a : b) * sizeof(float2);
}

// One setting of the q nonuniform FFT: oversampled grid length mg (sigma = mg/nq),
// kernel width w, frequencies per GFST workgroup ft, and its estimated relative error.
struct NufftChoice {
  int mg, w, ft;
  double est;
  int res;  // 1: resident-slice kernels
  int bs;   // threads per workgroup (512, 768 or 1024 for the resident kernels, else kBlockG)
  bool fwd = true, adj = true;  // a setting the interpolation (fwd) / spreading (adj) kernel may take
};

// Per-output records of the transpose U^T from its start table and per-input weights:
// output i takes the inputs [start[i-1], start[i+1]), those below start[i] by their upper
// weight (.y) and the others by their lower one (.x).
std::vector<LerpRec> lerp_records(const std::vector<int>& start, const std::vector<float2>& w, int nout) {
  std::vector<LerpRec> rec(nout);
  for (int i = 0; i < nout; ++i) {
    const int b = start[i], c = start[i + 1], a = i > 0 ? start[i - 1] : b;
    LerpRec r{a, 0.f, 0.f, c - a <= 2 ? c - a : -1};
    if (r.n >= 1) r.w0 = a < b ? w[a].y : w[a].x;
    if (r.n >= 2) r.w1 = a + 1 < b ? w[a + 1].y : w[a + 1].x;
    rec[i] = r;
  }
  return rec;
}

// Shape parameter of the exponential-of-semicircle kernel, beta = 0.98 pi (1 - 1/(2 sigma)) w:
// the rule of Barnett, Magland and af Klinteberg (SIAM J. Sci. Comput. 41, 2019) for the
// width of the kernel's spectrum at oversampling sigma (2.31 w at sigma = 2).  Above
// sigma = 2 the sigma = 2 shape is kept: a larger grid only lowers its aliasing, the width
// rule measures the result, and the kernels then evaluate the taps by the per-tap
// polynomials fitted to that shape (es_poly.hpp).
double es_beta(double sigma, int w) {
  const double s = std::min(sigma, 2.0);
  return 0.98 * M_PI * (1.0 - 1.0 / (2.0 * s)) * w;
}

// Estimated relative error of one q nonuniform FFT (white mode coefficients) at grid length
// mg, kernel width w and shape beta, as the root sum of squares of two parts:
//  * truncation: mode k interpolated by the w kernel taps around a point d of a cell past a
//    grid node, deapodised, against the exact exponential.  It depends on d alone, so its
//    root mean square is taken over 32 offsets in [0, 1) and over (at most 256 of) the modes;
//  * FP32 rounding: the grid transform rounds relative to the grid's content, which the
//    deapodisation scales up towards the band edge, so this part grows with the ratio r of
//    its largest to smallest factor: 7e-8 (r + 5), fitted to an FP32 emulation of the
//    transform and the interpolation at nq = 32, 64 and 128 (within 20%).
double nufft_error_estimate(int nq, int mg, int w, double beta) {
  const int qh = nq / 2;
  const int kstep = std::max(1, nq / 256);
  std::vector<int> modes;
  for (int l = 0; l < nq; l += kstep) modes.push_back(l - qh);
  if (modes.back() != nq - 1 - qh) modes.push_back(nq - 1 - qh);
  std::vector<double> deap(modes.size());
  double dmin = 1e300, dmax = 0.0;
  for (size_t i = 0; i < modes.size(); ++i) {
    deap[i] = 1.0 / es_transform(2.0 * M_PI * modes[i] / mg, w, beta);
    dmin = std::min(dmin, std::fabs(deap[i]));
    dmax = std::max(dmax, std::fabs(deap[i]));
  }
  const int nd = 32;
  double acc = 0.0;
  for (int id = 0; id < nd; ++id) {
    const double d = (id + 0.5) / nd;
    const int off = (w % 2 == 0) ? -w / 2 : (d < 0.5 ? -(w + 1) / 2 : -(w - 1) / 2);
    for (size_t i = 0; i < modes.size(); ++i) {
      double re = 0.0, im = 0.0;
      for (int t = 0; t < w; ++t) {
        const int j = off + 1 + t;
        const double ph = es_kernel_host(d - j, w, beta);
        const double a = -2.0 * M_PI * modes[i] * j / mg;
        re += ph * std::cos(a);
        im += ph * std::sin(a);
      }
      const double a0 = -2.0 * M_PI * modes[i] * d / mg;
      const double er = re * deap[i] - std::cos(a0), ei = im * deap[i] - std::sin(a0);
      acc += er * er + ei * ei;
    }
  }
  const double trunc = std::sqrt(acc / (nd * (double)modes.size()));
  const double fp32 = 7e-8 * (dmax / dmin + 5.0);
  return std::sqrt(trunc * trunc + fp32 * fp32);
}

// Kernel width for a target error at grid length mg (mg grows to 2w when w needs it): the
// narrowest w in 3..12 whose estimate meets tol.  When none does, best is false and the
// width with the smallest estimate is returned.
void width_for(double tol, int nq, int mg0, int* w_out, int* mg_out, double* est_out, bool* best_out) {
  int bw = 12, bmg = mg0;
  double best = 1e300;
  for (int w = 3; w <= 12; ++w) {
    const int mg = std::max(mg0, next_smooth_even(2 * w));
    const double e = nufft_error_estimate(nq, mg, w, es_beta((double)mg / nq, w));
    if (e <= tol) {
      *w_out = w;
      *mg_out = mg;
      *est_out = e;
      *best_out = true;
      return;
    }
    if (e < best) { best = e; bw = w; bmg = mg; }
  }
  *w_out = bw;
  *mg_out = bmg;
  *est_out = best;
  *best_out = false;
}

// Row length of a q-grid slot: the ghost cells, and room for the padded first FFT pass.
int slot_row(int mg, int w) {
  int ldr = std::max(mg + w - 1, (mg - 1) + ((mg - 1) >> 4) + 1);
  return ldr % 2 == 0 ? ldr + 1 : ldr;
}

// Row length of the resident-slice layout: the ghost cells and the register transform's
// padded exchange (mg + L - 1 cells), odd.
int res_row(int mg, int w) {
  int ldr = std::max(mg + w - 1, mg + res_lanes(mg) - 1);
  return ldr % 2 == 0 ? ldr + 1 : ldr;
}

// The resident-slice kernels cover FP32 q-grids of 64, 128 or 256 cells whose slices for a
// tile of ft frequencies fit the LDS of a CU.
bool res_fits(const Dims& dm, int mg, int w, int ft) {
  if (dm.gdt != AAHRT_GRID_F32 || (mg != 64 && mg != 128 && mg != 256)) return false;
  const size_t bytes = res_lds_f2(ft, res_row(mg, w), dm.ntheta, mg) * sizeof(float2) + dm.ntheta * sizeof(float2);
  return bytes <= 160 * 1024;
}

// A setting fits when its LDS fits a CU, its coefficients fit the register prefetch, and
// every pass of the in-place q-grid transform has at most one butterfly per thread.
bool choice_fits(const Dims& dm, int mg, int w, int ft) {
  FftPlan fp;
  if (!make_grid_fft_plan(mg, fp)) return false;
  for (int i = 0; i < fp.npass; ++i)
    if ((long)fp.pass[i].nb * ft > kBlockG) return false;
  return grid_lds(ft, slot_row(mg, w), dm.ntheta, mg, dm.gdt) <= 160 * 1024 && dm.nq * ft <= kPrefetchCells;
}

// The (tile, workgroup) settings of one grid shape.  Each kernel takes its requested tile
// (freq_tile; for spreading freq_tile_adjoint when set), halved until it fits, or any of
// `free_ft` that fits, and its requested workgroup size (block_threads, block_threads_adjoint;
// the resident-slice kernels only) or any of 512, 768 and 1024.  A setting is listed once, marked
// with the kernels that may take it.
template <class Fits>
void add_tile_choices(const aahrt_params& prm, int mg, int w, double est, int res, const std::vector<int>& free_ft,
                      Fits fits, std::vector<NufftChoice>& out) {
  auto pinned = [&](int ft) {
    while (ft > 1 && !fits(ft)) ft /= 2;
    return fits(ft) ? ft : 0;
  };
  const int ft_f = prm.freq_tile != 0 ? pinned(prm.freq_tile) : -1;
  const int ft_a = prm.freq_tile_adjoint != 0 ? pinned(prm.freq_tile_adjoint) : ft_f;
  const int bs_f = res ? prm.block_threads : 0;
  const int bs_a = res ? (prm.block_threads_adjoint != 0 ? prm.block_threads_adjoint : prm.block_threads) : 0;
  std::vector<int> tiles;
  for (int ft : {ft_f, ft_a})
    if (ft > 0 && std::find(tiles.begin(), tiles.end(), ft) == tiles.end()) tiles.push_back(ft);
  if (ft_f < 0 || ft_a < 0)
    for (int ft : free_ft)
      if (fits(ft) && std::find(tiles.begin(), tiles.end(), ft) == tiles.end()) tiles.push_back(ft);
  const std::vector<int> sizes = res ? std::vector<int>{512, 768, 1024} : std::vector<int>{kBlockG};
  for (int ft : tiles) {
    for (int bs : sizes) {
      NufftChoice c{mg, w, ft, est, res, bs};
      c.fwd = (ft_f < 0 || ft == ft_f) && (bs_f == 0 || bs == bs_f);
      c.adj = (ft_a < 0 || ft == ft_a) && (bs_a == 0 || bs == bs_a);
      if (c.fwd || c.adj) out.push_back(c);
    }
  }
}

// Candidates: the requested sigma (or 2, 1.5 and 1.25 when it is free) with the narrowest
// width whose estimated error meets the tolerance (or the requested width), and the
// requested tile (or 4..32 when free).  A free sigma that no width brings within the
// tolerance is left out (in FP32 the deapodisation range of sigma = 1.25 holds it near 6e-6);
// a requested sigma, or the last one when all miss, keeps the width of smallest estimate.
// The first candidate is the default setting.
int nufft_candidates(const aahrt_params& prm, const Dims& dm, std::vector<NufftChoice>& out) {
  const double tol = prm.nufft_tol == 0.0 ? 1e-6 : prm.nufft_tol;
  if (dm.nq > kPrefetchCells) return fail(AAHRT_E_UNSUPPORTED, "nq too large for the q-coefficient prefetch");
  std::vector<double> sig;
  if (prm.sigma != 0.0) sig.push_back(prm.sigma);
  else sig = {2.0, 1.5, 1.25};
  const std::vector<int> fts = {16, 8, 32, 4};
  out.clear();
  std::vector<int> seen_mg;
  NufftChoice fallback{0, 0, 0, 1e300, 0, kBlockG};
  for (double sg : sig) {
    // (less a rounding margin, so that a sigma reported as mg/nq gives back mg)
    const int mg0 = next_smooth_even((long)std::ceil(sg * dm.nq - 1e-9));
    int w = prm.kernel_width, mg = mg0;
    double est = 0.0;
    if (w != 0) {
      if (mg < 2 * w) mg = next_smooth_even(2 * w);
      est = w == 2 ? 1.0 : nufft_error_estimate(dm.nq, mg, w, es_beta((double)mg / dm.nq, w));
    } else {
      bool meets = false;
      width_for(tol, dm.nq, mg0, &w, &mg, &est, &meets);
      if (!meets && prm.sigma == 0.0) {
        if (est < fallback.est) fallback = NufftChoice{mg, w, 0, est, 0, kBlockG};
        continue;
      }
    }
    if (std::find(seen_mg.begin(), seen_mg.end(), mg) != seen_mg.end()) continue;
    seen_mg.push_back(mg);
    FftPlan fp;
    if (!make_grid_fft_plan(mg, fp)) continue;
    // the resident-slice kernels where they apply (unless the sweep is requested), with
    // tiles of 4, 8, 2 or 1 frequencies in workgroups of 512, 768 or 1024 threads; otherwise the
    // slice sweep with tiles of 4..32
    const bool res = prm.gfst_kind != 1 && res_fits(dm, mg, w, 1);
    if (res) {
      add_tile_choices(prm, mg, w, est, 1, {4, 8, 2, 1}, [&](int ft) { return res_fits(dm, mg, w, ft); }, out);
      continue;
    }
    const size_t before = out.size();
    add_tile_choices(prm, mg, w, est, 0, fts, [&](int ft) { return choice_fits(dm, mg, w, ft); }, out);
    if (out.size() == before) {
      int ft = 16;
      while (ft > 1 && !choice_fits(dm, mg, w, ft)) ft /= 2;
      if (choice_fits(dm, mg, w, ft)) out.push_back({mg, w, ft, est, 0, kBlockG});
    }
  }
  if (out.empty() && fallback.mg != 0) {
    // no free sigma meets the tolerance: the setting with the smallest estimate
    add_tile_choices(prm, fallback.mg, fallback.w, fallback.est, 0, {16},
                     [&](int ft) { return choice_fits(dm, fallback.mg, fallback.w, ft); }, out);
  }
  if (out.empty()) return fail(AAHRT_E_UNSUPPORTED, "q-grid too large for LDS");
  return AAHRT_OK;
}

// Make one candidate current: grid dimensions, kernel shape, q-grid FFT plan, and
// the device deapodisation and q-grid twiddle tables.
int set_nufft(Plan& P, const NufftChoice& c) {
  Dims& dm = P.dm;
  if (!make_grid_fft_plan(c.mg, P.fft_grid)) return fail(AAHRT_E_UNSUPPORTED, "q-grid length not 5-smooth");
  dm.mg = c.mg;
  dm.w = c.w;
  P.sigma = (double)c.mg / dm.nq;
  P.nufft_est = c.est;
  const double beta = es_beta(P.sigma, c.w);
  dm.beta = (float)beta;
  dm.cbeta = (float)(beta / std::log(2.0));
  dm.res = c.res;
  dm.poly = (P.sigma >= 2.0 && c.w >= 5) ? 1 : 0;
  dm.ldr = c.res ? res_row(c.mg, c.w) : slot_row(c.mg, c.w);
  dm.qhalf = dm.nq / 2;
  dm.ft = c.ft;
  dm.nftile = (dm.nf + c.ft - 1) / c.ft;
  P.ft_interp = c.ft;
  P.ft_spread = c.ft;
  P.bs_interp = c.bs;
  P.bs_spread = c.bs;
  dm.bsz = c.bs;
  // deapodisation 1/Phi(2 pi k/mg) of mode k = l - nq/2
  std::vector<float> deapod(dm.nq);
  for (int l = 0; l < dm.nq; ++l) {
    const int k = l - dm.qhalf;
    // w = 2: the paper's linear interpolation in k, which it applies without correction
    deapod[l] = c.w == 2 ? 1.0f : (float)(1.0 / es_transform(2.0 * M_PI * k / c.mg, c.w, beta));
  }
  std::vector<float2> tw_grid(c.mg);
  for (int t = 0; t < c.mg; ++t) {
    const double a = -2.0 * M_PI * t / c.mg;
    tw_grid[t] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  HIP_TRY(hipMemcpy(P.deapod_dev, deapod.data(), deapod.size() * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(P.twgrid_dev, tw_grid.data(), tw_grid.size() * sizeof(float2), hipMemcpyHostToDevice));
  return AAHRT_OK;
}

// Time the GFST stage for every candidate, on zeroed spectra: the interpolation
// and the spreading kernels are timed separately, each keeps its fastest tile for
// a given oversampling, and the oversampling with the smallest sum is kept (the first,
// default one unless another is at least 5% faster).  The
// oversamplings give the same result to within the tolerance; the tiles change no
// result.
int autotune_nufft(Plan& P, const std::vector<NufftChoice>& cands) {
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t s = nullptr;
  HIP_TRY(hipStreamCreate(&s));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = AAHRT_OK;
  // time one kernel (0: interpolation, 1: spreading): a warm-up launch, then 1 or 3 timed
  auto run = [&](int which, float* ms) -> int {
    for (int pass = 0; pass < 2; ++pass) {
      const int reps = pass == 0 ? 1 : (*ms > 25.f ? 1 : 3);
      HIP_TRY(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) {
        if (which == 0) HIP_TRY(launch_nufft_interp(P, P.mhat, P.dhat, s));
        else HIP_TRY(launch_nufft_spread(P, P.dhat, P.tr_bound, P.slice_scale, P.mhat, s));
      }
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      HIP_TRY(hipEventElapsedTime(ms, e0, e1));
      *ms /= reps;
    }
    return AAHRT_OK;
  };
  NufftChoice best{0, 0, 0, 0.0, 0, kBlockG};
  int best_fi = 0, best_fs = 0, best_bi = kBlockG, best_bs = kBlockG;
  float best_total = 0.f, default_total = 0.f;
  do {
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      rc = fail(AAHRT_E_HIP, "hipEventCreate failed");
      break;
    }
    const size_t rows = (size_t)P.dm.batch * P.dm.ntheta * P.dm.nq;
    if (launch_fill(reinterpret_cast<float*>(P.mhat), 0.f, 2 * rows * P.dm.nf, s) != hipSuccess ||
        launch_fill(reinterpret_cast<float*>(P.dhat), 0.f, 2 * (size_t)P.dm.ntr * P.dm.nf, s) != hipSuccess ||
        launch_fill(P.tr_bound, 1.f, (size_t)P.dm.ntr, s) != hipSuccess) {
      rc = fail(AAHRT_E_HIP, "autotune fill failed");
      break;
    }
    for (size_t i = 0; i < cands.size() && rc == AAHRT_OK;) {
      // candidates of one oversampling are consecutive
      size_t j = i;
      float bi = 0.f, bs = 0.f;
      int fi = 0, fs = 0, ni = kBlockG, ns = kBlockG;
      bool have_i = false, have_s = false;
      for (; j < cands.size() && cands[j].mg == cands[i].mg && rc == AAHRT_OK; ++j) {
        if ((rc = set_nufft(P, cands[j])) != AAHRT_OK) break;
        float t = 0.f;
        if (cands[j].fwd) {
          if ((rc = run(0, &t)) != AAHRT_OK) break;
          P.tune_ms.push_back(t);
          if (!have_i || t < bi) { bi = t; fi = cands[j].ft; ni = cands[j].bs; have_i = true; }
        }
        if (cands[j].adj) {
          if ((rc = run(1, &t)) != AAHRT_OK) break;
          P.tune_ms.push_back(t);
          if (!have_s || t < bs) { bs = t; fs = cands[j].ft; ns = cands[j].bs; have_s = true; }
        }
      }
      if (rc != AAHRT_OK) break;
      // another oversampling (which changes results within the tolerance) replaces the
      // default only when it is at least 5% faster, so that timing noise rarely flips it
      if (i == 0) default_total = bi + bs;
      if (best.mg == 0 || (bi + bs < best_total && bi + bs < 0.95f * default_total)) {
        best = cands[i];
        best_fi = fi;
        best_fs = fs;
        best_bi = ni;
        best_bs = ns;
        best_total = bi + bs;
      }
      i = j;
    }
  } while (false);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  if (rc != AAHRT_OK) return rc;
  TRY(set_nufft(P, best));
  P.ft_interp = best_fi;
  P.ft_spread = best_fs;
  P.bs_interp = best_bi;
  P.bs_spread = best_bs;
  P.autotune_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return AAHRT_OK;
}

// One axis of a regular offset grid: the distinct values (closer than 1e-9 km count as one)
// must be v0 + i step, i = 0..count-1, to 1e-6 of the step.
static bool grid_axis(const double* v, int64_t lo, int64_t hi, double& v0, double& step, int& count) {
  std::vector<double> u(v + lo, v + hi);
  std::sort(u.begin(), u.end());
  std::vector<double> q;
  for (double a : u)
    if (q.empty() || a - q.back() > 1e-9) q.push_back(a);
  if (q.size() < 2) return false;
  step = (q.back() - q.front()) / (double)(q.size() - 1);
  if (!(step > 0.0)) return false;
  for (size_t i = 0; i < q.size(); ++i)
    if (std::fabs(q[i] - (q.front() + step * (double)i)) > 1e-6 * step) return false;
  v0 = q.front();
  count = (int)q.size();
  return true;
}

// Tables of Algorithm 2 (aahrt_adjoint_grid).  A plan whose gathers are not complete
// regular grids, or whose nq has a prime factor above 5, records why and keeps going.
int build_grid_tables(Plan& P, const int64_t* trace_ptr, const double* x, const double* y) {
  const Dims& dm = P.dm;
  const aahrt_params& prm = P.prm;
  P.grid_ok = false;
  if (!make_fft_plan(dm.nq, P.fft_q)) {
    P.grid_why = "nq must have no prime factor above 5 for the grid adjoint";
    return AAHRT_OK;
  }
  const int ld = (dm.nq - 1) + ((dm.nq - 1) >> 4) + 1;  // padded sequence stride of the LDS transform
  int ft = 16;
  while (ft > 1 && 2 * (size_t)ft * ld * sizeof(float2) > 65536) ft >>= 1;
  if (2 * (size_t)ft * ld * sizeof(float2) > 65536) {
    P.grid_why = "nq is too large for the grid adjoint";
    return AAHRT_OK;
  }
  P.grid_ft = ft;
  std::vector<GridGather> gg(dm.batch);
  std::vector<int> node;
  for (int b = 0; b < dm.batch; ++b) {
    const int64_t lo = trace_ptr[b], hi = trace_ptr[b + 1];
    GridGather G{0.0, 1.0, 0.0, 1.0, 0, 0, (int)node.size(), 0};
    if (hi > lo) {
      int mx = 0, my = 0;
      if (!grid_axis(x, lo, hi, G.x0, G.dx, mx) || !grid_axis(y, lo, hi, G.y0, G.dy, my) ||
          (int64_t)mx * my != hi - lo) {
        P.grid_why = "gather " + std::to_string(b) + " is not a complete regular offset grid";
        return AAHRT_OK;
      }
      G.mx = mx;
      G.my = my;
      node.resize(node.size() + (size_t)mx * my, -1);
      for (int64_t n = lo; n < hi; ++n) {
        const long m = std::lround((x[n] - G.x0) / G.dx);
        const long k = std::lround((y[n] - G.y0) / G.dy);
        const bool inside = m >= 0 && m < mx && k >= 0 && k < my;
        if (!inside || node[G.node0 + (size_t)m * my + k] >= 0) {
          P.grid_why = "gather " + std::to_string(b) + " does not fill its offset grid exactly once";
          return AAHRT_OK;
        }
        node[G.node0 + (size_t)m * my + k] = (int)n;
      }
    }
    gg[b] = G;
  }
  const double dts = P.dt_str;
  std::vector<Tap> dtap(dm.nts), vtap(dm.ntau);
  for (int r = 0; r < dm.nts; ++r) {
    const double pos = std::sqrt(r * dts) / prm.dt;
    const long i = (long)std::floor(pos);
    const double a = pos - (double)i;
    Tap t{0, 0, 0.f, 0.f};
    if (i >= 0 && i < dm.nt) { t.i0 = (int)i; t.w0 = (float)(1.0 - a); }
    if (i + 1 >= 0 && i + 1 < dm.nt) { t.i1 = (int)(i + 1); t.w1 = (float)a; }
    dtap[r] = t;
  }
  for (int i = 0; i < dm.ntau; ++i) {
    const double tau = i * prm.dtau;
    const double pos = tau * tau / dts;
    const long r = (long)std::floor(pos);
    const double a = pos - (double)r;
    Tap t{0, 0, 0.f, 0.f};
    if (r >= 0 && r < dm.nts) { t.i0 = (int)r; t.w0 = (float)(1.0 - a); }
    if (r + 1 >= 0 && r + 1 < dm.nts) { t.i1 = (int)(r + 1); t.w1 = (float)a; }
    vtap[i] = t;
  }
  const double dq = (prm.q_max - prm.q_min) / (prm.nq - 1);
  std::vector<double> kp(dm.nq);
  std::vector<float2> phase(dm.nq), tw(dm.nq);
  for (int p = 0; p < dm.nq; ++p) {
    const int ps = p < (dm.nq + 1) / 2 ? p : p - dm.nq;
    kp[p] = ps / (dm.nq * dq);
    // exp(2 pi i k_p q_min) with the revolutions reduced in FP64
    double rev = (double)ps * prm.q_min / (dm.nq * dq);
    rev -= std::floor(rev);
    phase[p] = make_float2((float)(std::cos(2.0 * M_PI * rev) / dm.nq), (float)(std::sin(2.0 * M_PI * rev) / dm.nq));
    tw[p] = make_float2((float)std::cos(-2.0 * M_PI * p / dm.nq), (float)std::sin(-2.0 * M_PI * p / dm.nq));
  }
  std::vector<double2> cs(dm.ntheta);
  for (int j = 0; j < dm.ntheta; ++j) {
    const double th = M_PI * j / dm.ntheta;
    cs[j] = make_double2(std::cos(th), std::sin(th));
  }
  const std::vector<float> one(1, 1.0f);
  GridTables& gt = P.gt;
  TRY(upload(P, dtap, &gt.dtap));
  TRY(upload(P, vtap, &gt.vtap));
  TRY(upload(P, one, &gt.one));
  TRY(upload(P, phase, &gt.phase));
  TRY(upload(P, tw, &gt.tw));
  TRY(upload(P, kp, &gt.kp));
  TRY(upload(P, cs, &gt.cs));
  TRY(upload(P, gg, &gt.g));
  TRY(upload(P, node, &gt.node));
  gt.fscale = 1.0 / ((double)dm.nfft * dts);
  P.grid_ok = true;
  return AAHRT_OK;
}

int build_plan(Plan& P, const aahrt_params& prm, int32_t batch, const int64_t* trace_ptr,
               const double* x, const double* y) {
  P.prm = prm;
  Dims& dm = P.dm;
  dm.batch = batch;
  P.trace_ptr.assign(trace_ptr, trace_ptr + batch + 1);
  const int64_t ntr64 = trace_ptr[batch];
  if (ntr64 > (int64_t)1 << 30) return fail(AAHRT_E_UNSUPPORTED, "too many traces");
  dm.ntr = (int)ntr64;
  dm.nt = prm.nt;
  dm.ntau = prm.ntau;
  dm.nq = prm.nq;
  dm.ntheta = prm.ntheta;
  const int K = prm.stretch == 0 ? 2 : prm.stretch;
  dm.nts = K * prm.nt;
  if (dm.nts < 2) return fail(AAHRT_E_INVALID, "nt' must be >= 2");
  const double T = (prm.nt - 1) * prm.dt;
  const double dts = T * T / (dm.nts - 1);
  P.dt_str = dts;

  double h2max = 0.0;
  for (int64_t n = 0; n < ntr64; ++n) h2max = std::max(h2max, x[n] * x[n] + y[n] * y[n]);
  if (prm.nfft == 0) {
    const double need = dm.nts + std::ceil(std::max(prm.q_max, 0.0) * h2max / dts) +
                        std::ceil(std::max(-prm.q_min, 0.0) * h2max / dts);
    if (need > 1 << 22) return fail(AAHRT_E_UNSUPPORTED, "required FFT length too large");
    dm.nfft = next_smooth_even((long)need);
  } else {
    if (prm.nfft < dm.nts || prm.nfft % 2 || !smooth235(prm.nfft))
      return fail(AAHRT_E_INVALID, "nfft must be even, 2^a3^b5^c and >= nt'");
    dm.nfft = prm.nfft;
  }
  dm.nh = dm.nfft / 2;
  dm.nf = dm.nh;
  dm.nhp = (dm.nh - 1) + ((dm.nh - 1) >> 4) + 1;
  if (!make_fft_plan(dm.nh, P.fft_half))
    return fail(AAHRT_E_UNSUPPORTED, "FFT length N/2 = " + std::to_string(dm.nh) + " exceeds the LDS FFT limits");
  // Rows whose passes exceed the threads stay ping-pong while its two buffers leave room
  // for four or more workgroups per CU; longer rows run in place with several butterflies
  // per thread (half the LDS), which measured faster there.
  dm.row_ip = row_plan_kind(P.fft_half);
  if (dm.row_ip != 1) {
    dm.row_ip = 0;
    FftPlan alt;
    if (2 * (size_t)dm.nhp * sizeof(float2) > 32 * 1024 && make_row_fft_plan(dm.nh, alt)) {
      P.fft_half = alt;
      dm.row_ip = row_plan_kind(alt);
    }
  }
  // a plan that is also compiled in with constant sizes (kStaticRows) runs that instantiation
  if (dm.row_ip == 1) {
    for (const StaticRowSpec& sp : kStaticRows) {
      bool same = sp.n == dm.nh && sp.npass == P.fft_half.npass && (!sp.half || dm.nts <= dm.nh);
      for (int i = 0; same && i < sp.npass; ++i) same = sp.r[i] == P.fft_half.pass[i].r;
      if (same) dm.row_ip = sp.ip;
    }
  }

  // nonuniform FFT parameters: the candidate (sigma, w, ft) list; the first one
  // is built now, the others are timed by the autotuner once the plan is complete
  dm.qhalf = dm.nq / 2;
  dm.gdt = prm.grid_dtype;
  dm.nw = 0;
  dm.wc = 0;
  dm.res = 0;
  dm.poly = 0;
  P.tb.wav = nullptr;
  std::vector<NufftChoice> cands;
  TRY(nufft_candidates(prm, dm, cands));
  if (2 * (size_t)dm.nhp * sizeof(float2) > 160 * 1024 || std::max(dm.nt, dm.ntau) > 2 * dm.nh)
    return fail(AAHRT_E_UNSUPPORTED, "row FFT too large for LDS");

  // anti-alias rule of Section 3.5 (informational)
  const double fmax = (dm.nf - 1) / (dm.nfft * dts);
  P.q_alias_ok = dm.nq >= 2.0 * std::max(std::fabs(prm.q_max), std::fabs(prm.q_min)) * fmax * h2max ? 1 : 0;

  // ---- stretch tables (FP64 positions).  Forward: two taps per output.  Transpose:
  // the inputs of each output form contiguous ranges (positions are monotone), so it
  // keeps per-input weights (w0, w1) and the first input whose lower tap is >= i.
  std::vector<Tap> s_tap(dm.nts);
  std::vector<float2> s_w(dm.nts + 4, make_float2(0.f, 0.f));
  std::vector<int> s_start(dm.ntau + 1, dm.nts);
  {
    long next = 0;  // next output index whose start is not yet set
    for (int r = 0; r < dm.nts; ++r) {
      const double pos = std::sqrt(r * dts) / prm.dtau;
      const long i = (long)std::floor(pos);
      const double a = pos - (double)i;
      int i0 = 0, i1 = 0;
      double w0 = 0.0, w1 = 0.0;
      if (i >= 0 && i < dm.ntau) { i0 = (int)i; w0 = 1.0 - a; }
      if (i + 1 >= 0 && i + 1 < dm.ntau) { i1 = (int)(i + 1); w1 = a; }
      s_tap[r] = Tap{i0, i1, (float)w0, (float)w1};
      s_w[r] = make_float2((float)w0, (float)w1);
      for (; next <= std::min<long>(i, dm.ntau); ++next) s_start[next] = r;
    }
  }
  std::vector<Tap> u_tap(dm.nt);
  std::vector<float2> u_w(dm.nt + 4, make_float2(0.f, 0.f));
  std::vector<int> u_start(dm.nts + 1, dm.nt);
  {
    long next = 0;
    for (int t = 0; t < dm.nt; ++t) {
      const double ts = t * prm.dt;
      const double pos = ts * ts / dts;
      const long r = (long)std::floor(pos);
      const double b = pos - (double)r;
      int r0 = 0, r1 = 0;
      double w0 = 0.0, w1 = 0.0;
      if (r >= 0 && r < dm.nts) { r0 = (int)r; w0 = 1.0 - b; }
      if (r + 1 >= 0 && r + 1 < dm.nts) { r1 = (int)(r + 1); w1 = b; }
      u_tap[t] = Tap{r0, r1, (float)w0, (float)w1};
      u_w[t] = make_float2((float)w0, (float)w1);
      for (; next <= std::min<long>(r, dm.nts); ++next) u_start[next] = t;
    }
  }

  // ---- twiddles of the row transforms
  std::vector<float2> tw_half(dm.nh), tw_real(dm.nh);
  for (int t = 0; t < dm.nh; ++t) {
    const double a = -2.0 * M_PI * t / dm.nh;
    tw_half[t] = make_float2((float)std::cos(a), (float)std::sin(a));
    const double b = -2.0 * M_PI * t / dm.nfft;
    tw_real[t] = make_float2((float)std::cos(b), (float)std::sin(b));
  }

  // ---- per-trace tables in bin order
  const double dq = (prm.q_max - prm.q_min) / (prm.nq - 1);
  const double qc = prm.q_min + dm.qhalf * dq;
  const double dth = M_PI / prm.ntheta;
  std::vector<int> tr_row(dm.ntr), bin_ptr((size_t)batch * (prm.ntheta + 1)), gather_of_row(dm.ntr);
  std::vector<unsigned long long> tr_b(dm.ntr), tr_a(dm.ntr);
  std::vector<float> tr_alpha(dm.ntr);
  std::vector<float2> tr_rot(dm.ntr);
  std::vector<int> tr_bin(dm.ntr);
  std::vector<double> tr_h2(dm.ntr);
  std::vector<int> jbin(dm.ntr);
  std::vector<double> alpha(dm.ntr);
  for (int n = 0; n < dm.ntr; ++n) {
    double th = 0.0;
    if (!(x[n] == 0.0 && y[n] == 0.0)) th = std::fmod(std::atan2(y[n], x[n]), M_PI);
    if (th < 0.0) th += M_PI;
    const double u = th / dth;
    long j = (long)std::floor(u);
    double a = u - (double)j;
    if (j >= prm.ntheta) j -= prm.ntheta;
    if (j < 0) j = 0;
    jbin[n] = (int)j;
    alpha[n] = a;
  }
  for (int b = 0; b < batch; ++b) {
    const int lo = (int)trace_ptr[b], hi = (int)trace_ptr[b + 1];
    std::vector<int> cnt(prm.ntheta + 1, 0);
    for (int n = lo; n < hi; ++n) cnt[jbin[n] + 1]++;
    for (int j = 0; j < prm.ntheta; ++j) cnt[j + 1] += cnt[j];
    int* bp = &bin_ptr[(size_t)b * (prm.ntheta + 1)];
    for (int j = 0; j <= prm.ntheta; ++j) bp[j] = lo + cnt[j];
    std::vector<int> fill(prm.ntheta, 0);
    for (int n = lo; n < hi; ++n) {
      const int j = jbin[n];
      const int pos = bp[j] + fill[j]++;
      const double h2 = x[n] * x[n] + y[n] * y[n];
      tr_row[pos] = n;
      tr_b[pos] = to_fix64(dq * h2 / (dm.nfft * dts));
      tr_a[pos] = to_fix64(qc * h2 / (dm.nfft * dts));
      {
        const double fa = qc * h2 / (dm.nfft * dts);
        const double rev = fa - std::floor(fa);
        tr_rot[pos] = make_float2((float)std::cos(2.0 * M_PI * rev), (float)-std::sin(2.0 * M_PI * rev));
      }
      tr_alpha[pos] = (float)alpha[n];
      tr_bin[pos] = j;
      tr_h2[pos] = h2;
      gather_of_row[n] = b;
    }
  }
  P.h_bin_ptr = bin_ptr;

  // ---- upload
  Tables& tb = P.tb;
  TRY(upload(P, s_tap, &tb.s_tap));
  TRY(upload(P, s_start, &tb.s_start)); TRY(upload(P, s_w, &tb.s_w));
  TRY(upload(P, u_tap, &tb.u_tap));
  TRY(upload(P, u_start, &tb.u_start)); TRY(upload(P, u_w, &tb.u_w));
  TRY(upload(P, lerp_records(u_start, u_w, dm.nts), &tb.u_rec));
  TRY(upload(P, tw_half, &tb.tw_half)); TRY(upload(P, tw_real, &tb.tw_real));
  {
    int mg_cap = 0;
    for (const NufftChoice& c : cands) mg_cap = std::max(mg_cap, c.mg);
    TRY(alloc(P, (size_t)dm.nq, &P.deapod_dev));
    TRY(alloc(P, (size_t)mg_cap, &P.twgrid_dev));
    tb.deapod = P.deapod_dev;
    tb.tw_grid = P.twgrid_dev;
  }
  TRY(upload(P, tr_row, &tb.tr_row)); TRY(upload(P, tr_b, &tb.tr_b)); TRY(upload(P, tr_a, &tb.tr_a));
  TRY(upload(P, tr_alpha, &tb.tr_alpha)); TRY(upload(P, bin_ptr, &tb.bin_ptr));
  TRY(upload(P, tr_rot, &tb.tr_rot));
  TRY(upload(P, tr_bin, &tb.tr_bin));
  TRY(upload(P, tr_h2, &tb.tr_h2));
  TRY(upload(P, gather_of_row, &tb.gather_of_row));
  std::vector<int64_t> tp(P.trace_ptr);
  const int64_t* tpd = nullptr;
  TRY(upload(P, tp, &tpd));
  P.trace_ptr_dev = tpd;

  // ---- workspace
  const size_t model = (size_t)batch * dm.ntheta * dm.nq * dm.ntau;
  const size_t rows = (size_t)batch * dm.ntheta * dm.nq;
  const size_t per = (size_t)dm.ntheta * dm.nq * dm.ntau;
  P.red_blocks_model = (int)std::min<size_t>(64, std::max<size_t>(1, per / (kBlock * 16)));
  TRY(alloc(P, rows * dm.nf, &P.mhat));
  TRY(alloc(P, (size_t)dm.ntr * dm.nf, &P.dhat));
  TRY(alloc(P, model, &P.ybuf));
  TRY(alloc(P, model, &P.gbuf));
  TRY(alloc(P, (size_t)dm.ntr * dm.nt, &P.dscr));
  TRY(alloc(P, (size_t)batch, &P.gam));
  TRY(alloc(P, (size_t)batch, &P.lam));
  TRY(alloc(P, (size_t)batch, &P.tmpb));
  TRY(alloc(P, (size_t)batch * P.red_blocks_model, &P.red));
  TRY(alloc(P, rows, &P.l1row));
  TRY(alloc(P, (size_t)dm.ntr, &P.rss));
  TRY(alloc(P, (size_t)dm.ntr, &P.tr_bound));
  TRY(alloc(P, (size_t)batch * dm.ntheta, &P.slice_scale));

  TRY(build_grid_tables(P, trace_ptr, x, y));
  TRY(set_nufft(P, cands[0]));
  // timed only when a kernel has a choice; otherwise each kernel takes its one setting
  const auto n_fwd = std::count_if(cands.begin(), cands.end(), [](const NufftChoice& c) { return c.fwd; });
  const auto n_adj = std::count_if(cands.begin(), cands.end(), [](const NufftChoice& c) { return c.adj; });
  if (n_fwd > 1 || n_adj > 1) {
    TRY(autotune_nufft(P, cands));
  } else {
    for (const NufftChoice& c : cands) {
      if (c.fwd) { P.ft_interp = c.ft; P.bs_interp = c.bs; }
      if (c.adj) { P.ft_spread = c.ft; P.bs_spread = c.bs; }
    }
  }
  return AAHRT_OK;
}

hipStream_t as_stream(aahrt_stream s) { return reinterpret_cast<hipStream_t>(s); }

int check_plan(const aahrt_plan* plan) {
  if (!plan) return fail(AAHRT_E_INVALID, "plan is NULL");
  return AAHRT_OK;
}

const Plan& P_of(const aahrt_plan* p) { return *reinterpret_cast<const Plan*>(p); }
Plan& P_of(aahrt_plan* p) { return *reinterpret_cast<Plan*>(p); }

constexpr size_t kEventPairs = 8192;

// Event pair around one kernel launch when timing is on.
struct ProfScope {
  Plan& P;
  hipStream_t s;
  int pair = -1;
  ProfScope(Plan& p, int kind, hipStream_t st) : P(p), s(st) {
    if (P.prof && P.ev_used < kEventPairs) {
      pair = (int)P.ev_used++;
      P.ev_kind[pair] = kind;
      (void)hipEventRecord(P.ev_pool[2 * pair], s);
    }
  }
  ~ProfScope() {
    if (pair >= 0) (void)hipEventRecord(P.ev_pool[2 * pair + 1], s);
  }
};

int drain_profile(Plan& P) {
  for (size_t i = 0; i < P.ev_used; ++i) {
    HIP_TRY(hipEventSynchronize(P.ev_pool[2 * i + 1]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, P.ev_pool[2 * i], P.ev_pool[2 * i + 1]));
    P.prof_ms[P.ev_kind[i]] += ms;
    P.prof_n[P.ev_kind[i]] += 1;
  }
  P.ev_used = 0;
  return AAHRT_OK;
}

#define KCALL(KIND, expr)                  \
  do {                                     \
    ProfScope ps_(P, KIND, s);             \
    HIP_TRY(expr);                         \
  } while (0)

int do_forward(Plan& P, const float* m, float* d, hipStream_t s) {
  KCALL(AAHRT_K_MODEL_R2C, launch_model_r2c(P, m, P.mhat, s));
  KCALL(AAHRT_K_NUFFT_INTERP, launch_nufft_interp(P, P.mhat, P.dhat, s));
  KCALL(AAHRT_K_DATA_C2R, launch_data_c2r(P, P.dhat, d, s));
  return AAHRT_OK;
}

int do_adjoint(Plan& P, const float* d, float* m, hipStream_t s) {
  KCALL(AAHRT_K_DATA_R2C, launch_data_r2c(P, d, P.dhat, P.tr_bound, s));
  KCALL(AAHRT_K_NUFFT_SPREAD, launch_nufft_spread(P, P.dhat, P.tr_bound, P.slice_scale, P.mhat, s));
  KCALL(AAHRT_K_MODEL_C2R, launch_model_c2r(P, P.mhat, m, s));
  return AAHRT_OK;
}

int do_norm2(Plan& P, int n_iter, float* out, hipStream_t s) {
  const size_t model = (size_t)P.dm.batch * P.dm.ntheta * P.dm.nq * P.dm.ntau;
  float* v = P.ybuf;
  float* w = P.gbuf;
  HIP_TRY(launch_seed_vector(v, model, 12345u, s));
  HIP_TRY(launch_gather_reduce(P, v, RED_SUMSQ, P.tmpb, s));
  HIP_TRY(launch_gather_scalar(P, GS_SQRT, P.tmpb, P.tmpb, 0.f, s));
  HIP_TRY(launch_scale_per_gather(P, v, P.tmpb, s));
  if (n_iter == 0) HIP_TRY(launch_fill(out, 0.f, (size_t)P.dm.batch, s));
  for (int it = 0; it < n_iter; ++it) {
    TRY(do_forward(P, v, P.dscr, s));
    TRY(do_adjoint(P, P.dscr, w, s));
    HIP_TRY(launch_gather_reduce(P, w, RED_SUMSQ, P.tmpb, s));
    HIP_TRY(launch_gather_scalar(P, GS_SQRT, P.tmpb, out, 0.f, s));
    HIP_TRY(launch_scale_per_gather(P, w, out, s));
    std::swap(v, w);
  }
  return AAHRT_OK;
}

int do_lambda_max(Plan& P, const float* d, float* out, hipStream_t s) {
  TRY(do_adjoint(P, d, P.gbuf, s));
  HIP_TRY(launch_gather_reduce(P, P.gbuf, RED_MAXABS, out, s));
  return AAHRT_OK;
}

std::vector<double> fista_betas(int n, bool ista) {
  std::vector<double> b(std::max(n, 0), 0.0);
  double t = 1.0;
  for (int k = 0; k < n; ++k) {
    const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
    b[k] = ista ? 0.0 : (t - 1.0) / tn;
    t = tn;
  }
  return b;
}

int enqueue_iterations(Plan& P, const float* d, float* m, int n_iter, bool ista, float* objective,
                       hipStream_t s) {
  const std::vector<double> betas = fista_betas(n_iter, ista);
  // the forward spectra of y come from model_r2c for the first iteration and from the
  // fused update kernel of the previous iteration afterwards
  if (n_iter > 0) KCALL(AAHRT_K_MODEL_R2C, launch_model_r2c(P, P.ybuf, P.mhat, s));
  for (int k = 0; k < n_iter; ++k) {
    const bool next = k + 1 < n_iter;
    KCALL(AAHRT_K_NUFFT_INTERP, launch_nufft_interp(P, P.mhat, P.dhat, s));
    KCALL(AAHRT_K_RESIDUAL_R2C, launch_residual_r2c(P, P.dhat, d, objective ? P.rss : nullptr, s));
    KCALL(AAHRT_K_NUFFT_SPREAD, launch_nufft_spread(P, P.dhat, P.tr_bound, P.slice_scale, P.mhat, s));
    KCALL(next ? AAHRT_K_MODEL_UPDATE_R2C : AAHRT_K_MODEL_C2R_UPDATE,
          launch_model_c2r_update(P, P.mhat, P.ybuf, m, P.gam, P.lam, (float)betas[k], ista ? 1 : 0,
                                  objective ? P.l1row : nullptr, next, s));
    if (objective)
      HIP_TRY(launch_objective(P, P.rss, P.trace_ptr_dev, P.l1row, P.lam,
                               objective + (size_t)k * P.dm.batch, s));
  }
  return AAHRT_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char* aahrt_version(void) { return "aahrt-mi355x 0.1 (gfx950)"; }

const char* aahrt_last_error(void) { return g_last_error.c_str(); }

int aahrt_plan_create(aahrt_plan** out, const aahrt_params* p, int32_t batch, const int64_t* trace_ptr,
                      const double* x_km, const double* y_km, int32_t device) {
  if (!out) return fail(AAHRT_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!p) return fail(AAHRT_E_INVALID, "params is NULL");
  TRY(validate_params(*p));
  if (batch < 1) return fail(AAHRT_E_INVALID, "batch must be >= 1");
  if (!trace_ptr) return fail(AAHRT_E_INVALID, "trace_ptr is NULL");
  if (trace_ptr[0] != 0) return fail(AAHRT_E_INVALID, "trace_ptr[0] must be 0");
  for (int b = 0; b < batch; ++b)
    if (trace_ptr[b + 1] < trace_ptr[b]) return fail(AAHRT_E_INVALID, "trace_ptr must be non-decreasing");
  const int64_t ntr = trace_ptr[batch];
  if (ntr > 0 && (!x_km || !y_km)) return fail(AAHRT_E_INVALID, "offsets are NULL");
  for (int64_t n = 0; n < ntr; ++n)
    if (!std::isfinite(x_km[n]) || !std::isfinite(y_km[n])) return fail(AAHRT_E_INVALID, "non-finite offset");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(AAHRT_E_INVALID, "device ordinal out of range");
  HIP_TRY(hipSetDevice(device));
  Plan* P = new (std::nothrow) Plan();
  if (!P) return fail(AAHRT_E_NOMEM, "host allocation failed");
  P->device = device;
  const int rc = build_plan(*P, *p, batch, trace_ptr, x_km, y_km);
  if (rc != AAHRT_OK) {
    free_plan(P);
    return rc;
  }
  *out = reinterpret_cast<aahrt_plan*>(P);
  return AAHRT_OK;
}

int aahrt_plan_destroy(aahrt_plan* plan) {
  if (!plan) return AAHRT_OK;
  Plan* P = reinterpret_cast<Plan*>(plan);
  (void)hipSetDevice(P->device);
  (void)hipDeviceSynchronize();
  free_plan(P);
  return AAHRT_OK;
}

int aahrt_plan_query(const aahrt_plan* plan, aahrt_plan_info* info) {
  TRY(check_plan(plan));
  if (!info) return fail(AAHRT_E_INVALID, "info is NULL");
  const Plan& P = P_of(plan);
  info->batch = P.dm.batch;
  info->ntraces = P.dm.ntr;
  info->nt_stretch = P.dm.nts;
  info->dt_stretch = P.dt_str;
  info->nfft = P.dm.nfft;
  info->nfreq = P.dm.nf;
  info->grid_size = P.dm.mg;
  info->kernel_width = P.dm.w;
  info->sigma = P.sigma;
  info->beta = P.dm.beta;
  info->freq_tile = P.ft_interp;
  info->freq_tile_adjoint = P.ft_spread;
  info->workspace_bytes = (int64_t)P.workspace_bytes;
  info->q_alias_ok = P.q_alias_ok;
  info->autotune_candidates = (int32_t)P.tune_ms.size();
  info->autotune_seconds = P.autotune_s;
  info->nufft_error_estimate = P.nufft_est;
  info->gfst_resident = P.dm.res;
  info->block_threads = P.bs_interp;
  info->block_threads_adjoint = P.bs_spread;
  return AAHRT_OK;
}

int aahrt_forward(aahrt_plan* plan, const float* m, float* d, aahrt_stream stream) {
  TRY(check_plan(plan));
  Plan& P = P_of(plan);
  if (!m) return fail(AAHRT_E_INVALID, "m is NULL");
  if (!d && P.dm.ntr > 0) return fail(AAHRT_E_INVALID, "d is NULL");
  HIP_TRY(hipSetDevice(P.device));
  return do_forward(P, m, d, as_stream(stream));
}

int aahrt_adjoint(aahrt_plan* plan, const float* d, float* m, aahrt_stream stream) {
  TRY(check_plan(plan));
  Plan& P = P_of(plan);
  if (!m) return fail(AAHRT_E_INVALID, "m is NULL");
  if (!d && P.dm.ntr > 0) return fail(AAHRT_E_INVALID, "d is NULL");
  HIP_TRY(hipSetDevice(P.device));
  return do_adjoint(P, d, m, as_stream(stream));
}

int aahrt_lambda_max(aahrt_plan* plan, const float* d, float* lmax, aahrt_stream stream) {
  TRY(check_plan(plan));
  Plan& P = P_of(plan);
  if (!lmax) return fail(AAHRT_E_INVALID, "lmax is NULL");
  if (!d && P.dm.ntr > 0) return fail(AAHRT_E_INVALID, "d is NULL");
  HIP_TRY(hipSetDevice(P.device));
  return do_lambda_max(P, d, lmax, as_stream(stream));
}

int aahrt_velocity(aahrt_plan* plan, const float* m, float* qbar, float* vel, aahrt_stream stream) {
  TRY(check_plan(plan));
  Plan& P = P_of(plan);
  if (!m || !qbar || !vel) return fail(AAHRT_E_INVALID, "m, qbar and vel must not be NULL");
  HIP_TRY(hipSetDevice(P.device));
  HIP_TRY(launch_velocity(P, m, qbar, vel, as_stream(stream)));
  return AAHRT_OK;
}

int aahrt_set_wavelet(aahrt_plan* plan, const float* w, int32_t nw, int32_t center) {
  TRY(check_plan(plan));
  Plan& P = P_of(plan);
  if (nw < 0 || nw > 4096) return fail(AAHRT_E_INVALID, "nw must be in 0..4096");
  if (nw > 0 && !w) return fail(AAHRT_E_INVALID, "w is NULL");
  if (nw > 0 && (center < 0 || center >= nw)) return fail(AAHRT_E_INVALID, "center must be in 0..nw-1");
  for (int j = 0; j < nw; ++j)
    if (!std::isfinite(w[j])) return fail(AAHRT_E_INVALID, "non-finite wavelet tap");
  HIP_TRY(hipSetDevice(P.device));
  HIP_TRY(hipDeviceSynchronize());
  if (P.wav_dev) {
    HIP_TRY(hipFree(P.wav_dev));
    P.wav_dev = nullptr;
  }
  if (nw > 0) {
    void* dptr = nullptr;
    if (hipMalloc(&dptr, (size_t)nw * sizeof(float)) != hipSuccess)
      return fail(AAHRT_E_NOMEM, "hipMalloc of the wavelet failed");
    P.wav_dev = static_cast<float*>(dptr);
    HIP_TRY(hipMemcpy(P.wav_dev, w, (size_t)nw * sizeof(float), hipMemcpyHostToDevice));
  }
  P.tb.wav = P.wav_dev;
  P.dm.nw = nw;
  P.dm.wc = nw > 0 ? center : 0;
  // a captured solver graph holds the kernels of the previous operator
  if (P.graph_exec) (void)hipGraphExecDestroy(P.graph_exec);
  if (P.graph) (void)hipGraphDestroy(P.graph);
  P.graph_exec = nullptr;
  P.graph = nullptr;
  P.graph_key.clear();
  return AAHRT_OK;
}

int aahrt_adjoint_noalloc(aahrt_plan* plan, const float* d, float* m, aahrt_stream stream) {
  TRY(check_plan(plan));
  Plan& P = P_of(plan);
  if (!m) return fail(AAHRT_E_INVALID, "m is NULL");
  if (!d && P.dm.ntr > 0) return fail(AAHRT_E_INVALID, "d is NULL");
  HIP_TRY(hipSetDevice(P.device));
  const int rc = adjoint_noalloc(P, d, m, as_stream(stream));
  if (rc != AAHRT_OK) return fail(rc, noalloc_last_message());
  return AAHRT_OK;
}

int aahrt_adjoint_direct(aahrt_plan* plan, const float* d, float* m, aahrt_stream stream) {
  TRY(check_plan(plan));
  Plan& P = P_of(plan);
  if (!m) return fail(AAHRT_E_INVALID, "m is NULL");
  if (!d && P.dm.ntr > 0) return fail(AAHRT_E_INVALID, "d is NULL");
  if (P.dm.nw > 0) return fail(AAHRT_E_UNSUPPORTED, "the direct adjoint covers the plain operator (no wavelet)");
  if ((long)P.dm.batch * P.dm.ntheta > 65535 || P.dm.nq > 65535)
    return fail(AAHRT_E_UNSUPPORTED, "batch*ntheta and nq must each be at most 65535 for the direct adjoint");
  if ((long)P.dm.batch * P.dm.ntau == 0) return AAHRT_OK;
  HIP_TRY(hipSetDevice(P.device));
  HIP_TRY(launch_direct_adjoint(P, d, m, as_stream(stream)));
  return AAHRT_OK;
}

int aahrt_adjoint_grid(aahrt_plan* plan, const float* d, float* m, aahrt_stream stream) {
  TRY(check_plan(plan));
  Plan& P = P_of(plan);
  if (!m) return fail(AAHRT_E_INVALID, "m is NULL");
  if (!d && P.dm.ntr > 0) return fail(AAHRT_E_INVALID, "d is NULL");
  if (!P.grid_ok) return fail(AAHRT_E_UNSUPPORTED, P.grid_why);
  if (P.dm.nw > 0) return fail(AAHRT_E_UNSUPPORTED, "the grid adjoint covers the plain operator (no wavelet)");
  if (P.dm.batch > 65535 || P.dm.ntheta > 65535)
    return fail(AAHRT_E_UNSUPPORTED, "batch and ntheta must each be at most 65535 for the grid adjoint");
  HIP_TRY(hipSetDevice(P.device));
  HIP_TRY(launch_grid_adjoint(P, d, m, as_stream(stream)));
  return AAHRT_OK;
}

int aahrt_operator_norm2(aahrt_plan* plan, int32_t n_iter, float* norm2, aahrt_stream stream) {
  TRY(check_plan(plan));
  Plan& P = P_of(plan);
  if (!norm2) return fail(AAHRT_E_INVALID, "norm2 is NULL");
  if (n_iter < 0) return fail(AAHRT_E_INVALID, "n_iter must be >= 0");
  HIP_TRY(hipSetDevice(P.device));
  return do_norm2(P, n_iter, norm2, as_stream(stream));
}

int aahrt_sparse_solve(aahrt_plan* plan, const float* d, float* m, const float* lambda, const float* step,
                       int32_t n_iter, int32_t flags, float* objective, aahrt_stream stream) {
  TRY(check_plan(plan));
  Plan& P = P_of(plan);
  if (!m) return fail(AAHRT_E_INVALID, "m is NULL");
  if (!d && P.dm.ntr > 0) return fail(AAHRT_E_INVALID, "d is NULL");
  if (n_iter < 0) return fail(AAHRT_E_INVALID, "n_iter must be >= 0");
  if (flags & ~(AAHRT_SOLVE_ISTA | AAHRT_SOLVE_NO_GRAPH)) return fail(AAHRT_E_INVALID, "unknown flags");
  HIP_TRY(hipSetDevice(P.device));
  hipStream_t s = as_stream(stream);
  const size_t model = (size_t)P.dm.batch * P.dm.ntheta * P.dm.nq * P.dm.ntau;
  const bool ista = (flags & AAHRT_SOLVE_ISTA) != 0;
  if (step) {
    HIP_TRY(launch_copy(P.gam, step, (size_t)P.dm.batch, s));
  } else {
    TRY(do_norm2(P, 30, P.tmpb, s));
    HIP_TRY(launch_gather_scalar(P, GS_STEP, P.tmpb, P.gam, 1.05f, s));
  }
  if (lambda) {
    HIP_TRY(launch_copy(P.lam, lambda, (size_t)P.dm.batch, s));
  } else {
    TRY(do_lambda_max(P, d, P.tmpb, s));
    HIP_TRY(launch_gather_scalar(P, GS_LAMBDA, P.tmpb, P.lam, 0.05f, s));
  }
  HIP_TRY(launch_copy(P.ybuf, m, model, s));
  if ((flags & AAHRT_SOLVE_NO_GRAPH) || P.prof || n_iter == 0)
    return enqueue_iterations(P, d, m, n_iter, ista, objective, s);
  // The iterations are captured once into a hipGraph (on the plan's capture stream) and
  // replayed on the caller's stream; the capture is reused while the arguments match.
  char key[160];
  snprintf(key, sizeof(key), "%p/%p/%d/%d/%p", (const void*)d, (void*)m, n_iter, (int)ista, (void*)objective);
  if (!P.graph_exec || P.graph_key != key) {
    if (P.graph_exec) { (void)hipGraphExecDestroy(P.graph_exec); P.graph_exec = nullptr; }
    if (P.graph) { (void)hipGraphDestroy(P.graph); P.graph = nullptr; }
    if (!P.cap_stream) HIP_TRY(hipStreamCreateWithFlags(&P.cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(P.cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_iterations(P, d, m, n_iter, ista, objective, P.cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(P.cap_stream, &g);
    if (rc != AAHRT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) return fail(AAHRT_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    P.graph = g;
    HIP_TRY(hipGraphInstantiate(&P.graph_exec, P.graph, nullptr, nullptr, 0));
    P.graph_key = key;
  }
  HIP_TRY(hipGraphLaunch(P.graph_exec, s));
  return AAHRT_OK;
}

int aahrt_profile_enable(aahrt_plan* plan, int32_t enable) {
  TRY(check_plan(plan));
  Plan& P = P_of(plan);
  HIP_TRY(hipSetDevice(P.device));
  if (enable && P.ev_pool.empty()) {
    P.ev_pool.resize(2 * kEventPairs);
    P.ev_kind.assign(kEventPairs, 0);
    for (auto& e : P.ev_pool) HIP_TRY(hipEventCreate(&e));
  }
  if (P.ev_used) TRY(drain_profile(P));
  for (int k = 0; k < AAHRT_K_COUNT; ++k) { P.prof_ms[k] = 0.0; P.prof_n[k] = 0; }
  P.prof = enable != 0;
  return AAHRT_OK;
}

int aahrt_profile_read(aahrt_plan* plan, int32_t kernel, double* total_ms, int64_t* launches) {
  TRY(check_plan(plan));
  if (kernel < 0 || kernel >= AAHRT_K_COUNT) return fail(AAHRT_E_INVALID, "kernel id out of range");
  if (!total_ms || !launches) return fail(AAHRT_E_INVALID, "output pointer is NULL");
  Plan& P = P_of(plan);
  HIP_TRY(hipSetDevice(P.device));
  TRY(drain_profile(P));
  *total_ms = P.prof_ms[kernel];
  *launches = P.prof_n[kernel];
  return AAHRT_OK;
}

}  // extern "C"
