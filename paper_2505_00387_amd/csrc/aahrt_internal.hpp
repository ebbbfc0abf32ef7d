// Internal definitions shared by the host plan code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/aahrt.h"

namespace aahrt {

constexpr int kMaxPasses = 12;
constexpr int kBlock = 256;     // threads per workgroup of the row kernels and small kernels
constexpr int kPrefetch = 4;    // samples per thread a row kernel loads before its transform
constexpr int kBlockG = 512;    // threads per workgroup of the GFST (nonuniform FFT) kernels
constexpr int kPrefetchCells = 4 * 512;  // q-coefficients (nq * ft) a GFST workgroup holds in registers

// x / d = (umulhi(x, m) + x) >> s for 0 <= x < 2^31 (d = 1: x).
struct FastDiv {
  unsigned d, m, s;
};

// One Stockham pass: radix r, nb = n/r butterflies per sequence, ns = product of
// the earlier radices, stride = n/(ns*r) into the twiddle table.
struct FftPass {
  int r, nb, ns, stride;
  FastDiv dnb, dns;
};

struct FftPlan {
  int n;
  int npass;
  FftPass pass[kMaxPasses];
};

// Butterflies of one in-place row-transform pass a thread may hold in registers
// (passes with more butterflies than threads), by radix.
__host__ __device__ constexpr int row_kmax(int r) { return r >= 15 ? 2 : (r == 5 ? 5 : 3); }

// Row transforms also compiled with their length and radices as constants (row_ip >= 3):
// N/2 of the stretched axis and the radices in pass order (each pass one butterfly per thread).
// half = 1: the plan also assumes nt' <= N/2, so that the second half of a forward
// transform's packed input is zero padding and the second half of an inverse transform's
// output is never read; both are left out of its first and last passes.
struct StaticRowSpec {
  int ip, n, npass, r[3], half;
};
constexpr StaticRowSpec kStaticRows[] = {{3, 2160, 3, {16, 15, 9}, 1}, {4, 480, 3, {16, 15, 2}, 0}};
constexpr int kRowKinds = 5;  // row_ip 0..4

// Two-tap linear interpolation entry: value = w0 * x[i0] + w1 * x[i1] (dropped taps have weight 0).
struct __attribute__((aligned(16))) Tap {
  int i0, i1;
  float w0, w1;
};

// One output of the transpose U^T, read with a single 16-byte load: its inputs a and a + 1
// with their weights w0, w1 (n = 0, 1 or 2 of them), or n = -1 where more than two inputs
// reach the output (the general gather over the start table then runs).  Past t = 0 the
// data samples are sparse on the stretched axis, so nearly every output takes this form; S^T,
// whose outputs gather up to eight inputs, keeps the start table alone.
struct __attribute__((aligned(16))) LerpRec {
  int a;
  float w0, w1;
  int n;
};

// Device tables of one plan.  Per-trace arrays are stored in "bin order":
// within a gather, traces are grouped by their lower azimuth bin j_n.
struct Tables {
  // stretch S (model side): for r < nt', M'(r) = interpolation s_tap[r] of M
  const Tap* s_tap;
  // S^T: weights (w0, w1) of every stretched sample (4 zero entries of padding) and
  // s_start[i] = first stretched sample whose lower tap is >= i (i <= ntau)
  const int* s_start;
  const float2* s_w;
  // unstretch U (data side): d(s) = interpolation u_tap[s] of D'
  const Tap* u_tap;
  // U^T: weights of every time sample (4 zero entries of padding) and u_start[r] =
  // first time sample whose lower tap is >= r (r <= nt')
  const int* u_start;
  const float2* u_w;
  const LerpRec* u_rec;   // [nt']
  // deapodisation 1/Phi(2 pi k/Mg), k = l - nq/2, per curvature sample l
  const float* deapod;
  // twiddles
  const float2* tw_half;   // exp(-2 pi i t/(N/2)), t < N/2
  const float2* tw_real;   // exp(-2 pi i k/N), k < N/2
  const float2* tw_grid;   // exp(-2 pi i t/Mg), t < Mg
  // per trace, bin order
  const int* tr_row;                   // data row of the trace
  const unsigned long long* tr_b;      // frac(dq h^2/(N dt')) as 0.64 fixed point
  const unsigned long long* tr_a;      // frac(q_c h^2/(N dt')) as 0.64 fixed point
  const float* tr_alpha;               // azimuth weight on the upper bin
  const float2* tr_rot;                // exp(-2 pi i frac(q_c h^2/(N dt'))), the pre-phase step per frequency
  const int* tr_bin;                   // lower azimuth bin j_n of the trace
  const int* bin_ptr;                  // [batch][ntheta+1] positions into the bin-ordered arrays
  const int* gather_of_row;            // data row -> gather
  const float* wav;                    // wavelet taps (deconvolutive operator), or null
  const double* tr_h2;                 // h^2 of the trace (direct time-domain operator)
};

struct Dims {
  int batch;
  int ntr;      // total traces
  int nt, ntau, nq, ntheta;
  int nts;      // nt'
  int nfft, nh, nf;  // N, N/2, bins carried (= N/2)
  int nhp;      // LDS cells of one row FFT buffer: room for the padded first pass
  int row_ip;   // row FFT in place: 1 = one butterfly per thread per pass, 2 = up to row_kmax; 0 = ping-pong;
                // 3, 4: as 1 with the plan of kStaticRows compiled in
  int mg;       // q-grid length
  int ldr;      // LDS row length of a q-grid slot: mg + w - 1 ghost cells, padded to odd
  int w;        // kernel width
  float beta;
  float cbeta;  // beta * log2(e)
  int ft;       // frequencies per GFST tile (set per launch: interpolation and spreading tile separately)
  int nftile;   // ceil(nf/ft)
  int qhalf;    // nq/2 (mode offset)
  int gdt;      // storage of the forward q-grid (aahrt_grid_dtype)
  int nw, wc;   // wavelet of the deconvolutive operator: taps and origin (nw = 0: none)
  int res;      // 1: GFST kernels with every azimuth slice resident in LDS (q-grid of 64, 128 or 256 cells)
  int poly;     // 1: kernel taps by the per-tap polynomials (w >= 5, sigma >= 2 shape)
  int bsz;      // threads per workgroup of the resident GFST kernels (512, 768 or 1024; set per launch)
};

// Algorithm 2 of Section 3.2 on a regular offset grid x_m = x0 + m dx, y_n = y0 + n dy.
struct GridGather {
  double x0, dx, y0, dy;
  int mx, my;  // grid lines along x and y (0 for an empty gather)
  int node0;   // first entry of the gather in the node table
  int pad;
};

struct GridTables {
  const Tap* dtap;      // [nt'] data stretch by interpolation: D'(r) = D(t = sqrt(r dt'))
  const Tap* vtap;      // [ntau] model unstretch by interpolation: M(tau_i) = M'(tau' = tau_i^2)
  const float* one;     // [1] = 1 (unit row scale of the data-side transform)
  const float2* phase;  // [nq] exp(2 pi i k_p q_min) / nq
  const float2* tw;     // [nq] exp(-2 pi i t / nq)
  const double* kp;     // [nq] k_p = p / (nq dq), FFT order, signed
  const double2* cs;    // [ntheta] (cos, sin) of theta_j
  const GridGather* g;  // [batch]
  const int* node;      // trace row of node (m, n): node[g.node0 + m * my + n]
  double fscale;        // f' of bin f is f * fscale = f / (N dt')
};

struct Plan {
  Dims dm;
  aahrt_params prm;
  int device = 0;
  double dt_str = 0.0;
  double sigma = 2.0;
  double nufft_est = 0.0;  // estimated relative error of the current q nonuniform FFT setting
  int q_alias_ok = 0;
  FftPlan fft_half{};   // N/2 complex
  FftPlan fft_grid{};   // Mg complex
  Tables tb{};
  std::vector<void*> allocations;
  // workspace
  float2* mhat = nullptr;   // [batch][ntheta][nq][nf]
  float2* dhat = nullptr;   // [ntr][nf]
  float* ybuf = nullptr;    // [batch][ntheta][nq][ntau]
  float* gbuf = nullptr;    // [batch][ntheta][nq][ntau]  (power iteration / scratch)
  float* dscr = nullptr;    // [ntr][nt]
  float* gam = nullptr;     // [batch]
  float* lam = nullptr;     // [batch]
  float* red = nullptr;     // reduction partials
  float* tmpb = nullptr;    // [batch] scratch scalars
  float* l1row = nullptr;   // [rows] per-row l1 norms (objective)
  float* rss = nullptr;     // [ntr] per-trace residual sums of squares (objective)
  float* tr_bound = nullptr; // [ntr] max_f |Re Dh| + |Im Dh| of each trace (spreading scale bound)
  float* slice_scale = nullptr; // [batch][ntheta] fixed-point scale of each azimuth slice (spreading)
  float* wav_dev = nullptr;      // wavelet taps (owned; replaced by each aahrt_set_wavelet)
  float* deapod_dev = nullptr;   // [nq] deapodisation of the current q-grid setting
  float2* twgrid_dev = nullptr;  // [mg] q-grid twiddles of the current setting
  int ft_interp = 16;            // frequency tile of the interpolation kernel
  int ft_spread = 16;            // frequency tile of the spreading kernel
  int bs_interp = kBlockG;       // workgroup threads of the interpolation kernel
  int bs_spread = kBlockG;       // workgroup threads of the spreading kernel
  std::vector<float> tune_ms;    // GFST stage time of each autotune candidate
  int tune_choice = 0;
  double autotune_s = 0.0;
  const int64_t* trace_ptr_dev = nullptr;
  int red_blocks_model = 0; // partial blocks per gather (model-sized reductions)
  size_t workspace_bytes = 0;
  // host copies
  std::vector<int64_t> trace_ptr;
  std::vector<int> h_bin_ptr;
  // per-kernel timing
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int> ev_kind;      // kernel id of each recorded pair
  double prof_ms[AAHRT_K_COUNT] = {0};
  int64_t prof_n[AAHRT_K_COUNT] = {0};
  // cached graph of the solver
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t cap_stream = nullptr;
  std::string graph_key;
  // Algorithm 2 on regular offset grids (aahrt_adjoint_grid)
  bool grid_ok = false;
  std::string grid_why;
  GridTables gt{};
  FftPlan fft_q{};  // nq complex
  int grid_ft = 1;  // frequencies per workgroup of the polar interpolation
};

// LDS of the GFST kernels in float2 units (q-grid transforms run in place).
// Interpolation: two slots (one if ntheta = 1; 16-bit grids pack a cell in 4
// bytes, plus one FP32 transform buffer) and the q-grid twiddles.  Spreading:
// two fixed-point slots and the twiddles.
__host__ __device__ inline size_t interp_slots_f2(int ft, int ldr, int ntheta, int gdt) {
  const int nslot = ntheta >= 2 ? 2 : 1;
  const size_t cells = (size_t)nslot * ft * ldr;
  return gdt == AAHRT_GRID_F32 ? cells : (cells + 1) / 2;
}
__host__ __device__ inline size_t interp_lds_f2(int ft, int ldr, int ntheta, int mg, int gdt) {
  return interp_slots_f2(ft, ldr, ntheta, gdt) + (gdt == AAHRT_GRID_F32 ? 0 : (size_t)ft * ldr) + mg;
}
__host__ __device__ inline size_t spread_lds_f2(int ft, int ldr, int mg) {
  return 2 * (size_t)ft * ldr + mg;
}
// Resident-slice kernels: every slice of the tile ([ntheta][ft][ldr] cells) and the q-grid
// twiddles (the spreading kernel adds one float per slice for its scales).
__host__ __device__ inline size_t res_lds_f2(int ft, int ldr, int ntheta, int mg) {
  return (size_t)ntheta * ft * ldr + mg;
}
// Lanes per q-grid row of the resident kernels' register transform (mg = 64, 128, 256).
__host__ __device__ inline int res_lanes(int mg) { return mg == 256 ? 16 : 8; }

// ---- kernels (kernels.hip) ----
hipError_t launch_model_r2c(const Plan& p, const float* m, float2* mhat, hipStream_t s);
// steps 1-2 of L on nrows rows of dm.ntau samples with the given tables (rows of dm.ntau in,
// dm.nf bins out), for Algorithm 2's data-side stretch and transform
hipError_t launch_rows_r2c(const Dims& dm, const Tables& tb, const FftPlan& fp, const float* in, float2* out,
                           unsigned nrows, hipStream_t s);
hipError_t launch_nufft_interp(const Plan& p, const float2* mhat, float2* dhat, hipStream_t s);
hipError_t launch_data_c2r(const Plan& p, const float2* dhat, float* d, hipStream_t s);
hipError_t launch_data_r2c(const Plan& p, const float* d, float2* dhat, float* tr_bound, hipStream_t s);
hipError_t launch_residual_r2c(const Plan& p, float2* dhat, const float* dobs, float* rss,
                               hipStream_t s);
hipError_t launch_nufft_spread(const Plan& p, const float2* dhat, const float* tr_bound, float* slice_scale,
                               float2* mhat, hipStream_t s);
hipError_t launch_model_c2r(const Plan& p, const float2* mhat, float* m, hipStream_t s);
hipError_t launch_model_c2r_update(const Plan& p, float2* mhat, float* y, float* x, const float* gam,
                                   const float* lam, float beta, int ista, float* l1, bool next,
                                   hipStream_t s);
hipError_t launch_velocity(const Plan& p, const float* m, float* qbar, float* vel, hipStream_t s);
hipError_t launch_direct_adjoint(const Plan& p, const float* d, float* m, hipStream_t s);
hipError_t launch_grid_adjoint(const Plan& p, const float* d, float* m, hipStream_t s);
hipError_t launch_fill(float* p, float v, size_t n, hipStream_t s);
hipError_t launch_copy(float* dst, const float* src, size_t n, hipStream_t s);
hipError_t launch_seed_vector(float* v, size_t n, unsigned seed, hipStream_t s);
// per-gather reductions over model-sized arrays [batch][per]
hipError_t launch_gather_reduce(const Plan& p, const float* x, int op, float* out, hipStream_t s);
hipError_t launch_scale_per_gather(const Plan& p, float* x, const float* norms, hipStream_t s);
hipError_t launch_gather_scalar(const Plan& p, int op, const float* a, float* out, float c,
                                hipStream_t s);
hipError_t launch_trace_to_gather_sum(const Plan& p, const float* per_trace, float* out,
                                      const float* l1, const float* lam, hipStream_t s);

// ---- the adjoint without allocation (noalloc.hip) ----
size_t noalloc_scratch_limit();
size_t noalloc_adjoint_bytes(const Dims& dm);
int adjoint_noalloc(Plan& P, const float* d, float* m, hipStream_t s);
const char* noalloc_last_message();

enum { RED_SUMSQ = 0, RED_MAXABS = 1, RED_SUMABS = 2 };
enum { GS_STEP = 0, GS_LAMBDA = 1, GS_SQRT = 2 };

}  // namespace aahrt
