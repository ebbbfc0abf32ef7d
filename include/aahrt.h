/*
 * aahrt.h -- C ABI of the MI355X (gfx950) azimuthally anisotropic hyperbolic
 * Radon transform (AAHRT) library, computed through the generalized Fourier
 * slice theorem (GFST).
 *
 * Operators (notation of the paper, Sections 2.2, 3 and 4):
 *   L   : model M(tau, q, theta) -> CMP data D(t, x, y)      (the paper's R^-1, Algorithm 1)
 *   L^T : data -> model, the exact transpose of L            (the paper's R^-T, Section 4)
 *   sparse solve: argmin_m 0.5 ||d - L m||^2 + lambda ||m||_1 by forward-backward
 *   splitting with soft shrinkage (Section 4) and FISTA momentum.
 *
 * Discretisation of L (one gather; n = trace, t_s = s dt, tau_i = i dtau,
 * q_l = q_min + l dq with dq = (q_max - q_min)/(nq - 1), theta_j = j pi/ntheta):
 *   1. stretch tau' = tau^2 by linear interpolation (Section 3.4, operator S),
 *      nt' = stretch * nt samples, dt' = ((nt-1) dt)^2 / (nt' - 1);
 *   2. real DFT of length N along tau', bins f = 0 .. N/2-1 (f'_f = f/(N dt'));
 *   3. GFST map (Section 3.1): Dh[n,f] = sum_j w[n,j] sum_l Mh[j,l,f] exp(-2 pi i f'_f q_l h_n^2),
 *      h_n^2 = x_n^2 + y_n^2, w = linear weights of theta_n = atan2(y_n, x_n) mod pi
 *      onto theta_j and theta_{j+1 mod ntheta} (theta part of Section 3.4);
 *      the sum over q is computed by a type-2 nonuniform FFT (exponential-of-
 *      semicircle kernel on a sigma-times oversampled q-grid), the azimuth by
 *      the linear weights;
 *   4. inverse real DFT (1/N, Nyquist bin zero), first nt' samples;
 *   5. unstretch t' = t^2 by linear interpolation (operator S^-1).
 *
 * Conventions shared by every entry point:
 *   - All array pointers passed to aahrt_forward / aahrt_adjoint /
 *     aahrt_sparse_solve / aahrt_lambda_max / aahrt_operator_norm2 are DEVICE
 *     pointers owned by the caller; aahrt_plan_create takes HOST arrays and
 *     copies them.
 *   - Layouts (row-major, FP32):
 *       model m : [batch][ntheta][nq][ntau]
 *       data  d : [ntraces][nt], traces of gather b are rows trace_ptr[b] .. trace_ptr[b+1]-1
 *   - stream is a hipStream_t (NULL = the null stream); every call is
 *     asynchronous on it.  Outputs are overwritten, never accumulated.
 *   - Errors: a negative aahrt_status is returned and nothing is enqueued when
 *     an argument is invalid; aahrt_last_error() gives a message (per thread).
 *   - Calls that share one plan must not overlap in time (the plan owns one
 *     workspace); plans are independent of each other.
 */
#ifndef AAHRT_H
#define AAHRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* aahrt_stream; /* hipStream_t */

typedef enum {
  AAHRT_OK = 0,
  AAHRT_E_INVALID = -1,     /* bad argument; nothing enqueued */
  AAHRT_E_HIP = -2,         /* HIP runtime error */
  AAHRT_E_NOMEM = -3,       /* device allocation failed */
  AAHRT_E_UNSUPPORTED = -4  /* valid but not supported by this library */
} aahrt_status;

typedef enum {
  AAHRT_GRID_F32 = 0,  /* oversampled q-grid of the nonuniform FFT held in FP32 */
  AAHRT_GRID_F16 = 1,  /* ... stored in FP16, accumulated in FP32.  FP16 holds magnitudes up to 65504 only: a
                          grid cell is a sum over the nq curvature modes of a model spectrum value (the DFT of a
                          stretched model row) times its deapodisation factor, and a cell above that range
                          becomes inf, unchecked.  Scale the model (L is linear) or use FP32/BF16 */
  AAHRT_GRID_BF16 = 2  /* ... stored in BF16, accumulated in FP32 */
} aahrt_grid_dtype;

/* Axes and numerical options of a plan.  Zero in an option field selects its default. */
typedef struct aahrt_params {
  int32_t nt;            /* data time samples (>= 2) */
  double dt;             /* data time step [s] (> 0) */
  int32_t ntau;          /* model intercept-time samples (>= 1) */
  double dtau;           /* model intercept-time step [s] (> 0) */
  int32_t nq;            /* curvature samples (>= 2) */
  double q_min, q_max;   /* curvature range, squared slowness [s^2/km^2], q_min < q_max, inclusive */
  int32_t ntheta;        /* azimuth samples over [0, pi) (>= 1) */
  int32_t stretch;       /* nt' = stretch * nt; 0 -> 2 */
  int32_t nfft;          /* length N of the stretched-axis DFT; 0 -> smallest even 2^a3^b5^c
                            >= nt' + ceil(max(q_max,0) h2max/dt') + ceil(max(-q_min,0) h2max/dt');
                            otherwise it must be even, 2^a3^b5^c and >= nt' */
  double nufft_tol;      /* target relative error of the q nonuniform FFT; 0 -> 1e-6 */
  double sigma;          /* q-grid oversampling in [1.25, 4]; 0 -> autotune among those of 2, 1.5 and 1.25
                            that some width brings within nufft_tol */
  int32_t kernel_width;  /* spreading kernel width w (3..12); 0 -> the narrowest whose estimated error
                            (kernel truncation and FP32 rounding, see aahrt_plan_create) meets nufft_tol,
                            or, where none does at a requested sigma, the one of smallest estimate;
                            2 -> the paper's own step 3 (Section 3.4): linear interpolation in k on the
                            sigma-oversampled grid, no deapodisation (low accuracy, reported only) */
  int32_t freq_tile;     /* frequencies per workgroup tile of the GFST kernels (power of 2, 1..64; halved until
                            the tile fits LDS); 0 -> autotune.  The spreading kernel takes freq_tile_adjoint
                            instead when that is set */
  int32_t grid_dtype;    /* aahrt_grid_dtype */
  int32_t gfst_kind;     /* 0: GFST kernels with every azimuth slice of a frequency tile resident in LDS where
                            they apply (FP32 q-grid of 64, 128 or 256 cells that fits), else the slice sweep;
                            1: always the slice sweep.  The two differ only in the FP32 rounding of the q-grid
                            transform; the tile changes no result within a kind */
  int32_t block_threads; /* threads per workgroup of the resident-slice GFST kernels: 512, 768 or 1024; 0 -> autotune
                            (the slice sweep always uses 512); changes no result.  The spreading kernel takes
                            block_threads_adjoint instead when that is set */
  int32_t freq_tile_adjoint;     /* tile of the spreading (adjoint) GFST kernel alone, as freq_tile; 0 -> as
                                    freq_tile.  With freq_tile and the two workgroup sizes this re-creates an
                                    autotuned setting (aahrt_plan_info) without timing it again */
  int32_t block_threads_adjoint; /* workgroup size of the spreading kernel alone, as block_threads; 0 -> as
                                    block_threads */
} aahrt_params;

typedef struct aahrt_plan aahrt_plan;

/* Facts about a built plan (filled by aahrt_plan_query). */
typedef struct aahrt_plan_info {
  int32_t batch;         /* number of gathers */
  int64_t ntraces;       /* total traces */
  int32_t nt_stretch;    /* nt' */
  double dt_stretch;     /* dt' [s^2] */
  int32_t nfft;          /* N */
  int32_t nfreq;         /* N/2 frequency bins carried */
  int32_t grid_size;     /* oversampled q-grid length */
  int32_t kernel_width;  /* w */
  double sigma;          /* grid_size / nq */
  double beta;           /* kernel shape parameter */
  int32_t freq_tile;     /* frequencies per workgroup tile of the forward GFST kernel (interpolation) */
  int64_t workspace_bytes;
  int32_t q_alias_ok;    /* 1 if nq >= 2 q_max f'_max h2max (Section 3.5 anti-alias rule), else 0 (informational) */
  int32_t autotune_candidates; /* GFST settings timed at plan creation (0: none, the setting was fixed) */
  double autotune_seconds;     /* wall time of that autotuning */
  int32_t freq_tile_adjoint;   /* frequencies per workgroup tile of the adjoint GFST kernel (spreading) */
  int32_t gfst_resident;       /* 1 if the resident-slice GFST kernels run, 0 for the slice sweep */
  double nufft_error_estimate; /* estimated relative error of one q nonuniform FFT at the chosen setting
                                  (kernel truncation and FP32 rounding; 1 for kernel_width = 2) */
  int32_t block_threads;         /* threads per workgroup of the forward GFST kernel */
  int32_t block_threads_adjoint; /* threads per workgroup of the adjoint GFST kernel */
} aahrt_plan_info;

/* Version string of the library. */
const char* aahrt_version(void);

/* Message for the last non-OK status returned on this thread. */
const char* aahrt_last_error(void);

/*
 * Build a plan for a batch of CMP gathers sharing one set of axes.
 *   out        : receives the plan (owned by the caller, release with aahrt_plan_destroy)
 *   p          : axes and options (host)
 *   batch      : number of gathers (>= 1)
 *   trace_ptr  : host int64[batch+1], trace_ptr[0] = 0, non-decreasing (empty gathers allowed)
 *   x_km, y_km : host double[trace_ptr[batch]] offsets of every trace [km], finite
 *   device     : HIP device ordinal the plan lives on
 * Computes the FP64 tables (stretch taps, azimuth weights, 64-bit fixed-point
 * phase increments, kernel deapodisation), allocates the device tables and the
 * workspace (hipMalloc).  The kernel width at an oversampling sigma is the narrowest
 * whose estimated error meets nufft_tol.  The estimate is the root sum of squares of the
 * kernel's truncation error (computed in FP64 for white mode coefficients) and an FP32
 * rounding term that grows with the range of the deapodisation; in FP32 it keeps
 * sigma = 1.25 above about 6e-6 and sigma = 1.5 above about 1.1e-6, so at the default
 * tolerance only sigma = 2 is admitted.  When a kernel has more than one admissible setting
 * (sigma 0, or a tile or workgroup size that applies to it left at 0) it then autotunes the
 * GFST stage: every admissible setting (sigma in {2, 1.5, 1.25}; for the resident-slice
 * kernels freq_tile in {1, 2, 4, 8} and block_threads in {512, 768, 1024}, for the slice sweep
 * freq_tile in {4, 8, 16, 32}, each narrowed by the requested values) is timed on the
 * interpolation and on the spreading launch over the batch (on zeroed spectra, in a stream
 * of its own, synchronously); each kernel keeps its fastest tile and workgroup size, and the
 * sigma with the smallest sum is kept, the default sigma = 2 unless another is at least 5% faster.
 * Tiles and workgroup sizes change no result; sigma changes results within the tolerance.
 */
int aahrt_plan_create(aahrt_plan** out, const aahrt_params* p, int32_t batch,
                      const int64_t* trace_ptr, const double* x_km, const double* y_km,
                      int32_t device);

/* Release a plan and its device memory (NULL is a no-op). */
int aahrt_plan_destroy(aahrt_plan* plan);

/* Fill *info with the plan's derived sizes. */
int aahrt_plan_query(const aahrt_plan* plan, aahrt_plan_info* info);

/*
 * d = L m  (Algorithm 1, Section 3.1; factorisation S^-1 F1^-1 P F2 S of Section 4).
 *   m : device float[batch][ntheta][nq][ntau] (read)
 *   d : device float[ntraces][nt] (written)
 */
int aahrt_forward(aahrt_plan* plan, const float* m, float* d, aahrt_stream stream);

/*
 * m = L^T d, the exact transpose of aahrt_forward (Section 3.2 defines the
 * adjoint as the velocity stack; this is the transpose of the discrete L).
 *   d : device float[ntraces][nt] (read)
 *   m : device float[batch][ntheta][nq][ntau] (written)
 */
int aahrt_adjoint(aahrt_plan* plan, const float* d, float* m, aahrt_stream stream);

/*
 * m = L^T d exactly as aahrt_adjoint (same kernels, bitwise the same result), for callers
 * that cannot allocate (code under stream capture, serving loops, harnesses that forbid
 * hipMalloc): the call allocates nothing.  Its intermediates (trace spectra, model spectra,
 * per-trace spreading bounds, per-slice scales) live in a file-scope device array of
 * 64 MiB = 67108864 bytes in the library, not in the plan's workspace; each GPU holds its
 * own copy until the process ends.  It needs
 *   256-byte-aligned sum of ntraces*nf*8, batch*ntheta*nq*nf*8, ntraces*4 and batch*ntheta*4
 * bytes (nf = N/2, aahrt_plan_info.nfreq); a plan that needs more returns AAHRT_E_UNSUPPORTED
 * before anything is enqueued.  All calls on one GPU share the array: calls that overlap in
 * time on one GPU race and must not be made.
 *   d : device float[ntraces][nt] (read)
 *   m : device float[batch][ntheta][nq][ntau] (written)
 */
int aahrt_adjoint_noalloc(aahrt_plan* plan, const float* d, float* m, aahrt_stream stream);

/*
 * Per-gather max |L^T d| (the lambda scale of Section 4).
 *   d    : device float[ntraces][nt] (read)
 *   lmax : device float[batch] (written)
 */
int aahrt_lambda_max(aahrt_plan* plan, const float* d, float* lmax, aahrt_stream stream);

/*
 * Per-gather ||L_b||^2 by n_iter power iterations on L^T L from a fixed
 * pseudo-random start vector (the step length of Section 4 is 1/(1.05 ||L_b||^2)).
 *   norm2 : device float[batch] (written)
 */
int aahrt_operator_norm2(aahrt_plan* plan, int32_t n_iter, float* norm2, aahrt_stream stream);

enum {
  AAHRT_SOLVE_FISTA = 0,     /* forward-backward splitting with FISTA momentum (default) */
  AAHRT_SOLVE_ISTA = 1,      /* plain iteration of Section 4 */
  AAHRT_SOLVE_NO_GRAPH = 2   /* enqueue kernels one by one instead of replaying a captured hipGraph */
};

/*
 * Sparse AAHRT: n_iter iterations of m <- soft(y + gamma_b L^T (d - L y), gamma_b lambda_b)
 * (Section 4), with y the FISTA extrapolation (or y = m for ISTA).
 *   d         : device float[ntraces][nt] observed data (read)
 *   m         : device float[batch][ntheta][nq][ntau]; in: starting model (zeros for a cold
 *               start), out: the last iterate
 *   lambda    : device float[batch] per-gather lambda_b, or NULL for 0.05 * max|L_b^T d_b|
 *   step      : device float[batch] per-gather gamma_b, or NULL for 1/(1.05 ||L_b||^2)
 *               (30 power iterations)
 *   n_iter    : iterations (>= 0)
 *   flags     : AAHRT_SOLVE_* bits
 *   objective : device float[n_iter][batch] receiving 0.5||d_b - L_b y||^2 + lambda_b ||m_b||_1
 *               per iteration (the residual of the extrapolated point), or NULL
 */
int aahrt_sparse_solve(aahrt_plan* plan, const float* d, float* m, const float* lambda,
                       const float* step, int32_t n_iter, int32_t flags, float* objective,
                       aahrt_stream stream);

/*
 * Algorithm 2 of Section 3.2, the paper's fast velocity stack, for gathers whose traces
 * fill a regular offset grid x_m = x0 + m dx, y_n = y0 + n dy (each node once, any order):
 *   1. stretch every trace by interpolation, D'(t') = D(t = sqrt(t'));
 *   2. real DFT along t' (bins below N/2);
 *   3. the model spectrum at (f', k_p, theta_j) is the data spectrum at the offset
 *      x = sqrt(k_p/f') cos(theta_j), y = sqrt(k_p/f') sin(theta_j), interpolated with the
 *      bilinear coefficients B1..B4 of Section 3.4 (0 for k_p < 0, f' = 0 or outside the grid);
 *      k_p = p/(nq dq), p = -nq/2 .. nq/2-1 (odd nq: -(nq-1)/2 .. (nq-1)/2);
 *   4. inverse DFT along k (1/nq, onto q_l = q_min + l dq) and along f' (1/N, real);
 *   5. unstretch by interpolation, M(tau_i) = M'(tau' = tau_i^2).
 * Not the transpose of aahrt_forward (that is aahrt_adjoint): the paper's approximation, for
 * comparison.  Layouts as aahrt_adjoint; m is overwritten.  Returns AAHRT_E_UNSUPPORTED when a
 * gather is not a complete regular grid (a gather with no traces gives zeros), when nq has a
 * prime factor above 5 or exceeds 3856, or when a wavelet is set.
 */
int aahrt_adjoint_grid(aahrt_plan* plan, const float* d, float* m, aahrt_stream stream);

/*
 * Conventional time-domain adjoint (Section 5's direct summation, the method the
 * paper's timing table compares against): for every gather b, azimuth theta_j,
 * curvature q_l and intercept tau_i, the Riemann sum over the traces n of
 *   w[n][j] ((1 - a) d[n][s] + a d[n][s+1]),  s + a = sqrt(tau_i^2 + q_l h_n^2)/dt,
 * with the linear azimuth weights of the plan and taps at or beyond nt dropped.  A
 * second discretisation of the continuous adjoint, for timing comparison; positions
 * in FP64, sums in FP32.  Layouts as aahrt_adjoint; m is overwritten.  Returns
 * AAHRT_E_UNSUPPORTED when a wavelet is set or batch*ntheta or nq exceeds 65535.
 */
int aahrt_adjoint_direct(aahrt_plan* plan, const float* d, float* m, aahrt_stream stream);

/*
 * Deconvolutive AAHRT (Section 4, "Deconvolutive AAHRT"): from this call on, every
 * operator of the plan is L_w = W L and L_w^T = L^T W^T, with W the linear convolution
 * of every trace with the wavelet along t (the basis functions carry the wavelet
 * instead of a delta in time):
 *   (W d)[s] = sum_j w[j] d[s - j + center],  samples outside 0..nt-1 taken as zero.
 *   w      : host float[nw] wavelet taps (copied); nw = 0 returns to the plain operator
 *   nw     : 0..4096
 *   center : index of the tap at zero lag, 0..nw-1
 * Synchronises the device and drops a captured solver graph; must not overlap other
 * calls on the plan.
 */
int aahrt_set_wavelet(aahrt_plan* plan, const float* w, int32_t nw, int32_t center);

/*
 * Automatic anisotropic velocity estimate of a Radon cube (Section 3, "Automatic
 * Anisotropic Velocity Peaking"): for every gather b, azimuth theta_j and intercept
 * tau_i, the curvature-weighted mean
 *   qbar = v^-2 = sum_l q_l |m[b][j][l][i]| / sum_l |m[b][j][l][i]|
 * (weights |m|, as a sparse-inversion cube is signed; 0 where the cube holds no energy)
 * and the velocity v = qbar^(-1/2) [km/s] (0 where qbar <= 0).
 *   m    : device float[batch][ntheta][nq][ntau] (read)
 *   qbar : device float[batch][ntheta][ntau] (written) [s^2/km^2]
 *   vel  : device float[batch][ntheta][ntau] (written) [km/s]
 */
int aahrt_velocity(aahrt_plan* plan, const float* m, float* qbar, float* vel, aahrt_stream stream);

/* Kernels of the library, for per-kernel timing. */
typedef enum {
  AAHRT_K_MODEL_R2C = 0,        /* model rows: stretch S, deapodise, real DFT along tau' (L steps 1-2) */
  AAHRT_K_NUFFT_INTERP = 1,     /* GFST map: q-grid FFT + kernel interpolation + azimuth weights (L step 3) */
  AAHRT_K_DATA_C2R = 2,         /* traces: inverse real DFT, unstretch (L steps 4-5) */
  AAHRT_K_DATA_R2C = 3,         /* traces: unstretch transpose, real DFT (L^T) */
  AAHRT_K_NUFFT_SPREAD = 4,     /* transpose of the GFST map: spreading + inverse q-grid FFT (L^T) */
  AAHRT_K_MODEL_C2R = 5,        /* model rows: inverse real DFT, stretch transpose (L^T) */
  AAHRT_K_RESIDUAL_R2C = 6,     /* solver: residual d - L y fused with the data side of L^T */
  AAHRT_K_MODEL_C2R_UPDATE = 7, /* solver: model side of L^T fused with shrinkage + momentum */
  AAHRT_K_MODEL_UPDATE_R2C = 8, /* solver: the same, then L steps 1-2 on the new y (next iteration) */
  AAHRT_K_COUNT = 9
} aahrt_kernel_id;

/*
 * Per-kernel timing (Section 5 reports wall-clock cost; this splits it per kernel).
 * enable = 1 records a HIP event pair on the launch stream around every kernel of the
 * kinds above (up to 8192 launches between reads) and clears the totals; 0 stops recording.
 * Recording is for eager calls (AAHRT_SOLVE_NO_GRAPH for the solver).
 */
int aahrt_profile_enable(aahrt_plan* plan, int32_t enable);

/*
 * Accumulated time of one kernel kind since the last enable: waits for the recorded
 * events, adds their durations, then reports the totals.
 *   total_ms : host double, milliseconds summed over launches
 *   launches : host int64, number of timed launches
 */
int aahrt_profile_read(aahrt_plan* plan, int32_t kernel, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* AAHRT_H */
